/*
 * spa_oracle.c -- plain, slow CPU oracle for sum-product BP over the BPSK-AWGN
 * channel (the paper's classical channel-coding benchmark of its ZSZ-2BGA
 * codes, Sec. "Classical channel coding" of the numerics appendix).
 *
 * TEST INFRASTRUCTURE ONLY.  Compiled into liboracle.so with rbp_oracle.c; the
 * product library never links, loads or calls it, and it shares no code,
 * header or table with the product library.
 *
 * What it computes:
 *
 *   channel   all-zero codeword, x_j = +1, y_j = 1 + sigma z_j, z_j ~ N(0, 1);
 *             channel LLR_j = 2 y_j / sigma^2.  z comes from Philox4x32-10
 *             (key = seed, counter = (j / 4, shot lo, shot hi, 2)) by the
 *             Box-Muller transform: words 2h and 2h+1 give u1 = (w >> 8 + 1) 2^-24
 *             in (0, 1] and u2 = (w >> 8) 2^-24 in [0, 1), then
 *             r = sqrt(-2 ln u1), z_{4q+2h} = r cos(2 pi u2), z_{4q+2h+1} = r sin(2 pi u2).
 *             Evaluated in double.
 *   decoder   flooding sum-product BP in single precision:
 *               L_j        = clip(LLR_j, +-llr_max)
 *               nu(0)      = L_j on every edge of j
 *               mu_{i->j}  = prod_{j' != j} s(nu_{j'->i}) * phi( sum_{j' != j} phi(|nu_{j'->i}|) )
 *                            (the exclusive sum accumulated over the row's other
 *                            edges in ascending column order; s(x) = -1 iff x < 0)
 *               M_j        = L_j + sum_i mu_{i->j}   (ascending check index)
 *               nu_{j->i}  = clip(M_j - mu_{i->j}, +-llr_max)
 *               c_j        = [M_j < 0]; stop after the first iteration with H c = 0
 *                            (if stopping is on), else after max_iterations
 *             phi(x) = -ln tanh(x / 2) = log1p(2 / expm1(x)), with phi(0) = +inf
 *             and phi(+inf) = 0 as IEEE limits.
 *
 * Compiled with -O2 -ffp-contract=off and no fast-math.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

float orc_spa_phi(float x) { return log1pf(2.0f / expm1f(x)); }

static float clip_llr(float x, float c) { return x > c ? c : (x < -c ? -c : x); }

void orc_awgn(int32_t N, uint64_t shots, double sigma, uint64_t seed, uint64_t offset, double* llr) {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const double two_pi = 6.283185307179586476925286766559;
    for (uint64_t s = 0; s < shots; ++s) {
        const uint64_t sid = offset + s;
        for (int32_t q = 0; 4 * q < N; ++q) {
            const uint32_t ctr[4] = {(uint32_t)q, (uint32_t)sid, (uint32_t)(sid >> 32), 2u};
            uint32_t w[4];
            orc_philox4x32_10(ctr, key, w);
            for (int h = 0; h < 2; ++h) {
                const double u1 = ((double)(w[2 * h] >> 8) + 1.0) * 0x1p-24;
                const double u2 = (double)(w[2 * h + 1] >> 8) * 0x1p-24;
                const double r = sqrt(-2.0 * log(u1));
                const double z[2] = {r * cos(two_pi * u2), r * sin(two_pi * u2)};
                for (int b = 0; b < 2; ++b) {
                    const int32_t j = 4 * q + 2 * h + b;
                    if (j < N) llr[s * (uint64_t)N + (uint64_t)j] = 2.0 * (1.0 + sigma * z[b]) / (sigma * sigma);
                }
            }
        }
    }
}

typedef struct {
    int32_t M, N, E;
    const int32_t *col_ptr, *row_idx; /* CSC of H (input) */
    int32_t *row_ptr, *col_idx;       /* CSR of H, columns ascending in a row */
    int32_t* csc2csr;
} spa_graph;

static int spa_graph_build(spa_graph* g, int32_t M, int32_t N, const int32_t* col_ptr, const int32_t* row_idx) {
    g->M = M; g->N = N; g->E = col_ptr[N]; g->col_ptr = col_ptr; g->row_idx = row_idx;
    g->row_ptr = (int32_t*)calloc((size_t)M + 1, sizeof(int32_t));
    g->col_idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->E > 0 ? g->E : 1));
    g->csc2csr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->E > 0 ? g->E : 1));
    int32_t* fill = (int32_t*)calloc((size_t)M + 1, sizeof(int32_t));
    if (!g->row_ptr || !g->col_idx || !g->csc2csr || !fill) { free(fill); return -4; }
    for (int32_t e = 0; e < g->E; ++e) g->row_ptr[row_idx[e] + 1]++;
    for (int32_t i = 0; i < M; ++i) g->row_ptr[i + 1] += g->row_ptr[i];
    for (int32_t j = 0; j < N; ++j)
        for (int32_t e = col_ptr[j]; e < col_ptr[j + 1]; ++e) {
            const int32_t i = row_idx[e];
            const int32_t pos = g->row_ptr[i] + fill[i]++;
            g->col_idx[pos] = j;
            g->csc2csr[e] = pos;
        }
    free(fill);
    return 0;
}

static void spa_graph_free(spa_graph* g) {
    free(g->row_ptr);
    free(g->col_idx);
    free(g->csc2csr);
}

typedef struct {
    float *L, *nu, *mu, *a, *Mg;
    uint8_t* c;
} spa_work;

/* One shot.  Returns the number of iterations run; *conv = 1 iff H c = 0 at the end. */
static int32_t spa_shot(const spa_graph* g, const float* llr, int32_t T, float llr_max, int32_t stop, spa_work* w,
                        int* conv) {
    const int32_t M = g->M, N = g->N;
    for (int32_t j = 0; j < N; ++j) w->L[j] = clip_llr(llr[j], llr_max);
    for (int32_t e = 0; e < g->E; ++e) w->nu[e] = w->L[g->col_idx[e]];
    *conv = 0;
    int32_t t;
    for (t = 1; t <= T; ++t) {
        /* check -> variable */
        for (int32_t i = 0; i < M; ++i) {
            const int32_t a = g->row_ptr[i], b = g->row_ptr[i + 1];
            for (int32_t e = a; e < b; ++e) w->a[e] = orc_spa_phi(fabsf(w->nu[e]));
            for (int32_t e = a; e < b; ++e) {
                float s = 0.0f;
                int neg = 0;
                for (int32_t f = a; f < b; ++f) {
                    if (f == e) continue;
                    s = s + w->a[f];
                    if (w->nu[f] < 0.0f) neg ^= 1;
                }
                const float m = orc_spa_phi(s);
                w->mu[e] = neg ? -m : m;
            }
        }
        /* marginals and hard decision */
        for (int32_t j = 0; j < N; ++j) {
            float acc = w->L[j];
            for (int32_t e = g->col_ptr[j]; e < g->col_ptr[j + 1]; ++e) acc = acc + w->mu[g->csc2csr[e]];
            w->Mg[j] = acc;
            w->c[j] = acc < 0.0f;
        }
        /* variable -> check (extrinsic, clipped) */
        for (int32_t e = 0; e < g->E; ++e) w->nu[e] = clip_llr(w->Mg[g->col_idx[e]] - w->mu[e], llr_max);
        /* parity of the hard decision */
        int ok = 1;
        for (int32_t i = 0; i < M && ok; ++i) {
            int par = 0;
            for (int32_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) par ^= w->c[g->col_idx[e]];
            if (par) ok = 0;
        }
        if (ok) *conv = 1;
        if (ok && stop) break;
    }
    return t > T ? T : t;
}

typedef struct {
    const spa_graph* g;
    const float* llr;
    int32_t T, stop;
    float llr_max;
    uint8_t *bits, *conv;
    int32_t* iters;
    float* marg;
    uint64_t begin, end;
    int status;
} spa_job;

static void* spa_worker(void* arg) {
    spa_job* J = (spa_job*)arg;
    const spa_graph* g = J->g;
    spa_work w;
    const size_t E = (size_t)(g->E > 0 ? g->E : 1), N = (size_t)g->N;
    w.L = (float*)malloc(sizeof(float) * N);
    w.Mg = (float*)malloc(sizeof(float) * N);
    w.c = (uint8_t*)malloc(N);
    w.nu = (float*)malloc(sizeof(float) * E);
    w.mu = (float*)malloc(sizeof(float) * E);
    w.a = (float*)malloc(sizeof(float) * E);
    if (!w.L || !w.Mg || !w.c || !w.nu || !w.mu || !w.a) {
        J->status = -4;
    } else {
        for (uint64_t s = J->begin; s < J->end; ++s) {
            int conv = 0;
            const int32_t it = spa_shot(g, J->llr + s * N, J->T, J->llr_max, J->stop, &w, &conv);
            memcpy(J->bits + s * N, w.c, N);
            if (J->marg) memcpy(J->marg + s * N, w.Mg, sizeof(float) * N);
            J->conv[s] = (uint8_t)conv;
            J->iters[s] = it;
        }
        J->status = 0;
    }
    free(w.L); free(w.Mg); free(w.c); free(w.nu); free(w.mu); free(w.a);
    return NULL;
}

/* Decode `shots` rows of channel LLRs (float[shots][N]).  Outputs: bits
   uint8[shots][N] (the hard decision at the stop), conv uint8[shots], iters
   int32[shots], and optionally the marginals float[shots][N]. */
int orc_spa_decode(int32_t M, int32_t N, const int32_t* col_ptr, const int32_t* row_idx, const float* llr,
                   uint64_t shots, int32_t max_iterations, float llr_max, int32_t stop, uint8_t* bits, uint8_t* conv,
                   int32_t* iters, float* marg, int32_t nthreads) {
    spa_graph g;
    if (spa_graph_build(&g, M, N, col_ptr, row_idx)) { spa_graph_free(&g); return -4; }
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > shots) nthreads = (int32_t)(shots > 0 ? shots : 1);
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    spa_job* jobs = (spa_job*)calloc((size_t)nthreads, sizeof(spa_job));
    int status = 0;
    const uint64_t per = (shots + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    for (int32_t t = 0; t < nthreads; ++t) {
        spa_job* J = &jobs[t];
        J->g = &g; J->llr = llr; J->T = max_iterations; J->stop = stop; J->llr_max = llr_max;
        J->bits = bits; J->conv = conv; J->iters = iters; J->marg = marg;
        J->begin = (uint64_t)t * per;
        if (J->begin > shots) J->begin = shots;
        J->end = J->begin + per > shots ? shots : J->begin + per;
        pthread_create(&th[t], NULL, spa_worker, J);
    }
    for (int32_t t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].status) status = jobs[t].status;
    }
    free(th); free(jobs);
    spa_graph_free(&g);
    return status;
}
