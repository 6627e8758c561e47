/*
 * rbp_oracle.c -- plain, slow CPU oracle for the Relay-BP Monte-Carlo path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which is
 * loaded by the tests, by the smoke check and by the benchmark's cpu_baseline
 * leg.  The product library never links, loads or calls it, and it shares no
 * code, header or table with the product library.
 *
 * What it computes (paper Sec. 6.1; the decoder is the Relay-BP method the
 * paper cites for its memory experiments, run with flooding schedule,
 * sequential relay legs and single-precision messages):
 *
 *   sampling      independent faults e_j ~ Bernoulli(p_j): the mechanisms are cut
 *                 into 64 segments; in each, candidates follow geometric gaps of
 *                 parameter pmax = max p_j read off an integer table of
 *                 floor((1 - pmax)^k 2^32), and a candidate is kept with
 *                 probability p_j / pmax (integer thresholds); words from
 *                 Philox4x32-10 (see sample_shot)
 *   syndromes     sigma = H e, observables o = O e over GF(2)
 *   LLRs          Lambda_j = (float) ln((1 - p_j) / p_j), evaluated in double
 *   Relay-BP      per shot, legs r = 0..R; leg 0 has memory strength gamma0 for
 *                 every variable and pre_iter iterations; relay legs have
 *                 gamma_j^(r) drawn uniformly from [gamma_min, gamma_max]
 *                 (shared by all shots) and max_iterations iterations; every
 *                 leg restarts its messages and starts from the marginals the
 *                 previous leg ended with.  One flooding iteration:
 *                   mu_{i->j}  = (-1)^sigma_i prod_{j' != j} s(nu_{j'->i})
 *                                min_{j' != j} |nu_{j'->i}|   (min-sum)
 *                   Lt_j       = fmaf(gamma_j, M_j - Lambda_j, Lambda_j)
 *                   M_j        = sat(Lt_j + sum_i mu_{i->j})  (ascending check index)
 *                   nu_{j->i}  = M_j - mu_{i->j}
 *                   e^_j       = [M_j < 0];  converged iff H e^ = sigma
 *                 with s(x) = -1 iff x < 0 and sat(x) = min(max(x, -2^90), 2^90).
 *                 The paper does not say what happens when FP32 messages
 *                 overflow.  Without the saturation, shots that never converge
 *                 reach inf and then NaN (inf - inf) within a few legs, and the
 *                 outcome depends on how an implementation compares NaN; with
 *                 it, every value stays finite (|mu| grows by at most 2^90 per
 *                 iteration, far below the FP32 range for the iteration budgets
 *                 allowed), and shots that stay below 2^90, i.e. every shot
 *                 that converges in practice, are unchanged.  Converged legs give solutions of
 *                 weight W = sum_j e^_j Lambda_j (double); the lowest weight
 *                 wins (ties keep the earlier one).  Stop after stop_nconv
 *                 solutions (criterion 0) or after all legs (criterion 1).
 *                 A zero syndrome returns e^ = 0 directly.
 *
 * Compiled with -O2 -ffp-contract=off and no fast-math, so every float
 * operation above is one IEEE single-precision operation in the stated order.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the        */
/* multiply-hi/lo bijection with key schedule bumped by the Weyl constants.  */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

void orc_llr(int64_t n, const double* p, float* llr) {
    for (int64_t j = 0; j < n; ++j) llr[j] = (float)log((1.0 - p[j]) / p[j]);
}

/* Memory strengths of relay legs r = 1..R: out[(r-1)*N + j]. */
void orc_gamma_table(int32_t N, int32_t R, float gmin, float gmax, uint64_t seed, float* out) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    float span = gmax - gmin;
    for (int32_t r = 1; r <= R; ++r) {
        for (int32_t j = 0; j < N; ++j) {
            uint32_t ctr[4] = {(uint32_t)(j / 4), (uint32_t)r, 0u, 1u};
            uint32_t o[4];
            orc_philox4x32_10(ctr, key, o);
            float u = (float)(o[j % 4] >> 8) * (1.0f / 16777216.0f);
            out[(int64_t)(r - 1) * N + j] = fmaf(u, span, gmin);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Sampling and syndromes                                                     */
/* ------------------------------------------------------------------------- */
static int get_bit(const uint32_t* w, int64_t b) { return (int)((w[b >> 5] >> (b & 31)) & 1u); }
static void flip_bit(uint32_t* w, int64_t b) { w[b >> 5] ^= (1u << (b & 31)); }
static void set_bit(uint32_t* w, int64_t b) { w[b >> 5] |= (1u << (b & 31)); }

/* Geometric gap table of the sampler: T_k = floor((1 - pmax)^k 2^32), k = 1..L,
   with (1 - pmax)^k evaluated as exp(k log1p(-pmax)) in double, at most 2^32 - 1. */
void orc_gap_table(double pmax, int32_t L, uint32_t* T) {
    const double lq = log1p(-pmax);
    for (int32_t k = 1; k <= L; ++k) {
        double t = floor(exp((double)k * lq) * 4294967296.0);
        T[k - 1] = t >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)t;
    }
}

/* Acceptance thresholds: A_j = floor(p_j / pmax 2^32) (at most 2^32 - 2) when
   p_j < pmax; 0xFFFFFFFF marks p_j = pmax (accepted without a draw). */
void orc_accept_table(int64_t n, const double* p, double pmax, uint32_t* A) {
    for (int64_t j = 0; j < n; ++j) {
        if (p[j] >= pmax) { A[j] = 0xFFFFFFFFu; continue; }
        double t = floor(p[j] / pmax * 4294967296.0);
        A[j] = t >= 4294967294.0 ? 0xFFFFFFFEu : (uint32_t)t;
    }
}

/* Faults of one shot.  The N mechanisms are cut into 64 segments of
   L = ceil(N / 64); in each, candidate positions follow geometric gaps of
   parameter pmax (gap G = number of k in 1..len with T_k > w for the next
   word w), and a candidate j with p_j < pmax is kept when the next word is
   below A_j.  Words of segment g come from Philox4x32-10 with key = seed and
   counter (g 2^24 + d / 4, shot lo, shot hi, 3), word d mod 4, d = 0, 1, ... */
static void sample_shot(int32_t N, const uint32_t* T, const uint32_t* A, const uint32_t key[2], uint64_t sid,
                        void (*fault)(int32_t j, void* ctx), void* ctx) {
    const int32_t L = (N + 63) / 64;
    for (int32_t g = 0; g < 64; ++g) {
        const int32_t base = g * L;
        const int32_t len = N - base < L ? N - base : L;
        if (len <= 0) break;
        uint32_t buf[4];
        int64_t d = 0, have = -1;
        int32_t pos = -1;
        for (;;) {
            if (d / 4 != have) {
                const uint32_t ctr[4] = {((uint32_t)g << 24) + (uint32_t)(d / 4), (uint32_t)sid,
                                         (uint32_t)(sid >> 32), 3u};
                orc_philox4x32_10(ctr, key, buf);
                have = d / 4;
            }
            const uint32_t w = buf[d % 4];
            ++d;
            int32_t G = 0;
            while (G < len && T[G] > w) ++G; /* T[G] is T_{G+1} */
            pos += G + 1;
            if (pos >= len) break;
            const int32_t j = base + pos;
            if (A[j] != 0xFFFFFFFFu) {
                if (d / 4 != have) {
                    const uint32_t ctr[4] = {((uint32_t)g << 24) + (uint32_t)(d / 4), (uint32_t)sid,
                                             (uint32_t)(sid >> 32), 3u};
                    orc_philox4x32_10(ctr, key, buf);
                    have = d / 4;
                }
                const uint32_t a = buf[d % 4];
                ++d;
                if (a >= A[j]) continue;
            }
            fault(j, ctx);
        }
    }
}

typedef struct {
    const int32_t *col_ptr, *row_idx, *ocol_ptr, *orow_idx;
    uint32_t *sy, *ob, *er;
} fault_ctx;

static void apply_fault(int32_t j, void* vctx) {
    fault_ctx* c = (fault_ctx*)vctx;
    for (int32_t e = c->col_ptr[j]; e < c->col_ptr[j + 1]; ++e) flip_bit(c->sy, c->row_idx[e]);
    for (int32_t e = c->ocol_ptr[j]; e < c->ocol_ptr[j + 1]; ++e) flip_bit(c->ob, c->orow_idx[e]);
    if (c->er) set_bit(c->er, j);
}

int orc_sample(int32_t M, int32_t N, const int32_t* col_ptr, const int32_t* row_idx, int32_t k,
               const int32_t* ocol_ptr, const int32_t* orow_idx, const double* priors, uint64_t shots,
               uint64_t seed, uint64_t shot_offset, uint32_t* synd, uint32_t* obs, uint32_t* err) {
    int64_t wm = (M + 31) / 32, wk = (k + 31) / 32, wn = (N + 31) / 32;
    const int32_t L = (N + 63) / 64;
    double pmax = 0.0;
    for (int32_t j = 0; j < N; ++j) pmax = priors[j] > pmax ? priors[j] : pmax;
    uint32_t* T = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(L > 0 ? L : 1));
    uint32_t* A = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(N > 0 ? N : 1));
    if (!T || !A) { free(T); free(A); return -4; }
    orc_gap_table(pmax, L, T);
    orc_accept_table(N, priors, pmax, A);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint64_t s = 0; s < shots; ++s) {
        fault_ctx c = {col_ptr, row_idx, ocol_ptr, orow_idx, synd + s * wm, obs + s * wk,
                       err ? err + s * wn : NULL};
        memset(c.sy, 0, sizeof(uint32_t) * wm);
        memset(c.ob, 0, sizeof(uint32_t) * wk);
        if (c.er) memset(c.er, 0, sizeof(uint32_t) * wn);
        sample_shot(N, T, A, key, shot_offset + s, apply_fault, &c);
    }
    free(T);
    free(A);
    return 0;
}

/* The plain definition of the fault law, kept beside the gap sampler as the
   reference its law is pinned against: each mechanism j draws its own word,
   word (j mod 4) of Philox4x32-10 with key = seed and counter
   (j / 4, shot lo, shot hi, 0), and faults iff that word is below
   thr_j = min(floor(p_j 2^32), 2^32 - 1).  One Philox call per four
   mechanisms, so P(fault) = thr_j / 2^32 exactly, independently over j and
   shots.  (A different stream from the gap sampler's: the two draw different
   faults, with the same law.) */
int orc_sample_plain(int32_t N, const double* priors, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                     uint32_t* err) {
    int64_t wn = (N + 31) / 32;
    uint32_t* thr = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(N > 0 ? N : 1));
    if (!thr) return -4;
    for (int32_t j = 0; j < N; ++j) {
        double t = floor(priors[j] * 4294967296.0);
        thr[j] = t >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)t;
    }
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint64_t s = 0; s < shots; ++s) {
        const uint64_t sid = shot_offset + s;
        uint32_t* e = err + s * wn;
        memset(e, 0, sizeof(uint32_t) * (size_t)wn);
        for (int32_t j = 0; j < N; ++j) {
            uint32_t w[4];
            const uint32_t ctr[4] = {(uint32_t)(j / 4), (uint32_t)sid, (uint32_t)(sid >> 32), 0u};
            orc_philox4x32_10(ctr, key, w);
            if (w[j % 4] < thr[j]) set_bit(e, j);
        }
    }
    free(thr);
    return 0;
}

/* sigma = H e and o = O e for given error words (used to pin the syndrome map). */
void orc_syndrome(int32_t M, int32_t N, const int32_t* col_ptr, const int32_t* row_idx, uint64_t shots,
                  const uint32_t* err, uint32_t* synd) {
    int64_t wm = (M + 31) / 32, wn = (N + 31) / 32;
    for (uint64_t s = 0; s < shots; ++s) {
        uint32_t* sy = synd + s * wm;
        memset(sy, 0, sizeof(uint32_t) * wm);
        for (int32_t j = 0; j < N; ++j)
            if (get_bit(err + s * wn, j))
                for (int32_t e = col_ptr[j]; e < col_ptr[j + 1]; ++e) flip_bit(sy, row_idx[e]);
    }
}

/* ------------------------------------------------------------------------- */
/* Relay-BP                                                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    float gamma0, gamma_min, gamma_max;
    int32_t pre_iter, max_iterations, num_sets, stop_nconv, stopping_criterion;
    uint64_t gamma_seed;
} orc_params;

typedef struct {
    int32_t M, N, E, k;
    const int32_t *col_ptr, *row_idx;   /* CSC of H (input) */
    int32_t *row_ptr, *col_idx;         /* CSR of H (built here) */
    int32_t* csc2csr;                   /* CSC edge -> CSR edge */
    const int32_t *ocol_ptr, *orow_idx; /* CSC of O */
} orc_graph;

static int graph_build(orc_graph* g, int32_t M, int32_t N, const int32_t* col_ptr, const int32_t* row_idx,
                       int32_t k, const int32_t* ocol_ptr, const int32_t* orow_idx) {
    g->M = M; g->N = N; g->E = col_ptr[N]; g->k = k;
    g->col_ptr = col_ptr; g->row_idx = row_idx; g->ocol_ptr = ocol_ptr; g->orow_idx = orow_idx;
    g->row_ptr = (int32_t*)calloc((size_t)M + 1, sizeof(int32_t));
    g->col_idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->E > 0 ? g->E : 1));
    g->csc2csr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->E > 0 ? g->E : 1));
    int32_t* fill = (int32_t*)calloc((size_t)M + 1, sizeof(int32_t));
    if (!g->row_ptr || !g->col_idx || !g->csc2csr || !fill) return -4;
    for (int32_t e = 0; e < g->E; ++e) g->row_ptr[row_idx[e] + 1]++;
    for (int32_t i = 0; i < M; ++i) g->row_ptr[i + 1] += g->row_ptr[i];
    /* visiting columns in ascending order keeps each row's columns ascending */
    for (int32_t j = 0; j < N; ++j)
        for (int32_t e = col_ptr[j]; e < col_ptr[j + 1]; ++e) {
            int32_t i = row_idx[e];
            int32_t pos = g->row_ptr[i] + fill[i]++;
            g->col_idx[pos] = j;
            g->csc2csr[e] = pos;
        }
    free(fill);
    return 0;
}

static void graph_free(orc_graph* g) {
    free(g->row_ptr);
    free(g->col_idx);
    free(g->csc2csr);
}

typedef struct {
    float *Mg, *nu, *mu, *lamL;
    uint8_t *ehat, *best, *sig;
} shot_work;

static int sgn_neg(float x) { return x < 0.0f; }

/* saturation bound of the marginals, 2^90 */
#define ORC_M_SAT 0x1p90f

/* One flooding iteration on the current leg.  Returns 1 iff H e^ = sigma after it. */
static int bp_iteration(const orc_graph* g, shot_work* w, const float* gam, float gamma_const, int use_const) {
    const int32_t M = g->M, N = g->N;
    /* check -> variable messages from the variable -> check messages of t-1 */
    for (int32_t i = 0; i < M; ++i) {
        int32_t a = g->row_ptr[i], b = g->row_ptr[i + 1];
        for (int32_t e = a; e < b; ++e) {
            int neg = w->sig[i];
            float mn = INFINITY;
            for (int32_t f = a; f < b; ++f) {
                if (f == e) continue;
                float v = w->nu[f];
                if (sgn_neg(v)) neg ^= 1;
                float av = fabsf(v);
                if (av < mn) mn = av;
            }
            w->mu[e] = neg ? -mn : mn;
        }
    }
    /* marginals with the memory prior */
    for (int32_t j = 0; j < N; ++j) {
        float gj = use_const ? gamma_const : gam[j];
        float lam = w->lamL[j];
        float d = w->Mg[j] - lam;
        float acc = fmaf(gj, d, lam);
        for (int32_t e = g->col_ptr[j]; e < g->col_ptr[j + 1]; ++e) acc = acc + w->mu[g->csc2csr[e]];
        if (acc > ORC_M_SAT) acc = ORC_M_SAT;
        if (acc < -ORC_M_SAT) acc = -ORC_M_SAT;
        w->Mg[j] = acc;
        w->ehat[j] = acc < 0.0f;
    }
    /* variable -> check messages (extrinsic, subtractive form) */
    for (int32_t i = 0; i < M; ++i)
        for (int32_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e)
            w->nu[e] = w->Mg[g->col_idx[e]] - w->mu[e];
    /* syndrome check */
    for (int32_t i = 0; i < M; ++i) {
        int par = w->sig[i];
        for (int32_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) par ^= w->ehat[g->col_idx[e]];
        if (par) return 0;
    }
    return 1;
}

typedef struct {
    uint8_t converged, nconv, path;
    int32_t legs, iters;
} shot_result;

/* Trace request: stop after iteration trace_t of leg trace_leg of phase trace_phase. */
typedef struct {
    int active, phase, leg, t, hit;
    float *M_out, *mu_out; /* mu in CSC edge order */
} trace_req;

/* Runs one decode phase (plain Relay-BP from leg 0, or the single proposal leg).
   Returns the number of solutions found; updates best/bestW. */
static int run_phase(const orc_graph* g, shot_work* w, const float* lam, const float* lam_leg0,
                     const float* gtab, const orc_params* prm, int phase, int proposal_only,
                     double* bestW, int* have_best, shot_result* res, trace_req* tr) {
    const int32_t N = g->N, E = g->E;
    int nconv = 0;
    int legs_total = proposal_only ? 0 : prm->num_sets;
    for (int32_t j = 0; j < N; ++j) w->Mg[j] = lam_leg0[j];
    for (int32_t leg = 0; leg <= legs_total; ++leg) {
        const float* lamL = leg == 0 ? lam_leg0 : lam;
        memcpy(w->lamL, lamL, sizeof(float) * (size_t)N);
        for (int32_t e = 0; e < E; ++e) w->nu[e] = lamL[g->col_idx[e]];
        int32_t T = leg == 0 ? prm->pre_iter : prm->max_iterations;
        const float* gam = leg == 0 ? NULL : gtab + (int64_t)(leg - 1) * N;
        int conv = 0;
        res->legs++;
        for (int32_t t = 1; t <= T; ++t) {
            conv = bp_iteration(g, w, gam, prm->gamma0, leg == 0);
            res->iters++;
            if (tr && tr->active && tr->phase == phase && tr->leg == leg && tr->t == t) {
                memcpy(tr->M_out, w->Mg, sizeof(float) * (size_t)N);
                for (int32_t e = 0; e < E; ++e) tr->mu_out[e] = w->mu[g->csc2csr[e]];
                tr->hit = 1;
                return -1;
            }
            if (conv) break;
        }
        if (conv) {
            double W = 0.0;
            for (int32_t j = 0; j < N; ++j)
                if (w->ehat[j]) W += (double)lam[j];
            if (!*have_best || W < *bestW) {
                *bestW = W;
                *have_best = 1;
                memcpy(w->best, w->ehat, (size_t)N);
            }
            nconv++;
            if (prm->stopping_criterion == 0 && nconv >= prm->stop_nconv) break;
        }
    }
    return nconv;
}

static void decode_shot(const orc_graph* g, const float* lam, const float* gtab, const orc_params* prm,
                        const uint32_t* syn_words, const float* delta, shot_work* w, uint32_t* corr,
                        uint32_t* obsp, shot_result* res, trace_req* tr) {
    const int32_t M = g->M, N = g->N, k = g->k;
    memset(res, 0, sizeof(*res));
    int any = 0;
    for (int32_t i = 0; i < M; ++i) {
        w->sig[i] = (uint8_t)get_bit(syn_words, i);
        any |= w->sig[i];
    }
    memset(corr, 0, sizeof(uint32_t) * (size_t)((N + 31) / 32));
    memset(obsp, 0, sizeof(uint32_t) * (size_t)((k + 31) / 32));
    if (!any) {
        res->converged = 1;
        res->path = 3;
        return;
    }
    double bestW = 0.0;
    int have_best = 0;
    int nconv = 0;
    int path = 0;
    if (delta) {
        /* proposal leg: leg 0 with the adjusted priors Lambda + delta */
        float* lp = (float*)malloc(sizeof(float) * (size_t)N);
        for (int32_t j = 0; j < N; ++j) lp[j] = lam[j] + delta[j];
        nconv = run_phase(g, w, lam, lp, gtab, prm, 1, 1, &bestW, &have_best, res, tr);
        free(lp);
        if (nconv < 0) return;
        path = nconv > 0 ? 1 : 2;
    }
    if (!delta || nconv == 0) {
        nconv = run_phase(g, w, lam, lam, gtab, prm, 0, 0, &bestW, &have_best, res, tr);
        if (nconv < 0) return;
    }
    res->path = (uint8_t)path;
    res->nconv = (uint8_t)(nconv > 255 ? 255 : nconv);
    res->converged = (uint8_t)(have_best != 0);
    const uint8_t* out = have_best ? w->best : w->ehat;
    for (int32_t j = 0; j < N; ++j)
        if (out[j]) {
            set_bit(corr, j);
            for (int32_t e = g->ocol_ptr[j]; e < g->ocol_ptr[j + 1]; ++e) flip_bit(obsp, g->orow_idx[e]);
        }
}

static int work_alloc(shot_work* w, const orc_graph* g) {
    size_t N = (size_t)g->N + 1, E = (size_t)g->E + 1, M = (size_t)g->M + 1;
    w->Mg = (float*)malloc(sizeof(float) * N);
    w->lamL = (float*)malloc(sizeof(float) * N);
    w->nu = (float*)malloc(sizeof(float) * E);
    w->mu = (float*)malloc(sizeof(float) * E);
    w->ehat = (uint8_t*)calloc(N, 1);
    w->best = (uint8_t*)calloc(N, 1);
    w->sig = (uint8_t*)calloc(M, 1);
    return (w->Mg && w->lamL && w->nu && w->mu && w->ehat && w->best && w->sig) ? 0 : -4;
}

static void work_free(shot_work* w) {
    free(w->Mg); free(w->lamL); free(w->nu); free(w->mu); free(w->ehat); free(w->best); free(w->sig);
}

typedef struct {
    const orc_graph* g;
    const float *lam, *gtab, *delta;
    const orc_params* prm;
    const uint32_t* syn;
    uint32_t *corr, *obsp;
    uint8_t *conv, *nconv, *path;
    int32_t *legs, *iters;
    double* seconds;
    uint64_t begin, end;
    int status;
} job;

#include <time.h>
static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static void* worker(void* arg) {
    job* J = (job*)arg;
    const orc_graph* g = J->g;
    shot_work w;
    if (work_alloc(&w, g)) { J->status = -4; work_free(&w); return NULL; }
    int64_t wm = (g->M + 31) / 32, wn = (g->N + 31) / 32, wk = (g->k + 31) / 32;
    for (uint64_t s = J->begin; s < J->end; ++s) {
        shot_result r;
        double t0 = J->seconds ? now_s() : 0.0;
        decode_shot(g, J->lam, J->gtab, J->prm, J->syn + s * wm, J->delta ? J->delta + s * (uint64_t)g->N : NULL,
                    &w, J->corr + s * wn, J->obsp + s * wk, &r, NULL);
        if (J->seconds) J->seconds[s] = now_s() - t0;
        if (J->conv) J->conv[s] = r.converged;
        if (J->nconv) J->nconv[s] = r.nconv;
        if (J->path) J->path[s] = r.path;
        if (J->legs) J->legs[s] = r.legs;
        if (J->iters) J->iters[s] = r.iters;
    }
    work_free(&w);
    J->status = 0;
    return NULL;
}

int orc_decode(int32_t M, int32_t N, const int32_t* col_ptr, const int32_t* row_idx, int32_t k,
               const int32_t* ocol_ptr, const int32_t* orow_idx, const double* priors, const uint32_t* syn,
               uint64_t shots, const orc_params* prm, const float* delta, uint32_t* corr, uint32_t* obsp,
               uint8_t* conv, uint8_t* nconv, uint8_t* path, int32_t* legs, int32_t* iters, double* seconds,
               int32_t nthreads) {
    orc_graph g;
    if (graph_build(&g, M, N, col_ptr, row_idx, k, ocol_ptr, orow_idx)) { graph_free(&g); return -4; }
    float* lam = (float*)malloc(sizeof(float) * (size_t)(N + 1));
    float* gtab = (float*)malloc(sizeof(float) * ((size_t)N * (size_t)(prm->num_sets > 0 ? prm->num_sets : 1) + 1));
    if (!lam || !gtab) { free(lam); free(gtab); graph_free(&g); return -4; }
    orc_llr(N, priors, lam);
    orc_gamma_table(N, prm->num_sets, prm->gamma_min, prm->gamma_max, prm->gamma_seed, gtab);
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > shots) nthreads = (int32_t)(shots > 0 ? shots : 1);
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    job* jobs = (job*)calloc((size_t)nthreads, sizeof(job));
    int status = 0;
    /* interleaved chunks keep the threads evenly loaded */
    uint64_t per = (shots + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    for (int32_t t = 0; t < nthreads; ++t) {
        job* J = &jobs[t];
        J->g = &g; J->lam = lam; J->gtab = gtab; J->delta = delta; J->prm = prm; J->syn = syn;
        J->corr = corr; J->obsp = obsp; J->conv = conv; J->nconv = nconv; J->path = path;
        J->legs = legs; J->iters = iters; J->seconds = seconds;
        J->begin = (uint64_t)t * per;
        J->end = J->begin + per > shots ? shots : J->begin + per;
        if (J->begin > shots) J->begin = shots;
        pthread_create(&th[t], NULL, worker, J);
    }
    for (int32_t t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].status) status = jobs[t].status;
    }
    free(th); free(jobs); free(lam); free(gtab);
    graph_free(&g);
    return status;
}

/* Marginals M (N floats) and check->variable messages (nnz floats, CSC edge
   order) right after iteration t of leg `leg` in phase `phase` (0 plain,
   1 proposal) of one shot.  Returns 1 if that point was reached, 0 if the
   decode finished earlier, <0 on error. */
int orc_trace(int32_t M, int32_t N, const int32_t* col_ptr, const int32_t* row_idx, int32_t k,
              const int32_t* ocol_ptr, const int32_t* orow_idx, const double* priors, const uint32_t* syn,
              const orc_params* prm, const float* delta, int32_t phase, int32_t leg, int32_t t, float* M_out,
              float* mu_out) {
    orc_graph g;
    if (graph_build(&g, M, N, col_ptr, row_idx, k, ocol_ptr, orow_idx)) { graph_free(&g); return -4; }
    float* lam = (float*)malloc(sizeof(float) * (size_t)(N + 1));
    float* gtab = (float*)malloc(sizeof(float) * ((size_t)N * (size_t)(prm->num_sets > 0 ? prm->num_sets : 1) + 1));
    shot_work w;
    if (!lam || !gtab || work_alloc(&w, &g)) { free(lam); free(gtab); graph_free(&g); return -4; }
    orc_llr(N, priors, lam);
    orc_gamma_table(N, prm->num_sets, prm->gamma_min, prm->gamma_max, prm->gamma_seed, gtab);
    trace_req tr = {1, phase, leg, t, 0, M_out, mu_out};
    uint32_t* corr = (uint32_t*)calloc((size_t)(N + 31) / 32 + 1, 4);
    uint32_t* obsp = (uint32_t*)calloc((size_t)(k + 31) / 32 + 1, 4);
    shot_result r;
    decode_shot(&g, lam, gtab, prm, syn, delta, &w, corr, obsp, &r, &tr);
    int hit = tr.hit;
    free(corr); free(obsp); work_free(&w); free(lam); free(gtab);
    graph_free(&g);
    return hit;
}

/* Marginals after T flooding iterations of one leg with a constant memory
   strength, starting from M = nu = Lambda and ignoring convergence.  This runs
   the same iteration as the decoder and exists to pin its arithmetic. */
int orc_bp_marginals(int32_t M, int32_t N, const int32_t* col_ptr, const int32_t* row_idx, const double* priors,
                     const uint32_t* syn, float gamma, int32_t T, float* M_out) {
    orc_graph g;
    if (graph_build(&g, M, N, col_ptr, row_idx, 0, col_ptr, row_idx)) { graph_free(&g); return -4; }
    shot_work w;
    float* lam = (float*)malloc(sizeof(float) * (size_t)(N + 1));
    if (!lam || work_alloc(&w, &g)) { free(lam); graph_free(&g); return -4; }
    orc_llr(N, priors, lam);
    for (int32_t i = 0; i < M; ++i) w.sig[i] = (uint8_t)get_bit(syn, i);
    memcpy(w.lamL, lam, sizeof(float) * (size_t)N);
    memcpy(w.Mg, lam, sizeof(float) * (size_t)N);
    for (int32_t e = 0; e < g.E; ++e) w.nu[e] = lam[g.col_idx[e]];
    for (int32_t t = 1; t <= T; ++t) (void)bp_iteration(&g, &w, NULL, gamma, 1);
    memcpy(M_out, w.Mg, sizeof(float) * (size_t)N);
    work_free(&w);
    free(lam);
    graph_free(&g);
    return 0;
}
