// librbp: sampling and Relay-BP decoding kernels for gfx950, and their C ABI.
//
// Paper Sec. 6.1: syndromes of a detector error model are decoded with Relay-BP
// (flooding min-sum with memory, sequential relay legs, lowest weight of
// stop_nconv solutions, FP32 messages).  The work here is organised for CDNA4:
//
//  * sample_kernel     one wavefront per shot; counter-based Philox draws four
//                      mechanisms per call; the rare faults XOR their detector
//                      and observable columns into LDS bit arrays.
//  * relay_bp_kernel   persistent: each workgroup is a shot slot that pulls shots
//                      from a device queue until none are left, so a shot that
//                      converges early frees its slot at once.  The slot's
//                      per-shot state (marginals M[N], check->variable messages
//                      mu[nnz] in CSR order) sits in LDS when it fits, else in a
//                      per-slot device buffer.  One flooding iteration is a check
//                      sweep over CSR rows (min / second-min / sign parity kept in
//                      registers; a check's new messages are written to its own
//                      contiguous CSR slots) and a variable sweep over CSC columns
//                      (memory prior, marginal, hard decision).  The syndrome of
//                      the hard decision is tracked incrementally: a variable
//                      whose decision flips XORs its checks' parity bits with LDS
//                      atomics and the workgroup keeps the count of unsatisfied
//                      checks, so convergence costs no extra sweep.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rbp_common.h"

namespace rbp {

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
rbp_status fail(rbp_status st, const std::string& m) {
    g_err = m;
    return st;
}

rbp_status DevBuf::reserve(size_t n) {
    if (n <= bytes && p) return RBP_OK;
    if (p) {
        hipError_t e = hipFree(p);
        p = nullptr;
        bytes = 0;
        if (e != hipSuccess) return fail(RBP_ERR_HIP, std::string("hipFree: ") + hipGetErrorString(e));
    }
    size_t want = n ? n : 4;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        p = nullptr;
        return fail(e == hipErrorOutOfMemory ? RBP_ERR_OOM : RBP_ERR_HIP,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    bytes = want;
    return RBP_OK;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

// ---------------------------------------------------------------------------
// Sampling: e_j = [Philox(seed; j/4, shot, 0)_{j%4} < thr_j]; sigma = H e; o = O e
// ---------------------------------------------------------------------------
struct SampleArgs {
    int32_t M, N, k, WM, WK, WN;
    const int32_t* col_ptr;
    const int32_t* csc_row;
    const int32_t* ocol_ptr;
    const int32_t* orow_idx;
    const uint32_t* thr;
    uint64_t shots, seed, offset;
    uint32_t* syn;
    uint32_t* obs;
    uint32_t* err;
};

constexpr int kSampleWaves = 4;

__global__ void __launch_bounds__(64 * kSampleWaves) sample_kernel(const SampleArgs a) {
    extern __shared__ uint32_t sm_sample[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t s = (uint64_t)blockIdx.x * kSampleWaves + wid;
    const bool live = s < a.shots;
    const int words = a.WM + a.WK;
    uint32_t* sy = sm_sample + wid * words;
    uint32_t* ob = sy + a.WM;
    for (int x = lane; x < words; x += 64) sy[x] = 0u;
    __syncthreads();
    const uint64_t sid = a.offset + s;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const int nq = (a.N + 3) >> 2;
    for (int qb = 0; qb < nq; qb += 64) {
        const int q = qb + lane;
        uint32_t nib = 0;
        if (live && q < nq) {
            const U4 r = philox4x32_10(U4{(uint32_t)q, (uint32_t)sid, (uint32_t)(sid >> 32), 0u}, k0, k1);
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int j = 4 * q + w;
                if (j < a.N && u4_get(r, w) < a.thr[j]) {
                    nib |= 1u << w;
                    for (int e = a.col_ptr[j]; e < a.col_ptr[j + 1]; ++e) {
                        const int i = a.csc_row[e];
                        atomicXor(sy + (i >> 5), 1u << (i & 31));
                    }
                    for (int e = a.ocol_ptr[j]; e < a.ocol_ptr[j + 1]; ++e) {
                        const int i = a.orow_idx[e];
                        atomicXor(ob + (i >> 5), 1u << (i & 31));
                    }
                }
            }
        }
        if (a.err) {
            // eight consecutive lanes hold the eight nibbles of one 32-bit word
            uint32_t v = nib << (4 * (lane & 7));
            v |= __shfl_xor(v, 1);
            v |= __shfl_xor(v, 2);
            v |= __shfl_xor(v, 4);
            if (live && (lane & 7) == 0 && q < nq) a.err[s * a.WN + (q >> 3)] = v;
        }
    }
    __syncthreads();
    if (live) {
        for (int x = lane; x < a.WM; x += 64) a.syn[s * a.WM + x] = sy[x];
        if (a.obs)
            for (int x = lane; x < a.WK; x += 64) a.obs[s * a.WK + x] = ob[x];
    }
}

// ---------------------------------------------------------------------------
// Relay-leg memory strengths gamma_j^(r), r = 1..R: table[(r-1)*N + j]
// ---------------------------------------------------------------------------
__global__ void gamma_table_kernel(float* out, int32_t N, int32_t R, float gmin, float gmax, uint64_t seed) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)N * R;
    if (idx >= total) return;
    const int32_t r = (int32_t)(idx / N) + 1, j = (int32_t)(idx % N);
    const U4 o = philox4x32_10(U4{(uint32_t)(j >> 2), (uint32_t)r, 0u, 1u}, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float u = (float)(u4_get(o, j & 3) >> 8) * (1.0f / 16777216.0f);
    const float span = gmax - gmin;
    out[idx] = __builtin_fmaf(u, span, gmin);
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------------------
// Persistent Relay-BP
// ---------------------------------------------------------------------------
constexpr int kMaxModels = 8;

struct DecodeModel {
    int32_t M, N, E, k, WM, WN, WK;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const int32_t* col_ptr;
    const int32_t* csc_row;
    const int32_t* csc_edge;
    const int32_t* orow_ptr;
    const int32_t* ocol_idx;
    const float* lam;
    const float* gtab;
    const uint32_t* syn;
    uint32_t* corr;
    uint32_t* obsp;
};

struct DecodeLaunch {
    DecodeModel m[kMaxModels];
    int32_t n_models;
    const uint8_t* shot_code;
    const uint32_t* shot_index;
    uint64_t shots;
    const float* delta;
    rbp_shot_stats* stats;
    unsigned long long* queue;
    float* gstate;
    int64_t gstate_stride;
    int32_t Nmax;
    int32_t off_sig, off_par, off_best;  // byte offsets in dynamic LDS
    float gamma0;
    int32_t T0, Tr, R, S, crit;
    int32_t trace_on, trace_phase, trace_leg, trace_t;
    float* trace_M;
    float* trace_mu;
    int32_t* trace_hit;
};

template <class T>
__device__ __forceinline__ T block_sum(T v, T* red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    T s = 0;
    for (int i = 0; i < nw; ++i) s += red[i];
    __syncthreads();
    return s;
}

// Packs the hard decisions [M_j < 0] into bit words with one ballot per wave.
__device__ __forceinline__ void capture_decisions(const float* Ms, uint32_t* bits, int N, int WN) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int jb = wid * 64; jb < N; jb += blockDim.x) {
        const int j = jb + lane;
        const bool neg = j < N && Ms[j] < 0.0f;
        const unsigned long long b = __ballot(neg);
        if (lane == 0) {
            bits[jb >> 5] = (uint32_t)b;
            if ((jb >> 5) + 1 < WN) bits[(jb >> 5) + 1] = (uint32_t)(b >> 32);
        }
    }
}

template <int MAXDEG, bool LDS_STATE>
__global__ void __launch_bounds__(1024) relay_bp_kernel(const DecodeLaunch a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long sh_shot;
    __shared__ int sh_count;
    __shared__ double sh_red_d[16];
    __shared__ int sh_red_i[16];

    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63;
    float* Ms;
    if constexpr (LDS_STATE) {
        Ms = reinterpret_cast<float*>(smem);
    } else {
        Ms = a.gstate + (int64_t)blockIdx.x * a.gstate_stride;
    }
    float* mu = Ms + a.Nmax;
    uint32_t* sig = reinterpret_cast<uint32_t*>(smem + a.off_sig);
    uint32_t* par = reinterpret_cast<uint32_t*>(smem + a.off_par);
    uint32_t* best = reinterpret_cast<uint32_t*>(smem + a.off_best);

    for (;;) {
        if (tid == 0) sh_shot = atomicAdd(a.queue, 1ull);
        __syncthreads();
        const unsigned long long s = sh_shot;
        if (s >= a.shots) break;
        const uint64_t t_start = wall_clock64();
        const int mi = a.shot_code ? (int)a.shot_code[s] : 0;
        const DecodeModel& m = a.m[mi];
        const uint64_t row = a.shot_index ? (uint64_t)a.shot_index[s] : (uint64_t)s;
        const int M = m.M, N = m.N, WM = m.WM, WN = m.WN;
        const float* lam = m.lam;
        const float* dlt = a.delta ? a.delta + row * (uint64_t)N : nullptr;

        // syndrome into LDS, parity := sigma, count of unsatisfied checks
        if (tid == 0) sh_count = 0;
        int pc = 0;
        for (int w = tid; w < WM; w += nth) {
            const uint32_t v = m.syn[row * WM + w];
            sig[w] = v;
            par[w] = v;
            pc += __popc(v);
        }
        const int base_sig = block_sum<int>(pc, sh_red_i);

        int nconv = 0, legs = 0, iters = 0, path = 0;
        bool have_best = false;
        double bestW = 0.0;
        bool traced = false;
        int base = base_sig;

        if (base_sig == 0) {
            path = 3;
            have_best = true;
            for (int w = tid; w < WN; w += nth) best[w] = 0u;
            __syncthreads();
        } else {
            const int first_phase = dlt ? 1 : 0;
            for (int phase = first_phase; phase >= 0; --phase) {
                const bool prop = phase == 1;
                if (phase == 0 && first_phase == 1) {
                    // plain Relay-BP from scratch after a failed proposal
                    __syncthreads();
                    if (tid == 0) sh_count = 0;
                    for (int w = tid; w < WM; w += nth) par[w] = sig[w];
                    __syncthreads();
                    base = base_sig;
                }
                // M(0) = Lambda (or Lambda + delta); parity := sigma xor H [M(0) < 0]
                int dc = 0;
                for (int j = tid; j < N; j += nth) {
                    const float v = prop ? lam[j] + dlt[j] : lam[j];
                    Ms[j] = v;
                    if (v < 0.0f) {
                        for (int e = m.col_ptr[j]; e < m.col_ptr[j + 1]; ++e) {
                            const int i = m.csc_row[e];
                            const uint32_t bit = 1u << (i & 31);
                            const uint32_t old = atomicXor(par + (i >> 5), bit);
                            dc += (old & bit) ? -1 : 1;
                        }
                    }
                }
                if (dc) atomicAdd(&sh_count, dc);
                __syncthreads();

                const int nlegs = prop ? 0 : a.R;
                for (int leg = 0; leg <= nlegs; ++leg) {
                    const bool leg0 = leg == 0;
                    const bool lp = prop && leg0;  // priors of this leg are Lambda + delta
                    const int T = leg0 ? a.T0 : a.Tr;
                    const float* gam = leg0 ? nullptr : m.gtab + (int64_t)(leg - 1) * N;
                    bool conv = false;
                    ++legs;
                    for (int t = 1; t <= T; ++t) {
                        const bool first = t == 1;
                        // ---- check sweep: mu(t) from nu(t-1) = M(t-1) - mu(t-1) (or the priors at t = 1)
                        for (int i = tid; i < M; i += nth) {
                            const int rs = m.row_ptr[i];
                            const int deg = m.row_ptr[i + 1] - rs;
                            uint32_t sgn = ((sig[i >> 5] >> (i & 31)) & 1u) << 31;
                            float min1 = INFINITY, min2 = INFINITY;
                            float nu[MAXDEG];
#pragma unroll
                            for (int p = 0; p < MAXDEG; ++p) {
                                if (p < deg) {
                                    const int j = m.col_idx[rs + p];
                                    float v;
                                    if (first) {
                                        v = lp ? lam[j] + dlt[j] : lam[j];
                                    } else {
                                        v = Ms[j] - mu[rs + p];
                                    }
                                    nu[p] = v;
                                    sgn ^= __float_as_uint(v);
                                    const float av = fabsf(v);
                                    min2 = __builtin_amdgcn_fmed3f(min1, min2, av);
                                    min1 = fminf(min1, av);
                                }
                            }
#pragma unroll
                            for (int p = 0; p < MAXDEG; ++p) {
                                if (p < deg) {
                                    const float av = fabsf(nu[p]);
                                    const float mag = (av == min1) ? min2 : min1;
                                    const uint32_t sb = (sgn ^ __float_as_uint(nu[p])) & 0x80000000u;
                                    mu[rs + p] = __uint_as_float(__float_as_uint(mag) | sb);
                                }
                            }
                        }
                        __syncthreads();
                        // ---- variable sweep: memory prior, marginal, decision flips
                        int dcount = 0;
                        for (int j = tid; j < N; j += nth) {
                            const float lt = lp ? lam[j] + dlt[j] : lam[j];
                            const float g = leg0 ? a.gamma0 : gam[j];
                            const float mo = Ms[j];
                            float acc = __builtin_fmaf(g, mo - lt, lt);
                            const int e0 = m.col_ptr[j], e1 = m.col_ptr[j + 1];
                            for (int e = e0; e < e1; ++e) acc = acc + mu[m.csc_edge[e]];
                            Ms[j] = acc;
                            if ((acc < 0.0f) != (mo < 0.0f)) {
                                for (int e = e0; e < e1; ++e) {
                                    const int i = m.csc_row[e];
                                    const uint32_t bit = 1u << (i & 31);
                                    const uint32_t old = atomicXor(par + (i >> 5), bit);
                                    dcount += (old & bit) ? -1 : 1;
                                }
                            }
                        }
                        if (dcount) atomicAdd(&sh_count, dcount);
                        __syncthreads();
                        ++iters;
                        if (a.trace_on && phase == a.trace_phase && leg == a.trace_leg && t == a.trace_t) {
                            for (int j = tid; j < N; j += nth) a.trace_M[j] = Ms[j];
                            for (int e = tid; e < m.E; e += nth) a.trace_mu[e] = mu[m.csc_edge[e]];
                            if (tid == 0) *a.trace_hit = 1;
                            traced = true;
                            break;
                        }
                        if (base + sh_count == 0) {
                            conv = true;
                            break;
                        }
                    }
                    if (traced) break;
                    if (conv) {
                        double wsum = 0.0;
                        for (int j = tid; j < N; j += nth)
                            if (Ms[j] < 0.0f) wsum += (double)lam[j];
                        const double W = block_sum<double>(wsum, sh_red_d);
                        if (!have_best || W < bestW) {
                            bestW = W;
                            have_best = true;
                            capture_decisions(Ms, best, N, WN);
                        }
                        ++nconv;
                        if (a.crit == 0 && nconv >= a.S) break;
                    }
                }
                if (traced) break;
                if (prop) {
                    if (nconv > 0) {
                        path = 1;
                        break;
                    }
                    path = 2;
                }
            }
            if (!have_best) capture_decisions(Ms, best, N, WN);
            __syncthreads();
        }
        if (!traced && !a.trace_on) {
            for (int w = tid; w < WN; w += nth) m.corr[row * WN + w] = best[w];
            if (m.obsp) {
                const int wid = tid >> 6;
                for (int rb = wid * 64; rb < m.k; rb += nth) {
                    const int r = rb + lane;
                    uint32_t pbit = 0;
                    if (r < m.k)
                        for (int e = m.orow_ptr[r]; e < m.orow_ptr[r + 1]; ++e) {
                            const int j = m.ocol_idx[e];
                            pbit ^= (best[j >> 5] >> (j & 31)) & 1u;
                        }
                    const unsigned long long b = __ballot(pbit != 0);
                    if (lane == 0) {
                        m.obsp[row * m.WK + (rb >> 5)] = (uint32_t)b;
                        if ((rb >> 5) + 1 < m.WK) m.obsp[row * m.WK + (rb >> 5) + 1] = (uint32_t)(b >> 32);
                    }
                }
            }
            if (a.stats && tid == 0) {
                rbp_shot_stats st;
                st.converged = have_best ? 1 : 0;
                st.nconv = (uint8_t)(nconv > 255 ? 255 : nconv);
                st.path = (uint8_t)path;
                st.reserved = 0;
                st.legs = (uint16_t)(legs > 65535 ? 65535 : legs);
                st.reserved2 = 0;
                st.iters = (uint32_t)iters;
                st.reserved3 = 0;
                st.t_start = t_start;
                st.t_end = wall_clock64();
                a.stats[s] = st;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

template <class T>
static rbp_status upload(DevBuf& b, const std::vector<T>& v) {
    rbp_status st = b.reserve(sizeof(T) * std::max<size_t>(v.size(), 1));
    if (st) return st;
    if (!v.empty()) RBP_HIP_CHECK(hipMemcpy(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return RBP_OK;
}

static rbp_status check_priors(const double* priors, int N) {
    if (!priors) return fail(RBP_ERR_INVALID_ARG, "priors is NULL");
    for (int j = 0; j < N; ++j)
        if (!(priors[j] > 0.0 && priors[j] <= 0.5))
            return fail(RBP_ERR_UNSUPPORTED, "prior " + std::to_string(j) + " outside (0, 0.5]");
    return RBP_OK;
}

// LLRs Lambda_j = (float) ln((1-p)/p) in double, uploaded when the priors change.
static rbp_status ensure_llr(rbp_code* c, const double* priors, hipStream_t stream) {
    if (c->lam.p && c->lam_key.size() == (size_t)c->N &&
        std::memcmp(c->lam_key.data(), priors, sizeof(double) * c->N) == 0)
        return RBP_OK;
    std::vector<float> lam(c->N);
    for (int j = 0; j < c->N; ++j) lam[j] = (float)std::log((1.0 - priors[j]) / priors[j]);
    rbp_status st = c->lam.reserve(sizeof(float) * std::max(c->N, 1));
    if (st) return st;
    RBP_HIP_CHECK(hipStreamSynchronize(stream));
    RBP_HIP_CHECK(hipMemcpy(c->lam.p, lam.data(), sizeof(float) * c->N, hipMemcpyHostToDevice));
    c->lam_key.assign(priors, priors + c->N);
    return RBP_OK;
}

static rbp_status ensure_thresholds(rbp_code* c, const double* priors, hipStream_t stream) {
    if (c->thr.p && c->thr_key.size() == (size_t)c->N &&
        std::memcmp(c->thr_key.data(), priors, sizeof(double) * c->N) == 0)
        return RBP_OK;
    std::vector<uint32_t> thr(c->N);
    for (int j = 0; j < c->N; ++j) {
        const double t = std::floor(priors[j] * 4294967296.0);
        thr[j] = t >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)t;
    }
    rbp_status st = c->thr.reserve(sizeof(uint32_t) * std::max(c->N, 1));
    if (st) return st;
    RBP_HIP_CHECK(hipStreamSynchronize(stream));
    RBP_HIP_CHECK(hipMemcpy(c->thr.p, thr.data(), sizeof(uint32_t) * c->N, hipMemcpyHostToDevice));
    c->thr_key.assign(priors, priors + c->N);
    return RBP_OK;
}

static rbp_status ensure_gamma(rbp_code* c, const rbp_relay_params* p, hipStream_t stream) {
    const int R = p->num_sets;
    if (c->gtab.p && c->gtab_R == R && c->gtab_seed == p->gamma_seed && c->gtab_lo == p->gamma_min &&
        c->gtab_hi == p->gamma_max)
        return RBP_OK;
    const int64_t total = (int64_t)c->N * std::max(R, 0);
    RBP_HIP_CHECK(hipStreamSynchronize(stream));
    rbp_status st = c->gtab.reserve(sizeof(float) * std::max<int64_t>(total, 1));
    if (st) return st;
    if (total > 0) {
        hipLaunchKernelGGL(gamma_table_kernel, dim3(ceil_div(total, 256)), dim3(256), 0, stream,
                           c->gtab.as<float>(), c->N, R, p->gamma_min, p->gamma_max, p->gamma_seed);
        RBP_HIP_CHECK(hipGetLastError());
    }
    c->gtab_R = R;
    c->gtab_seed = p->gamma_seed;
    c->gtab_lo = p->gamma_min;
    c->gtab_hi = p->gamma_max;
    return RBP_OK;
}

static rbp_status check_params(const rbp_relay_params* p) {
    if (!p) return fail(RBP_ERR_INVALID_ARG, "params is NULL");
    if (p->pre_iter < 1 || p->max_iterations < 1 || p->num_sets < 0 || p->stop_nconv < 1 ||
        p->stop_nconv > 255 || (p->stopping_criterion != 0 && p->stopping_criterion != 1))
        return fail(RBP_ERR_INVALID_ARG, "relay parameters out of range");
    if (!std::isfinite(p->gamma0) || !std::isfinite(p->gamma_min) || !std::isfinite(p->gamma_max))
        return fail(RBP_ERR_INVALID_ARG, "gamma values must be finite");
    if ((int64_t)p->num_sets + 1 > 32767) return fail(RBP_ERR_INVALID_ARG, "num_sets too large");
    return RBP_OK;
}

static DecodeModel model_of(const rbp_code* c, const uint32_t* syn, uint32_t* corr, uint32_t* obsp) {
    DecodeModel m;
    m.M = c->M;
    m.N = c->N;
    m.E = c->E;
    m.k = c->k;
    m.WM = ceil_div(c->M, 32);
    m.WN = ceil_div(c->N, 32);
    m.WK = ceil_div(c->k, 32);
    m.row_ptr = c->row_ptr.as<int32_t>();
    m.col_idx = c->col_idx.as<int32_t>();
    m.col_ptr = c->col_ptr.as<int32_t>();
    m.csc_row = c->csc_row.as<int32_t>();
    m.csc_edge = c->csc_edge.as<int32_t>();
    m.orow_ptr = c->orow_ptr.as<int32_t>();
    m.ocol_idx = c->ocol_idx.as<int32_t>();
    m.lam = c->lam.as<float>();
    m.gtab = c->gtab.as<float>();
    m.syn = syn;
    m.corr = corr;
    m.obsp = c->k > 0 ? obsp : nullptr;
    return m;
}

typedef void (*DecodeKernel)(const DecodeLaunch);

static DecodeKernel pick_kernel(int maxdeg, bool lds) {
    if (maxdeg <= 12) return lds ? relay_bp_kernel<12, true> : relay_bp_kernel<12, false>;
    return lds ? relay_bp_kernel<32, true> : relay_bp_kernel<32, false>;
}

static constexpr int kMaxLds = 160 * 1024;

struct LaunchShape {
    int waves = 1;
    bool lds_state = true;
    int lds_bytes = 0;
    int slots = 1;
    int64_t gstride = 0;
    int off_sig = 0, off_par = 0, off_best = 0;
};

// Launch shape for a set of models decoded together (max sizes over models).
static rbp_status plan_launch(rbp_code* const* cs, int n, uint64_t shots, LaunchShape* out) {
    int Nmax = 0, Emax = 0, WMmax = 0, WNmax = 0, maxdeg = 0;
    for (int i = 0; i < n; ++i) {
        Nmax = std::max(Nmax, cs[i]->N);
        Emax = std::max(Emax, cs[i]->E);
        WMmax = std::max(WMmax, ceil_div(cs[i]->M, 32));
        WNmax = std::max(WNmax, ceil_div(cs[i]->N, 32));
        maxdeg = std::max(maxdeg, cs[i]->max_row_deg);
    }
    const LaunchCfg& cfg = cs[0]->cfg;
    int waves = cfg.waves_per_shot;
    if (waves <= 0) {
        const int want = ceil_div(Nmax, 512);
        waves = 1;
        while (waves < want && waves < 8) waves <<= 1;
    }
    waves = std::min(std::max(waves, 1), 16);
    const int small = 4 * (2 * WMmax + WNmax) + 512;  // + static shared variables
    const int state_bytes = 4 * (Nmax + Emax);
    bool lds = state_bytes + small <= kMaxLds;
    if (cfg.state == 1 && !lds) return fail(RBP_ERR_UNSUPPORTED, "per-shot state does not fit in LDS");
    if (cfg.state == 2) lds = false;
    LaunchShape L;
    L.waves = waves;
    L.lds_state = lds;
    int off = lds ? state_bytes : 0;
    off = (off + 15) & ~15;
    L.off_sig = off;
    off += 4 * WMmax;
    L.off_par = off;
    off += 4 * WMmax;
    L.off_best = off;
    off += 4 * WNmax;
    L.lds_bytes = (off + 15) & ~15;
    L.gstride = lds ? 0 : ((int64_t)Nmax + Emax + 63) / 64 * 64;
    int per_cu = 0;
    DecodeKernel k = pick_kernel(maxdeg, lds);
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k), 64 * waves,
                                                                L.lds_bytes);
    if (e != hipSuccess) return fail(RBP_ERR_HIP, std::string("occupancy query: ") + hipGetErrorString(e));
    per_cu = std::max(per_cu, 1);
    int64_t slots = (int64_t)per_cu * std::max(cs[0]->num_cus, 1);
    if (cfg.max_slots > 0) slots = std::min<int64_t>(slots, cfg.max_slots);
    slots = std::min<int64_t>(slots, std::max<uint64_t>(shots, 1));
    L.slots = (int)std::max<int64_t>(slots, 1);
    *out = L;
    return RBP_OK;
}

static rbp_status launch_decode(rbp_code* const* cs, int n, DecodeLaunch& a, uint64_t shots, hipStream_t stream) {
    LaunchShape L;
    rbp_status st = plan_launch(cs, n, shots, &L);
    if (st) return st;
    rbp_code* c0 = cs[0];
    st = c0->queue.reserve(64);
    if (st) return st;
    if (!L.lds_state) {
        st = c0->gstate.reserve(sizeof(float) * (size_t)L.gstride * L.slots);
        if (st) return st;
    }
    int Nmax = 0, maxdeg = 0;
    for (int i = 0; i < n; ++i) {
        Nmax = std::max(Nmax, cs[i]->N);
        maxdeg = std::max(maxdeg, cs[i]->max_row_deg);
    }
    a.queue = c0->queue.as<unsigned long long>();
    a.gstate = L.lds_state ? nullptr : c0->gstate.as<float>();
    a.gstate_stride = L.gstride;
    a.Nmax = Nmax;
    a.off_sig = L.off_sig;
    a.off_par = L.off_par;
    a.off_best = L.off_best;
    a.shots = shots;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, stream, a.queue, 1);
    RBP_HIP_CHECK(hipGetLastError());
    DecodeKernel k = pick_kernel(maxdeg, L.lds_state);
    RBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      L.lds_bytes));
    hipLaunchKernelGGL(k, dim3(L.slots), dim3(64 * L.waves), L.lds_bytes, stream, a);
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

static void fill_params(DecodeLaunch& a, const rbp_relay_params* p) {
    a.gamma0 = p->gamma0;
    a.T0 = p->pre_iter;
    a.Tr = p->max_iterations;
    a.R = p->num_sets;
    a.S = p->stop_nconv;
    a.crit = p->stopping_criterion;
}

}  // namespace rbp

using namespace rbp;

extern "C" {

const char* rbp_last_error(void) { return rbp::g_err.c_str(); }

rbp_status rbp_code_create(int32_t M, int32_t N, const int32_t* col_ptr, const int32_t* row_idx, int32_t k,
                           const int32_t* obs_col_ptr, const int32_t* obs_row_idx, rbp_code_t* out) {
    if (!out) return fail(RBP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (M < 1 || N < 1 || k < 0) return fail(RBP_ERR_SHAPE, "need M >= 1, N >= 1, k >= 0");
    if (!col_ptr || !row_idx) return fail(RBP_ERR_INVALID_ARG, "H arrays are NULL");
    if (k > 0 && (!obs_col_ptr || !obs_row_idx)) return fail(RBP_ERR_INVALID_ARG, "O arrays are NULL");
    if (col_ptr[0] != 0) return fail(RBP_ERR_SHAPE, "col_ptr[0] must be 0");
    for (int j = 0; j < N; ++j) {
        if (col_ptr[j + 1] < col_ptr[j]) return fail(RBP_ERR_SHAPE, "col_ptr not monotone");
        for (int e = col_ptr[j]; e < col_ptr[j + 1]; ++e) {
            if (row_idx[e] < 0 || row_idx[e] >= M) return fail(RBP_ERR_SHAPE, "row index out of range");
            if (e > col_ptr[j] && row_idx[e] <= row_idx[e - 1])
                return fail(RBP_ERR_SHAPE, "rows must be strictly ascending within a column");
        }
    }
    const int E = col_ptr[N];
    std::vector<int32_t> deg(M, 0);
    int maxcol = 0;
    for (int j = 0; j < N; ++j) {
        maxcol = std::max(maxcol, col_ptr[j + 1] - col_ptr[j]);
        for (int e = col_ptr[j]; e < col_ptr[j + 1]; ++e) deg[row_idx[e]]++;
    }
    int maxrow = 0;
    for (int i = 0; i < M; ++i) {
        if (deg[i] == 1 || deg[i] > 32)
            return fail(RBP_ERR_UNSUPPORTED, "row " + std::to_string(i) + " has degree " + std::to_string(deg[i]) +
                                                 " (supported: 0 or 2..32)");
        maxrow = std::max(maxrow, deg[i]);
    }
    int nnzO = 0;
    if (k > 0) {
        if (obs_col_ptr[0] != 0) return fail(RBP_ERR_SHAPE, "obs_col_ptr[0] must be 0");
        for (int j = 0; j < N; ++j) {
            if (obs_col_ptr[j + 1] < obs_col_ptr[j]) return fail(RBP_ERR_SHAPE, "obs_col_ptr not monotone");
            for (int e = obs_col_ptr[j]; e < obs_col_ptr[j + 1]; ++e) {
                if (obs_row_idx[e] < 0 || obs_row_idx[e] >= k) return fail(RBP_ERR_SHAPE, "observable row out of range");
                if (e > obs_col_ptr[j] && obs_row_idx[e] <= obs_row_idx[e - 1])
                    return fail(RBP_ERR_SHAPE, "observable rows must be strictly ascending");
            }
        }
        nnzO = obs_col_ptr[N];
    }
    // CSR of H (columns ascending within a row) and the CSC -> CSR edge map
    std::vector<int32_t> rp(M + 1, 0), ci(std::max(E, 1)), cedge(std::max(E, 1)), fillc(M, 0);
    for (int i = 0; i < M; ++i) rp[i + 1] = rp[i] + deg[i];
    for (int j = 0; j < N; ++j)
        for (int e = col_ptr[j]; e < col_ptr[j + 1]; ++e) {
            const int i = row_idx[e];
            const int pos = rp[i] + fillc[i]++;
            ci[pos] = j;
            cedge[e] = pos;
        }
    // CSR of O
    std::vector<int32_t> orp(k + 1, 0), oci(std::max(nnzO, 1)), ofill(std::max(k, 1), 0);
    if (k > 0) {
        for (int e = 0; e < nnzO; ++e) orp[obs_row_idx[e] + 1]++;
        for (int r = 0; r < k; ++r) orp[r + 1] += orp[r];
        for (int j = 0; j < N; ++j)
            for (int e = obs_col_ptr[j]; e < obs_col_ptr[j + 1]; ++e) {
                const int r = obs_row_idx[e];
                oci[orp[r] + ofill[r]++] = j;
            }
    }
    rbp_code* c = new rbp_code();
    c->M = M;
    c->N = N;
    c->E = E;
    c->k = k;
    c->nnzO = nnzO;
    c->max_row_deg = maxrow;
    c->max_col_deg = maxcol;
    hipError_t he = hipGetDevice(&c->device);
    if (he == hipSuccess) he = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, c->device);
    if (he != hipSuccess) {
        delete c;
        return fail(RBP_ERR_HIP, std::string("device query: ") + hipGetErrorString(he));
    }
    std::vector<int32_t> cp(col_ptr, col_ptr + N + 1), cr(row_idx, row_idx + E);
    std::vector<int32_t> ocp(N + 1, 0), ori;
    if (k > 0) {
        ocp.assign(obs_col_ptr, obs_col_ptr + N + 1);
        ori.assign(obs_row_idx, obs_row_idx + nnzO);
    }
    ci.resize(std::max(E, 1));
    rbp_status st = RBP_OK;
    if (!st) st = upload(c->row_ptr, rp);
    if (!st) st = upload(c->col_idx, ci);
    if (!st) st = upload(c->col_ptr, cp);
    if (!st) st = upload(c->csc_row, cr);
    if (!st) st = upload(c->csc_edge, cedge);
    if (!st) st = upload(c->orow_ptr, orp);
    if (!st) st = upload(c->ocol_idx, oci);
    if (!st) st = upload(c->ocol_ptr, ocp);
    if (!st) st = upload(c->orow_idx, ori);
    if (st) {
        rbp_code_destroy(c);
        return st;
    }
    *out = c;
    return RBP_OK;
}

rbp_status rbp_code_destroy(rbp_code_t c) {
    if (!c) return RBP_OK;
    (void)hipDeviceSynchronize();
    for (DevBuf* b : {&c->row_ptr, &c->col_idx, &c->col_ptr, &c->csc_row, &c->csc_edge, &c->orow_ptr, &c->ocol_idx,
                      &c->ocol_ptr, &c->orow_idx, &c->thr, &c->lam, &c->gtab, &c->queue, &c->gstate, &c->trace_hit})
        b->release();
    delete c;
    return RBP_OK;
}

rbp_status rbp_code_info(rbp_code_t c, int32_t* M, int32_t* N, int32_t* nnz, int32_t* k, int32_t* max_row_deg,
                         int32_t* max_col_deg) {
    if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
    if (M) *M = c->M;
    if (N) *N = c->N;
    if (nnz) *nnz = c->E;
    if (k) *k = c->k;
    if (max_row_deg) *max_row_deg = c->max_row_deg;
    if (max_col_deg) *max_col_deg = c->max_col_deg;
    return RBP_OK;
}

rbp_status rbp_sample(rbp_code_t c, const double* priors, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                      uint32_t* syndromes, uint32_t* obs, uint32_t* errors, void* stream_) {
    if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
    if (shots == 0) return RBP_OK;
    if (!syndromes) return fail(RBP_ERR_INVALID_ARG, "syndromes is NULL");
    if (c->k > 0 && !obs) return fail(RBP_ERR_INVALID_ARG, "obs is NULL");
    rbp_status st = check_priors(priors, c->N);
    if (st) return st;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    st = ensure_thresholds(c, priors, stream);
    if (st) return st;
    SampleArgs a;
    a.M = c->M;
    a.N = c->N;
    a.k = c->k;
    a.WM = ceil_div(c->M, 32);
    a.WK = ceil_div(c->k, 32);
    a.WN = ceil_div(c->N, 32);
    a.col_ptr = c->col_ptr.as<int32_t>();
    a.csc_row = c->csc_row.as<int32_t>();
    a.ocol_ptr = c->ocol_ptr.as<int32_t>();
    a.orow_idx = c->orow_idx.as<int32_t>();
    a.thr = c->thr.as<uint32_t>();
    a.seed = seed;
    a.offset = shot_offset;
    a.syn = syndromes;
    a.obs = c->k > 0 ? obs : nullptr;
    a.err = errors;
    const size_t lds = sizeof(uint32_t) * (size_t)kSampleWaves * (a.WM + a.WK);
    if (lds > (size_t)kMaxLds) return fail(RBP_ERR_UNSUPPORTED, "detector/observable count too large for sampler");
    const uint64_t max_blocks = 1ull << 30;
    for (uint64_t done = 0; done < shots;) {
        const uint64_t n = std::min<uint64_t>(shots - done, max_blocks * kSampleWaves);
        a.shots = n;
        a.offset = shot_offset + done;
        a.syn = syndromes + done * a.WM;
        a.obs = c->k > 0 ? obs + done * a.WK : nullptr;
        a.err = errors ? errors + done * a.WN : nullptr;
        hipLaunchKernelGGL(sample_kernel, dim3((unsigned)ceil_div(n, kSampleWaves)), dim3(64 * kSampleWaves), lds,
                           stream, a);
        RBP_HIP_CHECK(hipGetLastError());
        done += n;
    }
    return RBP_OK;
}

rbp_status rbp_decode(rbp_code_t c, const double* priors, const uint32_t* syndromes, uint64_t shots,
                      const rbp_relay_params* params, const float* prior_delta, uint32_t* corrections,
                      uint32_t* obs_pred, rbp_shot_stats* stats, void* stream_) {
    if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
    rbp_status st = check_params(params);
    if (st) return st;
    if (shots == 0) return RBP_OK;
    if (!syndromes || !corrections) return fail(RBP_ERR_INVALID_ARG, "syndromes/corrections is NULL");
    if (c->k > 0 && !obs_pred) return fail(RBP_ERR_INVALID_ARG, "obs_pred is NULL");
    st = check_priors(priors, c->N);
    if (st) return st;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    st = ensure_llr(c, priors, stream);
    if (!st) st = ensure_gamma(c, params, stream);
    if (st) return st;
    DecodeLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.m[0] = model_of(c, syndromes, corrections, obs_pred);
    a.n_models = 1;
    a.delta = prior_delta;
    a.stats = stats;
    fill_params(a, params);
    rbp_code* cs[1] = {c};
    return launch_decode(cs, 1, a, shots, stream);
}

rbp_status rbp_decode_multi(int32_t n_codes, const rbp_code_t* codes, const double* const* priors,
                            const uint8_t* shot_code, const uint32_t* shot_index, uint64_t shots,
                            const uint32_t* const* syndromes, const rbp_relay_params* params,
                            uint32_t* const* corrections, uint32_t* const* obs_pred, rbp_shot_stats* stats,
                            void* stream_) {
    if (n_codes < 1 || n_codes > kMaxModels) return fail(RBP_ERR_INVALID_ARG, "n_codes must be 1..8");
    if (!codes || !priors || !syndromes || !corrections) return fail(RBP_ERR_INVALID_ARG, "NULL array");
    if (!shot_code || !shot_index) return fail(RBP_ERR_INVALID_ARG, "shot_code/shot_index is NULL");
    rbp_status st = check_params(params);
    if (st) return st;
    if (shots == 0) return RBP_OK;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    DecodeLaunch a;
    std::memset(&a, 0, sizeof(a));
    std::vector<rbp_code*> cs(n_codes);
    for (int i = 0; i < n_codes; ++i) {
        rbp_code* c = codes[i];
        if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
        for (int j = 0; j < i; ++j)
            if (cs[j] == c) return fail(RBP_ERR_INVALID_ARG, "each handle may appear once");
        if (!syndromes[i] || !corrections[i]) return fail(RBP_ERR_INVALID_ARG, "syndromes/corrections is NULL");
        if (c->k > 0 && (!obs_pred || !obs_pred[i])) return fail(RBP_ERR_INVALID_ARG, "obs_pred is NULL");
        st = check_priors(priors[i], c->N);
        if (!st) st = ensure_llr(c, priors[i], stream);
        if (!st) st = ensure_gamma(c, params, stream);
        if (st) return st;
        cs[i] = c;
        a.m[i] = model_of(c, syndromes[i], corrections[i], obs_pred ? obs_pred[i] : nullptr);
    }
    a.n_models = n_codes;
    a.shot_code = shot_code;
    a.shot_index = shot_index;
    a.stats = stats;
    fill_params(a, params);
    return launch_decode(cs.data(), n_codes, a, shots, stream);
}

rbp_status rbp_set_launch_config(rbp_code_t c, const rbp_launch_config* cfg) {
    if (!c || !cfg) return fail(RBP_ERR_INVALID_ARG, "NULL argument");
    if (cfg->waves_per_shot < 0 || cfg->waves_per_shot > 16 || cfg->state < 0 || cfg->state > 2 ||
        cfg->max_slots < 0)
        return fail(RBP_ERR_INVALID_ARG, "launch config out of range");
    c->cfg.waves_per_shot = cfg->waves_per_shot;
    c->cfg.state = cfg->state;
    c->cfg.max_slots = cfg->max_slots;
    return RBP_OK;
}

rbp_status rbp_get_launch_config(rbp_code_t c, rbp_launch_config* cfg, int32_t* slots, int32_t* lds_bytes) {
    if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
    LaunchShape L;
    rbp_code* cs[1] = {c};
    rbp_status st = plan_launch(cs, 1, ~0ull, &L);
    if (st) return st;
    if (cfg) {
        cfg->waves_per_shot = L.waves;
        cfg->state = L.lds_state ? 1 : 2;
        cfg->max_slots = c->cfg.max_slots;
    }
    if (slots) *slots = L.slots;
    if (lds_bytes) *lds_bytes = L.lds_bytes;
    return RBP_OK;
}

rbp_status rbp_trace(rbp_code_t c, const double* priors, const uint32_t* syndrome, const rbp_relay_params* params,
                     const float* prior_delta, int32_t phase, int32_t leg, int32_t t, float* M_out, float* mu_out,
                     int32_t* reached, void* stream_) {
    if (!c || !syndrome || !M_out || !mu_out || !reached) return fail(RBP_ERR_INVALID_ARG, "NULL argument");
    if (phase < 0 || phase > 1 || leg < 0 || t < 1) return fail(RBP_ERR_INVALID_ARG, "bad trace point");
    rbp_status st = check_params(params);
    if (!st) st = check_priors(priors, c->N);
    if (st) return st;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    st = ensure_llr(c, priors, stream);
    if (!st) st = ensure_gamma(c, params, stream);
    if (!st) st = c->trace_hit.reserve(16);
    if (st) return st;
    RBP_HIP_CHECK(hipMemsetAsync(c->trace_hit.p, 0, 16, stream));
    DecodeLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.m[0] = model_of(c, syndrome, nullptr, nullptr);
    a.n_models = 1;
    a.delta = prior_delta;
    fill_params(a, params);
    a.trace_on = 1;
    a.trace_phase = phase;
    a.trace_leg = leg;
    a.trace_t = t;
    a.trace_M = M_out;
    a.trace_mu = mu_out;
    a.trace_hit = c->trace_hit.as<int32_t>();
    rbp_code* cs[1] = {c};
    st = launch_decode(cs, 1, a, 1, stream);
    if (st) return st;
    int32_t hit = 0;
    RBP_HIP_CHECK(hipMemcpyAsync(&hit, c->trace_hit.p, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    RBP_HIP_CHECK(hipStreamSynchronize(stream));
    *reached = hit;
    return RBP_OK;
}

}  // extern "C"
