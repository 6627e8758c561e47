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
//                      converges early frees its slot at once.  The slot's state
//                      is one float per edge, in place (see below), in LDS when
//                      it fits, else in a per-slot device buffer; the threads'
//                      index lists and the marginals of their variables stay in
//                      registers for the life of the kernel.  The syndrome of the
//                      hard decision and the weight of the current solution are
//                      tracked incrementally: a variable whose decision flips XORs
//                      its checks' parity bits with LDS atomics and moves the
//                      weight, so convergence and solution weights cost no extra
//                      sweep or reduction.
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

// one thread per shot; a wave-level ballot count, one atomic per wave
__global__ void count_failures_kernel(const uint32_t* obsp, const uint32_t* obs, const rbp_shot_stats* st,
                                      uint64_t shots, int words, unsigned long long* count) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool fail = false;
    if (s < shots) {
        fail = st[s].converged == 0;
        for (int w = 0; w < words; ++w) fail |= obsp[s * words + w] != obs[s * words + w];
    }
    const unsigned long long b = __ballot(fail);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (unsigned long long)__popcll(b));
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------------------
// Persistent Relay-BP
//
// State of a shot slot: one float per Tanner-graph edge, X[E], in CSC order
// (the edges of a variable are contiguous, checks ascending).  The check sweep
// reads nu_{j->i} from X and overwrites it with mu_{i->j}; the variable sweep
// reads mu, forms the marginal M_j and overwrites X with nu_{j->i} = M_j - mu.
// So the two sweeps work in place on a single array, and the marginals live in
// the registers of the thread that owns the variable (or in Mg[N] when the
// index lists are not cached in registers).  The first iteration of a plain
// leg reads no state: nu(0) = Lambda, so mu(1) = (-1)^sigma_i * (min of the
// other Lambda of the row), a per-model table m1[E] computed once per priors.
// ---------------------------------------------------------------------------
constexpr int kMaxModels = 8;

struct DecodeModel {
    int32_t M, N, E, k, WM, WN, WK, P;  // P: row stride of rpos/m1p (<= RD of the kernel)
    const int32_t* rpos;      // [M][P] CSC slot of each edge of a row (columns ascending), -1 padded
    const int32_t* col_ptr;   // [N+1]
    const int32_t* csc_row;   // [E] check of each CSC slot
    const int32_t* ocol_ptr;  // [N+1] observables, CSC
    const int32_t* orow_idx;
    const float* lam;         // [N] Lambda
    const float* m1p;         // [M][P] first-iteration message magnitudes, row layout
    const float* gtab;        // [R][N] relay-leg memory strengths
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
    int32_t Emax;
    int32_t off_sig, off_par, off_best, off_obs;  // byte offsets in dynamic LDS
    float gamma0;
    int32_t T0, Tr, R, S, crit;
    int32_t trace_on, trace_phase, trace_leg, trace_t;
    float* trace_M;
    float* trace_mu;
    int32_t* trace_hit;
};

// first-iteration magnitudes in the padded row layout:
// m1p[i*P + p] = min over the other variables j' of row i of Lambda_j'
__global__ void first_message_kernel(const int32_t* row_ptr, const int32_t* col_idx, const float* lam, float* m1p,
                                     int32_t M, int32_t P) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int rs = row_ptr[i], re = row_ptr[i + 1];
    float min1 = INFINITY, min2 = INFINITY;
    for (int e = rs; e < re; ++e) {
        const float av = fabsf(lam[col_idx[e]]);
        min2 = __builtin_amdgcn_fmed3f(min1, min2, av);
        min1 = fminf(min1, av);
    }
    for (int e = rs; e < re; ++e) {
        const float av = fabsf(lam[col_idx[e]]);
        m1p[(int64_t)i * P + (e - rs)] = (av == min1) ? min2 : min1;
    }
}

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

// One check row of the min-sum update, in place on X.  pos[p] is the CSC slot
// of the row's p-th edge; slots past the row's degree hold E, the index of a
// read-only +inf cell (neutral for both minima and for the sign product), and
// their results go to the write-only cell E + 1.  nu -> mu with
//   mu_p = (-1)^sigma * prod_{q != p} s(nu_q) * min_{q != p} |nu_q|.
// The sign product is the XOR of the IEEE sign bits (nu is never -0: it is a
// difference of floats or a positive prior, and x - x = +0); |nu| is compared as
// an unsigned integer, which orders non-negative floats exactly as the floats;
// the minimum over the others is the second minimum exactly when |nu_p| is the
// first (with a tie both are equal).
template <int RD>
__device__ __forceinline__ void check_row(float* X, const int (&pos)[RD], int E, uint32_t sbit, bool first,
                                          const float (&m1v)[RD]) {
    const int wdummy = E + 1;
    if (first) {
#pragma unroll
        for (int p = 0; p < RD; ++p) {
            const int w = pos[p] == E ? wdummy : pos[p];
            X[w] = __uint_as_float(__float_as_uint(m1v[p]) | sbit);
        }
        return;
    }
    uint32_t nu[RD];
    uint32_t sgn = sbit;
    uint32_t min1 = 0x7f800000u, min2 = 0x7f800000u;
#pragma unroll
    for (int p = 0; p < RD; ++p) {
        const uint32_t v = __float_as_uint(X[pos[p]]);
        nu[p] = v;
        sgn ^= v;
        const uint32_t av = v & 0x7fffffffu;
        const uint32_t lo2 = min2 < av ? min2 : av;
        min2 = min1 > lo2 ? min1 : lo2;  // median of (min1, min2, av) given min1 <= min2
        min1 = min1 < av ? min1 : av;
    }
#pragma unroll
    for (int p = 0; p < RD; ++p) {
        const uint32_t av = nu[p] & 0x7fffffffu;
        const uint32_t mag = (av == min1) ? min2 : min1;
        const int w = pos[p] == E ? wdummy : pos[p];
        X[w] = __uint_as_float(mag | ((sgn ^ nu[p]) & 0x80000000u));
    }
}

// A variable whose hard decision flips toggles the parity of its checks and
// moves the solution weight by +-Lambda_j (double; sums of FP32 values of
// this range are exact, so the order of the atomics does not matter).
__device__ __forceinline__ void flip_variable(const int32_t* csc_row, int s0, int d, bool now_neg, float lamj,
                                              uint32_t* par, int& dcount, double& dW) {
    for (int e = s0; e < s0 + d; ++e) {
        const int i = csc_row[e];
        const uint32_t bit = 1u << (i & 31);
        const uint32_t old = atomicXor(par + (i >> 5), bit);
        dcount += (old & bit) ? -1 : 1;
    }
    dW += now_neg ? (double)lamj : -(double)lamj;
}

// Hides a register value from loop-invariant code motion: address arithmetic on
// the cached index lists is then redone per sweep (one add) instead of being
// hoisted out of the persistent loop as one 64-bit address per edge.
__device__ __forceinline__ void opaque(int& x) { asm volatile("" : "+v"(x)); }

template <int RD, int CD, int CPT, int VPT, bool LDS_STATE, int WAVES>
__global__ void __launch_bounds__(64 * WAVES, (WAVES >= 4 ? 4 : WAVES)) relay_bp_kernel(const DecodeLaunch a) {
    constexpr bool CACHED = CPT > 0;
    constexpr int CP = CACHED ? CPT : 1;
    constexpr int VP = CACHED ? VPT : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long sh_shot;
    __shared__ int sh_count;
    __shared__ double sh_W;
    __shared__ int sh_red_i[16];

    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wid = tid >> 6;
    float* X;
    if constexpr (LDS_STATE) {
        X = reinterpret_cast<float*>(smem);
    } else {
        X = a.gstate + (int64_t)blockIdx.x * a.gstate_stride;
    }
    float* Mg = X + a.Emax + 4;  // marginals of the uncached variant (after the two dummy cells)
    uint32_t* sig = reinterpret_cast<uint32_t*>(smem + a.off_sig);
    uint32_t* par = reinterpret_cast<uint32_t*>(smem + a.off_par);
    uint32_t* best = reinterpret_cast<uint32_t*>(smem + a.off_best);
    uint32_t* obw = reinterpret_cast<uint32_t*>(smem + a.off_obs);

    // Register caches of the persistent thread: its checks tid + c*nth and its
    // variables tid + v*nth never change, so their index lists are loaded once.
    int cpos[CP][RD];
    int cdeg[CP];
    int vstart[VP], vdeg[VP];
    float vlam[VP], Mreg[VP], greg[VP];
    if constexpr (CACHED) {
        const DecodeModel m0 = a.m[0];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int i = tid + c * nth;
            cdeg[c] = 0;
#pragma unroll
            for (int p = 0; p < RD; ++p) cpos[c][p] = (i < m0.M && p < m0.P) ? m0.rpos[(int64_t)i * m0.P + p] : m0.E;
        }
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int j = tid + v * nth;
            int s0 = 0, d = 0;
            float l = 0.f;
            if (j < m0.N) {
                s0 = m0.col_ptr[j];
                d = m0.col_ptr[j + 1] - s0;
                l = m0.lam[j];
            }
            vstart[v] = s0;
            vdeg[v] = d;
            vlam[v] = l;
            Mreg[v] = 0.f;
            greg[v] = 0.f;
        }
    }

    for (;;) {
        if (tid == 0) {
            sh_shot = atomicAdd(a.queue, 1ull);
            sh_count = 0;
            sh_W = 0.0;
        }
        __syncthreads();
        // the shot, its model and its row are uniform over the workgroup: keep them scalar
        const unsigned long long s = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(sh_shot >> 32)) << 32) |
                                     __builtin_amdgcn_readfirstlane((uint32_t)sh_shot);
        if (s >= a.shots) break;
        const uint64_t t_start = wall_clock64();
        const int mi = (CACHED || !a.shot_code) ? 0 : __builtin_amdgcn_readfirstlane((int)a.shot_code[s]);
        const DecodeModel m = a.m[mi];
        const uint64_t row = a.shot_index ? (uint64_t)__builtin_amdgcn_readfirstlane(a.shot_index[s]) : (uint64_t)s;
        const int M = m.M, N = m.N, WM = m.WM, WN = m.WN;
        const float* lam = m.lam;
        const float* dlt = a.delta ? a.delta + row * (uint64_t)N : nullptr;

        if (tid == 0) X[m.E] = INFINITY;  // read-only cell of the padded row slots
        int pc = 0;
        for (int w = tid; w < WM; w += nth) {
            const uint32_t v = m.syn[row * WM + w];
            sig[w] = v;
            par[w] = v;
            pc += __popc(v);
        }
        const int base = block_sum<int>(pc, sh_red_i);

        int nconv = 0, legs = 0, iters = 0, path = 0;
        bool have_best = false;
        double bestW = 0.0;
        bool traced = false;

        if (base == 0) {
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
                    if (tid == 0) {
                        sh_count = 0;
                        sh_W = 0.0;
                    }
                    for (int w = tid; w < WM; w += nth) par[w] = sig[w];
                    __syncthreads();
                }
                // M(0) = Lambda (or Lambda + delta; then also nu(0) = Lambda + delta on every edge)
                {
                    int dc = 0;
                    double dW = 0.0;
                    if constexpr (CACHED) {
#pragma unroll
                        for (int v = 0; v < VPT; ++v) {
                            const int j = tid + v * nth;
                            if (j < N) {
                                const float x = prop ? vlam[v] + dlt[j] : vlam[v];
                                Mreg[v] = x;
                                if (prop)
                                    for (int e = vstart[v]; e < vstart[v] + vdeg[v]; ++e) X[e] = x;
                                if (x < 0.0f) flip_variable(m.csc_row, vstart[v], vdeg[v], true, vlam[v], par, dc, dW);
                            }
                        }
                    } else {
                        for (int j = tid; j < N; j += nth) {
                            const float x = prop ? lam[j] + dlt[j] : lam[j];
                            Mg[j] = x;
                            if (prop) {
                                const int s0 = m.col_ptr[j], d = m.col_ptr[j + 1] - s0;
                                for (int e = s0; e < s0 + d; ++e) X[e] = x;
                                if (x < 0.0f) flip_variable(m.csc_row, s0, d, true, lam[j], par, dc, dW);
                            }
                        }
                    }
                    if (dc) atomicAdd(&sh_count, dc);
                    if (dW != 0.0) atomicAdd(&sh_W, dW);
                    __syncthreads();
                }

                const int nlegs = prop ? 0 : a.R;
                for (int leg = 0; leg <= nlegs; ++leg) {
                    const bool leg0 = leg == 0;
                    const bool lp = prop && leg0;  // priors of this leg are Lambda + delta
                    const int T = leg0 ? a.T0 : a.Tr;
                    const float* gam = leg0 ? nullptr : m.gtab + (int64_t)(leg - 1) * N;
                    bool conv = false;
                    ++legs;
                    if constexpr (CACHED) {
#pragma unroll
                        for (int v = 0; v < VPT; ++v) {
                            const int j = tid + v * nth;
                            greg[v] = (leg0 || j >= N) ? a.gamma0 : gam[j];
                        }
                    }
                    for (int t = 1; t <= T; ++t) {
                        const bool first_plain = t == 1 && !lp;
                        // ---- check sweep
                        if constexpr (CACHED) {
#pragma unroll
                            for (int c = 0; c < CPT; ++c) {
#pragma unroll
                                for (int p = 0; p < RD; ++p) opaque(cpos[c][p]);
                                const int i = tid + c * nth;
                                if (i < M) {
                                    float m1v[RD];
#pragma unroll
                                    for (int p = 0; p < RD; ++p)
                                        m1v[p] = (first_plain && p < m.P) ? m.m1p[(int64_t)i * m.P + p] : 0.f;
                                    check_row<RD>(X, cpos[c], m.E, ((sig[i >> 5] >> (i & 31)) & 1u) << 31, first_plain, m1v);
                                }
                                __builtin_amdgcn_sched_barrier(0);
                            }
                        } else {
                            // rounds of CR rows per thread: the position lists of all
                            // rounds are loaded before any row is processed
                            constexpr int CR = RD <= 12 ? 2 : 1;
                            static_assert(RD % 4 == 0, "row stride must be a multiple of 4");
                            for (int i0 = tid; i0 < M; i0 += CR * nth) {
                                int pos[CR][RD];
                                float m1v[CR][RD];
#pragma unroll
                                for (int r = 0; r < CR; ++r) {
                                    const int i = i0 + r * nth;
                                    const uint32_t b = (uint32_t)(i < M ? i : 0) * (uint32_t)RD;
                                    const int4* pp = reinterpret_cast<const int4*>(m.rpos + b);
                                    const float4* mp = reinterpret_cast<const float4*>(m.m1p + b);
#pragma unroll
                                    for (int q = 0; q < RD / 4; ++q) {
                                        const int4 v = pp[q];
                                        pos[r][4 * q] = v.x;
                                        pos[r][4 * q + 1] = v.y;
                                        pos[r][4 * q + 2] = v.z;
                                        pos[r][4 * q + 3] = v.w;
                                        if (first_plain) {
                                            const float4 f = mp[q];
                                            m1v[r][4 * q] = f.x;
                                            m1v[r][4 * q + 1] = f.y;
                                            m1v[r][4 * q + 2] = f.z;
                                            m1v[r][4 * q + 3] = f.w;
                                        } else {
                                            m1v[r][4 * q] = m1v[r][4 * q + 1] = m1v[r][4 * q + 2] = m1v[r][4 * q + 3] = 0.f;
                                        }
                                    }
                                }
#pragma unroll
                                for (int r = 0; r < CR; ++r) {
                                    const int i = i0 + r * nth;
                                    if (i < M)
                                        check_row<RD>(X, pos[r], m.E, ((sig[i >> 5] >> (i & 31)) & 1u) << 31, first_plain,
                                                      m1v[r]);
                                }
                            }
                        }
                        __syncthreads();
                        // ---- variable sweep
                        const bool tr = a.trace_on && phase == a.trace_phase && leg == a.trace_leg && t == a.trace_t;
                        int dcount = 0;
                        double dW = 0.0;
                        if constexpr (CACHED) {
#pragma unroll
                            for (int v = 0; v < VPT; ++v) {
                                opaque(vstart[v]);
                                opaque(vdeg[v]);
                                const int j = tid + v * nth;
                                if (j < N) {
                                    const float lt = lp ? vlam[v] + dlt[j] : vlam[v];
                                    const float mo = Mreg[v];
                                    float acc = __builtin_fmaf(greg[v], mo - lt, lt);
                                    const int s0 = vstart[v], d = vdeg[v];
                                    float mu[CD];
#pragma unroll
                                    for (int e = 0; e < CD; ++e)
                                        if (e < d) mu[e] = X[s0 + e];
#pragma unroll
                                    for (int e = 0; e < CD; ++e)
                                        if (e < d) acc = acc + mu[e];
#pragma unroll
                                    for (int e = 0; e < CD; ++e)
                                        if (e < d) X[s0 + e] = acc - mu[e];
                                    if (tr) {
                                        a.trace_M[j] = acc;
#pragma unroll
                                        for (int e = 0; e < CD; ++e)
                                            if (e < d) a.trace_mu[s0 + e] = mu[e];
                                    }
                                    Mreg[v] = acc;
                                    if ((acc < 0.0f) != (mo < 0.0f))
                                        flip_variable(m.csc_row, s0, d, acc < 0.0f, vlam[v], par, dcount, dW);
                                }
                                __builtin_amdgcn_sched_barrier(0);
                            }
                        } else {
                            // rounds of VR variables per thread, scalars of all rounds loaded first
                            constexpr int VR = 4;
                            for (int j0 = tid; j0 < N; j0 += VR * nth) {
                                int s0[VR], dg[VR];
                                float lt[VR], g[VR], mo[VR];
#pragma unroll
                                for (int r = 0; r < VR; ++r) {
                                    const int j = j0 + r * nth;
                                    const uint32_t jj = j < N ? (uint32_t)j : 0u;
                                    s0[r] = m.col_ptr[jj];
                                    dg[r] = j < N ? m.col_ptr[jj + 1u] - s0[r] : 0;
                                    lt[r] = lp ? lam[jj] + dlt[jj] : lam[jj];
                                    g[r] = leg0 ? a.gamma0 : gam[jj];
                                    mo[r] = Mg[jj];
                                }
#pragma unroll
                                for (int r = 0; r < VR; ++r) {
                                    const int j = j0 + r * nth;
                                    if (j < N) {
                                        float acc = __builtin_fmaf(g[r], mo[r] - lt[r], lt[r]);
                                        const uint32_t b = (uint32_t)s0[r];
                                        const int d = dg[r];
                                        for (uint32_t e = b; e < b + d; ++e) acc = acc + X[e];
                                        for (uint32_t e = b; e < b + d; ++e) {
                                            const float mu = X[e];
                                            if (tr) a.trace_mu[e] = mu;
                                            X[e] = acc - mu;
                                        }
                                        if (tr) a.trace_M[j] = acc;
                                        Mg[j] = acc;
                                        if ((acc < 0.0f) != (mo[r] < 0.0f))
                                            flip_variable(m.csc_row, b, d, acc < 0.0f, lam[j], par, dcount, dW);
                                    }
                                }
                            }
                        }
                        if (dcount) atomicAdd(&sh_count, dcount);
                        if (dW != 0.0) atomicAdd(&sh_W, dW);
                        __syncthreads();
                        ++iters;
                        if (tr) {
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
                        const double W = sh_W;
                        if (!have_best || W < bestW) {
                            bestW = W;
                            have_best = true;
                            // best := current hard decision (one ballot per 64 variables)
                            if constexpr (CACHED) {
#pragma unroll
                                for (int v = 0; v < VPT; ++v) {
                                    const int jb = wid * 64 + v * nth;
                                    if (jb < N) {
                                        const unsigned long long b = __ballot(jb + lane < N && Mreg[v] < 0.0f);
                                        if (lane == 0) {
                                            best[jb >> 5] = (uint32_t)b;
                                            if ((jb >> 5) + 1 < WN) best[(jb >> 5) + 1] = (uint32_t)(b >> 32);
                                        }
                                    }
                                }
                            } else {
                                for (int jb = wid * 64; jb < N; jb += nth) {
                                    const int j = jb + lane;
                                    const unsigned long long b = __ballot(j < N && Mg[j] < 0.0f);
                                    if (lane == 0) {
                                        best[jb >> 5] = (uint32_t)b;
                                        if ((jb >> 5) + 1 < WN) best[(jb >> 5) + 1] = (uint32_t)(b >> 32);
                                    }
                                }
                            }
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
            if (!have_best) {
                // no solution: report the last hard decision
                if constexpr (CACHED) {
#pragma unroll
                    for (int v = 0; v < VPT; ++v) {
                        const int jb = wid * 64 + v * nth;
                        if (jb < N) {
                            const unsigned long long b = __ballot(jb + lane < N && Mreg[v] < 0.0f);
                            if (lane == 0) {
                                best[jb >> 5] = (uint32_t)b;
                                if ((jb >> 5) + 1 < WN) best[(jb >> 5) + 1] = (uint32_t)(b >> 32);
                            }
                        }
                    }
                } else {
                    for (int jb = wid * 64; jb < N; jb += nth) {
                        const int j = jb + lane;
                        const unsigned long long b = __ballot(j < N && Mg[j] < 0.0f);
                        if (lane == 0) {
                            best[jb >> 5] = (uint32_t)b;
                            if ((jb >> 5) + 1 < WN) best[(jb >> 5) + 1] = (uint32_t)(b >> 32);
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (!a.trace_on) {
            // corrections out; O * correction from the columns of O at its set bits
            for (int w = tid; w < m.WK; w += nth) obw[w] = 0u;
            __syncthreads();
            for (int w = tid; w < WN; w += nth) {
                const uint32_t bits = best[w];
                m.corr[row * WN + w] = bits;
                uint32_t b = bits;
                while (b) {
                    const int j = w * 32 + __builtin_ctz(b);
                    b &= b - 1u;
                    for (int e = m.ocol_ptr[j]; e < m.ocol_ptr[j + 1]; ++e) {
                        const int r = m.orow_idx[e];
                        atomicXor(obw + (r >> 5), 1u << (r & 31));
                    }
                }
            }
            __syncthreads();
            if (m.obsp)
                for (int w = tid; w < m.WK; w += nth) m.obsp[row * m.WK + w] = obw[w];
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
    st = c->m1.reserve(sizeof(float) * std::max<int64_t>((int64_t)c->M * c->P, 1));
    if (st) return st;
    RBP_HIP_CHECK(hipStreamSynchronize(stream));
    RBP_HIP_CHECK(hipMemcpy(c->lam.p, lam.data(), sizeof(float) * c->N, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(first_message_kernel, dim3(ceil_div(c->M, 256)), dim3(256), 0, stream, c->row_ptr.as<int32_t>(),
                       c->col_idx.as<int32_t>(), c->lam.as<float>(), c->m1.as<float>(), c->M, c->P);
    RBP_HIP_CHECK(hipGetLastError());
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
    m.P = c->P;
    m.rpos = c->rpos.as<int32_t>();
    m.col_ptr = c->col_ptr.as<int32_t>();
    m.csc_row = c->csc_row.as<int32_t>();
    m.m1p = c->m1.as<float>();
    m.ocol_ptr = c->ocol_ptr.as<int32_t>();
    m.orow_idx = c->orow_idx.as<int32_t>();
    m.lam = c->lam.as<float>();
    m.gtab = c->gtab.as<float>();
    m.syn = syn;
    m.corr = corr;
    m.obsp = c->k > 0 ? obsp : nullptr;
    return m;
}

typedef void (*DecodeKernel)(const DecodeLaunch);

// Variants whose per-thread index lists live in registers: a thread owns at
// most CPT checks and VPT variables (rows <= 12, columns <= 8 edges).
struct CachedVariant {
    int waves, cpt, vpt;
    DecodeKernel k;
};
#define RBP_CACHED(W, C, V) {W, C, V, relay_bp_kernel<12, 8, C, V, true, W>}
// Register-cached variants are compiled on demand; none is enabled by default
// (their control state does not fit the register budget without spilling).
static const CachedVariant kCached[] = {
    {0, 0, 0, nullptr},
};
#undef RBP_CACHED

static DecodeKernel generic_kernel(int maxdeg, bool lds) {
    if (maxdeg <= 12) return lds ? relay_bp_kernel<12, 8, 0, 0, true, 16> : relay_bp_kernel<12, 8, 0, 0, false, 16>;
    return lds ? relay_bp_kernel<32, 8, 0, 0, true, 16> : relay_bp_kernel<32, 8, 0, 0, false, 16>;
}

static constexpr int kMaxLds = 160 * 1024;

struct LaunchShape {
    int waves = 1;
    bool lds_state = true;
    bool cached = false;
    int cpt = 0, vpt = 0;
    DecodeKernel kernel = nullptr;
    int lds_bytes = 0;
    int slots = 1;
    int64_t gstride = 0;
    int Emax = 0;
    int off_sig = 0, off_par = 0, off_best = 0, off_obs = 0;
};

static const CachedVariant* find_cached(int M, int N, int waves) {
    const int nth = 64 * waves;
    const int cpt = ceil_div(M, nth), vpt = ceil_div(N, nth);
    const CachedVariant* bestv = nullptr;
    for (const CachedVariant& v : kCached)
        if (v.k && v.waves == waves && cpt <= v.cpt && vpt <= v.vpt &&
            (!bestv || v.cpt * 12 + v.vpt * 5 < bestv->cpt * 12 + bestv->vpt * 5))
            bestv = &v;
    return bestv;
}

// Launch shape for a set of models decoded together (max sizes over models).
static rbp_status plan_launch(rbp_code* const* cs, int n, uint64_t shots, LaunchShape* out) {
    int Nmax = 0, Emax = 0, WMmax = 0, WNmax = 0, WKmax = 1, maxdeg = 0, maxcol = 0, Mmax = 0;
    for (int i = 0; i < n; ++i) {
        Mmax = std::max(Mmax, cs[i]->M);
        Nmax = std::max(Nmax, cs[i]->N);
        Emax = std::max(Emax, cs[i]->E);
        WMmax = std::max(WMmax, ceil_div(cs[i]->M, 32));
        WNmax = std::max(WNmax, ceil_div(cs[i]->N, 32));
        WKmax = std::max(WKmax, ceil_div(cs[i]->k, 32));
        maxdeg = std::max(maxdeg, cs[i]->max_row_deg);
        maxcol = std::max(maxcol, cs[i]->max_col_deg);
    }
    for (int i = 1; i < n; ++i)
        if (cs[i]->P != cs[0]->P)
            return fail(RBP_ERR_UNSUPPORTED, "models decoded together must all have rows of <= 12 or all > 12 edges");
    const LaunchCfg& cfg = cs[0]->cfg;
    const int small = 4 * (2 * WMmax + WNmax + WKmax) + 512;  // + static shared variables
    const bool cached_possible = n == 1 && maxdeg <= 12 && maxcol <= 8 && cfg.state != 2 &&
                                 4 * (Emax + 4) + small <= kMaxLds;
    LaunchShape L;
    int waves = cfg.waves_per_shot;
    const CachedVariant* cv = nullptr;
    if (waves <= 0) {
        if (cached_possible)
            for (int w : {1, 2, 3, 4, 6, 8, 12, 16})
                if ((cv = find_cached(Mmax, Nmax, w))) {
                    waves = w;
                    break;
                }
        if (waves <= 0) {
            const int want = ceil_div(Nmax, 512);
            waves = 1;
            while (waves < want && waves < 8) waves <<= 1;
        }
    } else if (cached_possible) {
        cv = find_cached(Mmax, Nmax, waves);
    }
    waves = std::min(std::max(waves, 1), 16);
    int state_bytes;
    bool lds;
    if (cv) {
        L.cached = true;
        L.cpt = cv->cpt;
        L.vpt = cv->vpt;
        L.kernel = cv->k;
        lds = true;
        state_bytes = 4 * (Emax + 4);
    } else {
        state_bytes = 4 * (Emax + 4 + Nmax);
        lds = state_bytes + small <= kMaxLds;
        if (cfg.state == 1 && !lds) return fail(RBP_ERR_UNSUPPORTED, "per-shot state does not fit in LDS");
        if (cfg.state == 2) lds = false;
        L.kernel = generic_kernel(maxdeg, lds);
    }
    L.waves = waves;
    L.lds_state = lds;
    L.Emax = Emax;
    int off = lds ? state_bytes : 0;
    off = (off + 15) & ~15;
    L.off_sig = off;
    off += 4 * WMmax;
    L.off_par = off;
    off += 4 * WMmax;
    L.off_best = off;
    off += 4 * WNmax;
    L.off_obs = off;
    off += 4 * WKmax;
    L.lds_bytes = (off + 15) & ~15;
    L.gstride = lds ? 0 : ((int64_t)Nmax + Emax + 4 + 63) / 64 * 64;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(L.kernel),
                                                                64 * waves, L.lds_bytes);
    if (e != hipSuccess) return fail(RBP_ERR_HIP, std::string("occupancy query: ") + hipGetErrorString(e));
    per_cu = std::max(per_cu, 1);
    int64_t slots = (int64_t)per_cu * std::max(cs[0]->num_cus, 1);
    if (cfg.max_slots > 0) slots = std::min<int64_t>(slots, cfg.max_slots);
    slots = std::min<int64_t>(slots, (int64_t)std::min<uint64_t>(std::max<uint64_t>(shots, 1), 1ull << 40));
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
    a.queue = c0->queue.as<unsigned long long>();
    a.gstate = L.lds_state ? nullptr : c0->gstate.as<float>();
    a.gstate_stride = L.gstride;
    a.Emax = L.Emax;
    a.off_sig = L.off_sig;
    a.off_par = L.off_par;
    a.off_best = L.off_best;
    a.off_obs = L.off_obs;
    a.shots = shots;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, stream, a.queue, 1);
    RBP_HIP_CHECK(hipGetLastError());
    RBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(L.kernel),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, L.lds_bytes));
    hipLaunchKernelGGL(L.kernel, dim3(L.slots), dim3(64 * L.waves), L.lds_bytes, stream, a);
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
    const int P = maxrow <= 12 ? 12 : 32;  // row stride of the padded position table
    std::vector<int32_t> rp(M + 1, 0), ci(std::max(E, 1)), rpos((size_t)M * P, E), fillc(M, 0);
    for (int i = 0; i < M; ++i) rp[i + 1] = rp[i] + deg[i];
    for (int j = 0; j < N; ++j)
        for (int e = col_ptr[j]; e < col_ptr[j + 1]; ++e) {
            const int i = row_idx[e];
            const int pos = rp[i] + fillc[i]++;
            ci[pos] = j;
            rpos[(size_t)i * P + (pos - rp[i])] = e;
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
    c->P = P;
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
    if (!st) st = upload(c->rpos, rpos);
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
    for (DevBuf* b : {&c->row_ptr, &c->col_idx, &c->col_ptr, &c->csc_row, &c->rpos, &c->orow_ptr, &c->ocol_idx,
                      &c->ocol_ptr, &c->orow_idx, &c->thr, &c->lam, &c->m1, &c->gtab, &c->queue, &c->gstate, &c->trace_hit})
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

rbp_status rbp_count_failures(const uint32_t* obsp, const uint32_t* obs, const rbp_shot_stats* st, uint64_t shots,
                              int32_t words, unsigned long long* count, void* stream_) {
    if (!obsp || !obs || !st || !count) return fail(RBP_ERR_INVALID_ARG, "NULL argument");
    if (words < 0) return fail(RBP_ERR_INVALID_ARG, "obs_words < 0");
    if (shots == 0) return RBP_OK;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    hipLaunchKernelGGL(count_failures_kernel, dim3((unsigned)ceil_div((int64_t)shots, 256)), dim3(256), 0, stream, obsp,
                       obs, st, shots, words, count);
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

rbp_status rbp_code_llr(rbp_code_t c, const double* priors, float* llr, void* stream_) {
    if (!c || !llr) return fail(RBP_ERR_INVALID_ARG, "NULL argument");
    rbp_status st = check_priors(priors, c->N);
    if (st) return st;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    st = ensure_llr(c, priors, stream);
    if (st) return st;
    RBP_HIP_CHECK(hipMemcpyAsync(llr, c->lam.p, sizeof(float) * c->N, hipMemcpyDeviceToDevice, stream));
    return RBP_OK;
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
    rbp_status st = plan_launch(cs, 1, 1ull << 40, &L);
    if (st) return st;
    if (cfg) {
        cfg->waves_per_shot = L.waves;
        cfg->state = (L.lds_state ? 1 : 2) + (L.cached ? 8 : 0);
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
