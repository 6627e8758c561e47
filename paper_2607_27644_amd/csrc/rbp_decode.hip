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
//                      it fits, else in a per-slot device buffer; variables and
//                      checks are processed in degree-sorted groups of 64, one
//                      group per wavefront step.  The syndrome of the hard
//                      decision and the weight of the current solution are
//                      tracked incrementally: a variable whose decision flips XORs
//                      its checks' parity bits with LDS atomics and moves the
//                      weight, so convergence and solution weights cost no extra
//                      sweep or reduction.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rbp_common.h"
#include "../../include/rbp_test.h"

namespace rbp {

// ---------------------------------------------------------------------------
// Sampling: independent faults e_j ~ Bernoulli(p_j); sigma = H e; o = O e.
// The mechanisms are cut into 64 segments of L = ceil(N / 64), one per lane.
// In a segment, candidate positions follow geometric gaps of parameter
// pmax = max p_j: the gap G before the next candidate is the number of k in
// 1..len with T_k > w for the next 32-bit word w, T_k = floor((1 - pmax)^k 2^32)
// (a host table), so P(G >= k) = (1 - pmax)^k to 2^-32; a candidate j with
// p_j < pmax is kept when the next word is below A_j = floor(p_j / pmax 2^32).
// Words of segment g: Philox4x32-10, key = seed, counter (g 2^24 + d / 4,
// shot lo, shot hi, 3), word d mod 4 for d = 0, 1, ...  At p = 1e-3 a lane
// draws about one word per shot instead of one per mechanism.
// ---------------------------------------------------------------------------
struct SampleArgs {
    int32_t M, N, k, WM, WK, WN, L;
    const int32_t* col_ptr;
    const int32_t* csc_row;
    const int32_t* ocol_ptr;
    const int32_t* orow_idx;
    const uint32_t* gap;  // [L] T_k, decreasing
    const uint32_t* acc;  // [N] A_j; 0xFFFFFFFF where p_j = pmax (kept without a draw)
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
    const int words = a.WM + a.WK + (a.err ? a.WN : 0);
    uint32_t* sy = sm_sample + wid * words;
    uint32_t* ob = sy + a.WM;
    uint32_t* er = ob + a.WK;
    for (int x = lane; x < words; x += 64) sy[x] = 0u;
    __syncthreads();
    const int base = lane * a.L;
    const int len = min(a.L, a.N - base);
    if (live && len > 0) {
        const uint64_t sid = a.offset + s;
        const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
        const uint32_t c0 = (uint32_t)lane << 24;
        U4 buf{0u, 0u, 0u, 0u};
        uint32_t have = 0xFFFFFFFFu, d = 0;
        int pos = -1;
        for (;;) {
            if ((d >> 2) != have) {
                have = d >> 2;
                buf = philox4x32_10(U4{c0 + have, (uint32_t)sid, (uint32_t)(sid >> 32), 3u}, k0, k1);
            }
            const uint32_t w = u4_get(buf, (int)(d & 3u));
            ++d;
            // G = number of leading table entries above w (T decreasing)
            int G;
            if (a.gap[len - 1] > w) {
                G = len;
            } else {
                int lo = 0, hi = len - 1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (a.gap[mid] > w)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                G = lo;
            }
            pos += G + 1;
            if (pos >= len) break;
            const int j = base + pos;
            const uint32_t A = a.acc[j];
            if (A != 0xFFFFFFFFu) {
                if ((d >> 2) != have) {
                    have = d >> 2;
                    buf = philox4x32_10(U4{c0 + have, (uint32_t)sid, (uint32_t)(sid >> 32), 3u}, k0, k1);
                }
                const uint32_t u = u4_get(buf, (int)(d & 3u));
                ++d;
                if (u >= A) continue;
            }
            for (int e = a.col_ptr[j]; e < a.col_ptr[j + 1]; ++e) {
                const int i = a.csc_row[e];
                atomicXor(sy + (i >> 5), 1u << (i & 31));
            }
            for (int e = a.ocol_ptr[j]; e < a.ocol_ptr[j + 1]; ++e) {
                const int i = a.orow_idx[e];
                atomicXor(ob + (i >> 5), 1u << (i & 31));
            }
            if (a.err) atomicOr(er + (j >> 5), 1u << (j & 31));
        }
    }
    __syncthreads();
    if (live) {
        for (int x = lane; x < a.WM; x += 64) a.syn[s * a.WM + x] = sy[x];
        if (a.obs)
            for (int x = lane; x < a.WK; x += 64) a.obs[s * a.WK + x] = ob[x];
        if (a.err)
            for (int x = lane; x < a.WN; x += 64) a.err[s * a.WN + x] = er[x];
    }
}

// ---------------------------------------------------------------------------
// Relay-leg memory strengths gamma_j^(r), r = 1..R, drawn per variable j from
// Philox (key = gamma seed, counter = (j/4, r, 0, 1), word j%4) and stored by
// variable position (see the layout below): table[(r-1)*Np + pos].
// ---------------------------------------------------------------------------
__global__ void gamma_table_kernel(float* out, const int32_t* vord, int32_t Np, int32_t R, float gmin, float gmax,
                                   uint64_t seed) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)Np * R;
    if (idx >= total) return;
    const int32_t r = (int32_t)(idx / Np) + 1, pos = (int32_t)(idx % Np);
    const int32_t j = vord[pos];
    if (j < 0) {
        out[idx] = 0.0f;
        return;
    }
    const U4 o = philox4x32_10(U4{(uint32_t)(j >> 2), (uint32_t)r, 0u, 1u}, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float u = (float)(u4_get(o, j & 3) >> 8) * (1.0f / 16777216.0f);
    const float span = gmax - gmin;
    out[idx] = __builtin_fmaf(u, span, gmin);
}

// {Lambda, gamma} by leg and position, read by the variable sweep with one
// 8-byte load: row 0 holds gamma0 (first leg), row r the gamma of relay leg r.
__global__ void lam_gamma_kernel(float2* out, const float* lamp, const float* gtab, int32_t Np, int32_t R,
                                 float gamma0) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)Np * (R + 1);
    if (idx >= total) return;
    const int32_t r = (int32_t)(idx / Np), pos = (int32_t)(idx % Np);
    out[idx] = make_float2(lamp[pos], r == 0 ? gamma0 : gtab[(int64_t)(r - 1) * Np + pos]);
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
// Shot order for rbp_decode: heaviest syndromes first.  A shot's decoding time
// grows with its syndrome weight, and the batch ends when its slowest shot
// ends; handing the heavy shots out first lets them overlap the light ones
// instead of finishing last.  Counting sort on min(weight, 255), descending;
// the order within a weight is arbitrary, which no output depends on.
// ---------------------------------------------------------------------------
constexpr int kOrderBins = 256;  // also the block size of the ordering kernels (one bin per thread)

__device__ __forceinline__ int weight_bin(const uint32_t* row, int words) {
    int w = 0;
    for (int x = 0; x < words; ++x) w += __popc(row[x]);
    return w < kOrderBins - 1 ? w : kOrderBins - 1;
}

// histogram of the batch: per-block counts in LDS, one global atomic per block
// and non-empty bin
__global__ void __launch_bounds__(256) order_hist_kernel(const uint32_t* syn, int words, uint64_t shots,
                                                          uint32_t* hist) {
    __shared__ uint32_t h[kOrderBins];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (s < shots) atomicAdd(&h[weight_bin(syn + s * words, words)], 1u);
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// counts -> first position of each bin, heaviest bin first (one thread; 256 bins)
__global__ void order_scan_kernel(uint32_t* hist) {
    if (threadIdx.x != 0) return;
    uint32_t run = 0;
    for (int b = kOrderBins - 1; b >= 0; --b) {
        const uint32_t c = hist[b];
        hist[b] = run;
        run += c;
    }
}

// each block reserves a range per non-empty bin (one global atomic), then ranks
// its shots inside the ranges with LDS atomics
__global__ void __launch_bounds__(256) order_scatter_kernel(const uint32_t* syn, int words, uint64_t shots,
                                                             uint32_t* cursor, uint32_t* order) {
    __shared__ uint32_t cnt[kOrderBins];
    __shared__ uint32_t base[kOrderBins];
    cnt[threadIdx.x] = 0u;
    __syncthreads();
    const uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    int bin = 0;
    uint32_t rank = 0;
    if (s < shots) {
        bin = weight_bin(syn + s * words, words);
        rank = atomicAdd(&cnt[bin], 1u);
    }
    __syncthreads();
    const uint32_t c = cnt[threadIdx.x];
    base[threadIdx.x] = c ? atomicAdd(&cursor[threadIdx.x], c) : 0u;
    __syncthreads();
    if (s < shots) order[base[bin] + rank] = (uint32_t)s;
}

__global__ void zero_u32_kernel(uint32_t* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Persistent Relay-BP
//
// A shot slot's state is one float per Tanner-graph edge slot, X[S], plus the
// marginals Mg[Np].  The check sweep reads nu_{j->i} from X and overwrites it
// in place with mu_{i->j}; the variable sweep reads mu, forms the marginal M_j
// and overwrites X with nu_{j->i} = M_j - mu_{i->j}.
//
// Layout, chosen for 64-lane wavefronts:
//  * Variables are sorted by degree (descending, stable) and cut into groups
//    of 64.  Lane l of group g owns the variable at position 64 g + l, and the
//    q-th edge of that variable (q-th check in ascending order) lives in slot
//    vbase_g + 64 q + l.  A wave's loads and stores of X in the variable sweep
//    are unit-stride (no LDS bank conflicts) with the slot step folded into the
//    instruction's offset, and Mg is kept by position.
//  * Checks are sorted and grouped the same way.  Lane l of row group g owns
//    the check at row position 64 g + l; the byte offsets of its edge slots
//    (columns ascending) sit contiguously at rposp[rbase_g + st_g l + p], read
//    with 16-byte loads (st_g: the group's degree rounded up to 4).
//  * Every member of a group has the group's degree, except in the few groups
//    that straddle a degree boundary or are partial ("mixed").  Loops over a
//    member's edges therefore have a wave-uniform trip count and are unrolled
//    per degree; mixed row groups pad their rows with the offset of X[S], a
//    read-only +inf cell (neutral for both minima and the sign product), and
//    redirect those writes to X[S+1]; mixed variable groups mask their sums.
//  * Lambda_j and the leg's gamma_j are read together, one 8-byte load per
//    lane and group, from a {Lambda, gamma} table with one row per leg.
// The first iteration of a plain leg reads no state: nu(0) = Lambda, so
// mu(1) = (-1)^sigma_i * (least |Lambda| of the other variables of the row),
// a per-model table (layout of rposp) computed once per priors.
// Waves of a slot spend most of their time waiting on table loads, so the
// launch aims at about 8 waves per SIMD: the kernel is also built for a
// 64-VGPR budget, used when that fits more slots per CU.
// ---------------------------------------------------------------------------
constexpr int kMaxModels = 8;
constexpr int kShotRun = 4;  // shots taken per queue atomic while many remain

struct DecodeModel {
    int32_t M, N, E, k, WM, WN, WK;
    int32_t S;             // edge slots; X[S] = +inf (read-only padding cell), X[S+1] write-only cell
    int32_t GR, GV, Np;    // row groups, variable groups, Np = 64 GV variable positions
    int32_t GRw;           // leading row groups stored with more than 32 edges (rows sorted by degree)
    const int4* rgrp;      // [GR] {offset in rposp, stored degree, mixed, lane stride}
    const int32_t* rposp;  // byte offsets 4 x slot of the edges of each row (lane-major per group), 4 S padding
    const int32_t* rposw;  // the same for writes, 4 (S + 1) for padding
    const float* m1pp;     // first-iteration magnitudes, layout of rposp
    const int32_t* rord;   // [64 GR] check at each row position, -1 for padding
    const int4* vgrp;      // [GV] {first slot, degree, mixed, 0}
    const int32_t* vord;   // [Np] variable at each position, -1 for padding (positions N.. are padding)
    const int32_t* vinv;   // [N] position of each variable
    const int32_t* vdeg;   // [Np] degree at each position (0 for padding)
    const int32_t* scheck; // [S] check of each slot (-1 unused)
    const int32_t* scsc;   // [S] CSC edge index of each slot (-1 unused)
    const float* lamp;     // [Np] Lambda by position (0 for padding)
    const float* gtabp;    // [max(R,1)][Np] relay-leg memory strengths by position
    const float2* lg;      // [R+1][Np] {Lambda, gamma} by leg and position
    const int32_t* ocol_ptr;  // [N+1] observables, CSC
    const int32_t* orow_idx;
    // compact state (rows of at most 16 edges; null otherwise)
    const int32_t* cvar;      // layout of rposp: LDS byte address of the marginal of each edge's variable
    const uint32_t* vrec;     // [S] 16 * (row position) + (edge code in the row) of each edge slot
    const uint4* r1rec;       // [64 GR] first-iteration row records of a plain leg
    int32_t coff_M;           // LDS offset of the marginals in the compact layout (16 * 64 GR + 16)
    const uint32_t* syn;
    uint32_t* corr;
    uint32_t* obsp;
};

struct DecodeLaunch {
    DecodeModel m[kMaxModels];
    int32_t n_models;
    const uint8_t* shot_code;
    const uint32_t* shot_index;
    int32_t stats_by_row;  // statistics at the shot's row (rbp_decode) or at its ticket (rbp_decode_multi)
    uint64_t shots;
    const float* delta;
    const uint16_t* delta16;  // BF16 proposal adjustments (rbp_decode_proposal), else null
    int32_t d16_pos;          // delta16 rows by position (Np entries), not by variable (N entries)
    rbp_shot_stats* stats;
    unsigned long long* queue;
    float* gstate;
    int64_t gstate_stride;
    int32_t Smax;  // device-memory state: marginals at X + Smax + 4
    // byte offsets in dynamic LDS (X itself starts at 0 when it lives there)
    int32_t off_M, off_sig, off_sigp, off_par, off_bestp, off_best, off_obs, off_misc;
    int32_t off_d16;  // compact state with BF16 adjustments: their LDS copy by position
    int32_t off_grp;  // compact state: the model's variable and row group descriptors (int4 each)
    int32_t nsub;        // shots per workgroup of the multi-shot kernel (1: the one-shot kernels)
    int32_t sub_stride;  // LDS bytes between the multi-shot kernel's shot sub-slots (a multiple of 256)
    float gamma0;
    int32_t T0, Tr, R, S, crit;
    int32_t trace_on, trace_phase, trace_leg, trace_t;
    float* trace_M;
    float* trace_mu;
    int32_t* trace_hit;
};

// Per-slot scalars, in dynamic LDS (the kernel has no static LDS, so that X
// can start at address 0 and a slot's byte offset is its LDS address).
struct SlotMisc {
    unsigned long long shot;
    double W;
    int32_t count;
    int32_t pad;
    int32_t red[16];
};

// mu(1) magnitudes of a plain leg in the layout of rposp:
// m1pp[rbase_g + l st_g + p] = least |Lambda_j'| over the other variables j' of the row
__global__ void first_message_kernel(const int32_t* row_ptr, const int32_t* col_idx, const int32_t* rord,
                                     const int4* rgrp, const float* lam, float* m1pp, int32_t npos) {
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= npos) return;
    const int i = rord[pos];
    if (i < 0) return;
    const int4 gi = rgrp[pos >> 6];
    float* out = m1pp + gi.x + (pos & 63) * gi.w;
    const int rs = row_ptr[i], re = row_ptr[i + 1];
    float min1 = INFINITY, min2 = INFINITY;
    for (int e = rs; e < re; ++e) {
        const float av = fabsf(lam[col_idx[e]]);
        min2 = __builtin_amdgcn_fmed3f(min1, min2, av);
        min1 = fminf(min1, av);
    }
    for (int e = rs; e < re; ++e) {
        const float av = fabsf(lam[col_idx[e]]);
        out[e - rs] = (av == min1) ? min2 : min1;
    }
}

// median of three unsigned values: the new second minimum, given min1 <= min2
__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

typedef __attribute__((address_space(3))) float lds_float;

// Access to a slot's state by byte offset.  In LDS the state starts at LDS
// address 0 (the kernel declares no static LDS, so its dynamic LDS begins
// there) and a byte offset is the address itself; in device memory it is
// added to the slot's base pointer.
template <bool LDS>
struct State {
    float* g;
    __device__ __forceinline__ float ld(uint32_t off) const {
        if constexpr (LDS)
            return *reinterpret_cast<const lds_float*>((size_t)off);
        else
            return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(g) + (uint64_t)off);
    }
    __device__ __forceinline__ void st(uint32_t off, float v) const {
        if constexpr (LDS)
            *reinterpret_cast<lds_float*>((size_t)off) = v;
        else
            *reinterpret_cast<float*>(reinterpret_cast<char*>(g) + (uint64_t)off) = v;
    }
};

// element i of a read-only table, addressed as base + 32-bit byte offset
template <class T>
__device__ __forceinline__ T ldg(const T* base, uint32_t i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint64_t)(i * (uint32_t)sizeof(T)));
}

// One check row of the min-sum update with D edge slots, in place on X.  The
// magnitudes compare as unsigned integers (|nu| bit patterns order like the
// floats); the outgoing sign is sigma_i times the signs of the other nu.  On the
// first iteration of a plain leg the messages come from the m1 table.  The
// row's entries of the read-offset, write-offset and m1 tables are contiguous
// (lane-major, stride (D + 3) & ~3), so each is read with 16-byte loads; rows
// of a mixed group read padding from the +inf cell and write it to the
// write-only cell.
template <int D, bool MIXED, bool LDS>
__device__ __forceinline__ void check_row(const State<LDS> X, const int32_t* rp, const int32_t* wp, const float* mp,
                                          uint32_t sbit, bool first) {
    constexpr int Q = (D + 3) / 4;
    uint32_t pos[4 * Q], wpos[4 * Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int4 v = reinterpret_cast<const int4*>(rp)[k];
        pos[4 * k] = (uint32_t)v.x;
        pos[4 * k + 1] = (uint32_t)v.y;
        pos[4 * k + 2] = (uint32_t)v.z;
        pos[4 * k + 3] = (uint32_t)v.w;
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        if (MIXED) {
            const int4 v = reinterpret_cast<const int4*>(wp)[k];
            wpos[4 * k] = (uint32_t)v.x;
            wpos[4 * k + 1] = (uint32_t)v.y;
            wpos[4 * k + 2] = (uint32_t)v.z;
            wpos[4 * k + 3] = (uint32_t)v.w;
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) wpos[4 * k + r] = pos[4 * k + r];
        }
    }
    if (first) {
        float m1v[4 * Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const float4 v = reinterpret_cast<const float4*>(mp)[k];
            m1v[4 * k] = v.x;
            m1v[4 * k + 1] = v.y;
            m1v[4 * k + 2] = v.z;
            m1v[4 * k + 3] = v.w;
        }
#pragma unroll
        for (int p = 0; p < D; ++p) X.st(wpos[p], __uint_as_float(__float_as_uint(m1v[p]) | sbit));
        return;
    }
    uint32_t nu[D], av[D];
#pragma unroll
    for (int p = 0; p < D; ++p) nu[p] = __float_as_uint(X.ld(pos[p]));
    uint32_t min1 = 0x7f800000u, min2 = 0x7f800000u, sgn = sbit;
#pragma unroll
    for (int p = 0; p < D; ++p) {
        av[p] = nu[p] & 0x7fffffffu;
        sgn ^= nu[p];
        min2 = umed3(min1, min2, av[p]);
        min1 = min1 < av[p] ? min1 : av[p];
    }
#pragma unroll
    for (int p = 0; p < D; ++p) {
        const uint32_t mag = (av[p] == min1) ? min2 : min1;
        X.st(wpos[p], __uint_as_float(mag | ((sgn ^ nu[p]) & 0x80000000u)));
    }
}

// rp, wp, mp: the group's blocks of the three tables; lane l's entries start at
// l * ((D + 3) & ~3)
template <int D, bool LDS>
__device__ __forceinline__ void check_row_d(const State<LDS> X, const int32_t* rp, const int32_t* wp, const float* mp,
                                            int lane, bool mixed, uint32_t sbit, bool first) {
    constexpr int ST = (D + 3) & ~3;
    const uint32_t o = (uint32_t)lane * ST;
    if (mixed)
        check_row<D, true>(X, rp + o, wp + o, mp + o, sbit, first);
    else
        check_row<D, false>(X, rp + o, wp + o, mp + o, sbit, first);
}

// Rows of more than 32 edges (circuit-level models) with D slots, D a multiple
// of 8: the same operations as check_row in two rolled passes over 16-byte
// chunks of the tables, the first for the two smallest magnitudes and the sign
// product, the second re-reading each nu before its own slot is overwritten.
template <bool MIXED, bool LDS>
__device__ __forceinline__ void check_row_rolled(const State<LDS> X, const int32_t* rp, const int32_t* wp,
                                                 const float* mp, int D, uint32_t sbit, bool first) {
    const int Q = D >> 2;
    const int4* r4 = reinterpret_cast<const int4*>(rp);
    const int4* w4 = reinterpret_cast<const int4*>(MIXED ? wp : rp);
    if (first) {
        const float4* m4 = reinterpret_cast<const float4*>(mp);
        for (int k = 0; k < Q; ++k) {
            const int4 w = w4[k];
            const float4 v = m4[k];
            X.st((uint32_t)w.x, __uint_as_float(__float_as_uint(v.x) | sbit));
            X.st((uint32_t)w.y, __uint_as_float(__float_as_uint(v.y) | sbit));
            X.st((uint32_t)w.z, __uint_as_float(__float_as_uint(v.z) | sbit));
            X.st((uint32_t)w.w, __uint_as_float(__float_as_uint(v.w) | sbit));
        }
        return;
    }
    uint32_t min1 = 0x7f800000u, min2 = 0x7f800000u, sgn = sbit;
    for (int k = 0; k < Q; ++k) {
        const int4 v = r4[k];
        const uint32_t n[4] = {__float_as_uint(X.ld((uint32_t)v.x)), __float_as_uint(X.ld((uint32_t)v.y)),
                               __float_as_uint(X.ld((uint32_t)v.z)), __float_as_uint(X.ld((uint32_t)v.w))};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t av = n[r] & 0x7fffffffu;
            sgn ^= n[r];
            min2 = umed3(min1, min2, av);
            min1 = min1 < av ? min1 : av;
        }
    }
    for (int k = 0; k < Q; ++k) {
        const int4 v = r4[k];
        const int4 w = w4[k];
        const uint32_t n[4] = {__float_as_uint(X.ld((uint32_t)v.x)), __float_as_uint(X.ld((uint32_t)v.y)),
                               __float_as_uint(X.ld((uint32_t)v.z)), __float_as_uint(X.ld((uint32_t)v.w))};
        const uint32_t wo[4] = {(uint32_t)w.x, (uint32_t)w.y, (uint32_t)w.z, (uint32_t)w.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t mag = ((n[r] & 0x7fffffffu) == min1) ? min2 : min1;
            X.st(wo[r], __uint_as_float(mag | ((sgn ^ n[r]) & 0x80000000u)));
        }
    }
}

// stored row degrees: 2..12 exactly, 13..32 padded to 16, 24 or 32 slots,
// larger rows to a multiple of 8 (rolled)
template <int RD, bool LDS>
__device__ __forceinline__ void check_dispatch(const State<LDS> X, const int32_t* rp, const int32_t* wp,
                                               const float* mp, int lane, int dg, bool mixed, uint32_t sbit,
                                               bool first) {
    switch (dg) {
#define RBP_ROW(D) \
    case D: check_row_d<D>(X, rp, wp, mp, lane, mixed, sbit, first); break;
        RBP_ROW(2) RBP_ROW(3) RBP_ROW(4) RBP_ROW(5) RBP_ROW(6) RBP_ROW(7)
        RBP_ROW(8) RBP_ROW(9) RBP_ROW(10) RBP_ROW(11) RBP_ROW(12)
        default:
            if constexpr (RD > 12) {
                switch (dg) {
                    RBP_ROW(16) RBP_ROW(24) RBP_ROW(32)
                    default: {
                        const uint32_t o = (uint32_t)lane * (uint32_t)dg;
                        if (mixed)
                            check_row_rolled<true>(X, rp + o, wp + o, mp + o, dg, sbit, first);
                        else
                            check_row_rolled<false>(X, rp + o, wp + o, mp + o, dg, sbit, first);
                    } break;
                }
            }
            break;
#undef RBP_ROW
    }
}

// One variable with D edge slots (byte offsets sb + 256 q): M = Lambda~ +
// sum_q mu_q (checks ascending), then nu_q = M - mu_q written back (WRITE), or
// mu left in place (see the first iteration of a plain leg in the kernel).  In
// a mixed group only the member's own vd edges enter the sum (its remaining
// slots are unused by any check).
// Marginals saturate at +-2^90: shots that never converge would otherwise
// overflow FP32 (inf, then inf - inf = NaN) within a few legs.  The bound keeps
// every message finite (a check message grows by at most 2^90 per iteration)
// and is never reached by shots that converge in practice.
constexpr float kMSat = 0x1p90f;
__device__ __forceinline__ float sat(float x) { return __builtin_amdgcn_fmed3f(x, -kMSat, kMSat); }

template <int D, bool MIXED, bool WRITE, bool LDS>
__device__ __forceinline__ float var_member(const State<LDS> X, uint32_t sb, int vd, float acc) {
    float mu[D];
#pragma unroll
    for (int q = 0; q < D; ++q) mu[q] = X.ld(sb + 256u * q);
#pragma unroll
    for (int q = 0; q < D; ++q) acc = (!MIXED || q < vd) ? acc + mu[q] : acc;
    acc = sat(acc);
    if (WRITE) {
#pragma unroll
        for (int q = 0; q < D; ++q) X.st(sb + 256u * q, acc - mu[q]);
    }
    return acc;
}

// rolled form for large degrees and traced iterations
template <bool LDS>
__device__ __forceinline__ float var_member_rolled(const State<LDS> X, bool write, uint32_t sb, int vd, float acc,
                                                   float* trace_mu, const int32_t* scsc) {
    for (int q = 0; q < vd; ++q) acc = acc + X.ld(sb + 256u * q);
    acc = sat(acc);
    for (int q = 0; q < vd; ++q) {
        const uint32_t o = sb + 256u * q;
        const float mu = X.ld(o);
        if (trace_mu) trace_mu[scsc[o >> 2]] = mu;
        if (write) X.st(o, acc - mu);
    }
    return acc;
}

template <int D, bool WRITE, bool LDS>
__device__ __forceinline__ float var_member_d(const State<LDS> X, uint32_t sb, bool mixed, int vd, float acc) {
    return mixed ? var_member<D, true, WRITE>(X, sb, vd, acc) : var_member<D, false, WRITE>(X, sb, vd, acc);
}

template <bool WRITE, bool LDS>
__device__ __forceinline__ float var_dispatch(const State<LDS> X, uint32_t sb, int dg, bool mixed, int vd, float acc) {
    switch (dg) {
        case 0: return sat(acc);
#define RBP_VAR(D) \
    case D: return var_member_d<D, WRITE>(X, sb, mixed, vd, acc);
        RBP_VAR(1) RBP_VAR(2) RBP_VAR(3) RBP_VAR(4) RBP_VAR(5) RBP_VAR(6) RBP_VAR(7) RBP_VAR(8)
#undef RBP_VAR
        default: return var_member_rolled(X, WRITE, sb, vd, acc, nullptr, nullptr);
    }
}

// nu_q = M - mu_q for one variable whose mu were left in X (same operands as
// the variable sweep's own write-back)
template <int D, bool LDS>
__device__ __forceinline__ void extrinsic_d(const State<LDS> X, uint32_t sb, float M) {
    float mu[D];
#pragma unroll
    for (int q = 0; q < D; ++q) mu[q] = X.ld(sb + 256u * q);
#pragma unroll
    for (int q = 0; q < D; ++q) X.st(sb + 256u * q, M - mu[q]);
}

template <bool LDS>
__device__ __forceinline__ void extrinsic_dispatch(const State<LDS> X, uint32_t sb, int dg, float M) {
    switch (dg) {
        case 0: return;
#define RBP_EXT(D) \
    case D: extrinsic_d<D>(X, sb, M); return;
        RBP_EXT(1) RBP_EXT(2) RBP_EXT(3) RBP_EXT(4) RBP_EXT(5) RBP_EXT(6) RBP_EXT(7) RBP_EXT(8)
#undef RBP_EXT
        default:
            for (int q = 0; q < dg; ++q) {
                const uint32_t o = sb + 256u * q;
                X.st(o, M - X.ld(o));
            }
    }
}

// A variable whose hard decision flips toggles the parity bits of its checks
// (LDS atomics); the caller moves the solution weight by +-Lambda_j.
__device__ __forceinline__ void flip_slots(const int32_t* scheck, uint32_t sb, int vd, uint32_t* par, int& dcount) {
    for (int q = 0; q < vd; ++q) {
        const int i = ldg(scheck, (sb >> 2) + 64u * q);
        const uint32_t bit = 1u << (i & 31);
        const uint32_t old = atomicXor(par + (i >> 5), bit);
        dcount += (old & bit) ? -1 : 1;
    }
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// the proposal's adjustment of variable j: FP32, or BF16 widened exactly
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float delta_of(const float* dlt, const uint16_t* dl16, int j) {
    return dl16 ? bf16_to_f32(dl16[j]) : dlt[j];
}

// the adjustment of the variable j at position pp: by position when the BF16
// rows are laid out by position
__device__ __forceinline__ float delta_at(const float* dlt, const uint16_t* dl16, bool by_pos, int j, uint32_t pp) {
    return by_pos ? bf16_to_f32(dl16[pp]) : delta_of(dlt, dl16, j);
}

constexpr int kQuarterRegs = 32;  // edges per lane kept in registers (rows up to 128)

// the four lanes of a row exchange their two smallest magnitudes and sign
// products: the two smallest of the row are the two smallest of the four pairs
template <int LPR = 4>
__device__ __forceinline__ void quarter_combine(uint32_t& min1, uint32_t& min2, uint32_t& sgn) {
#pragma unroll
    for (int d = 1; d < LPR; d <<= 1) {
        const uint32_t b1 = (uint32_t)__shfl_xor((int)min1, d, 64);
        const uint32_t b2 = (uint32_t)__shfl_xor((int)min2, d, 64);
        sgn ^= (uint32_t)__shfl_xor((int)sgn, d, 64);
        const uint32_t hi = min1 < b1 ? b1 : min1;
        const uint32_t lo2 = min2 < b2 ? min2 : b2;
        min1 = min1 < b1 ? min1 : b1;
        min2 = hi < lo2 ? hi : lo2;
    }
}

// A quarter of a row group of stored degree D > 32 (multiple of 8): rows
// q*16 + (lane >> 2) of the group, four lanes per row, lane k of a row taking
// the edges k, k + 4, ...  The lanes combine their two smallest magnitudes and
// sign products (quarter_combine), so every message equals the one-lane
// update's.
template <bool MIXED, bool LDS, bool KEEP = true, int REGS = kQuarterRegs, int LPR = 4>
__device__ __forceinline__ void check_quarter(const State<LDS> X, const int32_t* rp, const int32_t* wp,
                                              const float* mp, int lane, int q, int D, uint32_t sbit, bool first) {
    const int k = lane & (LPR - 1);
    const uint32_t o = (uint32_t)(q * (64 / LPR) + lane / LPR) * (uint32_t)D;
    const int32_t* r = rp + o;
    const int32_t* w = (MIXED ? wp : rp) + o;
    if (first) {
        const float* mm = mp + o;
        for (int p = k; p < D; p += LPR) X.st((uint32_t)w[p], __uint_as_float(__float_as_uint(mm[p]) | sbit));
        return;
    }
    uint32_t min1 = 0x7f800000u, min2 = 0x7f800000u, sgn = 0u;
    if (D <= LPR * REGS) {
        // rows of up to 128 edges: the lane's messages are gathered at once and
        // kept in registers for the write pass
        uint32_t pos[KEEP ? REGS : 1], nv[REGS];
        if constexpr (KEEP) {
#pragma unroll
            for (int i = 0; i < REGS; ++i) pos[i] = k + LPR * i < D ? (uint32_t)r[k + LPR * i] : 0u;
#pragma unroll
            for (int i = 0; i < REGS; ++i)
                nv[i] = k + LPR * i < D ? __float_as_uint(X.ld(pos[i])) : 0x7f800000u;
        } else {
#pragma unroll
            for (int i = 0; i < REGS; ++i)
                nv[i] = k + LPR * i < D ? __float_as_uint(X.ld((uint32_t)r[k + LPR * i])) : 0x7f800000u;
        }
#pragma unroll
        for (int i = 0; i < REGS; ++i) {
            const uint32_t av = nv[i] & 0x7fffffffu;
            sgn ^= nv[i];
            min2 = umed3(min1, min2, av);
            min1 = min1 < av ? min1 : av;
        }
        quarter_combine<LPR>(min1, min2, sgn);
        sgn ^= sbit;
#pragma unroll
        for (int i = 0; i < REGS; ++i) {
            if (k + LPR * i < D) {
                const uint32_t mag = ((nv[i] & 0x7fffffffu) == min1) ? min2 : min1;
                const uint32_t at = MIXED ? (uint32_t)w[k + LPR * i] : (KEEP ? pos[KEEP ? i : 0] : (uint32_t)r[k + LPR * i]);
                X.st(at, __uint_as_float(mag | ((sgn ^ nv[i]) & 0x80000000u)));
            }
        }
        return;
    }
    for (int p = k; p < D; p += LPR) {
        const uint32_t n = __float_as_uint(X.ld((uint32_t)r[p]));
        const uint32_t av = n & 0x7fffffffu;
        sgn ^= n;
        min2 = umed3(min1, min2, av);
        min1 = min1 < av ? min1 : av;
    }
    quarter_combine<LPR>(min1, min2, sgn);
    sgn ^= sbit;
    for (int p = k; p < D; p += LPR) {
        const uint32_t n = __float_as_uint(X.ld((uint32_t)r[p]));
        const uint32_t mag = ((n & 0x7fffffffu) == min1) ? min2 : min1;
        X.st((uint32_t)w[p], __uint_as_float(mag | ((sgn ^ n) & 0x80000000u)));
    }
}

// Rows over 32 edges go in parts of a group, several lanes per row
// (check_quarter: one gather pass, half the cache lines of the rolled update),
// in the build with state in device memory and 128 VGPRs.  Circuit-level
// ZSZ-LP-320 and -550 decode 1.5-1.7x the shots/s of the rolled update with
// four lanes per row.
template <int RD, bool LDS_STATE, int MINW>
constexpr bool kQuarterRows = RD > 12 && !LDS_STATE && MINW == 4;
// lanes per wide row there: 8 (13 messages per lane for rows up to 104
// edges) measured 8-17 % more shots/s than 4 on circuit-level ZSZ-LP-320/-550
constexpr int kPersLpr = 8;

// MINW: waves per SIMD the register allocation must allow (4: up to 128
// VGPRs; 8: up to 64, for launch shapes whose LDS permits 8 waves per SIMD).
template <int RD, bool LDS_STATE, int MINW>
__global__ void __launch_bounds__(1024, MINW) relay_bp_kernel(const DecodeLaunch a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63;
    const int wid = uniform(tid >> 6), nw = nth >> 6;
    State<LDS_STATE> X;
    float* Mg;
    if constexpr (LDS_STATE) {
        X.g = nullptr;
        Mg = reinterpret_cast<float*>(smem + a.off_M);
    } else {
        X.g = a.gstate + (int64_t)blockIdx.x * a.gstate_stride;
        Mg = X.g + a.Smax + 4;
    }
    uint32_t* sig = reinterpret_cast<uint32_t*>(smem + a.off_sig);
    uint32_t* sigp = reinterpret_cast<uint32_t*>(smem + a.off_sigp);
    uint32_t* par = reinterpret_cast<uint32_t*>(smem + a.off_par);
    uint32_t* bestp = reinterpret_cast<uint32_t*>(smem + a.off_bestp);
    uint32_t* best = reinterpret_cast<uint32_t*>(smem + a.off_best);
    uint32_t* obw = reinterpret_cast<uint32_t*>(smem + a.off_obs);
    SlotMisc* ms = reinterpret_cast<SlotMisc*>(smem + a.off_misc);
    // the current model's group descriptors in LDS when they fit (copied when
    // the model changes), else read from the model tables
    const bool grp_lds = a.off_grp >= 0;
    int4* lvg = reinterpret_cast<int4*>(smem + (grp_lds ? a.off_grp : 0));
    int cur_model = -1;

    // Shots come from a device-wide ticket counter in runs of kShotRun (one
    // atomic per run) while many shots remain, one at a time near the end.
    unsigned long long run_next = 0, run_end = 0, last_ticket = 0;
    for (;;) {
        if (tid == 0) {
            if (run_next == run_end) {
                const unsigned long long k =
                    last_ticket + 8ull * kShotRun * gridDim.x < a.shots ? (unsigned long long)kShotRun : 1ull;
                run_next = atomicAdd(a.queue, k);
                run_end = run_next + k;
                last_ticket = run_next;
            }
            ms->shot = run_next++;
            ms->count = 0;
            ms->W = 0.0;
            ms->red[0] = 0;
        }
        __syncthreads();
        // the shot, its model and its row are uniform over the workgroup: keep them scalar
        const unsigned long long s = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(ms->shot >> 32))
                                      << 32) |
                                     __builtin_amdgcn_readfirstlane((uint32_t)ms->shot);
        if (s >= a.shots) break;
        const uint64_t t_start = wall_clock64();
        const int mi = a.shot_code ? uniform((int)a.shot_code[s]) : 0;
        const DecodeModel m = a.m[mi < a.n_models ? mi : 0];  // the host checks shot codes; never read past
        const uint64_t row =
            a.shot_index ? (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(a.shot_index[s]) : (uint64_t)s;
        const int N = m.N, WM = m.WM, WN = m.WN;
        const float* dlt = a.delta ? a.delta + row * (uint64_t)N : nullptr;
        const uint16_t* dl16 = a.delta16 ? a.delta16 + row * (uint64_t)(a.d16_pos ? m.Np : N) : nullptr;
        if (tid == 0) X.st(4u * (uint32_t)m.S, INFINITY);  // read-only padding cell
        int4* const lrg = lvg + m.GV;
        if (grp_lds && mi != cur_model) {
            // ordered before the sweeps' reads by the set-up barrier below
            for (int i = tid; i < m.GV; i += nth) lvg[i] = m.vgrp[i];
            for (int i = tid; i < m.GR; i += nth) lrg[i] = m.rgrp[i];
            cur_model = mi;
        }
        auto vgrp_at = [&](int g) { return grp_lds ? lvg[g] : m.vgrp[g]; };
        auto rgrp_at = [&](int g) { return grp_lds ? lrg[g] : m.rgrp[g]; };
        int pc = 0;
        for (int w = tid; w < WM; w += nth) {
            const uint32_t v = m.syn[row * WM + w];
            sig[w] = v;
            par[w] = v;
            pc += __popc(v);
        }
        for (int w = tid; w < m.WK; w += nth) obw[w] = 0u;
        for (int w = tid; w < WN; w += nth) best[w] = 0u;  // the output bits, scattered at the end
        if (pc) atomicAdd(&ms->red[0], pc);
        __syncthreads();
        const int base = uniform(ms->red[0]);  // syndrome weight

        int nconv = 0, legs = 0, iters = 0, path = 0;
        bool x_mu1 = false;  // X holds mu(1) of a plain leg
        bool have_best = false;
        double bestW = 0.0;
        bool traced = false;

        if (base == 0) {
            path = 3;
            have_best = true;
        } else {
            // syndrome bits in row-position order, one ballot per row group
            for (int g = wid; g < m.GR; g += nw) {
                const int i = m.rord[g * 64 + lane];
                const bool b = i >= 0 && ((sig[i >> 5] >> (i & 31)) & 1u);
                const unsigned long long bb = __ballot(b);
                if (lane == 0) {
                    sigp[2 * g] = (uint32_t)bb;
                    sigp[2 * g + 1] = (uint32_t)(bb >> 32);
                }
            }
            const int first_phase = (dlt || dl16) ? 1 : 0;
            for (int phase = first_phase; phase >= 0; --phase) {
                const bool prop = phase == 1;
                if (phase == 0 && first_phase == 1) {
                    // plain Relay-BP from scratch after a failed proposal
                    __syncthreads();
                    if (tid == 0) {
                        ms->count = 0;
                        ms->W = 0.0;
                    }
                    for (int w = tid; w < WM; w += nth) par[w] = sig[w];
                    __syncthreads();
                }
                // M(0) = Lambda (or Lambda + delta; then also nu(0) = Lambda + delta on every edge)
                x_mu1 = false;
                {
                    int dc = 0;
                    double dW = 0.0;
                    for (int pp = tid; pp < m.Np; pp += nth) {
                        const float l = ldg(m.lamp, pp);
                        float x = l;
                        if (prop) {
                            const int j = ldg(m.vord, pp);
                            x = j >= 0 ? l + delta_at(dlt, dl16, a.d16_pos != 0, j, (uint32_t)pp) : 0.0f;
                            const int vd = ldg(m.vdeg, pp);
                            const uint32_t sb = 4u * ((uint32_t)ldg(m.vgrp, pp >> 6).x + (uint32_t)(pp & 63));
                            for (int q = 0; q < vd; ++q) X.st(sb + 256u * q, x);
                            if (x < 0.0f) {
                                flip_slots(m.scheck, sb, vd, par, dc);
                                dW += (double)l;
                            }
                        }
                        Mg[pp] = x;
                    }
                    if (dc) atomicAdd(&ms->count, dc);
                    if (dW != 0.0) atomicAdd(&ms->W, dW);
                    __syncthreads();
                }

                const int nlegs = prop ? 0 : a.R;
                for (int leg = 0; leg <= nlegs; ++leg) {
                    const bool leg0 = leg == 0;
                    const bool lp = prop && leg0;  // priors of this leg are Lambda + delta
                    const int T = leg0 ? a.T0 : a.Tr;
                    const float2* lgl = m.lg + (int64_t)leg * m.Np;  // {Lambda, gamma} of this leg
                    bool conv = false;
                    ++legs;
                    for (int t = 1; t <= T; ++t) {
                        // The first iteration of a plain leg starts from nu(0) = Lambda, so its
                        // check messages mu(1) are the same for every plain leg of the shot.  Its
                        // variable sweep leaves mu(1) in X; if the leg converges there, the next
                        // leg finds mu(1) in place and skips that check sweep, otherwise nu(1) is
                        // formed from the marginals before the second check sweep.
                        const bool first_plain = t == 1 && !lp;
                        if (!(first_plain && x_mu1)) {
                            // ---- check sweep: one row group per wave at a time
                            if constexpr (kQuarterRows<RD, LDS_STATE, MINW>) {
                                // device-memory state, 128-VGPR build: rows over 32 edges in
                                // quarters of 16 rows, four lanes per row (one gather pass)
                                // units: the kPersLpr parts of each wide group (they come
                                // first), then every narrower group whole
                                const int wide_units = kPersLpr * m.GRw;
                                for (int u = wid; u < wide_units + m.GR - m.GRw; u += nw) {
                                    const bool wide = u < wide_units;
                                    const int g = wide ? u / kPersLpr : m.GRw + (u - wide_units);
                                    const int qq = wide ? u % kPersLpr : 0;
                                    const int4 gi = rgrp_at(g);
                                    const int dg = uniform(gi.y);
                                    const uint32_t off = (uint32_t)uniform(gi.x);
                                    if (dg > 32) {
                                        const int rl = qq * (64 / kPersLpr) + lane / kPersLpr;
                                        const uint32_t sbit = ((sigp[2 * g + (rl >> 5)] >> (rl & 31)) & 1u) << 31;
                                        if (uniform(gi.z) != 0)
                                            check_quarter<true, LDS_STATE, false, 104 / kPersLpr, kPersLpr>(X, m.rposp + off, m.rposw + off,
                                                                           m.m1pp + off, lane, qq, dg, sbit,
                                                                           first_plain);
                                        else
                                            check_quarter<false, LDS_STATE, false, 104 / kPersLpr, kPersLpr>(X, m.rposp + off, m.rposw + off,
                                                                            m.m1pp + off, lane, qq, dg, sbit,
                                                                            first_plain);
                                    } else {
                                        const uint32_t sbit = ((sigp[2 * g + (lane >> 5)] >> (lane & 31)) & 1u)
                                                              << 31;
                                        check_dispatch<RD>(X, m.rposp + off, m.rposw + off, m.m1pp + off, lane, dg,
                                                           uniform(gi.z) != 0, sbit, first_plain);
                                    }
                                }
                            } else {
                                for (int g = wid; g < m.GR; g += nw) {
                                    const int4 gi = rgrp_at(g);
                                    const uint32_t off = (uint32_t)uniform(gi.x);
                                    const uint32_t sbit = ((sigp[2 * g + (lane >> 5)] >> (lane & 31)) & 1u) << 31;
                                    check_dispatch<RD>(X, m.rposp + off, m.rposw + off, m.m1pp + off, lane,
                                                       uniform(gi.y), uniform(gi.z) != 0, sbit, first_plain);
                                }
                            }
                            __syncthreads();
                            x_mu1 = first_plain;
                        } else {
                            // every thread has read the count and weight of the previous leg
                            // before this sweep's atomics change them
                            __syncthreads();
                        }
                        // ---- variable sweep: one variable group per wave at a time
                        const bool tr = a.trace_on && phase == a.trace_phase && leg == a.trace_leg && t == a.trace_t;
                        int dcount = 0;
                        double dW = 0.0;
                        for (int g = wid; g < m.GV; g += nw) {
                            const int4 gi = vgrp_at(g);
                            const int dg = uniform(gi.y);
                            const bool mixed = uniform(gi.z) != 0;
                            const uint32_t pp = (uint32_t)(g * 64 + lane);
                            const float2 lgv = ldg(lgl, pp);
                            const float l = lgv.x, gm = lgv.y;
                            float lt = l;
                            if (lp) {
                                const int j = ldg(m.vord, pp);
                                if (j >= 0) lt = l + delta_at(dlt, dl16, a.d16_pos != 0, j, pp);
                            }
                            const float mo = Mg[pp];
                            float acc = __builtin_fmaf(gm, mo - lt, lt);
                            const uint32_t sb = 4u * ((uint32_t)uniform(gi.x) + (uint32_t)lane);
                            const int vd = mixed ? ldg(m.vdeg, pp) : dg;
                            if (!tr) {
                                acc = first_plain ? var_dispatch<false>(X, sb, dg, mixed, vd, acc)
                                                  : var_dispatch<true>(X, sb, dg, mixed, vd, acc);
                            } else {
                                acc = var_member_rolled(X, !first_plain, sb, vd, acc, a.trace_mu, m.scsc);
                                const int j = ldg(m.vord, pp);
                                if (j >= 0) a.trace_M[j] = acc;
                            }
                            Mg[pp] = acc;
                            if ((acc < 0.0f) != (mo < 0.0f)) {
                                flip_slots(m.scheck, sb, vd, par, dcount);
                                dW += acc < 0.0f ? (double)l : -(double)l;
                            }
                        }
                        if (dcount) atomicAdd(&ms->count, dcount);
                        if (dW != 0.0) atomicAdd(&ms->W, dW);
                        __syncthreads();
                        ++iters;
                        if (tr) {
                            if (tid == 0) *a.trace_hit = 1;
                            traced = true;
                            break;
                        }
                        if (base + ms->count == 0) {
                            conv = true;
                            break;
                        }
                        if (first_plain) {
                            // not converged on mu(1): nu(1) = M - mu(1) for the second check sweep
                            for (int g = wid; g < m.GV; g += nw) {
                                const int4 gi = vgrp_at(g);
                                const uint32_t pp = (uint32_t)(g * 64 + lane);
                                extrinsic_dispatch(X, 4u * ((uint32_t)uniform(gi.x) + (uint32_t)lane), uniform(gi.y),
                                                   Mg[pp]);
                            }
                            __syncthreads();
                            x_mu1 = false;
                        }
                    }
                    if (traced) break;
                    if (conv) {
                        const double W = ms->W;
                        if (!have_best || W < bestW) {
                            bestW = W;
                            have_best = true;
                            // best := current hard decision, by position (one ballot per group)
                            for (int g = wid; g < m.GV; g += nw) {
                                const unsigned long long b = __ballot(Mg[g * 64 + lane] < 0.0f);
                                if (lane == 0) {
                                    bestp[2 * g] = (uint32_t)b;
                                    bestp[2 * g + 1] = (uint32_t)(b >> 32);
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
                for (int g = wid; g < m.GV; g += nw) {
                    const unsigned long long b = __ballot(Mg[g * 64 + lane] < 0.0f);
                    if (lane == 0) {
                        bestp[2 * g] = (uint32_t)b;
                        bestp[2 * g + 1] = (uint32_t)(b >> 32);
                    }
                }
            }
            // positions -> variable order: scatter the (few) set bits (each wave
            // reads the ballots it wrote itself; `best` was cleared at set-up)
            for (int g = wid; g < m.GV; g += nw) {
                if ((bestp[2 * g + (lane >> 5)] >> (lane & 31)) & 1u) {
                    const int j = ldg(m.vord, (uint32_t)(g * 64 + lane));
                    atomicOr(best + (j >> 5), 1u << (j & 31));
                }
            }
            __syncthreads();
        }
        if (!a.trace_on) {
            // corrections out; O * correction from the columns of O at its set bits
            // (obw was cleared with the shot's setup)
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
                a.stats[a.stats_by_row ? row : s] = st;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Compact Relay-BP state
//
// With min-sum, every message a check sends is fixed by a few numbers of its
// row: the least and second least |nu_{j->i}| over the row, an edge that
// attains the least, and the sign of each outgoing message,
//   mu_{i->j_p} = (p == p* ? m2 : m1) with sign sigma_i xor prod_{p' != p} s(nu_{j_p'->i}).
// One 16-byte record per row instead of one float per edge cuts a slot's
// state to 16 bytes per row and 4 per variable, so models such as the
// 12-round [[840,168]] one (43,680 edges, 13,776 variables) keep it in LDS.
// nu is not stored: the check sweep forms nu_{j->i}(t-1) = M_j(t-1) -
// mu_{i->j}(t-1) from the marginals and the previous record -- the subtraction
// of the extrinsic step on the same FP32 operands -- so every message and
// marginal equals the per-edge form's bit for bit.
//
// Edge p of a row stored with D slots has the code c = D - 1 - p (the order in
// which one funnel shift per edge collects the signs).  Record of the row at
// position rp (LDS byte address 16 rp):
//   .x m1   least |nu| of the row (float bits, sign clear)
//   .y m2   second least (equal to m1 on a tie)
//   .z sg   bit c (c < 16): sign bit of mu_{i->j} for the edge of code c;
//           bits 16..31 repeat 0..15
//   .w ax   16 rp + c*, c* the code of an edge attaining m1
// Per edge slot the variable sweep holds x = 16 rp + c (vrec): the record is
// at x & ~15, the message sign is bit (x mod 32) of sg (the repeat makes the
// low bit of rp that falls into x mod 32 harmless) and the magnitude is m2 iff
// x == ax.  The marginals follow the records at LDS offset coff_M =
// 16 * 64 GR + 16; the word at 16 * 64 GR holds +inf, the padding target of
// mixed row groups (neutral for both minima and the signs).
// ---------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) u32x4 lds_u32x4;

__device__ __forceinline__ uint4 lds_rec(uint32_t addr) {
    const u32x4 v = *reinterpret_cast<const lds_u32x4*>((size_t)addr);
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void lds_rec_st(uint32_t addr, uint4 v) {
    u32x4 w;
    w.x = v.x;
    w.y = v.y;
    w.z = v.z;
    w.w = v.w;
    *reinterpret_cast<lds_u32x4*>((size_t)addr) = w;
}
__device__ __forceinline__ float lds_f(uint32_t addr) { return *reinterpret_cast<const lds_float*>((size_t)addr); }

// the message of edge slot x from its row's record
__device__ __forceinline__ float rec_mu(uint4 r, uint32_t x) {
    const uint32_t mag = x == r.w ? r.y : r.x;
    return __uint_as_float(mag | ((r.z >> (x & 31u)) << 31));
}

// One row of the compact check update with D stored edges (entries of the
// lane's cvar block, 16-byte loads).  FIRST: nu = M, the first iteration of a
// proposal leg (its nu(0) equals its M(0)); otherwise nu = M - mu(old record).
template <int D, bool FIRST>
__device__ __forceinline__ void compact_row(const int32_t* cp, uint32_t rpx, uint32_t sigma) {
    constexpr int Q = (D + 3) / 4;
    uint32_t pos[4 * Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int4 v = reinterpret_cast<const int4*>(cp)[k];
        pos[4 * k] = (uint32_t)v.x;
        pos[4 * k + 1] = (uint32_t)v.y;
        pos[4 * k + 2] = (uint32_t)v.z;
        pos[4 * k + 3] = (uint32_t)v.w;
    }
    uint4 old = make_uint4(0u, 0u, 0u, 0u);
    if (!FIRST) old = lds_rec(rpx);
    const uint32_t pa = old.w - rpx;
    // the minima as floats: |nu| enters the float median and compare as a
    // source modifier; on these operands (no NaN, not negative) the float and
    // unsigned orders agree, and both results are one of the inputs' bits
    float m1 = __uint_as_float(0x7f800000u), m2 = m1;
    uint32_t nb = 0u, am = 0u;
#pragma unroll
    for (int p = 0; p < D; ++p) {
        const int c = D - 1 - p;  // the edge's code
        const float M = lds_f(pos[p]);
        float nu;
        if (FIRST) {
            nu = M;
        } else {
            const uint32_t mag = pa == (uint32_t)c ? old.y : old.x;
            const float mu = __uint_as_float(mag | ((old.z << (31 - c)) & 0x80000000u));
            nu = M - mu;
        }
        const float av = __builtin_fabsf(nu);
        nb = __builtin_amdgcn_alignbit(nb, __float_as_uint(nu), 31);  // (nb << 1) | sign: edge p lands on bit c
        m2 = __builtin_amdgcn_fmed3f(m1, m2, av);
        const bool lt = av < m1;
        m1 = lt ? av : m1;
        am = lt ? (uint32_t)c : am;
    }
    // sign of mu = sigma xor (parity of all signs) xor sign(nu)
    const uint32_t flip = 0u - ((((uint32_t)__popc(nb)) ^ sigma) & 1u);
    const uint32_t sg = (nb ^ flip) & 0xFFFFu;
    lds_rec_st(rpx, make_uint4(__float_as_uint(m1), __float_as_uint(m2), sg | (sg << 16), rpx + am));
}

// stored row degrees of the compact form: 2..12 exactly, 13..16 padded to 16
template <bool FIRST>
__device__ __forceinline__ void compact_row_dispatch(int dg, const int32_t* cp, uint32_t rpx, uint32_t sigma) {
    switch (dg) {
#define RBP_CROW(D) \
    case D: compact_row<D, FIRST>(cp, rpx, sigma); break;
        RBP_CROW(2) RBP_CROW(3) RBP_CROW(4) RBP_CROW(5) RBP_CROW(6) RBP_CROW(7)
        RBP_CROW(8) RBP_CROW(9) RBP_CROW(10) RBP_CROW(11) RBP_CROW(12) RBP_CROW(16)
#undef RBP_CROW
        default: break;
    }
}

// One variable with D edge slots (vrec entries slot + 64 q): the marginal
// Lambda~ + sum_q mu_q in ascending check order.  In a mixed group only the
// member's own vd edges enter the sum (unused slots hold x = 0, a valid read).
// vrec entry q of a variable slot (its q-th edge); 32-bit offsets (folding the
// constant 256 q into the loads' offset fields through 64-bit address
// arithmetic measured 2 % slower on the [[840,168]] model)
__device__ __forceinline__ uint32_t vrec_at(const uint32_t* vrec, uint32_t slot, int q) {
    return ldg(vrec, slot + 64u * (uint32_t)q);
}

template <int D, bool MIXED>
__device__ __forceinline__ float compact_var(const uint32_t* vrec, uint32_t slot, int vd, float acc) {
    uint32_t x[D];
#pragma unroll
    for (int q = 0; q < D; ++q) x[q] = vrec_at(vrec, slot, q);
#pragma unroll
    for (int q = 0; q < D; ++q) {
        const float mu = rec_mu(lds_rec(x[q] & ~15u), x[q]);
        acc = (!MIXED || q < vd) ? acc + mu : acc;
    }
    return acc;
}

// rolled form for larger degrees and traced iterations (then also writes each
// mu at its CSC edge index)
__device__ __forceinline__ float compact_var_rolled(const uint32_t* vrec, uint32_t slot, int vd, float acc,
                                                   float* trace_mu, const int32_t* scsc) {
    for (int q = 0; q < vd; ++q) {
        const uint32_t x = vrec_at(vrec, slot, q);
        const float mu = rec_mu(lds_rec(x & ~15u), x);
        acc = acc + mu;
        if (trace_mu) trace_mu[ldg(scsc, slot + 64u * (uint32_t)q)] = mu;
    }
    return acc;
}

__device__ __forceinline__ float compact_var_dispatch(const uint32_t* vrec, uint32_t slot, int dg, bool mixed, int vd,
                                                      float acc) {
    switch (dg) {
        case 0: return acc;
#define RBP_CVAR(D) \
    case D: return mixed ? compact_var<D, true>(vrec, slot, vd, acc) : compact_var<D, false>(vrec, slot, vd, acc);
        RBP_CVAR(1) RBP_CVAR(2) RBP_CVAR(3) RBP_CVAR(4) RBP_CVAR(5) RBP_CVAR(6) RBP_CVAR(7) RBP_CVAR(8)
#undef RBP_CVAR
        default: return compact_var_rolled(vrec, slot, vd, acc, nullptr, nullptr);
    }
}

// a flipped hard decision toggles the parity bits (by row position) of the
// variable's checks
__device__ __forceinline__ void compact_flip(const uint32_t* vrec, uint32_t slot, int vd, uint32_t* par,
                                             int& dcount) {
    for (int q = 0; q < vd; ++q) {
        const uint32_t rp = vrec_at(vrec, slot, q) >> 4;
        const uint32_t bit = 1u << (rp & 31u);
        const uint32_t old = atomicXor(par + (rp >> 5), bit);
        dcount += (old & bit) ? -1 : 1;
    }
}

// Runs of equal-degree groups.  Groups are sorted by degree, so the groups a
// wave takes in one sweep (g, g + nw, ...) come in long runs of one degree:
// the degree dispatch is taken once per run, and inside a run each group only
// checks that the next one still has the same degree.
template <int D, bool FIRST>
__device__ __forceinline__ int compact_row_run(int g, int nw, int GR, const int4* lrg, const int32_t* cvar,
                                               const uint32_t* sigp, int lane) {
    do {
        const int4 gi = lrg[g];
        const uint32_t rp = (uint32_t)(g * 64 + lane);
        const uint32_t sigma = (sigp[2 * g + (lane >> 5)] >> (lane & 31)) & 1u;
        const uint32_t off = (uint32_t)uniform(gi.x) + (uint32_t)lane * (uint32_t)uniform(gi.w);
        compact_row<D, FIRST>(cvar + off, 16u * rp, sigma);
        g += nw;
    } while (g < GR && uniform(lrg[g].y) == D);
    return g;
}

// a check sweep in runs: FIRST, the first iteration of a proposal leg (nu =
// M); else past a leg's first iteration (nu = M - mu of the old record)
template <bool FIRST>
__device__ __forceinline__ void compact_check_runs(int g, int nw, int GR, const int4* lrg, const int32_t* cvar,
                                                   const uint32_t* sigp, int lane) {
    while (g < GR) {
        switch (uniform(lrg[g].y)) {
#define RBP_CRUN(D) \
    case D: g = compact_row_run<D, FIRST>(g, nw, GR, lrg, cvar, sigp, lane); break;
            RBP_CRUN(2) RBP_CRUN(3) RBP_CRUN(4) RBP_CRUN(5) RBP_CRUN(6) RBP_CRUN(7)
            RBP_CRUN(8) RBP_CRUN(9) RBP_CRUN(10) RBP_CRUN(11) RBP_CRUN(12) RBP_CRUN(16)
#undef RBP_CRUN
            default: g += nw;  // no other stored degree occurs
        }
    }
}

// a run of unmixed variable groups of degree D; PROP: a proposal leg, whose
// prior is Lambda + delta with the shot's BF16 adjustments by position (dpos)
template <int D, bool PROP>
__device__ __forceinline__ int compact_var_run(int g, int nw, int GV, const int4* lvg, const uint32_t* vrec,
                                               const float2* lgl, const uint16_t* dpos, float* Mg, uint32_t* par,
                                               int& dcount, double& dW, int lane) {
    do {
        const int4 gi = lvg[g];
        const uint32_t pp = (uint32_t)(g * 64 + lane);
        const float2 lgv = ldg(lgl, pp);
        const float l = lgv.x;
        const float lt = PROP ? l + bf16_to_f32(dpos[pp]) : l;
        const float mo = Mg[pp];
        const uint32_t slot = (uint32_t)uniform(gi.x) + (uint32_t)lane;
        const float acc = sat(compact_var<D, false>(vrec, slot, D, __builtin_fmaf(lgv.y, mo - lt, lt)));
        Mg[pp] = acc;
        if ((acc < 0.0f) != (mo < 0.0f)) {
            compact_flip(vrec, slot, D, par, dcount);
            dW += acc < 0.0f ? (double)l : -(double)l;
        }
        g += nw;
    } while (g < GV && uniform(lvg[g].y) == D && uniform(lvg[g].z) == 0);
    return g;
}

// Persistent Relay-BP on the compact state (always in LDS); the shot queue,
// phases, legs, stop rule, statistics and outputs are those of
// relay_bp_kernel.  The parity bits of the hard decision are kept by row
// position (initialised from the syndrome's row-position ballots).
template <int MINW, bool PROP>
__global__ void __launch_bounds__(1024, MINW) relay_bp_compact_kernel(const DecodeLaunch a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63;
    const int wid = uniform(tid >> 6), nw = nth >> 6;
    uint32_t* sig = reinterpret_cast<uint32_t*>(smem + a.off_sig);
    uint32_t* sigp = reinterpret_cast<uint32_t*>(smem + a.off_sigp);
    uint32_t* par = reinterpret_cast<uint32_t*>(smem + a.off_par);
    uint32_t* bestp = reinterpret_cast<uint32_t*>(smem + a.off_bestp);
    uint32_t* best = reinterpret_cast<uint32_t*>(smem + a.off_best);
    uint32_t* obw = reinterpret_cast<uint32_t*>(smem + a.off_obs);
    SlotMisc* ms = reinterpret_cast<SlotMisc*>(smem + a.off_misc);
    // the current model's group descriptors, copied to LDS when the model
    // changes: every group of both sweeps starts with one, and an LDS read of
    // a uniform address is far shorter than a load through the L2
    int4* lvg = reinterpret_cast<int4*>(smem + a.off_grp);
    int cur_model = -1;

    unsigned long long run_next = 0, run_end = 0, last_ticket = 0;
    for (;;) {
        if (tid == 0) {
            if (run_next == run_end) {
                const unsigned long long k =
                    last_ticket + 8ull * kShotRun * gridDim.x < a.shots ? (unsigned long long)kShotRun : 1ull;
                run_next = atomicAdd(a.queue, k);
                run_end = run_next + k;
                last_ticket = run_next;
            }
            ms->shot = run_next++;
            ms->count = 0;
            ms->W = 0.0;
            ms->red[0] = 0;
        }
        __syncthreads();
        const unsigned long long s = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(ms->shot >> 32))
                                      << 32) |
                                     __builtin_amdgcn_readfirstlane((uint32_t)ms->shot);
        if (s >= a.shots) break;
        const uint64_t t_start = wall_clock64();
        const int mi = a.shot_code ? uniform((int)a.shot_code[s]) : 0;
        const DecodeModel& m = a.m[mi < a.n_models ? mi : 0];
        const uint64_t row =
            a.shot_index ? (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(a.shot_index[s]) : (uint64_t)s;
        const int N = m.N, WM = m.WM, WN = m.WN;
        const float* dlt = a.delta ? a.delta + row * (uint64_t)N : nullptr;
        const uint16_t* dl16 = a.delta16 ? a.delta16 + row * (uint64_t)(a.d16_pos ? m.Np : N) : nullptr;
        // BF16 adjustments are copied to LDS by position once per shot and read
        // from there by every iteration of the proposal leg
        uint16_t* dpos = dl16 ? reinterpret_cast<uint16_t*>(smem + a.off_d16) : nullptr;
        float* Mg = reinterpret_cast<float*>(smem + m.coff_M);
        if (tid == 0) Mg[-4] = INFINITY;  // the padding cell at 16 * 64 GR
        int4* const lrg = lvg + m.GV;
        if (mi != cur_model) {
            // the previous shot's sweeps ended before the end-of-shot barrier;
            // the barrier below orders these stores before the next reads
            for (int i = tid; i < m.GV; i += nth) lvg[i] = m.vgrp[i];
            for (int i = tid; i < m.GR; i += nth) lrg[i] = m.rgrp[i];
            cur_model = mi;
        }
        if (PROP && dpos) {
            // the shot's BF16 adjustments, placed in LDS by position (padding 0) at
            // the shot's start, where their loads overlap the syndrome's (the
            // barrier after the syndrome orders the stores before any read:
            // 1-7 % off a proposal decode); by mechanism, a gather through the
            // mechanism-to-position table with four loads in flight per thread
            if (a.d16_pos) {
                // rows by position (Np entries, a multiple of 64, padding 0):
                // contiguous 16-byte copies
                for (int q = tid; q < (m.Np >> 3); q += nth)
                    reinterpret_cast<uint4*>(dpos)[q] = reinterpret_cast<const uint4*>(dl16)[q];
                __syncthreads();
            }
            int j = a.d16_pos ? N : tid;
            for (; j + 3 * nth < N; j += 4 * nth) {
                const uint16_t d0 = dl16[j + 0 * nth];
                const uint16_t d1 = dl16[j + 1 * nth];
                const uint16_t d2 = dl16[j + 2 * nth];
                const uint16_t d3 = dl16[j + 3 * nth];
                const int p0 = ldg(m.vinv, j + 0 * nth);
                const int p1 = ldg(m.vinv, j + 1 * nth);
                const int p2 = ldg(m.vinv, j + 2 * nth);
                const int p3 = ldg(m.vinv, j + 3 * nth);
                dpos[p0] = d0;
                dpos[p1] = d1;
                dpos[p2] = d2;
                dpos[p3] = d3;
            }
            for (; j < N; j += nth) dpos[ldg(m.vinv, j)] = dl16[j];
            for (int pp = N + tid; pp < m.Np; pp += nth) dpos[pp] = 0;
        }
        int pc = 0;
        for (int w = tid; w < WM; w += nth) {
            const uint32_t v = m.syn[row * WM + w];
            sig[w] = v;
            pc += __popc(v);
        }
        for (int w = tid; w < m.WK; w += nth) obw[w] = 0u;
        for (int w = tid; w < WN; w += nth) best[w] = 0u;
        if (pc) atomicAdd(&ms->red[0], pc);
        __syncthreads();
        const int base = uniform(ms->red[0]);

        int nconv = 0, legs = 0, iters = 0, path = 0;
        bool have_best = false;
        double bestW = 0.0;
        bool traced = false;

        if (base == 0) {
            path = 3;
            have_best = true;
        } else {
            // syndrome bits by row position (one ballot per row group)
            for (int g = wid; g < m.GR; g += nw) {
                const int i = m.rord[g * 64 + lane];
                const bool b = i >= 0 && ((sig[i >> 5] >> (i & 31)) & 1u);
                const unsigned long long bb = __ballot(b);
                if (lane == 0) {
                    sigp[2 * g] = (uint32_t)bb;
                    sigp[2 * g + 1] = (uint32_t)(bb >> 32);
                }
            }
            const int first_phase = PROP && (dlt || dl16) ? 1 : 0;  // PROP = false: no proposal code at all
            for (int phase = first_phase; phase >= 0; --phase) {
                const bool prop = phase == 1;
                __syncthreads();  // sigp complete; the previous phase's counters read
                if (tid == 0) {
                    ms->count = 0;
                    ms->W = 0.0;
                }
                for (int w = tid; w < 2 * m.GR; w += nth) par[w] = sigp[w];
                __syncthreads();
                {
                    // M(0) = Lambda (or Lambda + delta), then the starting hard decision:
                    // the (few) negative entries flip their checks.  Two passes, so that
                    // the first one's loads are independent of each other.
#pragma unroll 4
                    for (int pp = tid; pp < m.Np; pp += nth) {
                        const float l = ldg(m.lamp, pp);
                        float x = l;
                        if (prop) {
                            if (dpos) {
                                x = pp < N ? l + bf16_to_f32(dpos[pp]) : 0.0f;
                            } else {
                                const int j = ldg(m.vord, pp);
                                x = j >= 0 ? l + dlt[j] : 0.0f;
                            }
                        }
                        Mg[pp] = x;
                    }
                    if (prop) {
                        int dc = 0;
                        double dW = 0.0;
                        for (int pp = tid; pp < m.Np; pp += nth) {
                            if (Mg[pp] < 0.0f) {
                                const uint32_t slot = (uint32_t)ldg(m.vgrp, pp >> 6).x + (uint32_t)(pp & 63);
                                compact_flip(m.vrec, slot, ldg(m.vdeg, pp), par, dc);
                                dW += (double)ldg(m.lamp, pp);
                            }
                        }
                        if (dc) atomicAdd(&ms->count, dc);
                        if (dW != 0.0) atomicAdd(&ms->W, dW);
                    }
                    __syncthreads();
                }

                const int nlegs = prop ? 0 : a.R;
                for (int leg = 0; leg <= nlegs; ++leg) {
                    const bool lp = prop && leg == 0;
                    const int T = leg == 0 ? a.T0 : a.Tr;
                    const float2* lgl = m.lg + (int64_t)leg * m.Np;
                    bool conv = false;
                    ++legs;
                    for (int t = 1; t <= T; ++t) {
                        // ---- check sweep: one row group per wave at a time
                        const bool first_plain = t == 1 && !lp;
                        for (int g = wid; g < m.GR; g += nw) {
                            const uint32_t rp = (uint32_t)(g * 64 + lane);
                            const uint32_t sigma = (sigp[2 * g + (lane >> 5)] >> (lane & 31)) & 1u;
                            if (first_plain) {
                                // nu(0) = Lambda > 0: the model's first records, signs = sigma
                                const uint4 r = ldg(m.r1rec, rp);
                                lds_rec_st(16u * rp, make_uint4(r.x, r.y, 0u - sigma, r.w));
                            } else {
                                // in runs of equal degree (t = 1 here only in a proposal leg,
                                // whose nu(0) is its M(0))
                                if (t == 1)
                                    compact_check_runs<true>(g, nw, m.GR, lrg, m.cvar, sigp, lane);
                                else
                                    compact_check_runs<false>(g, nw, m.GR, lrg, m.cvar, sigp, lane);
                                break;  // the runs covered every remaining group of this wave
                            }
                        }
                        __syncthreads();
                        // ---- variable sweep
                        const bool tr = a.trace_on && phase == a.trace_phase && leg == a.trace_leg && t == a.trace_t;
                        int dcount = 0;
                        double dW = 0.0;
                        for (int g = wid; g < m.GV; g += nw) {
                            const int4 gi = lvg[g];
                            const int dg = uniform(gi.y);
                            const bool mixed = uniform(gi.z) != 0;
                            if ((!lp || dpos) && !tr && !mixed && dg >= 1 && dg <= 8) {
                                // runs of unmixed groups of one degree (plain legs, and
                                // proposal legs with BF16 adjustments)
                                int h = g;
                                if (lp) {
                                    switch (dg) {
#define RBP_VRUN(D) \
    case D: h = compact_var_run<D, true>(g, nw, m.GV, lvg, m.vrec, lgl, dpos, Mg, par, dcount, dW, lane); break;
                                        RBP_VRUN(1) RBP_VRUN(2) RBP_VRUN(3) RBP_VRUN(4)
                                        RBP_VRUN(5) RBP_VRUN(6) RBP_VRUN(7) RBP_VRUN(8)
#undef RBP_VRUN
                                    }
                                } else {
                                    switch (dg) {
#define RBP_VRUN(D) \
    case D: h = compact_var_run<D, false>(g, nw, m.GV, lvg, m.vrec, lgl, dpos, Mg, par, dcount, dW, lane); break;
                                        RBP_VRUN(1) RBP_VRUN(2) RBP_VRUN(3) RBP_VRUN(4)
                                        RBP_VRUN(5) RBP_VRUN(6) RBP_VRUN(7) RBP_VRUN(8)
#undef RBP_VRUN
                                    }
                                }
                                g = h - nw;  // the loop's increment takes the next group
                                continue;
                            }
                            const uint32_t pp = (uint32_t)(g * 64 + lane);
                            const float2 lgv = ldg(lgl, pp);
                            const float l = lgv.x, gm = lgv.y;
                            float lt = l;
                            if (lp) {
                                if (dpos) {
                                    lt = l + bf16_to_f32(dpos[pp]);  // 0 at padding positions, whose Lambda is 0 too
                                } else {
                                    const int j = ldg(m.vord, pp);
                                    if (j >= 0) lt = l + dlt[j];
                                }
                            }
                            const float mo = Mg[pp];
                            float acc = __builtin_fmaf(gm, mo - lt, lt);
                            const uint32_t slot = (uint32_t)uniform(gi.x) + (uint32_t)lane;
                            const int vd = mixed ? ldg(m.vdeg, pp) : dg;
                            if (!tr) {
                                acc = sat(compact_var_dispatch(m.vrec, slot, dg, mixed, vd, acc));
                            } else {
                                acc = sat(compact_var_rolled(m.vrec, slot, vd, acc, a.trace_mu, m.scsc));
                                const int j = ldg(m.vord, pp);
                                if (j >= 0) a.trace_M[j] = acc;
                            }
                            Mg[pp] = acc;
                            if ((acc < 0.0f) != (mo < 0.0f)) {
                                compact_flip(m.vrec, slot, vd, par, dcount);
                                dW += acc < 0.0f ? (double)l : -(double)l;
                            }
                        }
                        if (dcount) atomicAdd(&ms->count, dcount);
                        if (dW != 0.0) atomicAdd(&ms->W, dW);
                        __syncthreads();
                        ++iters;
                        if (tr) {
                            if (tid == 0) *a.trace_hit = 1;
                            traced = true;
                            break;
                        }
                        // (the next check sweep's barrier orders this read before the
                        // next variable sweep's atomics)
                        if (base + uniform(ms->count) == 0) {
                            conv = true;
                            break;
                        }
                    }
                    if (traced) break;
                    if (conv) {
                        const double W = ms->W;
                        if (!have_best || W < bestW) {
                            bestW = W;
                            have_best = true;
                            for (int g = wid; g < m.GV; g += nw) {
                                const unsigned long long b = __ballot(Mg[g * 64 + lane] < 0.0f);
                                if (lane == 0) {
                                    bestp[2 * g] = (uint32_t)b;
                                    bestp[2 * g + 1] = (uint32_t)(b >> 32);
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
                for (int g = wid; g < m.GV; g += nw) {
                    const unsigned long long b = __ballot(Mg[g * 64 + lane] < 0.0f);
                    if (lane == 0) {
                        bestp[2 * g] = (uint32_t)b;
                        bestp[2 * g + 1] = (uint32_t)(b >> 32);
                    }
                }
            }
            for (int g = wid; g < m.GV; g += nw) {
                if ((bestp[2 * g + (lane >> 5)] >> (lane & 31)) & 1u) {
                    const int j = ldg(m.vord, (uint32_t)(g * 64 + lane));
                    atomicOr(best + (j >> 5), 1u << (j & 31));
                }
            }
            __syncthreads();
        }
        if (!a.trace_on) {
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
                a.stats[a.stats_by_row ? row : s] = st;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Several shots per workgroup (compact state, one model, plain Relay-BP).
//
// The workgroup keeps K shots' compact states in LDS, sub-slot k at byte
// offset k * sub_stride (the tables hold LDS addresses of sub-slot 0, so each
// access adds the sub-slot's base; the bases are multiples of 256, which keeps
// the low bits that encode an edge's code), and runs them in lockstep: one
// round is one flooding iteration of every sub-slot.  The group descriptor,
// the cvar / vrec table loads and the degree dispatch of each row or
// variable group are shared by the K shots, which also gives each wave K
// independent gathers per group.  A sub-slot whose shot finishes takes the
// next ticket at the start of the next round; sub-slots without a shot at the
// end of the batch are skipped.  Every shot's arithmetic is that of
// relay_bp_compact_kernel.
// ---------------------------------------------------------------------------
template <int D, int K>
__device__ __forceinline__ void compact_row_multi(const int32_t* cp, uint32_t rpx, const uint32_t (&sigma)[K],
                                                  const uint32_t (&base)[K], uint32_t mask) {
    constexpr int Q = (D + 3) / 4;
    uint32_t pos[4 * Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int4 v = reinterpret_cast<const int4*>(cp)[k];
        pos[4 * k] = (uint32_t)v.x;
        pos[4 * k + 1] = (uint32_t)v.y;
        pos[4 * k + 2] = (uint32_t)v.z;
        pos[4 * k + 3] = (uint32_t)v.w;
    }
    uint4 old[K];
#pragma unroll
    for (int s = 0; s < K; ++s)
        if ((mask >> s) & 1u) old[s] = lds_rec(base[s] + rpx);
#pragma unroll
    for (int s = 0; s < K; ++s) {
        if (!((mask >> s) & 1u)) continue;
        const uint32_t rx = base[s] + rpx;
        const uint32_t pa = old[s].w - rx;
        uint32_t m1 = 0x7f800000u, m2 = 0x7f800000u, nb = 0u, am = 0u;
#pragma unroll
        for (int p = 0; p < D; ++p) {
            const int c = D - 1 - p;  // the edge's code
            const float M = lds_f(base[s] + pos[p]);
            const uint32_t mag = pa == (uint32_t)c ? old[s].y : old[s].x;
            const float mu = __uint_as_float(mag | ((old[s].z << (31 - c)) & 0x80000000u));
            const uint32_t nu = __float_as_uint(M - mu);
            const uint32_t av = nu & 0x7fffffffu;
            nb = __builtin_amdgcn_alignbit(nb, nu, 31);
            m2 = umed3(m1, m2, av);
            const bool lt = av < m1;
            m1 = lt ? av : m1;
            am = lt ? (uint32_t)c : am;
        }
        const uint32_t flip = 0u - ((((uint32_t)__popc(nb)) ^ sigma[s]) & 1u);
        const uint32_t sg = (nb ^ flip) & 0xFFFFu;
        lds_rec_st(rx, make_uint4(m1, m2, sg | (sg << 16), rx + am));
    }
}

// mask: the sub-slots (bit s) that take the update; uniform over the workgroup
template <int K>
__device__ __forceinline__ void compact_row_multi_dispatch(int dg, const int32_t* cp, uint32_t rpx,
                                                           const uint32_t (&sigma)[K], const uint32_t (&base)[K],
                                                           uint32_t mask) {
    switch (dg) {
#define RBP_CROWM(D) \
    case D: compact_row_multi<D, K>(cp, rpx, sigma, base, mask); break;
        RBP_CROWM(2) RBP_CROWM(3) RBP_CROWM(4) RBP_CROWM(5) RBP_CROWM(6) RBP_CROWM(7)
        RBP_CROWM(8) RBP_CROWM(9) RBP_CROWM(10) RBP_CROWM(11) RBP_CROWM(12) RBP_CROWM(16)
#undef RBP_CROWM
        default: break;
    }
}

// the K shots' marginals of one variable with D edge slots (in a mixed group
// only the member's own vd edges enter the sums)
template <int D, bool MIXED, int K>
__device__ __forceinline__ void compact_var_multi(const uint32_t* vrec, uint32_t slot, int vd, float (&acc)[K],
                                                  const uint32_t (&base)[K], uint32_t mask) {
    uint32_t x[D];
#pragma unroll
    for (int q = 0; q < D; ++q) x[q] = vrec_at(vrec, slot, q);
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (!((mask >> s) & 1u)) continue;
            const uint32_t xs = base[s] + x[q];
            const float mu = rec_mu(lds_rec(xs & ~15u), xs);
            acc[s] = (!MIXED || q < vd) ? acc[s] + mu : acc[s];
        }
}

template <int K>
__device__ __forceinline__ void compact_var_multi_dispatch(const uint32_t* vrec, uint32_t slot, int dg, bool mixed,
                                                           int vd, float (&acc)[K], const uint32_t (&base)[K],
                                                           uint32_t mask) {
    switch (dg) {
        case 0: return;
#define RBP_CVARM(D)                                                         \
    case D:                                                                  \
        if (mixed)                                                           \
            compact_var_multi<D, true, K>(vrec, slot, vd, acc, base, mask);  \
        else                                                                 \
            compact_var_multi<D, false, K>(vrec, slot, vd, acc, base, mask); \
        return;
        RBP_CVARM(1) RBP_CVARM(2) RBP_CVARM(3) RBP_CVARM(4) RBP_CVARM(5) RBP_CVARM(6) RBP_CVARM(7) RBP_CVARM(8)
#undef RBP_CVARM
        default:
            for (int q = 0; q < vd; ++q) {
                const uint32_t x = vrec_at(vrec, slot, q);
#pragma unroll
                for (int s = 0; s < K; ++s) {
                    if (!((mask >> s) & 1u)) continue;
                    const uint32_t xs = base[s] + x;
                    acc[s] = acc[s] + rec_mu(lds_rec(xs & ~15u), xs);
                }
            }
    }
}

template <int K, int MINW>
__global__ void __launch_bounds__(1024, MINW) relay_bp_multishot_kernel(const DecodeLaunch a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63;
    const int wid = uniform(tid >> 6), nw = nth >> 6;
    const DecodeModel& m = a.m[0];
    const uint32_t SS = (uint32_t)a.sub_stride;
    const int N = m.N, WM = m.WM, WN = m.WN;
    uint32_t base[K];
#pragma unroll
    for (int s = 0; s < K; ++s) base[s] = (uint32_t)s * SS;
    auto P = [&](int s, int32_t off) { return smem + base[s] + off; };
    int4* lvg = reinterpret_cast<int4*>(smem + a.off_grp);
    int4* lrg = lvg + m.GV;
    for (int i = tid; i < m.GV; i += nth) lvg[i] = m.vgrp[i];
    for (int i = tid; i < m.GR; i += nth) lrg[i] = m.rgrp[i];

    // per sub-slot state, kept identically by every thread (every decision
    // below depends only on values all threads read after a barrier)
    int status[K];  // 0: needs a shot, 1: decoding, 2: no shot left
    int sbase[K], leg[K], t[K], nconv[K], legs[K], iters[K];
    bool have[K];
    double bestW[K];
    unsigned long long shot[K];
    uint64_t row[K], t_start[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
        status[s] = 0;
        sbase[s] = leg[s] = t[s] = nconv[s] = legs[s] = iters[s] = 0;
        have[s] = false;
        bestW[s] = 0.0;
        shot[s] = 0;
        row[s] = t_start[s] = 0;
    }
    unsigned long long run_next = 0, run_end = 0, last_ticket = 0;
    __syncthreads();

    for (;;) {
        // ---- a new shot for every sub-slot that finished (zero syndromes are
        // answered at once, and the sub-slot takes the next ticket)
#pragma unroll
        for (int s = 0; s < K; ++s) {
            while (status[s] == 0) {
                SlotMisc* ms = reinterpret_cast<SlotMisc*>(P(s, a.off_misc));
                if (tid == 0) {
                    if (run_next == run_end) {
                        const unsigned long long k = last_ticket + 8ull * kShotRun * K * gridDim.x < a.shots
                                                         ? (unsigned long long)kShotRun
                                                         : 1ull;
                        run_next = atomicAdd(a.queue, k);
                        run_end = run_next + k;
                        last_ticket = run_next;
                    }
                    ms->shot = run_next++;
                    ms->count = 0;
                    ms->W = 0.0;
                    ms->red[0] = 0;
                }
                __syncthreads();
                const unsigned long long sh =
                    ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(ms->shot >> 32)) << 32) |
                    __builtin_amdgcn_readfirstlane((uint32_t)ms->shot);
                if (sh >= a.shots) {
                    status[s] = 2;
                    break;
                }
                shot[s] = sh;
                t_start[s] = wall_clock64();
                row[s] = a.shot_index ? (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(a.shot_index[sh])
                                      : (uint64_t)sh;
                uint32_t* sig = reinterpret_cast<uint32_t*>(P(s, a.off_sig));
                uint32_t* obw = reinterpret_cast<uint32_t*>(P(s, a.off_obs));
                uint32_t* best = reinterpret_cast<uint32_t*>(P(s, a.off_best));
                int pc = 0;
                for (int w = tid; w < WM; w += nth) {
                    const uint32_t v = m.syn[row[s] * WM + w];
                    sig[w] = v;
                    pc += __popc(v);
                }
                for (int w = tid; w < m.WK; w += nth) obw[w] = 0u;
                for (int w = tid; w < WN; w += nth) best[w] = 0u;
                if (pc) atomicAdd(&ms->red[0], pc);
                __syncthreads();
                sbase[s] = uniform(ms->red[0]);
                if (sbase[s] == 0) {
                    // zero syndrome: the zero correction, converged
                    for (int w = tid; w < WN; w += nth) m.corr[row[s] * WN + w] = 0u;
                    if (m.obsp)
                        for (int w = tid; w < m.WK; w += nth) m.obsp[row[s] * m.WK + w] = 0u;
                    if (a.stats && tid == 0) {
                        rbp_shot_stats st;
                        st.converged = 1;
                        st.nconv = 0;
                        st.path = 3;
                        st.reserved = 0;
                        st.legs = 0;
                        st.reserved2 = 0;
                        st.iters = 0;
                        st.reserved3 = 0;
                        st.t_start = t_start[s];
                        st.t_end = wall_clock64();
                        a.stats[a.stats_by_row ? row[s] : sh] = st;
                    }
                    __syncthreads();  // every thread has read ms before thread 0 rewrites it
                    continue;
                }
                uint32_t* sigp = reinterpret_cast<uint32_t*>(P(s, a.off_sigp));
                uint32_t* par = reinterpret_cast<uint32_t*>(P(s, a.off_par));
                float* Mg = reinterpret_cast<float*>(P(s, m.coff_M));
                for (int g = wid; g < m.GR; g += nw) {
                    const int i = m.rord[g * 64 + lane];
                    const bool b = i >= 0 && ((sig[i >> 5] >> (i & 31)) & 1u);
                    const unsigned long long bb = __ballot(b);
                    if (lane == 0) {
                        sigp[2 * g] = (uint32_t)bb;
                        sigp[2 * g + 1] = (uint32_t)(bb >> 32);
                    }
                }
                if (tid == 0) Mg[-4] = INFINITY;  // the padding cell at 16 * 64 GR
                for (int pp = tid; pp < m.Np; pp += nth) Mg[pp] = ldg(m.lamp, pp);
                __syncthreads();
                for (int w = tid; w < 2 * m.GR; w += nth) par[w] = sigp[w];
                leg[s] = 0;
                t[s] = 1;
                nconv[s] = 0;
                legs[s] = 1;
                iters[s] = 0;
                have[s] = false;
                bestW[s] = 0.0;
                status[s] = 1;
                __syncthreads();
            }
        }
        bool live = false;
#pragma unroll
        for (int s = 0; s < K; ++s) live = live || status[s] == 1;
        if (!live) break;

        // ---- check sweep: the min-sum update for the sub-slots past the first
        // iteration of their leg, the model's first records for those at it
        uint32_t normal = 0u, first = 0u, liveset = 0u;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (status[s] != 1) continue;
            liveset |= 1u << s;
            if (t[s] == 1)
                first |= 1u << s;
            else
                normal |= 1u << s;
        }
        for (int g = wid; g < m.GR; g += nw) {
            const int4 gi = lrg[g];
            const uint32_t rp = (uint32_t)(g * 64 + lane);
            uint32_t sigma[K];
#pragma unroll
            for (int s = 0; s < K; ++s)
                sigma[s] = (reinterpret_cast<const uint32_t*>(P(s, a.off_sigp))[2 * g + (lane >> 5)] >> (lane & 31)) &
                           1u;
            const uint32_t off = (uint32_t)uniform(gi.x) + (uint32_t)lane * (uint32_t)uniform(gi.w);
            if (normal) compact_row_multi_dispatch<K>(uniform(gi.y), m.cvar + off, 16u * rp, sigma, base, normal);
            if (first) {
                const uint4 r = ldg(m.r1rec, rp);
#pragma unroll
                for (int s = 0; s < K; ++s)
                    if ((first >> s) & 1u)
                        lds_rec_st(base[s] + 16u * rp, make_uint4(r.x, r.y, 0u - sigma[s], r.w + base[s]));
            }
        }
        __syncthreads();

        // ---- variable sweep
        int dcount[K];
        double dW[K];
        const float2* lgl[K];
#pragma unroll
        for (int s = 0; s < K; ++s) {
            dcount[s] = 0;
            dW[s] = 0.0;
            lgl[s] = m.lg + (int64_t)leg[s] * m.Np;
        }
        for (int g = wid; g < m.GV; g += nw) {
            const int4 gi = lvg[g];
            const int dg = uniform(gi.y);
            const bool mixed = uniform(gi.z) != 0;
            const uint32_t pp = (uint32_t)(g * 64 + lane);
            const uint32_t slot = (uint32_t)uniform(gi.x) + (uint32_t)lane;
            const int vd = mixed ? ldg(m.vdeg, pp) : dg;
            float acc[K], mo[K], l[K];
#pragma unroll
            for (int s = 0; s < K; ++s) {
                if (!((liveset >> s) & 1u)) continue;
                const float2 lgv = ldg(lgl[s], pp);
                l[s] = lgv.x;
                mo[s] = reinterpret_cast<const float*>(P(s, m.coff_M))[pp];
                acc[s] = __builtin_fmaf(lgv.y, mo[s] - lgv.x, lgv.x);
            }
            compact_var_multi_dispatch<K>(m.vrec, slot, dg, mixed, vd, acc, base, liveset);
#pragma unroll
            for (int s = 0; s < K; ++s) {
                if (!((liveset >> s) & 1u)) continue;
                const float v = sat(acc[s]);
                reinterpret_cast<float*>(P(s, m.coff_M))[pp] = v;
                if ((v < 0.0f) != (mo[s] < 0.0f)) {
                    compact_flip(m.vrec, slot, vd, reinterpret_cast<uint32_t*>(P(s, a.off_par)), dcount[s]);
                    dW[s] += v < 0.0f ? (double)l[s] : -(double)l[s];
                }
            }
        }
#pragma unroll
        for (int s = 0; s < K; ++s) {
            SlotMisc* ms = reinterpret_cast<SlotMisc*>(P(s, a.off_misc));
            if (dcount[s]) atomicAdd(&ms->count, dcount[s]);
            if (dW[s] != 0.0) atomicAdd(&ms->W, dW[s]);
        }
        __syncthreads();

        // ---- per sub-slot: convergence, solutions, legs, end of the shot
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (status[s] != 1) continue;
            SlotMisc* ms = reinterpret_cast<SlotMisc*>(P(s, a.off_misc));
            const float* Mg = reinterpret_cast<const float*>(P(s, m.coff_M));
            uint32_t* bestp = reinterpret_cast<uint32_t*>(P(s, a.off_bestp));
            ++iters[s];
            bool finish = false;
            const int T = leg[s] == 0 ? a.T0 : a.Tr;
            if (sbase[s] + uniform(ms->count) == 0) {
                const double W = ms->W;
                if (!have[s] || W < bestW[s]) {
                    bestW[s] = W;
                    have[s] = true;
                    for (int g = wid; g < m.GV; g += nw) {
                        const unsigned long long b = __ballot(Mg[g * 64 + lane] < 0.0f);
                        if (lane == 0) {
                            bestp[2 * g] = (uint32_t)b;
                            bestp[2 * g + 1] = (uint32_t)(b >> 32);
                        }
                    }
                }
                ++nconv[s];
                if ((a.crit == 0 && nconv[s] >= a.S) || leg[s] == a.R) {
                    finish = true;
                } else {
                    ++leg[s];
                    t[s] = 1;
                    ++legs[s];
                }
            } else if (t[s] == T) {
                if (leg[s] == a.R) {
                    finish = true;
                } else {
                    ++leg[s];
                    t[s] = 1;
                    ++legs[s];
                }
            } else {
                ++t[s];
            }
            if (!finish) continue;
            if (!have[s]) {
                for (int g = wid; g < m.GV; g += nw) {
                    const unsigned long long b = __ballot(Mg[g * 64 + lane] < 0.0f);
                    if (lane == 0) {
                        bestp[2 * g] = (uint32_t)b;
                        bestp[2 * g + 1] = (uint32_t)(b >> 32);
                    }
                }
            }
            __syncthreads();
            uint32_t* best = reinterpret_cast<uint32_t*>(P(s, a.off_best));
            uint32_t* obw = reinterpret_cast<uint32_t*>(P(s, a.off_obs));
            for (int g = wid; g < m.GV; g += nw) {
                if ((bestp[2 * g + (lane >> 5)] >> (lane & 31)) & 1u) {
                    const int j = ldg(m.vord, (uint32_t)(g * 64 + lane));
                    atomicOr(best + (j >> 5), 1u << (j & 31));
                }
            }
            __syncthreads();
            for (int w = tid; w < WN; w += nth) {
                const uint32_t bits = best[w];
                m.corr[row[s] * WN + w] = bits;
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
                for (int w = tid; w < m.WK; w += nth) m.obsp[row[s] * m.WK + w] = obw[w];
            if (a.stats && tid == 0) {
                rbp_shot_stats st;
                st.converged = have[s] ? 1 : 0;
                st.nconv = (uint8_t)(nconv[s] > 255 ? 255 : nconv[s]);
                st.path = 0;
                st.reserved = 0;
                st.legs = (uint16_t)(legs[s] > 65535 ? 65535 : legs[s]);
                st.reserved2 = 0;
                st.iters = (uint32_t)iters[s];
                st.reserved3 = 0;
                st.t_start = t_start[s];
                st.t_end = wall_clock64();
                a.stats[a.stats_by_row ? row[s] : shot[s]] = st;
            }
            status[s] = 0;
        }
        __syncthreads();
    }
}

// First-iteration records of a plain leg (nu(0) = Lambda > 0): per row
// position, the two least Lambda of the row and the edge of the least; sg = 0
// (the kernel inserts sigma); padding positions get +inf magnitudes.
__global__ void first_record_kernel(const int32_t* row_ptr, const int32_t* col_idx, const int32_t* rord,
                                    const int4* rgrp, const float* lam, uint4* r1rec, int32_t npos) {
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= npos) return;
    const int i = rord[pos];
    const int D = rgrp[pos >> 6].y;  // stored degree: edge p has the code D - 1 - p
    uint32_t m1 = 0x7f800000u, m2 = 0x7f800000u, am = 0u;
    if (i >= 0) {
        const int rs = row_ptr[i], re = row_ptr[i + 1];
        for (int e = rs; e < re; ++e) {
            const uint32_t av = __float_as_uint(lam[col_idx[e]]) & 0x7fffffffu;
            m2 = umed3(m1, m2, av);
            if (av < m1) {
                m1 = av;
                am = (uint32_t)(D - 1 - (e - rs));
            }
        }
    }
    r1rec[pos] = make_uint4(m1, m2, 0u, 16u * (uint32_t)pos + am);
}

// ---------------------------------------------------------------------------
// Cooperative single-shot Relay-BP (latency mode)
//
// One shot at a time, decoded by G workgroups together: the row and variable
// groups of each sweep are spread over all G x W waves, so a shot gets the
// memory bandwidth of G CUs instead of one.  The shot's state (messages,
// marginals), the parity bits, the unsatisfied-check count and the weight live
// in device memory; the sweeps are separated by grid barriers (two per
// iteration).  The per-group arithmetic is the persistent kernel's (the same
// check_dispatch / var_dispatch calls on the same operands in the same order),
// so results are identical; only the distribution over waves differs.
//
// Participants are the workgroups with index % stride == 0 (stride 8 keeps
// them on one XCD when workgroups are dealt round-robin to the 8 XCDs, so they
// share one L2; correctness does not depend on it).  The launch is
// cooperative, so all workgroups are resident.  A barrier wait polls a
// generation counter at most spin_limit times; on expiry it raises the abort
// flag and every workgroup leaves at its next barrier, so no launch can hang.
// ---------------------------------------------------------------------------
// lanes per wide row in the latency mode: 8 (16 messages per lane at most)
// measured 5-11 % faster per shot than 4 on circuit-level ZSZ-LP-320 and -550
constexpr int kCoopLpr = 8;

struct CoopShared {
    unsigned int abort, xmask;  // xmask: XCDs of the participants
    unsigned int go;            // resident mode: ((shot + 1) mod 2^30) << 2 | decision, from rank 0
    unsigned int pad;
};

// Resident mode: the mailbox in fine-grained (coherent) pinned host memory
// through which the host hands the resident kernel one shot at a time.  The
// header is followed by the shot's syndrome [WM words], correction [WN],
// observable prediction [WK] and statistics record, at offsets the launch
// carries in m.syn, m.corr, m.obsp and stats.
struct ResidentBox {
    unsigned long long published;  // host: shots handed over so far (shot s is decoded once published > s)
    unsigned long long done;       // kernel: shots whose outputs are written
    unsigned int stop;             // host: 1 = end at the next wait
    unsigned int state;            // kernel: kResident* below
    unsigned int xcds;             // kernel: bit mask of the XCDs the participants run on
    unsigned int pad[9];
};
static_assert(sizeof(ResidentBox) == 64, "mailbox header is one 64-byte line");
constexpr unsigned kResidentRunning = 1, kResidentStopped = 2, kResidentIdle = 3, kResidentAborted = 4;

struct CoopLaunch {
    DecodeModel m;
    uint64_t shots;
    rbp_shot_stats* stats;
    float* X;        // the shot's state: X[S + 2], marginals at X + Smax + 4
    int32_t Smax;
    uint32_t* par;   // [WM] parity of the current hard decision
    uint32_t* bestp; // [Np / 32] best solution by position
    uint32_t* best;  // [WN] best solution by variable
    CoopShared* sh;
    uint32_t* flags;   // [arrivals] barrier generation each workgroup has reached
    int32_t* cnt;      // [nwg] change of the unsatisfied-check count, per workgroup (cumulative)
    double* wsum;      // [nwg] weight of the hard decision, per workgroup (cumulative)
    int32_t nwg, stride;
    uint32_t arrivals;  // workgroups a barrier waits for (nwg, more only to test expiry)
    uint32_t spin_limit;
    int32_t force_device;  // device-scope fences even on one XCD (for comparison)
    int32_t T0, Tr, R, S, crit;
    int32_t off_sig, off_sigp, off_obs, off_misc;
    // resident mode only
    ResidentBox* box;
    uint64_t res_start;   // index of the first shot this launch waits for
    uint64_t res_idle;    // clock ticks rank 0 waits for a shot before the launch ends itself
    uint64_t res_grace;   // further ticks the other workgroups wait for rank 0's decision
};

struct CoopMisc {
    int32_t red, flag, dcnt, pad;
    double dW;
};

// Ordering of the shot's state around a barrier.  When every participant
// runs on one XCD (`local`), they share that XCD's L2 and the vector L1 is
// write-through: waiting for this wave's stores, then an agent-scope
// invalidate (which drops the L1 and only non-coherent L2 lines; a
// workgroup-scope one leaves the L1, coherent at that scope, in place)
// suffice, and the L2 keeps the state.  Otherwise device-scope fences also
// write the L2 back before the barrier.
__device__ __forceinline__ void coop_release(bool local) {
    if (local)
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    else
        __threadfence();
}

__device__ __forceinline__ void coop_acquire(bool local) {
    if (local)
        asm volatile("buffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
    else
        __threadfence();
}

// Grid barrier over the participating workgroups; false if the launch
// aborted.  Workgroup r announces barrier g by storing g in flags[r]; wave 0
// then polls all flags (one load per lane) until every one has reached g, at
// most spin_limit times.  No read-modify-write on a shared word is needed.
__device__ __forceinline__ bool grid_sync(CoopShared* sh, uint32_t* flags, int rank, unsigned nflags, unsigned& gen,
                                          uint32_t spin_limit, CoopMisc* ms, bool local) {
    coop_release(local);  // this wave's stores are complete (and visible to the other participants)
    __syncthreads();
    ++gen;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        if (lane == 0) __hip_atomic_store(flags + rank, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        uint32_t spins = 0;
        for (;;) {
            int reached = 1;
            for (unsigned i = (unsigned)lane; i < nflags; i += 64u)
                reached &= (int)(__hip_atomic_load(flags + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - gen) >= 0;
            if (__all(reached)) break;
            if (++spins > spin_limit) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (lane == 0) {
            if (!ok) atomicExch(&sh->abort, 1u);
            ms->flag = ok;
            // see the other workgroups' stores: the L1 is shared by the CU's waves,
            // which load again only after the barrier below
            coop_acquire(local);
        }
    }
    __syncthreads();
    return ms->flag != 0;
}

// sum of the per-workgroup slots (every wave computes it)
template <class T>
__device__ __forceinline__ T coop_total(const T* v, int n, int lane) {
    T acc = 0;
    for (int i = lane; i < n; i += 64) {
        if constexpr (sizeof(T) == 8) {
            const unsigned long long b = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(v + i),
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            acc += __longlong_as_double((long long)b);
        } else {
            acc += __hip_atomic_load(v + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) acc += __shfl_xor(acc, d, 64);
    return acc;
}

// Resident mode: whether shot s is decoded (true) or the launch ends.  Rank 0
// polls the mailbox (system-scope loads of host memory) until the host has
// published shot s, asked to stop, or res_idle ticks have passed; it records
// an ending in the mailbox and hands its decision, tagged with the shot, to
// the other workgroups through device memory.  They wait for it at most
// res_idle + res_grace ticks (then the launch aborts), so every wait ends.
// All of these loads and stores are relaxed: the only data that crosses with
// them is the syndrome, which is read with system-scope loads that bypass the
// caches, so no acquire is needed, and an acquire at system scope would
// invalidate the L2 that holds the model's tables on every poll.
__device__ __forceinline__ bool resident_next(const CoopLaunch& a, int rank, uint64_t s, CoopMisc* ms) {
    if (threadIdx.x == 0) {
        ResidentBox* box = a.box;
        const unsigned want = (unsigned)((s + 1) & 0x3fffffffu);
        const uint64_t t0 = wall_clock64();
        unsigned dec = 0;
        if (rank == 0) {
            for (;;) {
                const unsigned long long pub =
                    __hip_atomic_load(&box->published, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                if (pub > s) {
                    dec = kResidentRunning;
                    break;
                }
                if (__hip_atomic_load(&box->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
                    dec = kResidentStopped;
                    break;
                }
                if (wall_clock64() - t0 > a.res_idle) {
                    dec = kResidentIdle;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (dec != kResidentRunning)
                __hip_atomic_store(&box->state, dec, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&a.sh->go, (want << 2) | dec, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            for (;;) {
                const unsigned g = __hip_atomic_load(&a.sh->go, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((g >> 2) == want) {
                    dec = g & 3u;
                    break;
                }
                if (wall_clock64() - t0 > a.res_idle + a.res_grace) {
                    dec = kResidentAborted;
                    atomicExch(&a.sh->abort, 1u);
                    __hip_atomic_store(&box->state, dec, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        ms->flag = (int)dec;
    }
    __syncthreads();
    // (ms->flag is next written inside a grid barrier, after a __syncthreads
    // that every thread reaches only after this read)
    return ms->flag == (int)kResidentRunning;
}

// One grid-synchronous single-shot decoder.  RES = false: the `shots` shots of
// the launch's arrays in turn.  RES = true (resident mode): shots handed over
// one at a time through the mailbox, from res_start on, until the host stops
// the launch or none comes for res_idle ticks; the syndrome is read from and
// the outputs written to the mailbox (host memory, system scope), and rank 0
// raises `done` once a shot's outputs are visible to the host.
template <int RD, bool RES>
__global__ void __launch_bounds__(512, 1) relay_bp_coop_kernel(const CoopLaunch a) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (blockIdx.x % (unsigned)a.stride) return;
    const int rank = (int)(blockIdx.x / (unsigned)a.stride);
    if (rank >= a.nwg) return;
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63;
    const int wid = uniform(tid >> 6), nw = nth >> 6;
    const int gw = rank * nw + wid, GW = a.nwg * nw;
    const DecodeModel& m = a.m;
    State<false> X;
    X.g = a.X;
    float* Mg = a.X + a.Smax + 4;
    uint32_t* sig = reinterpret_cast<uint32_t*>(smem + a.off_sig);
    uint32_t* sigp = reinterpret_cast<uint32_t*>(smem + a.off_sigp);
    uint32_t* obw = reinterpret_cast<uint32_t*>(smem + a.off_obs);
    CoopMisc* ms = reinterpret_cast<CoopMisc*>(smem + a.off_misc);
    CoopShared* sh = a.sh;
    const unsigned nflags = a.arrivals;
    unsigned gen = 0;
    const int WM = m.WM, WN = m.WN;
    // a grid barrier; in resident mode an expired wait is also recorded in the mailbox
    auto sync = [&](bool loc) -> bool {
        if (grid_sync(sh, a.flags, rank, nflags, gen, a.spin_limit, ms, loc)) return true;
        if constexpr (RES) {
            if (tid == 0) __hip_atomic_store(&a.box->state, kResidentAborted, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        return false;
    };
    // which XCDs the participants run on (hardware register XCC_ID, bits 3:0)
    if (tid == 0) atomicOr(&sh->xmask, 1u << (__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u));
    if (!sync(false)) return;
    const unsigned xmask = __hip_atomic_load(&sh->xmask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool local = __popc(xmask) == 1 && !a.force_device;
    if constexpr (RES) {
        // which XCDs this launch runs on, for the host (rbp_resident_info)
        if (rank == 0 && tid == 0)
            __hip_atomic_store(&a.box->xcds, xmask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }

    for (uint64_t s = RES ? a.res_start : 0; RES || s < a.shots; ++s) {
        if constexpr (RES) {
            if (!resident_next(a, rank, s, ms)) return;
        }
        const uint64_t t_start = wall_clock64();
        const uint64_t row = RES ? 0 : s;  // the mailbox holds one shot
        // ---- set-up: every workgroup keeps the syndrome and its row-group
        // ballots in LDS; rank 0 resets the shared arrays
        if (tid == 0) {
            ms->red = 0;
            ms->dcnt = 0;
            ms->dW = 0.0;
            a.cnt[rank] = 0;
            a.wsum[rank] = 0.0;
        }
        __syncthreads();
        int pc = 0;
        for (int w = tid; w < WM; w += nth) {
            const uint32_t v = RES ? __hip_atomic_load(m.syn + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)
                                   : m.syn[s * WM + w];
            sig[w] = v;
            pc += __popc(v);
            if (rank == 0) a.par[w] = v;
        }
        if (rank == 0) {
            for (int w = tid; w < WN; w += nth) a.best[w] = 0u;
            for (int w = tid; w < m.WK; w += nth) obw[w] = 0u;
            if (tid == 0) X.st(4u * (uint32_t)m.S, INFINITY);  // read-only padding cell
        }
        if (pc) atomicAdd(&ms->red, pc);
        __syncthreads();
        const int base = uniform(ms->red);
        for (int g = wid; g < m.GR; g += nw) {
            const int i = m.rord[g * 64 + lane];
            const bool b = i >= 0 && ((sig[i >> 5] >> (i & 31)) & 1u);
            const unsigned long long bb = __ballot(b);
            if (lane == 0) {
                sigp[2 * g] = (uint32_t)bb;
                sigp[2 * g + 1] = (uint32_t)(bb >> 32);
            }
        }
        for (int g = gw; g < m.GV; g += GW) Mg[g * 64 + lane] = ldg(m.lamp, (uint32_t)(g * 64 + lane));
        if (!sync(local)) return;

        int nconv = 0, legs = 0, iters = 0, path = 0;
        bool x_mu1 = false, have_best = false;
        double bestW = 0.0;
        if (base == 0) {
            path = 3;
            have_best = true;
        } else {
            for (int leg = 0; leg <= a.R; ++leg) {
                const int T = leg == 0 ? a.T0 : a.Tr;
                const float2* lgl = m.lg + (int64_t)leg * m.Np;
                bool conv = false;
                ++legs;
                for (int t = 1; t <= T; ++t) {
                    const bool first_plain = t == 1;
                    if (!(first_plain && x_mu1)) {
                        // units: 1/kCoopLpr of a group of rows over 32 edges (kCoopLpr
                        // lanes per row), else a whole group
                        const int wide_units = kCoopLpr * m.GRw;
                        for (int u = gw; u < wide_units + m.GR - m.GRw; u += GW) {
                            const bool wide = u < wide_units;
                            const int g = wide ? u / kCoopLpr : m.GRw + (u - wide_units);
                            const int qq = wide ? u % kCoopLpr : 0;
                            const int4 gi = m.rgrp[g];
                            const int dg = uniform(gi.y);
                            const uint32_t off = (uint32_t)uniform(gi.x);
                            if (dg > 32) {
                                const int rl = qq * (64 / kCoopLpr) + lane / kCoopLpr;
                                const uint32_t sbit = ((sigp[2 * g + (rl >> 5)] >> (rl & 31)) & 1u) << 31;
                                if (uniform(gi.z) != 0)
                                    check_quarter<true, false, true, 128 / kCoopLpr, kCoopLpr>(
                                        X, m.rposp + off, m.rposw + off, m.m1pp + off, lane, qq, dg, sbit, first_plain);
                                else
                                    check_quarter<false, false, true, 128 / kCoopLpr, kCoopLpr>(
                                        X, m.rposp + off, m.rposw + off, m.m1pp + off, lane, qq, dg, sbit, first_plain);
                            } else {
                                const uint32_t sbit = ((sigp[2 * g + (lane >> 5)] >> (lane & 31)) & 1u) << 31;
                                check_dispatch<RD>(X, m.rposp + off, m.rposw + off, m.m1pp + off, lane, dg,
                                                   uniform(gi.z) != 0, sbit, first_plain);
                            }
                        }
                        x_mu1 = first_plain;
                    }
                    // after the check sweep (or, when it is skipped, after every
                    // workgroup has read the previous count and weight)
                    if (!sync(local)) return;
                    int dcount = 0;
                    double dW = 0.0;
                    for (int g = gw; g < m.GV; g += GW) {
                        const int4 gi = m.vgrp[g];
                        const int dg = uniform(gi.y);
                        const bool mixed = uniform(gi.z) != 0;
                        const uint32_t pp = (uint32_t)(g * 64 + lane);
                        const float2 lgv = ldg(lgl, pp);
                        const float l = lgv.x, gm = lgv.y;
                        const float mo = Mg[pp];
                        float acc = __builtin_fmaf(gm, mo - l, l);
                        const uint32_t sb = 4u * ((uint32_t)uniform(gi.x) + (uint32_t)lane);
                        const int vd = mixed ? ldg(m.vdeg, pp) : dg;
                        acc = first_plain ? var_dispatch<false>(X, sb, dg, mixed, vd, acc)
                                          : var_dispatch<true>(X, sb, dg, mixed, vd, acc);
                        Mg[pp] = acc;
                        if ((acc < 0.0f) != (mo < 0.0f)) {
                            flip_slots(m.scheck, sb, vd, a.par, dcount);
                            dW += acc < 0.0f ? (double)l : -(double)l;
                        }
                    }
                    // the workgroup's changes, added to its own slots
                    if (dcount) atomicAdd(&ms->dcnt, dcount);
                    if (dW != 0.0) atomicAdd(&ms->dW, dW);
                    __syncthreads();
                    if (tid == 0 && (ms->dcnt != 0 || ms->dW != 0.0)) {
                        a.cnt[rank] += ms->dcnt;
                        a.wsum[rank] += ms->dW;
                        ms->dcnt = 0;
                        ms->dW = 0.0;
                    }
                    if (!sync(local)) return;
                    ++iters;
                    const int cnt = coop_total(a.cnt, a.nwg, lane);
                    if (base + uniform(cnt) == 0) {
                        conv = true;
                        break;
                    }
                    if (first_plain) {
                        for (int g = gw; g < m.GV; g += GW) {
                            const int4 gi = m.vgrp[g];
                            const uint32_t pp = (uint32_t)(g * 64 + lane);
                            extrinsic_dispatch(X, 4u * ((uint32_t)uniform(gi.x) + (uint32_t)lane), uniform(gi.y),
                                               Mg[pp]);
                        }
                        if (!sync(local)) return;
                        x_mu1 = false;
                    }
                }
                if (conv) {
                    const double W = coop_total(a.wsum, a.nwg, lane);
                    if (!have_best || W < bestW) {
                        bestW = W;
                        have_best = true;
                        for (int g = gw; g < m.GV; g += GW) {
                            const unsigned long long b = __ballot(Mg[g * 64 + lane] < 0.0f);
                            if (lane == 0) {
                                a.bestp[2 * g] = (uint32_t)b;
                                a.bestp[2 * g + 1] = (uint32_t)(b >> 32);
                            }
                        }
                    }
                    ++nconv;
                    if (a.crit == 0 && nconv >= a.S) break;
                }
            }
            if (!have_best) {
                for (int g = gw; g < m.GV; g += GW) {
                    const unsigned long long b = __ballot(Mg[g * 64 + lane] < 0.0f);
                    if (lane == 0) {
                        a.bestp[2 * g] = (uint32_t)b;
                        a.bestp[2 * g + 1] = (uint32_t)(b >> 32);
                    }
                }
            }
            // positions -> variable order (each wave reads the ballots it wrote)
            for (int g = gw; g < m.GV; g += GW) {
                if ((a.bestp[2 * g + (lane >> 5)] >> (lane & 31)) & 1u) {
                    const int j = ldg(m.vord, (uint32_t)(g * 64 + lane));
                    atomicOr(a.best + (j >> 5), 1u << (j & 31));
                }
            }
        }
        if (!sync(local)) return;
        if (rank == 0) {
            for (int w = tid; w < WN; w += nth) {
                const uint32_t bits = __hip_atomic_load(a.best + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
                a.stats[row] = st;
            }
            if constexpr (RES) {
                // every thread's mailbox stores have left the CU (they sit in this
                // XCD's L2, which rank 0's waves share); then one system-scope
                // release (an L2 write-back, no invalidation) publishes them with
                // `done`
                coop_release(true);
                __syncthreads();
                if (tid == 0)
                    __hip_atomic_store(&a.box->done, (unsigned long long)(s + 1), __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        // the next shot's set-up rewrites the shared arrays
        if (!sync(local)) return;
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

// LLRs Lambda_j = (float) ln((1-p)/p) in double, uploaded (by variable and by
// position) when the priors change, and the first-iteration message table.
static rbp_status ensure_llr(rbp_code* c, const double* priors, hipStream_t stream) {
    if (c->lam.p && c->lam_key.size() == (size_t)c->N &&
        std::memcmp(c->lam_key.data(), priors, sizeof(double) * c->N) == 0)
        return RBP_OK;
    if (c->residents) return fail(RBP_ERR_INVALID_ARG, "a resident decoder runs on this code with other priors; stop it first");
    std::vector<float> lam(c->N), lamp(c->Np, 0.0f);
    for (int j = 0; j < c->N; ++j) lam[j] = (float)std::log((1.0 - priors[j]) / priors[j]);
    for (int p = 0; p < c->Np; ++p)
        if (c->h_vord[p] >= 0) lamp[p] = lam[c->h_vord[p]];
    RBP_HIP_CHECK(hipStreamSynchronize(stream));
    rbp_status st = upload(c->lam, lam);
    if (!st) st = upload(c->lamp, lamp);
    if (!st) st = c->m1.reserve(sizeof(float) * std::max<int64_t>(c->RB, 1));
    if (st) return st;
    const int npos = 64 * c->GR;
    hipLaunchKernelGGL(first_message_kernel, dim3(ceil_div(npos, 256)), dim3(256), 0, stream, c->row_ptr.as<int32_t>(),
                       c->col_idx.as<int32_t>(), c->rord.as<int32_t>(), c->rgrp.as<int4>(), c->lam.as<float>(),
                       c->m1.as<float>(), npos);
    RBP_HIP_CHECK(hipGetLastError());
    if (c->compact_ok) {
        st = c->r1rec.reserve(sizeof(uint4) * (size_t)npos);
        if (st) return st;
        hipLaunchKernelGGL(first_record_kernel, dim3(ceil_div(npos, 256)), dim3(256), 0, stream,
                           c->row_ptr.as<int32_t>(), c->col_idx.as<int32_t>(), c->rord.as<int32_t>(),
                           c->rgrp.as<int4>(), c->lam.as<float>(), c->r1rec.as<uint4>(), npos);
        RBP_HIP_CHECK(hipGetLastError());
    }
    c->lam_key.assign(priors, priors + c->N);
    ++c->lam_gen;
    return RBP_OK;
}

// Sampler tables for the priors: T_k = floor((1 - pmax)^k 2^32), k = 1..L, with
// (1 - pmax)^k evaluated as exp(k log1p(-pmax)) in double (at most 2^32 - 1),
// and A_j = floor(p_j / pmax 2^32) (at most 2^32 - 2) for p_j < pmax,
// 0xFFFFFFFF for p_j = pmax.
static rbp_status ensure_thresholds(rbp_code* c, const double* priors, hipStream_t stream) {
    if (c->thr.p && c->thr_key.size() == (size_t)c->N &&
        std::memcmp(c->thr_key.data(), priors, sizeof(double) * c->N) == 0)
        return RBP_OK;
    const int L = ceil_div(c->N, 64);
    double pmax = 0.0;
    for (int j = 0; j < c->N; ++j) pmax = std::max(pmax, priors[j]);
    std::vector<uint32_t> T(std::max(L, 1)), A(std::max(c->N, 1));
    const double lq = std::log1p(-pmax);
    for (int kk = 1; kk <= L; ++kk) {
        const double t = std::floor(std::exp((double)kk * lq) * 4294967296.0);
        T[kk - 1] = t >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)t;
    }
    for (int j = 0; j < c->N; ++j) {
        if (priors[j] >= pmax) {
            A[j] = 0xFFFFFFFFu;
        } else {
            const double t = std::floor(priors[j] / pmax * 4294967296.0);
            A[j] = t >= 4294967294.0 ? 0xFFFFFFFEu : (uint32_t)t;
        }
    }
    rbp_status st = c->thr.reserve(sizeof(uint32_t) * A.size());
    if (!st) st = c->gapt.reserve(sizeof(uint32_t) * T.size());
    if (st) return st;
    RBP_HIP_CHECK(hipStreamSynchronize(stream));
    RBP_HIP_CHECK(hipMemcpy(c->thr.p, A.data(), sizeof(uint32_t) * A.size(), hipMemcpyHostToDevice));
    RBP_HIP_CHECK(hipMemcpy(c->gapt.p, T.data(), sizeof(uint32_t) * T.size(), hipMemcpyHostToDevice));
    c->thr_key.assign(priors, priors + c->N);
    return RBP_OK;
}

static rbp_status ensure_gamma(rbp_code* c, const rbp_relay_params* p, hipStream_t stream) {
    const int R = p->num_sets;
    if (c->gtab.p && c->gtab_R == R && c->gtab_seed == p->gamma_seed && c->gtab_lo == p->gamma_min &&
        c->gtab_hi == p->gamma_max)
        return RBP_OK;
    if (c->residents)
        return fail(RBP_ERR_INVALID_ARG, "a resident decoder runs on this code with other relay parameters; stop it first");
    const int64_t total = (int64_t)c->Np * std::max(R, 0);
    RBP_HIP_CHECK(hipStreamSynchronize(stream));
    // at least one row: the first leg reads (and discards) row 0
    rbp_status st = c->gtab.reserve(sizeof(float) * std::max<int64_t>(total, c->Np));
    if (st) return st;
    if (total > 0) {
        hipLaunchKernelGGL(gamma_table_kernel, dim3(ceil_div(total, 256)), dim3(256), 0, stream, c->gtab.as<float>(),
                           c->vord.as<int32_t>(), c->Np, R, p->gamma_min, p->gamma_max, p->gamma_seed);
        RBP_HIP_CHECK(hipGetLastError());
    }
    c->gtab_R = R;
    ++c->gtab_gen;
    c->gtab_seed = p->gamma_seed;
    c->gtab_lo = p->gamma_min;
    c->gtab_hi = p->gamma_max;
    return RBP_OK;
}

// the {Lambda, gamma} table, rebuilt when the priors, the gamma table or gamma0 change
static rbp_status ensure_lam_gamma(rbp_code* c, const rbp_relay_params* p, hipStream_t stream) {
    const int R = p->num_sets;
    if (c->lg.p && c->lg_lam_gen == c->lam_gen && c->lg_gtab_gen == c->gtab_gen && c->lg_gamma0 == p->gamma0 &&
        c->lg_R == R)
        return RBP_OK;
    if (c->residents)
        return fail(RBP_ERR_INVALID_ARG, "a resident decoder runs on this code with other relay parameters; stop it first");
    const int64_t total = (int64_t)c->Np * (R + 1);
    RBP_HIP_CHECK(hipStreamSynchronize(stream));
    rbp_status st = c->lg.reserve(sizeof(float2) * total);
    if (st) return st;
    hipLaunchKernelGGL(lam_gamma_kernel, dim3(ceil_div(total, 256)), dim3(256), 0, stream, c->lg.as<float2>(),
                       c->lamp.as<float>(), c->gtab.as<float>(), c->Np, R, p->gamma0);
    RBP_HIP_CHECK(hipGetLastError());
    c->lg_lam_gen = c->lam_gen;
    c->lg_gtab_gen = c->gtab_gen;
    c->lg_gamma0 = p->gamma0;
    c->lg_R = R;
    return RBP_OK;
}

static rbp_status check_params(const rbp_relay_params* p) {
    if (!p) return fail(RBP_ERR_INVALID_ARG, "params is NULL");
    // iteration budgets and |gamma| are bounded so that saturated marginals keep
    // every message finite
    if (p->pre_iter < 1 || p->max_iterations < 1 || p->pre_iter > 65536 || p->max_iterations > 65536 ||
        p->num_sets < 0 || p->stop_nconv < 1 ||
        p->stop_nconv > 255 || (p->stopping_criterion != 0 && p->stopping_criterion != 1))
        return fail(RBP_ERR_INVALID_ARG, "relay parameters out of range");
    if (!(std::fabs(p->gamma0) <= 16.0f) || !(std::fabs(p->gamma_min) <= 16.0f) || !(std::fabs(p->gamma_max) <= 16.0f))
        return fail(RBP_ERR_INVALID_ARG, "gamma values must be finite, |gamma| <= 16");
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
    m.S = c->S;
    m.GR = c->GR;
    m.GRw = c->GRw;
    m.GV = c->GV;
    m.Np = c->Np;
    m.rgrp = c->rgrp.as<int4>();
    m.rposp = c->rposp.as<int32_t>();
    m.rposw = c->rposw.as<int32_t>();
    m.m1pp = c->m1.as<float>();
    m.rord = c->rord.as<int32_t>();
    m.vgrp = c->vgrp.as<int4>();
    m.vord = c->vord.as<int32_t>();
    m.vinv = c->vinv.as<int32_t>();
    m.vdeg = c->vdeg.as<int32_t>();
    m.scheck = c->scheck.as<int32_t>();
    m.scsc = c->scsc.as<int32_t>();
    m.lamp = c->lamp.as<float>();
    m.gtabp = c->gtab.as<float>();
    m.lg = c->lg.as<float2>();
    m.ocol_ptr = c->ocol_ptr.as<int32_t>();
    m.orow_idx = c->orow_idx.as<int32_t>();
    m.cvar = c->cvar.as<int32_t>();
    m.vrec = c->vrec.as<uint32_t>();
    m.r1rec = c->r1rec.as<uint4>();
    m.coff_M = c->coff_M;
    m.syn = syn;
    m.corr = corr;
    m.obsp = c->k > 0 ? obsp : nullptr;
    return m;
}

typedef void (*DecodeKernel)(const DecodeLaunch);

// prop: the launch carries proposal adjustments (built separately, so that the
// plain decode's code is not shaped by the proposal leg's)
static DecodeKernel compact_kernel(int minw, bool prop) {
    if (prop) return minw >= 8 ? relay_bp_compact_kernel<8, true> : relay_bp_compact_kernel<4, true>;
    return minw >= 8 ? relay_bp_compact_kernel<8, false> : relay_bp_compact_kernel<4, false>;
}

static DecodeKernel decode_kernel(int max_stored_row_deg, bool lds, int minw) {
    if (max_stored_row_deg <= 12) {
        if (minw >= 8) return lds ? relay_bp_kernel<12, true, 8> : relay_bp_kernel<12, false, 8>;
        return lds ? relay_bp_kernel<12, true, 4> : relay_bp_kernel<12, false, 4>;
    }
    if (minw >= 8) return lds ? relay_bp_kernel<32, true, 8> : relay_bp_kernel<32, false, 8>;
    return lds ? relay_bp_kernel<32, true, 4> : relay_bp_kernel<32, false, 4>;
}

static constexpr int kMaxLds = 160 * 1024;
// device-memory state of all slots together: about three quarters of the
// 256 MB Infinity Cache
static constexpr int64_t kStateCacheBytes = 192ll << 20;

struct LaunchShape {
    int waves = 1;
    bool lds_state = true;
    bool compact = false;  // compact row-record state (always in LDS)
    DecodeKernel kernel = nullptr;
    int lds_bytes = 0;
    int slots = 1;
    int64_t gstride = 0;
    int Smax = 0;
    int off_M = 0, off_sig = 0, off_sigp = 0, off_par = 0, off_bestp = 0, off_best = 0, off_obs = 0, off_misc = 0;
    int off_d16 = 0;
    int off_grp = 0;
    int nsub = 1;         // shots per workgroup (multi-shot kernel when > 1)
    int sub_stride = 0;   // LDS bytes per shot sub-slot of the multi-shot kernel
};

static int align16(int64_t x) { return (int)((x + 15) & ~(int64_t)15); }

// Launch shape for a set of models decoded together (max sizes over models).
// d16: the launch carries BF16 proposal adjustments (the compact state keeps a
// copy of a shot's adjustments in LDS, 2 bytes per variable position)
static DecodeKernel multishot_kernel(int k, int minw) {
    if (k == 4) return minw >= 8 ? relay_bp_multishot_kernel<4, 8> : relay_bp_multishot_kernel<4, 4>;
    return minw >= 8 ? relay_bp_multishot_kernel<2, 8> : relay_bp_multishot_kernel<2, 4>;
}

// multishot_ok: the launch decodes one model with plain Relay-BP (no proposal,
// no trace), so the handle's shots_per_wg setting applies
static rbp_status plan_launch(rbp_code* const* cs, int n, uint64_t shots, LaunchShape* out, bool d16 = false,
                              bool multishot_ok = false, bool prop = false) {
    int Smax = 0, Npmax = 0, GRmax = 0, WMmax = 0, WNmax = 0, WKmax = 1, rdmax = 0;
    for (int i = 0; i < n; ++i) {
        Smax = std::max(Smax, cs[i]->S);
        Npmax = std::max(Npmax, cs[i]->Np);
        GRmax = std::max(GRmax, cs[i]->GR);
        WMmax = std::max(WMmax, ceil_div(cs[i]->M, 32));
        WNmax = std::max(WNmax, ceil_div(cs[i]->N, 32));
        WKmax = std::max(WKmax, ceil_div(cs[i]->k, 32));
        rdmax = std::max(rdmax, cs[i]->max_stored_row_deg);
    }
    const LaunchCfg& cfg = cs[0]->cfg;
    // small per-slot arrays (always LDS)
    const int small = align16(4 * (int64_t)WMmax) + align16(8 * (int64_t)GRmax) + align16(4 * (int64_t)WMmax) +
                      align16(4 * (int64_t)(Npmax / 32)) + align16(4 * (int64_t)WNmax) + align16(4 * (int64_t)WKmax) +
                      align16(sizeof(SlotMisc));
    const int64_t state_bytes = align16(4 * ((int64_t)Smax + 2)) + align16(4 * (int64_t)Npmax);
    // compact row-record state: every model's rows within 16 edges; the
    // records and marginals of each model at its own offsets, the small arrays
    // after the largest
    bool compact_ok = true;
    int64_t compact_bytes = 0;
    for (int i = 0; i < n; ++i) {
        compact_ok = compact_ok && cs[i]->compact_ok;
        compact_bytes = std::max<int64_t>(compact_bytes, (int64_t)cs[i]->coff_M + 4 * (int64_t)cs[i]->Np);
    }
    compact_bytes = align16(compact_bytes);
    const int64_t d16_bytes = d16 ? align16(2 * (int64_t)Npmax) : 0;
    // the compact kernel keeps a model's group descriptors in LDS (GV + GR int4)
    int64_t grp_bytes = 0;
    for (int i = 0; i < n; ++i) grp_bytes = std::max<int64_t>(grp_bytes, 16 * ((int64_t)cs[i]->GV + cs[i]->GR));
    const bool compact_fits = compact_ok && compact_bytes + d16_bytes + grp_bytes + small <= kMaxLds;
    bool lds = state_bytes + small <= kMaxLds;
    bool compact = false;
    if (cfg.state == 1 && !lds) return fail(RBP_ERR_UNSUPPORTED, "per-shot state does not fit in LDS");
    if (cfg.state == 3 && !compact_fits)
        return fail(RBP_ERR_UNSUPPORTED, "compact state needs rows of at most 16 edges and must fit in LDS");
    if (cfg.state == 2) lds = false;
    if (cfg.state == 3 || (cfg.state == 0 && !lds && compact_fits)) {
        // the per-edge state does not fit in LDS but the row records do
        compact = true;
        lds = true;
    }
    int waves = cfg.waves_per_shot;
    if (waves <= 0) {
        if (lds) {
            // about 8 waves per SIMD (32 per CU) over the slots that fit in LDS, and
            // at least min(4, groups) waves so that a slow shot is not left to one wave
            const int64_t per_slot = (compact ? compact_bytes + d16_bytes + grp_bytes : state_bytes) + small;
            const int per_cu_lds = (int)std::max<int64_t>(kMaxLds / per_slot, 1);
            int groups = 0;
            for (int i = 0; i < n; ++i) groups = std::max(groups, std::max(cs[i]->GR, cs[i]->GV));
            waves = 1;
            while (waves * 2 * per_cu_lds <= 32 && waves < 16) waves <<= 1;
            while (waves < 4 && waves < groups) waves <<= 1;
        } else {
            const int want = ceil_div(Npmax, 512);
            waves = 1;
            while (waves < want && waves < 16) waves <<= 1;
        }
    }
    waves = std::min(std::max(waves, 1), 16);
    LaunchShape L;
    L.waves = waves;
    L.lds_state = lds;
    L.compact = compact;
    L.Smax = Smax;
    int64_t off = 0;
    if (compact) {
        off = compact_bytes;
    } else if (lds) {
        off = align16(4 * ((int64_t)Smax + 2));
        L.off_M = (int)off;
        off += align16(4 * (int64_t)Npmax);
    }
    L.off_sig = (int)off;
    off += align16(4 * (int64_t)WMmax);
    L.off_sigp = (int)off;
    off += align16(8 * (int64_t)GRmax);
    L.off_par = (int)off;
    off += align16(4 * (int64_t)WMmax);
    L.off_bestp = (int)off;
    off += align16(4 * (int64_t)(Npmax / 32));
    L.off_best = (int)off;
    off += align16(4 * (int64_t)WNmax);
    L.off_obs = (int)off;
    off += align16(4 * (int64_t)WKmax);
    L.off_misc = (int)off;
    off += align16(sizeof(SlotMisc));
    L.off_d16 = (int)off;
    if (compact) off += d16_bytes;
    // Group descriptors in LDS: measured 4-6 % faster with the compact state
    // ([[840,168]], ZSZ-LP-550) and 4 % with device-memory state (hgp56), 2-3 %
    // slower with the per-edge state in LDS (ZSZ-LP-160/320), which keeps them
    // in the model tables.
    L.off_grp = (int)off;
    if (compact || (!lds && off + grp_bytes <= kMaxLds))
        off += grp_bytes;
    else
        L.off_grp = -1;
    if (off > kMaxLds) return fail(RBP_ERR_UNSUPPORTED, "per-shot bit arrays do not fit in LDS");
    L.lds_bytes = (int)off;
    const int nsub = multishot_ok && n == 1 && !d16 ? cfg.shots_per_wg : 1;
    if (nsub > 1) {
        if (!compact) return fail(RBP_ERR_UNSUPPORTED, "several shots per workgroup need the compact state");
        // K sub-slots of the one-shot layout (without the descriptors), then the descriptors
        L.nsub = nsub;
        L.sub_stride = (L.off_grp + 255) & ~255;
        const int64_t total = (int64_t)nsub * L.sub_stride + grp_bytes;
        if (total > kMaxLds)
            return fail(RBP_ERR_UNSUPPORTED, "the shots of one workgroup do not fit in LDS together");
        L.off_grp = nsub * L.sub_stride;
        L.lds_bytes = (int)total;
        if (cfg.waves_per_shot <= 0) L.waves = 8;
    }
    L.gstride = lds ? 0 : ((int64_t)Smax + 4 + Npmax + 63) / 64 * 64;
    // the register budget (128 or 64 VGPRs) that fits more slots per CU; on a
    // tie the larger budget (no spills)
    int per_cu = 0;
    for (int minw : {4, 8}) {
        DecodeKernel k = L.nsub > 1 ? multishot_kernel(L.nsub, minw)
                                    : compact ? compact_kernel(minw, prop || d16) : decode_kernel(rdmax, lds, minw);
        int pc = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, reinterpret_cast<const void*>(k), 64 * waves,
                                                                    L.lds_bytes);
        if (e != hipSuccess) return fail(RBP_ERR_HIP, std::string("occupancy query: ") + hipGetErrorString(e));
        if (!L.kernel || pc > per_cu) {
            L.kernel = k;
            per_cu = pc;
        }
    }
    per_cu = std::max(per_cu, 1);
    if (!lds && cfg.max_slots <= 0 && rdmax > 12) {
        // rows over 12 edges with device-memory state: the 128-VGPR build (the
        // 64-VGPR one spills the unrolled 16- to 32-edge rows) when the cache
        // cap below leaves no more slots than it fits
        DecodeKernel k4 = decode_kernel(rdmax, lds, 4);
        int pc4 = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc4, reinterpret_cast<const void*>(k4),
                                                                    64 * waves, L.lds_bytes);
        if (e != hipSuccess) return fail(RBP_ERR_HIP, std::string("occupancy query: ") + hipGetErrorString(e));
        const int cus = std::max(cs[0]->num_cus, 1);
        const int64_t cap = std::max<int64_t>(kStateCacheBytes / (4 * L.gstride), cus);
        if ((int64_t)pc4 * cus >= std::min<int64_t>((int64_t)per_cu * cus, cap)) {
            L.kernel = k4;
            per_cu = std::max(pc4, 1);
        }
    }
    int64_t slots = (int64_t)per_cu * std::max(cs[0]->num_cus, 1);
    if (cfg.max_slots > 0) {
        slots = std::min<int64_t>(slots, cfg.max_slots);
    } else if (!lds) {
        // Per-slot state in device memory: keep the slots' state within the
        // Infinity Cache, which serves the check sweep's gathers (circuit-level
        // ZSZ-LP-320 memory: 1.44x the shots/s of the occupancy-limited slot
        // count), with one slot per CU at least.
        const int64_t cap = kStateCacheBytes / (4 * L.gstride);
        slots = std::min<int64_t>(slots, std::max<int64_t>(cap, std::max(cs[0]->num_cus, 1)));
    }
    slots = std::min<int64_t>(
        slots, (int64_t)std::min<uint64_t>(std::max<uint64_t>((shots + L.nsub - 1) / L.nsub, 1), 1ull << 40));
    L.slots = (int)std::max<int64_t>(slots, 1);
    *out = L;
    return RBP_OK;
}

// queue: the shot counter in caller-provided scratch (the launch then
// allocates nothing and needs the per-shot state in LDS), or null for the
// handle's own counter
static rbp_status launch_decode(rbp_code* const* cs, int n, DecodeLaunch& a, uint64_t shots, hipStream_t stream,
                                unsigned long long* queue = nullptr) {
    LaunchShape L;
    const bool multishot_ok = n == 1 && !a.delta && !a.delta16 && !a.trace_on && !a.shot_code;
    rbp_status st = plan_launch(cs, n, shots, &L, a.delta16 != nullptr, multishot_ok, a.delta != nullptr);
    if (st) return st;
    rbp_code* c0 = cs[0];
    if (queue) {
        if (!L.lds_state)
            return fail(RBP_ERR_UNSUPPORTED, "the per-shot state of this model lives in device memory, which the "
                                             "allocation-free decode cannot provide");
    } else {
        st = c0->queue.reserve(64);
        if (st) return st;
        if (!L.lds_state) {
            st = c0->gstate.reserve(sizeof(float) * (size_t)L.gstride * L.slots);
            if (st) return st;
        }
        queue = c0->queue.as<unsigned long long>();
    }
    a.queue = queue;
    a.gstate = L.lds_state ? nullptr : c0->gstate.as<float>();
    a.gstate_stride = L.gstride;
    a.Smax = L.Smax;
    a.off_M = L.off_M;
    a.off_sig = L.off_sig;
    a.off_sigp = L.off_sigp;
    a.off_par = L.off_par;
    a.off_bestp = L.off_bestp;
    a.off_best = L.off_best;
    a.off_obs = L.off_obs;
    a.off_misc = L.off_misc;
    a.off_d16 = L.off_d16;
    a.off_grp = L.off_grp;
    a.nsub = L.nsub;
    a.sub_stride = L.sub_stride;
    a.shots = shots;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, stream, a.queue, 1);
    RBP_HIP_CHECK(hipGetLastError());
    RBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(L.kernel),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, L.lds_bytes));
    hipLaunchKernelGGL(L.kernel, dim3(L.slots), dim3(64 * L.waves), L.lds_bytes, stream, a);
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

// Batches smaller than this keep their own order (the four small launches
// would cost more than the tail they save).  The learned path (a prior delta
// per shot) keeps its order too: it measured slower when sorted.
constexpr uint64_t kOrderMinShots = 8192;

// the heaviest-first order of the batch into order[shots], with a 256-bin
// histogram in hist (both device buffers the caller provides)
static rbp_status order_into(const rbp_code* c, const uint32_t* syn, uint64_t shots, uint32_t* hist, uint32_t* order,
                             hipStream_t stream) {
    const unsigned blocks = (unsigned)((shots + 255) / 256);
    const int words = ceil_div(c->M, 32);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(256), 0, stream, hist, kOrderBins);
    RBP_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(order_hist_kernel, dim3(blocks), dim3(256), 0, stream, syn, words, shots, hist);
    RBP_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(64), 0, stream, hist);
    RBP_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(order_scatter_kernel, dim3(blocks), dim3(256), 0, stream, syn, words, shots, hist, order);
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

static rbp_status order_by_weight(rbp_code* c, const uint32_t* syn, uint64_t shots, hipStream_t stream) {
    rbp_status st = c->order.reserve(sizeof(uint32_t) * shots);
    if (!st) st = c->ohist.reserve(sizeof(uint32_t) * kOrderBins);
    if (st) return st;
    return order_into(c, syn, shots, c->ohist.as<uint32_t>(), c->order.as<uint32_t>(), stream);
}

// ---------------------------------------------------------------------------
// Scratch of rbp_decode_noalloc: one fixed device array per GPU holding the
// shot counter, the ordering histogram and the shot order, so that the call
// allocates nothing.  In host code `scratch` names a host-side stand-in, never
// the device memory: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// passed to kernels.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = 4u << 20;
constexpr size_t kScratchOrderOff = 2048;  // counter at 0, histogram at 256, order from here
constexpr uint64_t kScratchMaxShots = (kScratchBytes - kScratchOrderOff) / sizeof(uint32_t);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static unsigned char* g_scratch[kMaxDevices];
// Side streams of rbp_decode_each, kMaxModels per device, created on first
// use (non-blocking, default priority) and kept until the process ends.
static std::mutex g_side_mu;
static std::vector<std::vector<hipStream_t>> g_side;

static rbp_status side_streams(int dev, hipStream_t** out) {
    std::lock_guard<std::mutex> lock(g_side_mu);
    if ((int)g_side.size() <= dev) g_side.resize(dev + 1);
    std::vector<hipStream_t>& v = g_side[dev];
    while ((int)v.size() < kMaxModels) {
        hipStream_t s = nullptr;
        RBP_HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        v.push_back(s);
    }
    *out = v.data();
    return RBP_OK;
}

static std::mutex g_scratch_mu;

// the device address of this device's scratch (set up on first use)
static rbp_status scratch_of(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(RBP_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        int cur = 0;
        RBP_HIP_CHECK(hipGetDevice(&cur));
        if (cur != dev) RBP_HIP_CHECK(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(RBP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch[dev];
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
        if (deg[i] == 1 || deg[i] > kMaxRowDeg)
            return fail(RBP_ERR_UNSUPPORTED, "row " + std::to_string(i) + " has degree " + std::to_string(deg[i]) +
                                                 " (supported: 0 or 2.." + std::to_string(kMaxRowDeg) + ")");
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
    // CSR of H (columns ascending within a row)
    std::vector<int32_t> rp(M + 1, 0), ci(std::max(E, 1)), fillc(M, 0);
    for (int i = 0; i < M; ++i) rp[i + 1] = rp[i] + deg[i];
    for (int j = 0; j < N; ++j)
        for (int e = col_ptr[j]; e < col_ptr[j + 1]; ++e) {
            const int i = row_idx[e];
            ci[rp[i] + fillc[i]++] = j;
        }
    // Variable groups: positions sorted by degree (descending, stable), 64 per
    // group; the q-th edge of the variable at position 64 g + l sits in slot
    // vbase_g + 64 q + l.
    const int GV = ceil_div(N, 64), Np = 64 * GV;
    std::vector<int32_t> cdeg(N), vperm(N);
    for (int j = 0; j < N; ++j) {
        cdeg[j] = col_ptr[j + 1] - col_ptr[j];
        vperm[j] = j;
    }
    std::stable_sort(vperm.begin(), vperm.end(), [&](int x, int y) { return cdeg[x] > cdeg[y]; });
    std::vector<int32_t> vord(Np, -1), vdeg(Np, 0), vgrp(4 * (size_t)GV, 0);
    for (int p = 0; p < N; ++p) {
        vord[p] = vperm[p];
        vdeg[p] = cdeg[vperm[p]];
    }
    int64_t S = 0;
    for (int g = 0; g < GV; ++g) {
        const int dg = vdeg[64 * g];
        bool mixed = false;
        for (int l = 0; l < 64; ++l) mixed |= vord[64 * g + l] < 0 || vdeg[64 * g + l] != dg;
        vgrp[4 * g] = (int32_t)S;
        vgrp[4 * g + 1] = dg;
        vgrp[4 * g + 2] = mixed ? 1 : 0;
        S += 64 * (int64_t)dg;
    }
    if (S + 2 > (int64_t)(INT32_MAX / 4)) return fail(RBP_ERR_UNSUPPORTED, "too many edges");
    std::vector<int32_t> slot_of(std::max(E, 1)), scheck(std::max<int64_t>(S, 1), -1), scsc(std::max<int64_t>(S, 1), -1);
    for (int p = 0; p < N; ++p) {
        const int j = vord[p], g = p >> 6, l = p & 63;
        for (int q = 0; q < cdeg[j]; ++q) {
            const int e = col_ptr[j] + q;
            const int slot = vgrp[4 * g] + 64 * q + l;
            slot_of[e] = slot;
            scheck[slot] = row_idx[e];
            scsc[slot] = e;
        }
    }
    // Row groups: checks sorted the same way; rows of up to 12 edges are stored
    // at their group's degree, up to 32 padded to 16, 24 or 32 slots, larger
    // ones to a multiple of 8.
    const int GR = ceil_div(M, 64);
    std::vector<int32_t> rperm(M), rord(64 * (size_t)GR, -1), rinv(M), rgrp(4 * (size_t)GR, 0);
    for (int i = 0; i < M; ++i) rperm[i] = i;
    std::stable_sort(rperm.begin(), rperm.end(), [&](int x, int y) { return deg[x] > deg[y]; });
    for (int p = 0; p < M; ++p) {
        rord[p] = rperm[p];
        rinv[rperm[p]] = p;
    }
    int64_t RB = 0;
    int maxstored = 0;
    for (int g = 0; g < GR; ++g) {
        const int dmax = deg[rord[64 * g]];
        const int dst = dmax <= 12 ? dmax : dmax <= 16 ? 16 : dmax <= 24 ? 24 : dmax <= 32 ? 32 : (dmax + 7) & ~7;
        bool mixed = false;
        for (int l = 0; l < 64; ++l) {
            const int i = rord[64 * g + l];
            mixed |= i < 0 || deg[i] != dst;
        }
        const int st = (dst + 3) & ~3;  // entries per lane, 16-byte aligned
        rgrp[4 * g] = (int32_t)RB;
        rgrp[4 * g + 1] = dst;
        rgrp[4 * g + 2] = mixed ? 1 : 0;
        rgrp[4 * g + 3] = st;
        RB += 64 * (int64_t)st;
        maxstored = std::max(maxstored, dst);
    }
    if (RB > (int64_t)INT32_MAX) return fail(RBP_ERR_UNSUPPORTED, "too many edges");
    std::vector<int32_t> rposp(std::max<int64_t>(RB, 1), (int32_t)(4 * S)),
        rposw(std::max<int64_t>(RB, 1), (int32_t)(4 * (S + 1))), rfill(M, 0);
    // compact state (rows of at most 16 edges): LDS address of each row edge's
    // marginal (records first, then the +inf cell, then the marginals), and
    // 16 * row position + edge code (stored degree - 1 - index) for each edge slot
    const bool compact_ok = maxstored <= 16;
    const int64_t crec = 16 * 64 * (int64_t)GR;
    const int32_t coff_M = (int32_t)(crec + 16);
    std::vector<int32_t> vinv(N), cvar(compact_ok ? std::max<int64_t>(RB, 1) : 1, (int32_t)crec);
    std::vector<uint32_t> vrec(compact_ok ? std::max<int64_t>(S, 1) : 1, 0u);
    for (int p = 0; p < N; ++p) vinv[vord[p]] = p;
    for (int j = 0; j < N; ++j)
        for (int e = col_ptr[j]; e < col_ptr[j + 1]; ++e) {
            const int i = row_idx[e], p = rfill[i]++, pos = rinv[i];
            const size_t at = (size_t)rgrp[4 * (pos >> 6)] + (size_t)(pos & 63) * rgrp[4 * (pos >> 6) + 3] + p;
            rposp[at] = 4 * slot_of[e];
            rposw[at] = 4 * slot_of[e];
            if (compact_ok) {
                cvar[at] = coff_M + 4 * vinv[j];
                vrec[slot_of[e]] = 16u * (uint32_t)pos + (uint32_t)(rgrp[4 * (pos >> 6) + 1] - 1 - p);
            }
        }
    if (compact_ok && (int64_t)coff_M + 4 * (int64_t)Np > (int64_t)INT32_MAX)
        return fail(RBP_ERR_UNSUPPORTED, "too many rows");
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
    c->S = (int32_t)S;
    c->GR = GR;
    c->GV = GV;
    c->Np = Np;
    c->RB = (int32_t)RB;
    c->max_stored_row_deg = maxstored;
    c->GRw = 0;
    while (c->GRw < GR && rgrp[4 * c->GRw + 1] > 32) ++c->GRw;
    c->compact_ok = compact_ok;
    c->coff_M = coff_M;
    c->h_vord = vord;
    hipError_t he = hipGetDevice(&c->device);
    if (he == hipSuccess) he = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, c->device);
    if (he != hipSuccess) {
        delete c;
        return fail(RBP_ERR_HIP, std::string("device query: ") + hipGetErrorString(he));
    }
    {
        unsigned char* sp = nullptr;
        const rbp_status sst = scratch_of(c->device, &sp);
        if (sst) {
            delete c;
            return sst;
        }
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
    if (!st) st = upload(c->rgrp, rgrp);
    if (!st) st = upload(c->rposp, rposp);
    if (!st) st = upload(c->rposw, rposw);
    if (!st) st = upload(c->rord, rord);
    if (!st) st = upload(c->vgrp, vgrp);
    if (!st) st = upload(c->vord, vord);
    if (!st) st = upload(c->vdeg, vdeg);
    if (!st) st = upload(c->scheck, scheck);
    if (!st) st = upload(c->scsc, scsc);
    if (!st) st = upload(c->orow_ptr, orp);
    if (!st) st = upload(c->ocol_idx, oci);
    if (!st) st = upload(c->ocol_ptr, ocp);
    if (!st) st = upload(c->orow_idx, ori);
    if (!st) st = upload(c->vinv, vinv);
    if (!st && compact_ok) st = upload(c->cvar, cvar);
    if (!st && compact_ok) st = upload(c->vrec, vrec);
    if (st) {
        rbp_code_destroy(c);
        return st;
    }
    *out = c;
    return RBP_OK;
}

rbp_status rbp_code_destroy(rbp_code_t c) {
    if (!c) return RBP_OK;
    if (c->residents) return fail(RBP_ERR_INVALID_ARG, "a resident decoder runs on this code; stop it first");
    (void)hipDeviceSynchronize();
    for (DevBuf* b : {&c->row_ptr, &c->col_idx, &c->col_ptr, &c->csc_row, &c->rgrp, &c->rposp, &c->rposw, &c->rord, &c->vgrp,
                      &c->vord, &c->vdeg, &c->scheck, &c->scsc, &c->orow_ptr, &c->ocol_idx, &c->ocol_ptr,
                      &c->orow_idx, &c->thr, &c->lam, &c->lamp, &c->m1, &c->gtab, &c->lg, &c->queue, &c->gstate,
                      &c->trace_hit, &c->spa_queue, &c->gapt, &c->order, &c->ohist, &c->coop, &c->cvar, &c->vrec,
                      &c->r1rec, &c->vinv})
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
    a.L = ceil_div(c->N, 64);
    a.gap = c->gapt.as<uint32_t>();
    a.acc = c->thr.as<uint32_t>();
    a.seed = seed;
    a.offset = shot_offset;
    a.syn = syndromes;
    a.obs = c->k > 0 ? obs : nullptr;
    a.err = errors;
    const size_t lds = sizeof(uint32_t) * (size_t)kSampleWaves * (a.WM + a.WK + (errors ? a.WN : 0));
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
    if (!st) st = ensure_lam_gamma(c, params, stream);
    if (st) return st;
    DecodeLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.m[0] = model_of(c, syndromes, corrections, obs_pred);
    a.n_models = 1;
    a.delta = prior_delta;
    a.stats = stats;
    fill_params(a, params);
    if (!prior_delta && shots >= kOrderMinShots && shots <= 0x7FFFFFFFull) {
        st = order_by_weight(c, syndromes, shots, stream);
        if (st) return st;
        a.shot_index = c->order.as<uint32_t>();
        a.stats_by_row = 1;
    }
    rbp_code* cs[1] = {c};
    return launch_decode(cs, 1, a, shots, stream);
}

rbp_status rbp_decode_proposal(rbp_code_t c, const double* priors, const uint32_t* syndromes, uint64_t shots,
                               const rbp_relay_params* params, const uint16_t* delta_bf16, uint32_t* corrections,
                               uint32_t* obs_pred, rbp_shot_stats* stats, void* stream_) {
    if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
    rbp_status st = check_params(params);
    if (st) return st;
    if (shots == 0) return RBP_OK;
    if (!syndromes || !corrections || !delta_bf16)
        return fail(RBP_ERR_INVALID_ARG, "syndromes/corrections/delta is NULL");
    if (c->k > 0 && !obs_pred) return fail(RBP_ERR_INVALID_ARG, "obs_pred is NULL");
    st = check_priors(priors, c->N);
    if (st) return st;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    st = ensure_llr(c, priors, stream);
    if (!st) st = ensure_gamma(c, params, stream);
    if (!st) st = ensure_lam_gamma(c, params, stream);
    if (st) return st;
    DecodeLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.m[0] = model_of(c, syndromes, corrections, obs_pred);
    a.n_models = 1;
    a.delta16 = delta_bf16;
    a.stats = stats;
    fill_params(a, params);
    rbp_code* cs[1] = {c};
    return launch_decode(cs, 1, a, shots, stream);
}

rbp_status rbp_decode_proposal_pos(rbp_code_t c, const double* priors, const uint32_t* syndromes, uint64_t shots,
                                   const rbp_relay_params* params, const uint16_t* delta_bf16_pos,
                                   uint32_t* corrections, uint32_t* obs_pred, rbp_shot_stats* stats, void* stream_) {
    if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
    if (delta_bf16_pos && (reinterpret_cast<uintptr_t>(delta_bf16_pos) & 15) != 0)
        return fail(RBP_ERR_INVALID_ARG, "delta (by position) must be 16-byte aligned");
    rbp_status st = check_params(params);
    if (st) return st;
    if (shots == 0) return RBP_OK;
    if (!syndromes || !corrections || !delta_bf16_pos)
        return fail(RBP_ERR_INVALID_ARG, "syndromes/corrections/delta is NULL");
    if (c->k > 0 && !obs_pred) return fail(RBP_ERR_INVALID_ARG, "obs_pred is NULL");
    st = check_priors(priors, c->N);
    if (st) return st;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    st = ensure_llr(c, priors, stream);
    if (!st) st = ensure_gamma(c, params, stream);
    if (!st) st = ensure_lam_gamma(c, params, stream);
    if (st) return st;
    DecodeLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.m[0] = model_of(c, syndromes, corrections, obs_pred);
    a.n_models = 1;
    a.delta16 = delta_bf16_pos;
    a.d16_pos = 1;
    a.stats = stats;
    fill_params(a, params);
    rbp_code* cs[1] = {c};
    return launch_decode(cs, 1, a, shots, stream);
}

rbp_status rbp_code_positions(rbp_code_t c, int32_t* np, int32_t* var_of_position) {
    if (!c || !np) return fail(RBP_ERR_INVALID_ARG, "code/np is NULL");
    *np = c->Np;
    if (var_of_position) std::memcpy(var_of_position, c->h_vord.data(), sizeof(int32_t) * (size_t)c->Np);
    return RBP_OK;
}

rbp_status rbp_decode_noalloc(rbp_code_t c, const double* priors, const uint32_t* syndromes, uint64_t shots,
                              const rbp_relay_params* params, const float* prior_delta, uint32_t* corrections,
                              uint32_t* obs_pred, rbp_shot_stats* stats, void* stream_) {
    if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
    rbp_status st = check_params(params);
    if (st) return st;
    if (shots == 0) return RBP_OK;
    if (shots > kScratchMaxShots)
        return fail(RBP_ERR_UNSUPPORTED, "allocation-free decode: at most " + std::to_string(kScratchMaxShots) +
                                             " shots per call (4 MiB of scratch)");
    if (!syndromes || !corrections) return fail(RBP_ERR_INVALID_ARG, "syndromes/corrections is NULL");
    if (c->k > 0 && !obs_pred) return fail(RBP_ERR_INVALID_ARG, "obs_pred is NULL");
    st = check_priors(priors, c->N);
    if (st) return st;
    // the handle's tables must already hold these priors and parameters (an
    // rbp_decode call builds them); rebuilding them would allocate
    const bool ready = c->lam.p && c->lam_key.size() == (size_t)c->N &&
                       std::memcmp(c->lam_key.data(), priors, sizeof(double) * c->N) == 0 && c->gtab.p &&
                       c->gtab_R == params->num_sets && c->gtab_seed == params->gamma_seed &&
                       c->gtab_lo == params->gamma_min && c->gtab_hi == params->gamma_max && c->lg.p &&
                       c->lg_lam_gen == c->lam_gen && c->lg_gtab_gen == c->gtab_gen &&
                       c->lg_gamma0 == params->gamma0 && c->lg_R == params->num_sets;
    if (!ready)
        return fail(RBP_ERR_INVALID_ARG, "allocation-free decode: call rbp_decode once with these priors and relay "
                                         "parameters first (it builds the handle's tables)");
    unsigned char* sp = nullptr;
    st = scratch_of(c->device, &sp);
    if (st) return st;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    DecodeLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.m[0] = model_of(c, syndromes, corrections, obs_pred);
    a.n_models = 1;
    a.delta = prior_delta;
    a.stats = stats;
    fill_params(a, params);
    if (!prior_delta && shots >= kOrderMinShots) {
        uint32_t* hist = reinterpret_cast<uint32_t*>(sp + 256);
        uint32_t* order = reinterpret_cast<uint32_t*>(sp + kScratchOrderOff);
        st = order_into(c, syndromes, shots, hist, order, stream);
        if (st) return st;
        a.shot_index = order;
        a.stats_by_row = 1;
    }
    rbp_code* cs[1] = {c};
    return launch_decode(cs, 1, a, shots, stream, reinterpret_cast<unsigned long long*>(sp));
}

// Launch shape, scratch layout and kernel of the latency mode, shared by
// rbp_decode_coop and the resident decoder.  Fills everything in `a` but the
// model (a.m), the shot range and the outputs; (re)serves the shot state in
// `xbuf` and the parity / best-solution / barrier words in `scratch`.
struct CoopPlan {
    CoopLaunch a;
    int64_t grid = 0;
    int waves = 0, lds = 0;
    int clear_words = 0;  // barrier words cleared before each launch, from a.sh on
    const void* kern = nullptr;
};

static rbp_status coop_plan(rbp_code* c, const rbp_relay_params* params, const rbp_coop_params& cp, bool resident,
                            DevBuf& xbuf, DevBuf& scratch, CoopPlan& P) {
    const int cus = std::max(c->num_cus, 1);
    const int waves = cp.waves > 0 ? cp.waves : 8;
    int nwg = cp.workgroups > 0 ? cp.workgroups : std::max(cus / 8, 1);
    nwg = std::min(nwg, cus);
    int stride = cp.stride > 0 ? cp.stride : (nwg * 8 <= cus ? 8 : 1);
    if ((int64_t)nwg * stride > cus) stride = 1;
    CoopLaunch& a = P.a;
    std::memset(&a, 0, sizeof(a));
    a.Smax = c->S;
    a.nwg = nwg;
    a.stride = stride;
    a.arrivals = (unsigned)(nwg + c->coop_phantom);
    a.force_device = cp.device_fences != 0;
    a.spin_limit = cp.spin_limit > 0 ? cp.spin_limit : (1u << 21);
    a.T0 = params->pre_iter;
    a.Tr = params->max_iterations;
    a.R = params->num_sets;
    a.S = params->stop_nconv;
    a.crit = params->stopping_criterion;
    const int64_t xfloats = ((int64_t)c->S + 4 + c->Np + 63) / 64 * 64;
    const int WM = ceil_div(c->M, 32), WN = ceil_div(c->N, 32), WK = std::max(ceil_div(c->k, 32), 1);
    const int64_t o_par = 0, o_bestp = align16(4 * (int64_t)WM), o_best = o_bestp + align16(4 * (int64_t)(c->Np / 32)),
                  o_sh = o_best + align16(4 * (int64_t)WN), o_flags = o_sh + (int64_t)sizeof(CoopShared),
                  o_cnt = o_flags + align16(4 * (int64_t)a.arrivals), o_wsum = o_cnt + align16(4 * (int64_t)nwg),
                  coop_bytes = o_wsum + 8 * (int64_t)nwg;
    rbp_status st = xbuf.reserve(sizeof(float) * (size_t)xfloats);
    if (!st) st = scratch.reserve((size_t)coop_bytes);
    if (st) return st;
    a.X = xbuf.as<float>();
    char* cb = reinterpret_cast<char*>(scratch.p);
    a.par = reinterpret_cast<uint32_t*>(cb + o_par);
    a.bestp = reinterpret_cast<uint32_t*>(cb + o_bestp);
    a.best = reinterpret_cast<uint32_t*>(cb + o_best);
    a.sh = reinterpret_cast<CoopShared*>(cb + o_sh);
    a.flags = reinterpret_cast<uint32_t*>(cb + o_flags);
    a.cnt = reinterpret_cast<int32_t*>(cb + o_cnt);
    a.wsum = reinterpret_cast<double*>(cb + o_wsum);
    P.clear_words = (int)((o_cnt - o_sh) / 4);
    int64_t off = 0;
    a.off_sig = (int)off;
    off += align16(4 * (int64_t)WM);
    a.off_sigp = (int)off;
    off += align16(8 * (int64_t)c->GR);
    a.off_obs = (int)off;
    off += align16(4 * (int64_t)WK);
    a.off_misc = (int)off;
    off += align16(sizeof(CoopMisc));
    if (off > kMaxLds) return fail(RBP_ERR_UNSUPPORTED, "syndrome bits do not fit in LDS");
    const int lds = (int)off;
    void (*kern)(CoopLaunch);
    if (resident)
        kern = c->max_stored_row_deg <= 12 ? relay_bp_coop_kernel<12, true> : relay_bp_coop_kernel<32, true>;
    else
        kern = c->max_stored_row_deg <= 12 ? relay_bp_coop_kernel<12, false> : relay_bp_coop_kernel<32, false>;
    RBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      lds));
    int per_cu = 0;
    RBP_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                                64 * waves, lds));
    const int64_t grid = (int64_t)nwg * stride;
    if (per_cu < 1 || grid > (int64_t)per_cu * cus)
        return fail(RBP_ERR_UNSUPPORTED, "coop: the workgroups cannot all be resident");
    P.grid = grid;
    P.waves = waves;
    P.lds = lds;
    P.kern = reinterpret_cast<const void*>(kern);
    return RBP_OK;
}

static rbp_status coop_check(const rbp_coop_params& cp) {
    if (cp.workgroups < 0 || cp.stride < 0 || cp.waves < 0 || cp.waves > 8)
        return fail(RBP_ERR_INVALID_ARG, "coop: workgroups, stride >= 0, waves in 0..8");
    return RBP_OK;
}

// clears the barrier words, then launches the plan's kernel cooperatively
static rbp_status coop_launch(CoopPlan& P, hipStream_t stream) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(256), 0, stream, reinterpret_cast<uint32_t*>(P.a.sh),
                       P.clear_words);
    RBP_HIP_CHECK(hipGetLastError());
    void* args[] = {&P.a};
    RBP_HIP_CHECK(hipLaunchCooperativeKernel(P.kern, dim3((unsigned)P.grid), dim3(64 * P.waves), args,
                                             (unsigned)P.lds, stream));
    return RBP_OK;
}

rbp_status rbp_decode_coop(rbp_code_t c, const double* priors, const uint32_t* syndromes, uint64_t shots,
                           const rbp_relay_params* params, const rbp_coop_params* coop, uint32_t* corrections,
                           uint32_t* obs_pred, rbp_shot_stats* stats, void* stream_) {
    if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
    rbp_status st = check_params(params);
    if (st) return st;
    if (!syndromes || !corrections) return fail(RBP_ERR_INVALID_ARG, "syndromes/corrections is NULL");
    if (c->k > 0 && !obs_pred) return fail(RBP_ERR_INVALID_ARG, "obs_pred is NULL");
    st = check_priors(priors, c->N);
    if (st) return st;
    rbp_coop_params cp = {0, 0, 0, 0u, 0};
    if (coop) cp = *coop;
    st = coop_check(cp);
    if (st) return st;
    if (shots == 0) return RBP_OK;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    st = ensure_llr(c, priors, stream);
    if (!st) st = ensure_gamma(c, params, stream);
    if (!st) st = ensure_lam_gamma(c, params, stream);
    if (st) return st;
    CoopPlan P;
    st = coop_plan(c, params, cp, false, c->gstate, c->coop, P);
    if (st) return st;
    P.a.m = model_of(c, syndromes, corrections, obs_pred);
    P.a.shots = shots;
    P.a.stats = stats;
    st = coop_launch(P, stream);
    if (st) return st;
    // the launch's end: an expired barrier wait is reported as ABORTED
    unsigned int aborted = 0;
    RBP_HIP_CHECK(hipMemcpyAsync(&aborted, &P.a.sh->abort, sizeof(aborted), hipMemcpyDeviceToHost, stream));
    RBP_HIP_CHECK(hipStreamSynchronize(stream));
    if (aborted) return fail(RBP_ERR_ABORTED, "latency mode: a barrier wait expired; later shots were not decoded");
    return RBP_OK;
}

// ---------------------------------------------------------------------------
// Resident decoder: the latency-mode kernel launched once and fed one shot at
// a time through a mailbox in pinned host memory (ResidentBox).
// ---------------------------------------------------------------------------
struct rbp_resident {
    rbp_code* c = nullptr;
    hipStream_t stream = nullptr;
    char* host = nullptr;  // the mailbox (hipHostMalloc, coherent)
    size_t bytes = 0;
    int64_t o_syn = 0, o_corr = 0, o_obs = 0, o_stats = 0;
    rbp::DevBuf x, scratch;
    CoopPlan P;
    uint64_t next = 0;     // shots handed over (and finished) so far
    int32_t launches = 0;
    bool running = false;
    double wait_s = 60.0;
    rbp::ResidentBox* box() { return reinterpret_cast<rbp::ResidentBox*>(host); }
};

static rbp_status resident_launch(rbp_resident* r) {
    ResidentBox* b = r->box();
    __atomic_store_n(&b->published, (unsigned long long)r->next, __ATOMIC_RELAXED);
    __atomic_store_n(&b->done, (unsigned long long)r->next, __ATOMIC_RELAXED);
    __atomic_store_n(&b->stop, 0u, __ATOMIC_RELAXED);
    __atomic_store_n(&b->xcds, 0u, __ATOMIC_RELAXED);
    __atomic_store_n(&b->state, 0u, __ATOMIC_RELEASE);
    r->P.a.res_start = r->next;
    rbp_status st = coop_launch(r->P, r->stream);
    if (st) return st;
    r->running = true;
    ++r->launches;
    return RBP_OK;
}

// ends the kernel (it finishes the shot it is decoding, if any) and waits for it
static rbp_status resident_halt(rbp_resident* r) {
    if (!r->running) return RBP_OK;
    __atomic_store_n(&r->box()->stop, 1u, __ATOMIC_RELEASE);
    r->running = false;
    RBP_HIP_CHECK(hipStreamSynchronize(r->stream));
    r->next = __atomic_load_n(&r->box()->done, __ATOMIC_ACQUIRE);
    return RBP_OK;
}

rbp_status rbp_resident_start(rbp_code_t c, const double* priors, const rbp_relay_params* params,
                              const rbp_resident_params* rp, rbp_resident_t* out) {
    if (!c || !out) return fail(RBP_ERR_INVALID_ARG, "code/out is NULL");
    *out = nullptr;
    rbp_status st = check_params(params);
    if (st) return st;
    st = check_priors(priors, c->N);
    if (st) return st;
    rbp_resident_params q;
    std::memset(&q, 0, sizeof(q));
    if (rp) q = *rp;
    st = coop_check(q.coop);
    if (st) return st;
    if (!(q.idle_seconds >= 0.0 && q.idle_seconds <= 3600.0) || !(q.wait_seconds >= 0.0 && q.wait_seconds <= 3600.0))
        return fail(RBP_ERR_INVALID_ARG, "resident: idle_seconds and wait_seconds in [0, 3600]");
    int dev = 0, khz = 0;
    RBP_HIP_CHECK(hipGetDevice(&dev));
    RBP_HIP_CHECK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return fail(RBP_ERR_UNSUPPORTED, "resident: device wall clock rate unknown");
    std::unique_ptr<rbp_resident> r(new (std::nothrow) rbp_resident());
    if (!r) return fail(RBP_ERR_OOM, "resident: handle");
    r->c = c;
    r->wait_s = q.wait_seconds > 0.0 ? q.wait_seconds : 60.0;
    // its own non-blocking stream, at the default priority: the resident kernel
    // never holds up work on the legacy default stream
    RBP_HIP_CHECK(hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking));
    auto undo = [&](rbp_status e) {
        if (r->stream) (void)hipStreamSynchronize(r->stream);
        r->x.release();
        r->scratch.release();
        if (r->host) (void)hipHostFree(r->host);
        if (r->stream) (void)hipStreamDestroy(r->stream);
        return e;
    };
    st = ensure_llr(c, priors, r->stream);
    if (!st) st = ensure_gamma(c, params, r->stream);
    if (!st) st = ensure_lam_gamma(c, params, r->stream);
    if (!st) st = coop_plan(c, params, q.coop, true, r->x, r->scratch, r->P);
    if (st) return undo(st);
    const int WM = ceil_div(c->M, 32), WN = ceil_div(c->N, 32), WK = std::max(ceil_div(c->k, 32), 1);
    r->o_syn = (int64_t)sizeof(ResidentBox);
    r->o_corr = r->o_syn + (4 * (int64_t)WM + 63) / 64 * 64;
    r->o_obs = r->o_corr + (4 * (int64_t)WN + 63) / 64 * 64;
    r->o_stats = r->o_obs + (4 * (int64_t)WK + 63) / 64 * 64;
    r->bytes = (size_t)(r->o_stats + 64);
    void* h = nullptr;
    if (hipHostMalloc(&h, r->bytes, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess || !h) {
        (void)hipGetLastError();
        return undo(fail(RBP_ERR_OOM, "resident: pinned mailbox"));
    }
    r->host = reinterpret_cast<char*>(h);
    std::memset(r->host, 0, r->bytes);
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess || !d) {
        (void)hipGetLastError();
        return undo(fail(RBP_ERR_HIP, "resident: no device view of the mailbox"));
    }
    char* db = reinterpret_cast<char*>(d);
    CoopLaunch& a = r->P.a;
    a.m = model_of(c, reinterpret_cast<const uint32_t*>(db + r->o_syn), reinterpret_cast<uint32_t*>(db + r->o_corr),
                   reinterpret_cast<uint32_t*>(db + r->o_obs));
    a.stats = reinterpret_cast<rbp_shot_stats*>(db + r->o_stats);
    a.box = reinterpret_cast<ResidentBox*>(db);
    const double ticks_per_s = 1e3 * (double)khz;
    a.res_idle = (uint64_t)((q.idle_seconds > 0.0 ? q.idle_seconds : 1.0) * ticks_per_s);
    a.res_grace = (uint64_t)ticks_per_s;
    st = resident_launch(r.get());
    if (st) return undo(st);
    ++c->residents;
    *out = r.release();
    return RBP_OK;
}

rbp_status rbp_resident_decode(rbp_resident_t r, const uint32_t* syndrome, uint32_t* correction, uint32_t* obs_pred,
                               rbp_shot_stats* stats) {
    if (!r) return fail(RBP_ERR_INVALID_ARG, "resident handle is NULL");
    if (!syndrome || !correction) return fail(RBP_ERR_INVALID_ARG, "syndrome/correction is NULL");
    rbp_code* c = r->c;
    if (c->k > 0 && !obs_pred) return fail(RBP_ERR_INVALID_ARG, "obs_pred is NULL");
    const int WM = ceil_div(c->M, 32), WN = ceil_div(c->N, 32), WK = ceil_div(c->k, 32);
    rbp_status st;
    if (!r->running) {
        st = resident_launch(r);
        if (st) return st;
    }
    ResidentBox* b = r->box();
    const uint64_t s = r->next;
    std::memcpy(r->host + r->o_syn, syndrome, 4 * (size_t)WM);
    __atomic_store_n(&b->published, (unsigned long long)(s + 1), __ATOMIC_RELEASE);
    const auto t0 = std::chrono::steady_clock::now();
    for (uint64_t k = 1;; ++k) {
        if (__atomic_load_n(&b->done, __ATOMIC_ACQUIRE) > s) break;
        const unsigned state = __atomic_load_n(&b->state, __ATOMIC_ACQUIRE);
        if (state == kResidentIdle) {
            // the kernel ended for want of a shot before it saw this one (it ends
            // only while waiting for shot `done`, and done <= s): launch it again
            r->running = false;
            RBP_HIP_CHECK(hipStreamSynchronize(r->stream));
            st = resident_launch(r);
            if (st) return st;
            __atomic_store_n(&b->published, (unsigned long long)(s + 1), __ATOMIC_RELEASE);
            continue;
        }
        if (state == kResidentAborted || state == kResidentStopped) {
            st = resident_halt(r);
            if (st) return st;
            return fail(RBP_ERR_ABORTED, "resident: the kernel ended (a barrier wait expired); the shot was not decoded");
        }
        if ((k & 1023u) == 0) {
            const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (el > r->wait_s) {
                st = resident_halt(r);
                if (st) return st;
                return fail(RBP_ERR_ABORTED, "resident: no result within wait_seconds; the kernel was stopped");
            }
        }
        __builtin_ia32_pause();
    }
    std::memcpy(correction, r->host + r->o_corr, 4 * (size_t)WN);
    if (obs_pred && WK > 0) std::memcpy(obs_pred, r->host + r->o_obs, 4 * (size_t)WK);
    if (stats) std::memcpy(stats, r->host + r->o_stats, sizeof(rbp_shot_stats));
    r->next = s + 1;
    return RBP_OK;
}

rbp_status rbp_resident_info(rbp_resident_t r, uint64_t* shots, int32_t* launches, int32_t* running,
                             uint32_t* xcds) {
    if (!r) return fail(RBP_ERR_INVALID_ARG, "resident handle is NULL");
    if (shots) *shots = r->next;
    if (launches) *launches = r->launches;
    if (xcds) *xcds = __atomic_load_n(&r->box()->xcds, __ATOMIC_ACQUIRE);
    if (running) {
        const unsigned state = __atomic_load_n(&r->box()->state, __ATOMIC_ACQUIRE);
        *running = r->running && state != kResidentIdle && state != kResidentAborted && state != kResidentStopped;
    }
    return RBP_OK;
}

rbp_status rbp_resident_stop(rbp_resident_t r) {
    if (!r) return RBP_OK;
    rbp_status st = resident_halt(r);
    (void)hipStreamSynchronize(r->stream);
    r->x.release();
    r->scratch.release();
    if (r->host) (void)hipHostFree(r->host);
    (void)hipStreamDestroy(r->stream);
    --r->c->residents;
    delete r;
    return st;
}

rbp_status rbp_test_set_coop_phantom(rbp_code_t c, int32_t phantom) {
    if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
    if (phantom < 0 || phantom > 1024) return fail(RBP_ERR_INVALID_ARG, "phantom must be 0..1024");
    c->coop_phantom = phantom;
    return RBP_OK;
}

rbp_status rbp_coop_aborted(rbp_code_t c, void* stream_, int32_t* aborted) {
    if (!c || !aborted) return fail(RBP_ERR_INVALID_ARG, "code or aborted is NULL");
    *aborted = 0;
    if (!c->coop.p) return RBP_OK;
    const int WM = ceil_div(c->M, 32), WN = ceil_div(c->N, 32);
    const int64_t o_sh = align16(4 * (int64_t)WM) + align16(4 * (int64_t)(c->Np / 32)) + align16(4 * (int64_t)WN);
    const CoopShared* sh = reinterpret_cast<const CoopShared*>(reinterpret_cast<const char*>(c->coop.p) + o_sh);
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    unsigned int v = 0;
    RBP_HIP_CHECK(hipMemcpyAsync(&v, &sh->abort, sizeof(v), hipMemcpyDeviceToHost, stream));
    RBP_HIP_CHECK(hipStreamSynchronize(stream));
    *aborted = v != 0u ? 1 : 0;
    return RBP_OK;
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
        if (!st) st = ensure_lam_gamma(c, params, stream);
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

rbp_status rbp_decode_each(int32_t n_codes, const rbp_code_t* codes, const double* const* priors,
                           const uint64_t* shots, const uint32_t* const* syndromes, const rbp_relay_params* params,
                           uint32_t* const* corrections, uint32_t* const* obs_pred, rbp_shot_stats* const* stats,
                           void* stream_) {
    if (n_codes < 1 || n_codes > kMaxModels) return fail(RBP_ERR_INVALID_ARG, "n_codes must be 1..8");
    if (!codes || !priors || !shots || !syndromes || !corrections) return fail(RBP_ERR_INVALID_ARG, "NULL array");
    rbp_status st = check_params(params);
    if (st) return st;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    // every argument and table first, on the caller's stream: nothing is
    // launched unless every model can be
    for (int i = 0; i < n_codes; ++i) {
        rbp_code* c = codes[i];
        if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
        for (int j = 0; j < i; ++j)
            if (codes[j] == c) return fail(RBP_ERR_INVALID_ARG, "each handle may appear once");
        if (shots[i] == 0) continue;
        if (!syndromes[i] || !corrections[i]) return fail(RBP_ERR_INVALID_ARG, "syndromes/corrections is NULL");
        if (c->k > 0 && (!obs_pred || !obs_pred[i])) return fail(RBP_ERR_INVALID_ARG, "obs_pred is NULL");
        st = check_priors(priors[i], c->N);
        if (!st) st = ensure_llr(c, priors[i], stream);
        if (!st) st = ensure_gamma(c, params, stream);
        if (!st) st = ensure_lam_gamma(c, params, stream);
        if (st) return st;
    }
    int dev = 0;
    RBP_HIP_CHECK(hipGetDevice(&dev));
    hipStream_t* pool = nullptr;
    st = side_streams(dev, &pool);
    if (st) return st;
    // fork: every side stream waits for the caller's stream; the largest
    // model is issued first, so the smaller launches fill its tail
    std::vector<int> order(n_codes);
    for (int i = 0; i < n_codes; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return (int64_t)codes[x]->E * (int64_t)shots[x] > (int64_t)codes[y]->E * (int64_t)shots[y];
    });
    hipEvent_t fork = nullptr;
    RBP_HIP_CHECK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    std::vector<hipEvent_t> joins;
    auto finish = [&](rbp_status e) {
        // join whatever was issued, so the caller's stream orders after it
        for (hipEvent_t j : joins) {
            (void)hipStreamWaitEvent(stream, j, 0);
            (void)hipEventDestroy(j);
        }
        (void)hipEventDestroy(fork);
        return e;
    };
    if (hipEventRecord(fork, stream) != hipSuccess) return finish(fail(RBP_ERR_HIP, "hipEventRecord failed"));
    for (int k = 0; k < n_codes; ++k) {
        const int i = order[k];
        if (shots[i] == 0) continue;
        hipStream_t side = pool[k];
        if (hipStreamWaitEvent(side, fork, 0) != hipSuccess)
            return finish(fail(RBP_ERR_HIP, "hipStreamWaitEvent failed"));
        st = rbp_decode(codes[i], priors[i], syndromes[i], shots[i], params, nullptr, corrections[i],
                        obs_pred ? obs_pred[i] : nullptr, stats ? stats[i] : nullptr, side);
        hipEvent_t j = nullptr;
        if (hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess || hipEventRecord(j, side) != hipSuccess)
            return finish(st ? st : fail(RBP_ERR_HIP, "join event failed"));
        joins.push_back(j);
        if (st) return finish(st);
    }
    return finish(RBP_OK);
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
    if (cfg->waves_per_shot < 0 || cfg->waves_per_shot > 16 || cfg->state < 0 || cfg->state > 3 ||
        cfg->max_slots < 0 || (cfg->shots_per_wg != 0 && cfg->shots_per_wg != 1 && cfg->shots_per_wg != 2 &&
                               cfg->shots_per_wg != 4))
        return fail(RBP_ERR_INVALID_ARG, "launch config out of range");
    c->cfg.waves_per_shot = cfg->waves_per_shot;
    c->cfg.state = cfg->state;
    c->cfg.max_slots = cfg->max_slots;
    c->cfg.shots_per_wg = cfg->shots_per_wg;
    return RBP_OK;
}

rbp_status rbp_get_launch_config(rbp_code_t c, rbp_launch_config* cfg, int32_t* slots, int32_t* lds_bytes) {
    if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
    LaunchShape L;
    rbp_code* cs[1] = {c};
    rbp_status st = plan_launch(cs, 1, 1ull << 40, &L, false, true);
    if (st) return st;
    if (cfg) {
        cfg->waves_per_shot = L.waves;
        cfg->state = L.compact ? 3 : L.lds_state ? 1 : 2;
        cfg->max_slots = c->cfg.max_slots;
        cfg->shots_per_wg = L.nsub;
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
    if (!st) st = ensure_lam_gamma(c, params, stream);
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
