// librbp: BPSK-AWGN channel sampling and sum-product BP decoding for gfx950.
//
// The paper benchmarks its classical ZSZ-2BGA codes by sending the all-zero
// codeword over an additive white Gaussian noise channel and decoding with
// flooding sum-product BP (phi-domain check update, LLRs clipped to
// +-llr_max, single-precision messages; numerics appendix, "classical channel
// coding").  The work is organised like the Relay-BP decoder, whose layout
// tables a code handle already holds:
//
//  * awgn_kernel   one thread per (shot, 4 code bits): one Philox call gives
//                  two Box-Muller pairs, stored as four consecutive LLRs.
//  * spa_kernel    persistent: each workgroup is a shot slot that pulls shots
//                  from a device counter.  The slot's messages live in LDS, one
//                  float per edge slot, in the variable-major layout of the
//                  handle (slot of the q-th edge of the variable at position
//                  64 g + l is vbase_g + 64 q + l); rows read and write their
//                  edges through the handle's per-row offset tables (16-byte
//                  loads), padded rows read a +inf cell, which phi maps to 0.
//                  The syndrome of the hard decision is kept incrementally:
//                  a variable whose decision flips toggles its checks' parity
//                  bits with LDS atomics, so the stop test is one counter.
#include <algorithm>
#include <cmath>
#include <string>

#include "rbp_common.h"

namespace rbp {

// ---------------------------------------------------------------------------
// Channel: llr = 2 (1 + sigma z) / sigma^2, z by Box-Muller from Philox words
// ---------------------------------------------------------------------------
struct AwgnArgs {
    int32_t N, Q;  // Q = ceil(N / 4) Philox calls per shot
    uint64_t shots, seed, offset;
    float sigma, scale;  // scale = 2 / sigma^2
    float* llr;
};

__device__ __forceinline__ float2 box_muller(uint32_t w0, uint32_t w1) {
    const float u1 = (float)((w0 >> 8) + 1u) * 0x1p-24f;  // (0, 1]
    const float u2 = (float)(w1 >> 8) * 0x1p-24f;         // [0, 1)
    const float r = sqrtf(-2.0f * logf(u1));
    float s, c;
    sincospif(2.0f * u2, &s, &c);
    return make_float2(r * c, r * s);
}

__global__ void __launch_bounds__(256) awgn_kernel(const AwgnArgs a) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t s = t / (uint64_t)a.Q;
    if (s >= a.shots) return;
    const int q = (int)(t - s * (uint64_t)a.Q);
    const uint64_t sid = a.offset + s;
    const U4 w = philox4x32_10(U4{(uint32_t)q, (uint32_t)sid, (uint32_t)(sid >> 32), 2u}, (uint32_t)a.seed,
                               (uint32_t)(a.seed >> 32));
    const float2 z01 = box_muller(w.x, w.y), z23 = box_muller(w.z, w.w);
    const float z[4] = {z01.x, z01.y, z23.x, z23.y};
    float* out = a.llr + s * (uint64_t)a.N;
    const int j0 = 4 * q;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        if (j0 + b < a.N) out[j0 + b] = __fmul_rn(__fadd_rn(1.0f, __fmul_rn(a.sigma, z[b])), a.scale);
}

// ---------------------------------------------------------------------------
// Sum-product BP
// ---------------------------------------------------------------------------
struct SpaLaunch {
    int32_t N, WN, WM, S, GR, GV, Np;
    const int4* rgrp;      // {offset in rposp, stored degree, mixed, lane stride}
    const int32_t* rposp;  // byte offsets of a row's edge slots (4 S = the +inf cell)
    const int32_t* rposw;  // the same for writes (4 (S + 1) = write-only cell)
    const int4* vgrp;      // {first slot, degree, mixed, 0}
    const int32_t* vord;   // variable at each position (-1 padding)
    const int32_t* vdeg;   // degree at each position
    const int32_t* scheck; // check of each slot
    const float* llr;
    uint64_t shots;
    int32_t T, stop;
    float llr_max;
    uint32_t* bits;
    float* marg;
    rbp_shot_stats* stats;
    unsigned long long* counts;
    unsigned long long* queue;
    int32_t off_L, off_M, off_par, off_dec, off_out, off_misc;
};

constexpr int kSpaRun = 8;  // frames taken per counter atomic while many remain

struct SpaMisc {
    unsigned long long shot;
    int32_t count;  // unsatisfied checks of the current hard decision
    int32_t nonzero;
};

typedef __attribute__((address_space(3))) float spa_lds_float;

// the slot's messages start at LDS address 0 (the kernel declares no static
// LDS), so a byte offset is an LDS address
__device__ __forceinline__ float xld(uint32_t off) { return *reinterpret_cast<const spa_lds_float*>((size_t)off); }
__device__ __forceinline__ void xst(uint32_t off, float v) { *reinterpret_cast<spa_lds_float*>((size_t)off) = v; }

__device__ __forceinline__ int spa_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// phi(x) = -ln tanh(x / 2) = log1p(2 / expm1(x)) for x >= 0, from the
// hardware exp2, log2 and reciprocal and two short series, about 25
// instructions instead of the ~150 of the math library's expm1f and log1pf:
//   e = expm1(x): Taylor polynomial through x^7/7! for x < 1/4 (truncation
//       below 1e-8 relative), else exp2(x log2 e) - 1;
//   y = 2 / e;
//   log1p(y): series through y^6/6 for y < 1/32 (x > 4.17), else
//       log2(1 + y) ln 2.
// Relative error at most 2e-6 for x <= 20 and 4e-6 up to x = 60 (where phi
// is below 1e-25), measured against a double-precision phi with the hardware
// operations rounded once.  phi(0) = +inf and phi(+inf) = 0 as before.
__device__ __forceinline__ float phi(float x) {
    float e;
    if (x < 0.25f) {
        float p = 1.0f / 5040.0f;
        p = __builtin_fmaf(p, x, 1.0f / 720.0f);
        p = __builtin_fmaf(p, x, 1.0f / 120.0f);
        p = __builtin_fmaf(p, x, 1.0f / 24.0f);
        p = __builtin_fmaf(p, x, 1.0f / 6.0f);
        p = __builtin_fmaf(p, x, 0.5f);
        p = __builtin_fmaf(p, x, 1.0f);
        e = p * x;
    } else {
        e = __builtin_amdgcn_exp2f(x * 1.44269504088896341f) - 1.0f;
    }
    const float y = 2.0f * __builtin_amdgcn_rcpf(e);
    if (y < 0.03125f) {
        float q = -1.0f / 6.0f;
        q = __builtin_fmaf(q, y, 0.2f);
        q = __builtin_fmaf(q, y, -0.25f);
        q = __builtin_fmaf(q, y, 1.0f / 3.0f);
        q = __builtin_fmaf(q, y, -0.5f);
        q = __builtin_fmaf(q, y, 1.0f);
        return q * y;
    }
    return __builtin_amdgcn_logf(1.0f + y) * 0.693147180559945309f;
}

__device__ __forceinline__ float clip(float x, float c) { return fminf(fmaxf(x, -c), c); }

// One check row with D stored edge slots: every outgoing message is the sign
// product times phi of the exclusive sum of phi(|nu|), the sum taken over the
// row's other edges in ascending order.  Padding reads +inf (phi -> 0, sign +)
// and writes to the write-only cell.
template <int D, bool MIXED>
__device__ __forceinline__ void spa_row(const int32_t* rp, const int32_t* wp) {
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
    float a[D];
    bool neg[D];
    bool sgn = false;
#pragma unroll
    for (int p = 0; p < D; ++p) {
        const float nu = xld(pos[p]);
        neg[p] = nu < 0.0f;
        sgn ^= neg[p];
        a[p] = phi(fabsf(nu));
    }
#pragma unroll
    for (int p = 0; p < D; ++p) {
        float s = 0.0f;
#pragma unroll
        for (int f = 0; f < D; ++f)
            if (f != p) s = __fadd_rn(s, a[f]);
        const float m = phi(s);
        xst(wpos[p], (sgn ^ neg[p]) ? -m : m);
    }
}

template <int D>
__device__ __forceinline__ void spa_row_d(const int32_t* rp, const int32_t* wp, int lane, int stride, bool mixed) {
    const uint32_t o = (uint32_t)(lane * stride);
    if (mixed)
        spa_row<D, true>(rp + o, wp + o);
    else
        spa_row<D, false>(rp + o, wp + o);
}

// stored row degrees: 2..12 exactly, larger rows padded to 16, 24 or 32 slots
// (compiled only into the RD = 32 kernel, so that codes with light rows keep a
// small register budget)
template <int RD>
__device__ __forceinline__ void spa_row_dispatch(const int32_t* rp, const int32_t* wp, int lane, int dg, int stride,
                                                 bool mixed) {
    switch (dg) {
#define RBP_SPA_ROW(D) \
    case D: spa_row_d<D>(rp, wp, lane, stride, mixed); break;
        RBP_SPA_ROW(2) RBP_SPA_ROW(3) RBP_SPA_ROW(4) RBP_SPA_ROW(5) RBP_SPA_ROW(6) RBP_SPA_ROW(7)
        RBP_SPA_ROW(8) RBP_SPA_ROW(9) RBP_SPA_ROW(10) RBP_SPA_ROW(11) RBP_SPA_ROW(12)
        default:
            if constexpr (RD > 12) {
                switch (dg) {
                    RBP_SPA_ROW(16) RBP_SPA_ROW(24) RBP_SPA_ROW(32)
                    default: break;
                }
            }
            break;
#undef RBP_SPA_ROW
    }
}

// One variable with D edge slots (byte offsets sb + 256 q): M = L + sum_q mu_q
// (checks ascending), nu_q = clip(M - mu_q).  In a mixed group only the
// member's own vd edges take part.
template <int D, bool MIXED>
__device__ __forceinline__ float spa_var(uint32_t sb, int vd, float acc, float c) {
    float mu[D];
#pragma unroll
    for (int q = 0; q < D; ++q) mu[q] = xld(sb + 256u * q);
#pragma unroll
    for (int q = 0; q < D; ++q) acc = (!MIXED || q < vd) ? __fadd_rn(acc, mu[q]) : acc;
#pragma unroll
    for (int q = 0; q < D; ++q)
        if (!MIXED || q < vd) xst(sb + 256u * q, clip(__fsub_rn(acc, mu[q]), c));
    return acc;
}

__device__ __forceinline__ float spa_var_rolled(uint32_t sb, int vd, float acc, float c) {
    for (int q = 0; q < vd; ++q) acc = __fadd_rn(acc, xld(sb + 256u * q));
    for (int q = 0; q < vd; ++q) {
        const uint32_t o = sb + 256u * q;
        xst(o, clip(__fsub_rn(acc, xld(o)), c));
    }
    return acc;
}

__device__ __forceinline__ float spa_var_dispatch(uint32_t sb, int dg, bool mixed, int vd, float acc, float c) {
    switch (dg) {
        case 0: return acc;
#define RBP_SPA_VAR(D) \
    case D: return mixed ? spa_var<D, true>(sb, vd, acc, c) : spa_var<D, false>(sb, vd, acc, c);
        RBP_SPA_VAR(1) RBP_SPA_VAR(2) RBP_SPA_VAR(3) RBP_SPA_VAR(4) RBP_SPA_VAR(5) RBP_SPA_VAR(6)
        RBP_SPA_VAR(7) RBP_SPA_VAR(8)
#undef RBP_SPA_VAR
        default: return spa_var_rolled(sb, vd, acc, c);
    }
}

// a flipped hard decision toggles the parity bits of the variable's checks
__device__ __forceinline__ void spa_flip(const int32_t* scheck, uint32_t sb, int vd, uint32_t* par, int& dcount) {
    for (int q = 0; q < vd; ++q) {
        const int i = scheck[(sb >> 2) + 64u * q];
        const uint32_t bit = 1u << (i & 31);
        const uint32_t old = atomicXor(par + (i >> 5), bit);
        dcount += (old & bit) ? -1 : 1;
    }
}

template <int RD>
__global__ void __launch_bounds__(1024) spa_kernel(const SpaLaunch a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63;
    const int wid = spa_uniform(tid >> 6), nw = nth >> 6;
    float* Lp = reinterpret_cast<float*>(smem + a.off_L);
    float* Mg = reinterpret_cast<float*>(smem + a.off_M);
    uint32_t* par = reinterpret_cast<uint32_t*>(smem + a.off_par);
    uint32_t* dec = reinterpret_cast<uint32_t*>(smem + a.off_dec);
    uint32_t* outw = reinterpret_cast<uint32_t*>(smem + a.off_out);
    SpaMisc* ms = reinterpret_cast<SpaMisc*>(smem + a.off_misc);
    const float c = a.llr_max;
    unsigned long long n_block = 0, n_undetected = 0, n_nonconv = 0;  // kept by thread 0
    // Frames come from the device counter in runs of kSpaRun (one atomic per
    // run) while many remain, one at a time near the end: at high E_b/N_0 a
    // frame takes about two iterations and one atomic per frame would bound
    // the rate.
    unsigned long long run_next = 0, run_end = 0, last_ticket = 0;

    for (;;) {
        if (tid == 0) {
            if (run_next == run_end) {
                const unsigned long long k =
                    last_ticket + 8ull * kSpaRun * gridDim.x < a.shots ? (unsigned long long)kSpaRun : 1ull;
                run_next = atomicAdd(a.queue, k);
                run_end = run_next + k;
                last_ticket = run_next;
            }
            ms->shot = run_next++;
            ms->count = 0;
            ms->nonzero = 0;
        }
        if (tid == 0) xst(4u * (uint32_t)a.S, INFINITY);
        for (int w = tid; w < a.WM; w += nth) par[w] = 0u;
        for (int w = tid; w < a.WN; w += nth) outw[w] = 0u;
        __syncthreads();
        const unsigned long long s =
            ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(ms->shot >> 32)) << 32) |
            __builtin_amdgcn_readfirstlane((uint32_t)ms->shot);
        if (s >= a.shots) break;
        const uint64_t t_start = wall_clock64();
        const float* llr = a.llr + s * (uint64_t)a.N;

        // nu(0) = L on every edge; the parity of the channel's hard decision
        {
            int dc = 0;
            for (int pp = tid; pp < a.Np; pp += nth) {
                const int j = a.vord[pp];
                const int vd = a.vdeg[pp];
                const float l = j >= 0 ? clip(llr[j], c) : 0.0f;
                Lp[pp] = l;
                Mg[pp] = l;
                const uint32_t sb = 4u * ((uint32_t)a.vgrp[pp >> 6].x + (uint32_t)(pp & 63));
                for (int q = 0; q < vd; ++q) xst(sb + 256u * q, l);
                if (l < 0.0f) spa_flip(a.scheck, sb, vd, par, dc);
            }
            if (dc) atomicAdd(&ms->count, dc);
        }
        __syncthreads();

        bool conv = false;
        int iters = 0;
        for (int t = 1; t <= a.T; ++t) {
            // ---- check sweep: one row group per wave at a time
            for (int g = wid; g < a.GR; g += nw) {
                const int4 gi = a.rgrp[g];
                const uint32_t off = (uint32_t)spa_uniform(gi.x);
                spa_row_dispatch<RD>(a.rposp + off, a.rposw + off, lane, spa_uniform(gi.y), spa_uniform(gi.w),
                                 spa_uniform(gi.z) != 0);
            }
            __syncthreads();
            // ---- variable sweep: one variable group per wave at a time
            int dcount = 0;
            for (int g = wid; g < a.GV; g += nw) {
                const int4 gi = a.vgrp[g];
                const int dg = spa_uniform(gi.y);
                const bool mixed = spa_uniform(gi.z) != 0;
                const int pp = g * 64 + lane;
                const int vd = mixed ? a.vdeg[pp] : dg;
                const float mo = Mg[pp];
                const uint32_t sb = 4u * ((uint32_t)spa_uniform(gi.x) + (uint32_t)lane);
                const float acc = spa_var_dispatch(sb, dg, mixed, vd, Lp[pp], c);
                Mg[pp] = acc;
                if ((acc < 0.0f) != (mo < 0.0f)) spa_flip(a.scheck, sb, vd, par, dcount);
            }
            if (dcount) atomicAdd(&ms->count, dcount);
            __syncthreads();
            iters = t;
            // every thread reads the count before the next sweep's atomics (a
            // barrier follows the next check sweep)
            conv = ms->count == 0;
            if (conv && a.stop) break;
        }

        // hard decision by position -> variable order (the few set bits are scattered)
        for (int g = wid; g < a.GV; g += nw) {
            const unsigned long long b = __ballot(Mg[g * 64 + lane] < 0.0f);
            if (lane == 0) {
                dec[2 * g] = (uint32_t)b;
                dec[2 * g + 1] = (uint32_t)(b >> 32);
            }
        }
        __syncthreads();
        for (int g = wid; g < a.GV; g += nw) {
            if ((dec[2 * g + (lane >> 5)] >> (lane & 31)) & 1u) {
                const int j = a.vord[g * 64 + lane];
                atomicOr(outw + (j >> 5), 1u << (j & 31));
                ms->nonzero = 1;
            }
        }
        if (a.marg)
            for (int pp = tid; pp < a.Np; pp += nth) {
                const int j = a.vord[pp];
                if (j >= 0) a.marg[s * (uint64_t)a.N + j] = Mg[pp];
            }
        __syncthreads();
        for (int w = tid; w < a.WN; w += nth) a.bits[s * (uint64_t)a.WN + w] = outw[w];
        if (tid == 0) {
            const bool nz = ms->nonzero != 0;
            n_block += nz ? 1 : 0;
            n_undetected += (nz && conv) ? 1 : 0;
            n_nonconv += conv ? 0 : 1;
            if (a.stats) {
                rbp_shot_stats st;
                st.converged = conv ? 1 : 0;
                st.nconv = conv ? 1 : 0;
                st.path = nz ? 1 : 0;
                st.reserved = 0;
                st.legs = 1;
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
    if (tid == 0 && a.counts) {
        if (n_block) atomicAdd(a.counts, n_block);
        if (n_undetected) atomicAdd(a.counts + 1, n_undetected);
        if (n_nonconv) atomicAdd(a.counts + 2, n_nonconv);
    }
}

__global__ void spa_zero_kernel(unsigned long long* p) {
    if (threadIdx.x == 0) *p = 0ull;
}

static constexpr int kSpaMaxLds = 160 * 1024;
static int spa_align16(int64_t x) { return (int)((x + 15) & ~(int64_t)15); }

}  // namespace rbp

using namespace rbp;

extern "C" {

rbp_status rbp_sample_awgn(rbp_code_t c, uint64_t shots, double sigma, uint64_t seed, uint64_t shot_offset,
                           float* llr, void* stream_) {
    if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
    if (shots == 0) return RBP_OK;
    if (!llr) return fail(RBP_ERR_INVALID_ARG, "llr is NULL");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(RBP_ERR_INVALID_ARG, "sigma must be positive and finite");
    AwgnArgs a;
    a.N = c->N;
    a.Q = (c->N + 3) / 4;
    a.seed = seed;
    a.sigma = (float)sigma;
    a.scale = (float)(2.0 / (sigma * sigma));
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    const uint64_t max_threads = (uint64_t)256 * (1u << 30);
    const uint64_t per_launch = std::max<uint64_t>(max_threads / (uint64_t)a.Q, 1);
    for (uint64_t done = 0; done < shots;) {
        const uint64_t n = std::min<uint64_t>(shots - done, per_launch);
        a.shots = n;
        a.offset = shot_offset + done;
        a.llr = llr + done * (uint64_t)a.N;
        const uint64_t threads = n * (uint64_t)a.Q;
        hipLaunchKernelGGL(awgn_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, stream, a);
        RBP_HIP_CHECK(hipGetLastError());
        done += n;
    }
    return RBP_OK;
}

rbp_status rbp_decode_spa(rbp_code_t c, const float* llr, uint64_t shots, const rbp_spa_params* p, uint32_t* bits,
                          float* marg, rbp_shot_stats* stats, unsigned long long* counts, void* stream_) {
    if (!c || !p) return fail(RBP_ERR_INVALID_ARG, "code or params is NULL");
    if (shots == 0) return RBP_OK;
    if (!llr || !bits) return fail(RBP_ERR_INVALID_ARG, "llr or bits is NULL");
    if (p->max_iterations < 1) return fail(RBP_ERR_INVALID_ARG, "max_iterations must be >= 1");
    if (!(p->llr_max > 0.0f) || !std::isfinite(p->llr_max)) return fail(RBP_ERR_INVALID_ARG, "llr_max must be > 0");
    if (p->waves_per_shot < 0 || p->waves_per_shot > 16) return fail(RBP_ERR_INVALID_ARG, "waves_per_shot in 0..16");
    if (p->stop != 0 && p->stop != 1) return fail(RBP_ERR_INVALID_ARG, "stop is 0 or 1");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    RBP_HIP_CHECK(hipSetDevice(c->device));
    SpaLaunch a;
    a.N = c->N;
    a.WN = (c->N + 31) / 32;
    a.WM = (c->M + 31) / 32;
    a.S = c->S;
    a.GR = c->GR;
    a.GV = c->GV;
    a.Np = c->Np;
    a.rgrp = c->rgrp.as<int4>();
    a.rposp = c->rposp.as<int32_t>();
    a.rposw = c->rposw.as<int32_t>();
    a.vgrp = c->vgrp.as<int4>();
    a.vord = c->vord.as<int32_t>();
    a.vdeg = c->vdeg.as<int32_t>();
    a.scheck = c->scheck.as<int32_t>();
    a.llr = llr;
    a.shots = shots;
    a.T = p->max_iterations;
    a.stop = p->stop;
    a.llr_max = p->llr_max;
    a.bits = bits;
    a.marg = marg;
    a.stats = stats;
    a.counts = counts;
    // LDS: messages (S slots + the +inf cell + the write-only cell) at 0, then
    // L and M by position, parity words, decision bits, output words, scalars
    int64_t off = spa_align16(4 * ((int64_t)c->S + 2));
    a.off_L = (int)off;
    off += spa_align16(4 * (int64_t)c->Np);
    a.off_M = (int)off;
    off += spa_align16(4 * (int64_t)c->Np);
    a.off_par = (int)off;
    off += spa_align16(4 * (int64_t)a.WM);
    a.off_dec = (int)off;
    off += spa_align16(4 * (int64_t)(c->Np / 32));
    a.off_out = (int)off;
    off += spa_align16(4 * (int64_t)a.WN);
    a.off_misc = (int)off;
    off += spa_align16(sizeof(SpaMisc));
    if (off > kSpaMaxLds) return fail(RBP_ERR_UNSUPPORTED, "sum-product state does not fit in LDS");
    const int lds = (int)off;
    int waves = p->waves_per_shot;
    if (waves == 0) {
        // one wave per 3 groups of the larger sweep, at most 4: the sweeps are
        // ALU-bound (two phi evaluations per edge), so more shots per CU beat
        // more waves per shot (measured on the [64,32] and [310,155] codes)
        const int groups = std::max(c->GR, c->GV);
        waves = std::min(4, std::max(1, (groups + 2) / 3));
    }
    if (c->max_stored_row_deg > 32)
        return fail(RBP_ERR_UNSUPPORTED, "the sum-product decoder takes rows of at most 32 edges");
    void (*kern)(SpaLaunch) = c->max_stored_row_deg <= 12 ? spa_kernel<12> : spa_kernel<32>;
    RBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      lds));
    int per_cu = 0;
    RBP_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                                64 * waves, lds));
    per_cu = std::max(per_cu, 1);
    const uint64_t slots = std::min<uint64_t>((uint64_t)per_cu * (uint64_t)std::max(c->num_cus, 1), shots);
    rbp_status st = c->spa_queue.reserve(64);
    if (st) return st;
    a.queue = c->spa_queue.as<unsigned long long>();
    hipLaunchKernelGGL(spa_zero_kernel, dim3(1), dim3(64), 0, stream, a.queue);
    RBP_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(kern, dim3((unsigned)slots), dim3(64 * waves), lds, stream, a);
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

}  // extern "C"
