// Shared host/device helpers of librbp (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rbp.h"

namespace rbp {

// ---------------------------------------------------------------------------
// Errors: status code + thread-local message.
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
rbp_status fail(rbp_status st, const std::string& msg);

#define RBP_HIP_CHECK(expr)                                                              \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::rbp::fail(RBP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Device buffer owned by a handle; grows on demand, never shrinks.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    rbp_status reserve(size_t n);
    void release();
    template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__host__ __device__ inline uint32_t u4_get(const U4& v, int w) {
    return w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
}

// ---------------------------------------------------------------------------
// Detector error model handle.
// ---------------------------------------------------------------------------
struct LaunchCfg {
    int waves_per_shot = 0;
    int state = 0;
    int max_slots = 0;
    int shots_per_wg = 0;  // 0 or 1: one shot per workgroup; 2 or 4: the multi-shot kernel
};

// largest row degree of H the decoder accepts (rows above 32 edges take the
// rolled check update)
constexpr int kMaxRowDeg = 1024;

}  // namespace rbp

struct rbp_code {
    int32_t M = 0, N = 0, E = 0, k = 0, nnzO = 0;
    int32_t max_row_deg = 0, max_col_deg = 0;
    int device = 0;
    int num_cus = 0;
    // wave-group layout of the decoder (64 rows or variables per group)
    int32_t S = 0;                      // edge slots (>= E)
    int32_t GR = 0, GV = 0, Np = 0;     // row groups, variable groups, 64 GV
    int32_t GRw = 0;                    // leading row groups stored with more than 32 edges
    int32_t RB = 0;                     // length of the row position table
    int32_t max_stored_row_deg = 0;     // largest stored row degree (<= 12, 16, 24, 32, then multiples of 8)
    std::vector<int32_t> h_vord;        // host copy of vord
    // device copies
    rbp::DevBuf row_ptr, col_idx;       // CSR of H: row_ptr[M+1], col_idx[E]
    rbp::DevBuf col_ptr, csc_row;       // CSC of H: col_ptr[N+1], csc_row[E]
    rbp::DevBuf rgrp, rposp, rposw;     // row groups {offset, degree, mixed, 0}; slot byte offsets (read, write)
    rbp::DevBuf rord;                   // check at each row position
    rbp::DevBuf vgrp, vord, vdeg;       // variable groups {first slot, degree, mixed, 0}, order, degrees
    rbp::DevBuf vinv;                   // position of each variable
    rbp::DevBuf scheck, scsc;           // check and CSC edge of each slot
    rbp::DevBuf orow_ptr, ocol_idx;     // CSR of O: orow_ptr[k+1], ocol_idx[nnzO]
    rbp::DevBuf ocol_ptr, orow_idx;     // CSC of O (sampler)
    // per-call data (cached by content)
    rbp::DevBuf thr;                    // uint32[N] sampler acceptance thresholds A_j
    rbp::DevBuf gapt;                   // uint32[ceil(N/64)] sampler gap thresholds T_k
    std::vector<double> thr_key;
    rbp::DevBuf lam, lamp;              // float LLRs by variable [N] and by position [Np]
    rbp::DevBuf m1;                     // float[RB] first-iteration message magnitudes (layout of rposp)
    std::vector<double> lam_key;
    rbp::DevBuf gtab;                   // float[max(R,1)][Np] relay-leg memory strengths by position
    rbp::DevBuf lg;                     // float2[R+1][Np] {Lambda, gamma} by leg and position
    uint64_t lam_gen = 0, gtab_gen = 0; // bumped when lam / gtab are rewritten
    uint64_t lg_lam_gen = ~0ull, lg_gtab_gen = ~0ull;
    float lg_gamma0 = 0.f;
    int32_t lg_R = -1;
    uint64_t gtab_seed = 0;
    float gtab_lo = 0.f, gtab_hi = 0.f;
    int32_t gtab_R = -1;
    rbp::DevBuf queue;                  // work counter of the persistent decoder
    rbp::DevBuf order, ohist;           // shot order of rbp_decode (heaviest syndrome first) and its histogram
    rbp::DevBuf coop;                   // rbp_decode_coop: parity, best solution, barrier words
    rbp::DevBuf spa_queue;              // work counter of the sum-product decoder
    rbp::DevBuf gstate;                 // per-slot state when it does not fit in LDS
    rbp::DevBuf trace_hit;
    // compact row-record state (rows of at most 16 edges)
    bool compact_ok = false;
    int32_t coff_M = 0;                 // LDS offset of the marginals: 16 * 64 GR + 16
    rbp::DevBuf cvar;                   // int32, layout of rposp: LDS address of each row edge's marginal
    rbp::DevBuf vrec;                   // uint32[S]: 16 * row position + edge code in the row, per edge slot
    rbp::DevBuf r1rec;                  // uint4[64 GR]: first-iteration records of a plain leg (per priors)
    int32_t residents = 0;              // resident decoders running on this handle
    int32_t coop_phantom = 0;           // test hook: extra barrier arrivals that never come
    rbp::LaunchCfg cfg;
};
