// librbp: bookkeeping kernels of sliding-window decoding (gfx950).
//
// A window decodes the syndrome of a run of consecutive rounds with the
// Relay-BP decoder and commits the mechanisms that start in its first rounds
// (the paper's sliding-window decoding with a commit region, Sec. 6.1 latency
// discussion).  Between window decodes two small kernels move bits:
//
//  * bits_extract_kernel   one thread per (shot, output word): the window's
//                          syndrome rows are a contiguous bit range of the
//                          round-major syndrome, shifted to bit 0.
//  * window_commit_kernel  one thread per shot: for each committed set bit of
//                          the window's correction (a few per shot), set the
//                          mechanism in the full correction and XOR its column
//                          of H and of O (CSC on the device) into the running
//                          syndrome and the predicted observables.
//  * bits_gather_kernel    one thread per (shot, output word): bit t of the
//                          output is bit rows[t] of the source (windows whose
//                          rows are not one contiguous range, and the rows that
//                          fix single columns in parallel-window decoding).
//  * residual_kernel       one thread per shot: a shot whose running syndrome
//                          is not zero after every window is not converged.
#include <algorithm>
#include <string>

#include "rbp_common.h"

namespace rbp {

__global__ void __launch_bounds__(256) bits_extract_kernel(const uint32_t* src, int32_t sw, uint64_t shots,
                                                            int64_t off, int32_t nbits, uint32_t* dst, int32_t dw) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t s = t / (uint64_t)dw;
    if (s >= shots) return;
    const int w = (int)(t - s * (uint64_t)dw);
    const int64_t b0 = off + 32 * (int64_t)w;
    const int64_t q = b0 >> 5;
    const int r = (int)(b0 & 31);
    const uint32_t* row = src + s * (uint64_t)sw;
    const uint32_t lo = q < sw ? row[q] : 0u;
    const uint32_t hi = (r != 0 && q + 1 < sw) ? row[q + 1] : 0u;
    uint32_t v = r ? (lo >> r) | (hi << (32 - r)) : lo;
    const int rem = nbits - 32 * w;
    if (rem < 32) v &= rem > 0 ? ((1u << rem) - 1u) : 0u;
    dst[s * (uint64_t)dw + w] = v;
}

__global__ void __launch_bounds__(256) bits_gather_kernel(const uint32_t* src, int32_t sw, uint64_t shots,
                                                           const int32_t* rows, int32_t n, uint32_t* dst, int32_t dw) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t s = t / (uint64_t)dw;
    if (s >= shots) return;
    const int w = (int)(t - s * (uint64_t)dw);
    const uint32_t* row = src + s * (uint64_t)sw;
    uint32_t v = 0u;
    const int b0 = 32 * w, b1 = n < b0 + 32 ? n : b0 + 32;
    const int nb = 32 * sw;
    for (int b = b0; b < b1; ++b) {
        const int i = rows[b];
        if (i >= 0 && i < nb) v |= ((row[i >> 5] >> (i & 31)) & 1u) << (b - b0);
    }
    dst[s * (uint64_t)dw + w] = v;
}

__global__ void __launch_bounds__(256) residual_kernel(const uint32_t* syn, int32_t sw, uint64_t shots,
                                                        rbp_shot_stats* acc) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= shots) return;
    uint32_t any = 0u;
    for (int w = 0; w < sw; ++w) any |= syn[s * (uint64_t)sw + w];
    if (any) acc[s].converged = 0;
}

struct CommitArgs {
    uint64_t shots;
    const uint32_t* win_corr;
    int32_t ww, n_win;
    const int32_t* cmap;
    int32_t N, WM, WN, WK;
    const int32_t* col_ptr;
    const int32_t* csc_row;
    const int32_t* ocol_ptr;
    const int32_t* orow_idx;
    uint32_t* syn;
    uint32_t* obs;
    uint32_t* corr;
    const rbp_shot_stats* win_stats;
    rbp_shot_stats* acc;
    int32_t first;
};

__global__ void __launch_bounds__(256) window_commit_kernel(const CommitArgs a) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.shots) return;
    const uint32_t* e = a.win_corr + s * (uint64_t)a.ww;
    uint32_t* syn = a.syn + s * (uint64_t)a.WM;
    uint32_t* corr = a.corr + s * (uint64_t)a.WN;
    uint32_t* obs = a.obs ? a.obs + s * (uint64_t)a.WK : nullptr;
    for (int w = 0; w < a.ww; ++w) {
        uint32_t b = e[w];
        while (b) {
            const int j = 32 * w + __builtin_ctz(b);
            b &= b - 1u;
            if (j >= a.n_win) break;
            const int J = a.cmap[j];
            if (J < 0 || J >= a.N) continue;
            corr[J >> 5] |= 1u << (J & 31);
            for (int k = a.col_ptr[J]; k < a.col_ptr[J + 1]; ++k) {
                const int i = a.csc_row[k];
                syn[i >> 5] ^= 1u << (i & 31);
            }
            if (obs)
                for (int k = a.ocol_ptr[J]; k < a.ocol_ptr[J + 1]; ++k) {
                    const int r = a.orow_idx[k];
                    obs[r >> 5] ^= 1u << (r & 31);
                }
        }
    }
    if (a.acc && a.win_stats) {
        const rbp_shot_stats w = a.win_stats[s];
        if (a.first) {
            a.acc[s] = w;
        } else {
            rbp_shot_stats t = a.acc[s];
            t.converged = (t.converged && w.converged) ? 1 : 0;
            t.nconv = w.nconv < t.nconv ? w.nconv : t.nconv;
            const uint32_t legs = (uint32_t)t.legs + w.legs;
            t.legs = (uint16_t)(legs > 65535u ? 65535u : legs);
            t.iters += w.iters;
            t.t_end = w.t_end;
            a.acc[s] = t;
        }
    }
}

}  // namespace rbp

using namespace rbp;

extern "C" {

rbp_status rbp_bits_extract(const uint32_t* src, int32_t src_words, uint64_t shots, int64_t bit_offset, int32_t nbits,
                            uint32_t* dst, int32_t dst_words, void* stream_) {
    if (shots == 0) return RBP_OK;
    if (!src || !dst) return fail(RBP_ERR_INVALID_ARG, "src or dst is NULL");
    if (src_words < 1 || dst_words < 1 || nbits < 0 || bit_offset < 0)
        return fail(RBP_ERR_INVALID_ARG, "word counts must be >= 1, nbits and bit_offset >= 0");
    if ((int64_t)nbits > 32 * (int64_t)dst_words) return fail(RBP_ERR_SHAPE, "nbits exceeds the destination");
    if (bit_offset + nbits > 32 * (int64_t)src_words) return fail(RBP_ERR_SHAPE, "bit range exceeds the source");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    const uint64_t threads = shots * (uint64_t)dst_words;
    const uint64_t max_blocks = 1ull << 31;
    if ((threads + 255) / 256 > max_blocks) return fail(RBP_ERR_UNSUPPORTED, "too many shots for one launch");
    hipLaunchKernelGGL(bits_extract_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, stream, src,
                       src_words, shots, bit_offset, nbits, dst, dst_words);
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

rbp_status rbp_bits_gather(const uint32_t* src, int32_t src_words, uint64_t shots, const int32_t* rows_dev,
                           int32_t nrows, uint32_t* dst, int32_t dst_words, void* stream_) {
    if (shots == 0) return RBP_OK;
    if (!src || !dst || (nrows > 0 && !rows_dev)) return fail(RBP_ERR_INVALID_ARG, "src, dst or rows is NULL");
    if (src_words < 1 || dst_words < 1 || nrows < 0) return fail(RBP_ERR_INVALID_ARG, "bad word or row counts");
    if ((int64_t)nrows > 32 * (int64_t)dst_words) return fail(RBP_ERR_SHAPE, "nrows exceeds the destination");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    const uint64_t threads = shots * (uint64_t)dst_words;
    if ((threads + 255) / 256 > (1ull << 31)) return fail(RBP_ERR_UNSUPPORTED, "too many shots for one launch");
    hipLaunchKernelGGL(bits_gather_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, stream, src,
                       src_words, shots, rows_dev, nrows, dst, dst_words);
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

rbp_status rbp_window_residual(const uint32_t* syn, int32_t words, uint64_t shots, rbp_shot_stats* acc,
                               void* stream_) {
    if (shots == 0) return RBP_OK;
    if (!syn || !acc) return fail(RBP_ERR_INVALID_ARG, "syn or acc is NULL");
    if (words < 1) return fail(RBP_ERR_INVALID_ARG, "words must be >= 1");
    if ((shots + 255) / 256 > (1ull << 31)) return fail(RBP_ERR_UNSUPPORTED, "too many shots for one launch");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)((shots + 255) / 256)), dim3(256), 0, stream, syn, words, shots,
                       acc);
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

rbp_status rbp_window_commit(rbp_code_t c, uint64_t shots, const uint32_t* win_corr, int32_t win_words,
                             const int32_t* cmap, int32_t n_win, uint32_t* syn, uint32_t* obs, uint32_t* corr,
                             const rbp_shot_stats* win_stats, rbp_shot_stats* acc, int32_t first, void* stream_) {
    if (!c) return fail(RBP_ERR_INVALID_ARG, "code is NULL");
    if (shots == 0) return RBP_OK;
    if (!win_corr || !cmap || !syn || !corr) return fail(RBP_ERR_INVALID_ARG, "a required array is NULL");
    if (c->k > 0 && !obs) return fail(RBP_ERR_INVALID_ARG, "obs_pred is NULL");
    if (win_words < 1 || n_win < 0 || (int64_t)n_win > 32 * (int64_t)win_words)
        return fail(RBP_ERR_SHAPE, "n_win must fit in win_words words");
    if (acc && !win_stats) return fail(RBP_ERR_INVALID_ARG, "acc_stats needs win_stats");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    CommitArgs a;
    a.shots = shots;
    a.win_corr = win_corr;
    a.ww = win_words;
    a.n_win = n_win;
    a.cmap = cmap;
    a.N = c->N;
    a.WM = (c->M + 31) / 32;
    a.WN = (c->N + 31) / 32;
    a.WK = std::max((c->k + 31) / 32, 1);
    a.col_ptr = c->col_ptr.as<int32_t>();
    a.csc_row = c->csc_row.as<int32_t>();
    a.ocol_ptr = c->ocol_ptr.as<int32_t>();
    a.orow_idx = c->orow_idx.as<int32_t>();
    a.syn = syn;
    a.obs = c->k > 0 ? obs : nullptr;
    a.corr = corr;
    a.win_stats = win_stats;
    a.acc = acc;
    a.first = first;
    if ((shots + 255) / 256 > (1ull << 31)) return fail(RBP_ERR_UNSUPPORTED, "too many shots for one launch");
    hipLaunchKernelGGL(window_commit_kernel, dim3((unsigned)((shots + 255) / 256)), dim3(256), 0, stream, a);
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

}  // extern "C"
