// Learned proposal network of librbp: a 3-layer perceptron trained and run with
// hand-written BF16 MFMA kernels for gfx950 (FP32 accumulation, FP32 master
// weights, Adam).
//
//   x = syndrome bits (0/1)            [B x in]
//   h1 = relu(W1 x + b1)               [B x hid]   (BF16)
//   h2 = relu(W2 h1 + b2)              [B x hid]   (BF16)
//   delta = W3 h2 + b3                 [B x out]   (FP32)  log-prior adjustment
//   loss = mean_b sum_j BCEWithLogits(z_bj, y_bj), z = -(Lambda + delta),
//          y = correction bits of Relay-BP (the network learns posterior
//          log-odds of each mechanism; delta is the correction to the prior).
//
// All products are one tiled GEMM kernel: C[MxN] = opA(A)[MxK] . opB(B)[KxN]
// with a 128x128 output tile per workgroup of 4 wavefronts, each computing a
// 64x64 block with v_mfma_f32_32x32x16_bf16, operands staged through two LDS
// buffers in a K-contiguous layout (operands stored M- or N-contiguous are
// transposed while staging; the next K step's tiles are loaded while the
// current ones are multiplied).  Tiles are numbered so that each XCD works on
// a contiguous run of row blocks.  Epilogues fuse the bias, ReLU, the ReLU
// mask of the backward pass and the BF16/FP32 stores.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rbp_common.h"

namespace rbp {
namespace mlp {

#ifdef RBP_MLP_FP32
// Test build: weights, activations and gradients kept in FP32 and the products
// run on the FP32 matrix cores (v_mfma_f32_32x32x2_f32), with the same tiling,
// staging, epilogues and reductions; its gradients are compared with the
// float64 reference at 1e-5.
typedef float elem;
typedef float elemx8 __attribute__((ext_vector_type(8)));
#else
typedef __bf16 elem;
typedef __bf16 elemx8 __attribute__((ext_vector_type(8)));
#endif
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = 128, BK = 32;
// Register budget: the 64 x 64 wave tile is built for 4 waves per SIMD (128
// VGPRs, accumulators included), which fits the 4 workgroups per CU that the
// LDS stages allow; the wider tile for 2.
#ifdef RBP_MLP_FP32
constexpr int kMinWaves64 = 2, kMinWaves128 = 1;  // FP32 operands: twice the registers and LDS
#else
constexpr int kMinWaves64 = 4, kMinWaves128 = 2;
#endif
constexpr int kFwdTN = 2;  // MFMA column blocks per wave in the forward products
constexpr int LDSK = BK + 8;  // padded row of the staged tiles (bank spread)

enum Layout { K_CONTIG = 0, MN_CONTIG = 1, BITS = 2 };  // BITS: A is packed 0/1 bits, 32 per word, rows of lda words
enum Epi {
    EPI_BIAS_RELU_BF16 = 0,  // out_bf16 = elem(relu(acc + bias[n]))
    EPI_BIAS_F32 = 1,        // out_f32 = acc + bias[n]
    EPI_MASK_BF16_F32 = 2,   // v = acc * [mask[m][n] > 0]; out_bf16 = elem(v), out_f32 = v
    EPI_F32 = 3,             // out_f32 = acc
    EPI_BIAS_BF16 = 4,       // out_bf16 = elem(acc + bias[n]) (round to nearest even)
};

struct GemmArgs {
    int M, N, K;
    const elem* A;  // K_CONTIG: A[m*lda + k]; MN_CONTIG: A[k*lda + m]
    int lda;
    const elem* B;  // K_CONTIG: B[n*ldb + k]; MN_CONTIG: B[k*ldb + n]
    int ldb;
    const float* bias;
    const elem* mask;  // [M x N] row-major, ld = ldc
    elem* out_bf16;
    float* out_f32;
    int ldc;
};

// A ROWS x BK tile of an operand in flight from device memory to LDS: each
// thread holds VPT vectors of 8 BF16 between the load (issued one K step
// ahead) and the store into tile[row][k].
template <int ROWS>
struct TileRegs {
    static constexpr int VPT = ROWS * BK / 8 / 256;
    static_assert(VPT * 256 * 8 == ROWS * BK, "tile shape");
    elemx8 x[VPT];
};

template <int LAYOUT, int ROWS>
__device__ __forceinline__ TileRegs<ROWS> load_tile(const elem* src, int ld, int rows, int K, int r0, int k0) {
    constexpr int VPT = TileRegs<ROWS>::VPT;
    const int t = threadIdx.x;
    TileRegs<ROWS> v;
    if constexpr (LAYOUT == BITS) {
        // rows x BK k as vectors of 8 bits, each inside one 32-bit word (k0 and
        // the vector offsets are multiples of 8): expanded to BF16 0/1 in registers
        const uint32_t* w = reinterpret_cast<const uint32_t*>(src);
#pragma unroll
        for (int pass = 0; pass < VPT; ++pass) {
            const int q = t + pass * 256;
            const int r = q / (BK / 8), kk = (q % (BK / 8)) * 8;
            const int gr = r0 + r, gk = k0 + kk;
            const uint32_t bits = gr < rows && gk < K ? (w[(int64_t)gr * ld + (gk >> 5)] >> (gk & 31)) : 0u;
#pragma unroll
            for (int i = 0; i < 8; ++i) v.x[pass][i] = ((bits >> i) & 1u) && gk + i < K ? (elem)1.0f : (elem)0.0f;
        }
        return v;
    }
    // 16-byte vector loads need a 16-byte aligned base and a leading dimension of 8k
    const bool vec = ((reinterpret_cast<uintptr_t>(src) & 15) == 0) && ((ld & 7) == 0);
#pragma unroll
    for (int pass = 0; pass < VPT; ++pass) {
        const int q = t + pass * 256;
        if constexpr (LAYOUT == K_CONTIG) {
            // rows x BK k as vectors of 8 k
            const int r = q / (BK / 8), kk = (q % (BK / 8)) * 8;
            const int gr = r0 + r, gk = k0 + kk;
            if (vec && gr < rows && gk + 7 < K) {
                v.x[pass] = *reinterpret_cast<const elemx8*>(src + (int64_t)gr * ld + gk);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    v.x[pass][i] = (gr < rows && gk + i < K) ? src[(int64_t)gr * ld + gk + i] : (elem)0.0f;
            }
        } else {
            // BK k x rows, rows contiguous in memory: vectors of 8 rows
            const int kk = q / (ROWS / 8), r = (q % (ROWS / 8)) * 8;
            const int gr = r0 + r, gk = k0 + kk;
            if (vec && gk < K && gr + 7 < rows) {
                v.x[pass] = *reinterpret_cast<const elemx8*>(src + (int64_t)gk * ld + gr);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    v.x[pass][i] = (gk < K && gr + i < rows) ? src[(int64_t)gk * ld + gr + i] : (elem)0.0f;
            }
        }
    }
    return v;
}

template <int LAYOUT, int ROWS>
__device__ __forceinline__ void store_tile(elem (*tile)[LDSK], const TileRegs<ROWS>& v) {
    constexpr int VPT = TileRegs<ROWS>::VPT;
    const int t = threadIdx.x;
#pragma unroll
    for (int pass = 0; pass < VPT; ++pass) {
        const int q = t + pass * 256;
        if constexpr (LAYOUT == K_CONTIG || LAYOUT == BITS) {
            const int r = q / (BK / 8), kk = (q % (BK / 8)) * 8;
            *reinterpret_cast<elemx8*>(&tile[r][kk]) = v.x[pass];
        } else {
            const int kk = q / (ROWS / 8), r = (q % (ROWS / 8)) * 8;
#pragma unroll
            for (int i = 0; i < 8; ++i) tile[r + i][kk] = v.x[pass][i];
        }
    }
}

// TN: 32-column MFMA blocks per wave, so a wave computes 64 x 32 TN and the
// workgroup (2 x 2 waves) a BM x 64 TN tile
template <int LA, int LB, int EPI, int TN>
__global__ void __launch_bounds__(256, TN == 2 ? kMinWaves64 : kMinWaves128) gemm_kernel(const GemmArgs g) {
    constexpr int BNT = 64 * TN;
    // two LDS stages: the tiles of step k are read by the matrix cores while
    // those of step k + 1 arrive in registers
    // the two operand stages in one buffer, which the BF16-only epilogues reuse
    // to stage the output tile
    __shared__ __align__(16) elem stage[2 * BM * LDSK + 2 * BNT * LDSK];
    elem(*As)[BM][LDSK] = reinterpret_cast<elem(*)[BM][LDSK]>(stage);
    elem(*Bs)[BNT][LDSK] = reinterpret_cast<elem(*)[BNT][LDSK]>(stage + 2 * BM * LDSK);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // Workgroups are dealt to the 8 XCDs round-robin.  Renumber them so that
    // each XCD takes a contiguous run of tiles in row-major order: the column
    // tiles of a row block then run on one XCD and share its L2 copy of the A
    // rows (the B operand, a weight matrix, fits every L2).
    const int tiles_n = (g.N + BNT - 1) / BNT, tiles = tiles_n * ((g.M + BM - 1) / BM);
    const int per_xcd = (tiles + 7) / 8;
    const int logical = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (logical >= tiles) return;
    const int m0 = (logical / tiles_n) * BM, n0 = (logical % tiles_n) * BNT;
    const int wm = (wid >> 1) * 64, wn = (wid & 1) * 32 * TN;  // this wave's 64 x 32 TN block
    f32x16 acc[2][TN];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x16{};

    {
        const TileRegs<BM> ra = load_tile<LA, BM>(g.A, g.lda, g.M, g.K, m0, 0);
        const TileRegs<BNT> rb = load_tile<LB, BNT>(g.B, g.ldb, g.N, g.K, n0, 0);
        store_tile<LA, BM>(As[0], ra);
        store_tile<LB, BNT>(Bs[0], rb);
    }
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < g.K; k0 += BK) {
        const bool more = k0 + BK < g.K;
        TileRegs<BM> ra;
        TileRegs<BNT> rb;
        if (more) {
            ra = load_tile<LA, BM>(g.A, g.lda, g.M, g.K, m0, k0 + BK);
            rb = load_tile<LB, BNT>(g.B, g.ldb, g.N, g.K, n0, k0 + BK);
        }
#ifdef RBP_MLP_FP32
#pragma unroll
        for (int ks = 0; ks < BK; ks += 2) {
            // lane: row (lane % 32) of a 32-row block, k = ks + lane / 32 (A and B alike)
            const int kk = ks + (lane >> 5);
            float af[2], bfr[TN];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = As[cur][wm + i * 32 + (lane & 31)][kk];
#pragma unroll
            for (int j = 0; j < TN; ++j) bfr[j] = Bs[cur][wn + j * 32 + (lane & 31)][kk];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
#else
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            // lane: row (lane % 32) of a 32-row block, 8 consecutive k from (lane / 32) * 8.
            // A and B use the same k order, so the product is independent of how the
            // matrix core pairs the k slots.
            const int kk = ks + (lane >> 5) * 8;
            elemx8 af[2], bfr[TN];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                af[i] = *reinterpret_cast<const elemx8*>(&As[cur][wm + i * 32 + (lane & 31)][kk]);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bfr[j] = *reinterpret_cast<const elemx8*>(&Bs[cur][wn + j * 32 + (lane & 31)][kk]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
#endif
        if (more) {
            // the other stage was last read before the previous barrier
            store_tile<LA, BM>(As[cur ^ 1], ra);
            store_tile<LB, BNT>(Bs[cur ^ 1], rb);
        }
        __syncthreads();
        cur ^= 1;
    }
    // 32x32 accumulator layout: register r of lane l is C[8*(r/4) + 4*(l/32) + r%4][l%32]
    if constexpr (EPI == EPI_BIAS_BF16 || EPI == EPI_BIAS_RELU_BF16) {
        // BF16-only outputs: the rounded tile is staged in LDS (the K loop ended
        // with a barrier, so the operand stages are free) and written with
        // 16-byte stores, eight consecutive columns per thread
        constexpr int CLD = BNT + 8;  // padded row of the staged tile
        static_assert(BM * CLD <= 2 * BM * LDSK + 2 * BNT * LDSK, "output tile fits the operand stages");
        elem* ct = stage;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int ml = wm + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    const int nl = wn + j * 32 + (lane & 31);
                    const int n = n0 + nl;
                    float v = acc[i][j][r] + (n < g.N ? g.bias[n] : 0.0f);
                    if constexpr (EPI == EPI_BIAS_RELU_BF16) v = fmaxf(v, 0.0f);
                    ct[ml * CLD + nl] = (elem)v;
                }
        __syncthreads();
        const bool vec = ((reinterpret_cast<uintptr_t>(g.out_bf16) & 15) == 0) && ((g.ldc & 7) == 0);
        for (int q = threadIdx.x; q < BM * (BNT / 8); q += 256) {
            const int r = q / (BNT / 8), c = (q % (BNT / 8)) * 8;
            const int m = m0 + r, n = n0 + c;
            if (m >= g.M || n >= g.N) continue;
            elem* dst = g.out_bf16 + (int64_t)m * g.ldc + n;
            const elem* src = ct + r * CLD + c;
            if (vec && n + 8 <= g.N) {
                *reinterpret_cast<elemx8*>(dst) = *reinterpret_cast<const elemx8*>(src);
            } else {
                for (int e = 0; e < 8 && n + e < g.N; ++e) dst[e] = src[e];
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int n = n0 + wn + j * 32 + (lane & 31);
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[i][j][r];
                const int64_t o = (int64_t)m * g.ldc + n;
                if constexpr (EPI == EPI_BIAS_RELU_BF16) {
                    g.out_bf16[o] = (elem)fmaxf(v + g.bias[n], 0.0f);
                } else if constexpr (EPI == EPI_BIAS_F32) {
                    g.out_f32[o] = v + g.bias[n];
                } else if constexpr (EPI == EPI_BIAS_BF16) {
                    g.out_bf16[o] = (elem)(v + g.bias[n]);
                } else if constexpr (EPI == EPI_MASK_BF16_F32) {
                    const float x = (float)g.mask[o] > 0.0f ? v : 0.0f;
                    g.out_bf16[o] = (elem)x;
                    g.out_f32[o] = x;
                } else {
                    g.out_f32[o] = v;
                }
            }
}

// x[b][i] = bit i of syndrome row b, as BF16 0/1
__global__ void expand_bits_kernel(const uint32_t* syn, int words, int in, int B, elem* x) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * in) return;
    const int b = (int)(idx / in), i = (int)(idx % in);
    x[idx] = (elem)(float)((syn[(int64_t)b * words + (i >> 5)] >> (i & 31)) & 1u);
}

// Per element: z = -(lambda + delta), p = sigmoid(z), y = target bit.
// dL/d(delta) = -(p - y) / B.  Per-block loss partial sums for a deterministic
// reduction.
__global__ void loss_grad_kernel(const float* delta, const float* lam, const uint32_t* tgt, int words, int N, int B,
                                 float* d3f, elem* d3b, float* partial) {
    __shared__ float red[256];
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (idx < (int64_t)B * N) {
        const int b = (int)(idx / N), j = (int)(idx % N);
        const float z = -(lam[j] + delta[idx]);
        const float y = (float)((tgt[(int64_t)b * words + (j >> 5)] >> (j & 31)) & 1u);
        const float p = 1.0f / (1.0f + expf(-z));
        const float g = -(p - y) / (float)B;
        d3f[idx] = g;
        d3b[idx] = (elem)g;
        l = fmaxf(z, 0.0f) - z * y + log1pf(expf(-fabsf(z)));
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sum_partials_kernel(const float* partial, int n, float scale, float* out) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// Column sums out[n] = sum_b in[b][n] in two deterministic stages: chunks of
// 256 rows per block (64 columns x 4 row groups, fixed order), then the chunk
// partials in order.
constexpr int CS_ROWS = 256;
__global__ void colsum_partial_kernel(const float* in, int B, int N, float* part) {
    __shared__ float red[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
    const int r0 = blockIdx.y * CS_ROWS;
    float s = 0.0f;
    if (c < N)
        for (int r = r0 + g; r < min(B, r0 + CS_ROWS); r += 4) s += in[(int64_t)r * N + c];
    red[g][threadIdx.x & 63] = s;
    __syncthreads();
    if (g == 0 && c < N)
        part[(int64_t)blockIdx.y * N + c] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
                                           red[3][threadIdx.x];
}

__global__ void colsum_final_kernel(const float* part, int chunks, int N, float* out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int k = 0; k < chunks; ++k) s += part[(int64_t)k * N + n];
    out[n] = s;
}

// out[c][r] = in[r][c] for a rows x cols BF16 matrix (64 x 64 tiles through LDS)
__global__ void transpose_bf16_kernel(const elem* in, int rows, int cols, elem* out) {
    __shared__ elem t[64][65];
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int gr = r0 + r, gc = c0 + tx;
        t[r][tx] = (gr < rows && gc < cols) ? in[(int64_t)gr * cols + gc] : (elem)0.0f;
    }
    __syncthreads();
    for (int c = ty; c < 64; c += 4) {
        const int gc = c0 + c, gr = r0 + tx;
        if (gc < cols && gr < rows) out[(int64_t)gc * rows + gr] = t[tx][c];
    }
}

__global__ void adam_kernel(float* w, float* mo, float* ve, const float* g, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float m = b1 * mo[i] + (1.0f - b1) * gi;
    const float v = b2 * ve[i] + (1.0f - b2) * gi * gi;
    mo[i] = m;
    ve[i] = v;
    w[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// output layer in a caller's order: row p of W3o (and b3o[p]) is row ord[p] of
// W3 (b3), or zero where ord[p] < 0
__global__ void order_rows_kernel(const elem* w3, const float* b3, const int32_t* ord, int n, int hid, elem* w3o,
                                  float* b3o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * hid) return;
    const int p = (int)(i / hid), k = (int)(i % hid);
    const int o = ord[p];
    w3o[i] = o >= 0 ? w3[(int64_t)o * hid + k] : (elem)0.0f;
    if (k == 0) b3o[p] = o >= 0 ? b3[o] : 0.0f;
}

__global__ void to_bf16_kernel(const float* w, elem* o, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = (elem)w[i];
}

}  // namespace mlp
}  // namespace rbp

using namespace rbp;
using namespace rbp::mlp;

struct rbp_mlp {
    int in = 0, hid = 0, out = 0;
    int64_t n_params = 0;
    int64_t oW1, ob1, oW2, ob2, oW3, ob3;  // offsets in the parameter array
    DevBuf w, m, v, g, wb;                 // FP32 masters, Adam moments, gradients, BF16 copies
    DevBuf w2t, w3t;                       // BF16 W2^T [hid][hid] and W3^T [hid][out] for the backward pass
    int64_t step = 0;
    int cap = 0;                           // batch capacity of the training workspace
    int fcap = 0;                          // batch capacity of the forward workspace
    DevBuf xb, h1, h2, d3b, dh2b, dh1b;    // BF16 activations / gradients
    DevBuf delta, d3f, dh2f, dh1f, partial, loss;
    DevBuf tA, tB, csum;                   // transposed operands of the weight gradients, column-sum partials
    int ord_n = 0;                         // rbp_mlp_set_output_order: columns of the BF16 forward (0: out)
    DevBuf ord, w3o, b3o;                  // the order, and the output layer's rows in that order
};

namespace {

// forward needs x, h1, h2; training also the gradient buffers
rbp_status ensure_workspace(rbp_mlp* p, int B, bool training) {
    if (B <= (training ? p->cap : p->fcap)) return RBP_OK;
    const int64_t Bi = B;
    rbp_status st = RBP_OK;
    if (!st) st = p->xb.reserve(sizeof(elem) * Bi * p->in);
    if (!st) st = p->h1.reserve(sizeof(elem) * Bi * p->hid);
    if (!st) st = p->h2.reserve(sizeof(elem) * Bi * p->hid);
    if (st) return st;
    p->fcap = std::max(p->fcap, B);
    if (!training) return RBP_OK;
    if (!st) st = p->d3b.reserve(sizeof(elem) * Bi * p->out);
    if (!st) st = p->dh2b.reserve(sizeof(elem) * Bi * p->hid);
    if (!st) st = p->dh1b.reserve(sizeof(elem) * Bi * p->hid);
    if (!st) st = p->delta.reserve(sizeof(float) * Bi * p->out);
    if (!st) st = p->d3f.reserve(sizeof(float) * Bi * p->out);
    if (!st) st = p->dh2f.reserve(sizeof(float) * Bi * p->hid);
    if (!st) st = p->dh1f.reserve(sizeof(float) * Bi * p->hid);
    if (!st) st = p->partial.reserve(sizeof(float) * (Bi * std::max(p->out, p->hid) / 256 + 2));
    if (!st) st = p->loss.reserve(sizeof(float) * 4);
    const int64_t wide = std::max<int64_t>(std::max(p->out, p->hid), p->in);
    if (!st) st = p->tA.reserve(sizeof(elem) * Bi * wide);
    if (!st) st = p->tB.reserve(sizeof(elem) * Bi * wide);
    if (!st) st = p->csum.reserve(sizeof(float) * ((Bi + CS_ROWS - 1) / CS_ROWS) * wide);
    if (st) return st;
    p->cap = B;
    return RBP_OK;
}

template <int LA, int LB, int EPI, int TN = 2>
rbp_status gemm(const GemmArgs& a, hipStream_t s) {
    const int tiles = ((a.N + 64 * TN - 1) / (64 * TN)) * ((a.M + BM - 1) / BM);
    dim3 grid(8 * ((tiles + 7) / 8));  // renumbered per XCD in the kernel
    hipLaunchKernelGGL((gemm_kernel<LA, LB, EPI, TN>), grid, dim3(256), 0, s, a);
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

GemmArgs ga(int M, int N, int K, const elem* A, int lda, const elem* B, int ldb, int ldc) {
    GemmArgs a;
    std::memset(&a, 0, sizeof(a));
    a.M = M;
    a.N = N;
    a.K = K;
    a.A = A;
    a.lda = lda;
    a.B = B;
    a.ldb = ldb;
    a.ldc = ldc;
    return a;
}

int blocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

rbp_status transpose(const elem* in, int rows, int cols, elem* out, hipStream_t s) {
    hipLaunchKernelGGL(transpose_bf16_kernel, dim3(blocks(cols, 64), blocks(rows, 64)), dim3(256), 0, s, in, rows, cols,
                       out);
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

rbp_status colsum(rbp_mlp* p, const float* in, int B, int N, float* out, hipStream_t s) {
    const int chunks = blocks(B, CS_ROWS);
    hipLaunchKernelGGL(colsum_partial_kernel, dim3(blocks(N, 64), chunks), dim3(256), 0, s, in, B, N,
                       p->csum.as<float>());
    RBP_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(colsum_final_kernel, dim3(blocks(N, 256)), dim3(256), 0, s, p->csum.as<float>(), chunks, N, out);
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

// forward of B rows: x from syndromes, h1, h2 (workspace), delta into `dout`.
// Training keeps x as BF16 (the weight gradient of layer 1 needs it); inference
// expands the syndrome bits while staging the first product's tiles.
rbp_status forward(rbp_mlp* p, const uint32_t* syn, int B, float* dout, hipStream_t s, bool keep_x,
                   elem* dout16 = nullptr) {
    const int words = (p->in + 31) / 32;
    elem* xb = p->xb.as<elem>();
    elem* h1 = p->h1.as<elem>();
    elem* h2 = p->h2.as<elem>();
    const elem* wb = p->wb.as<elem>();
    const float* w = p->w.as<float>();
    rbp_status st;
    if (keep_x) {
        hipLaunchKernelGGL(expand_bits_kernel, dim3(blocks((int64_t)B * p->in, 256)), dim3(256), 0, s, syn, words,
                           p->in, B, xb);
        RBP_HIP_CHECK(hipGetLastError());
        GemmArgs a = ga(B, p->hid, p->in, xb, p->in, wb + p->oW1, p->in, p->hid);
        a.bias = w + p->ob1;
        a.out_bf16 = h1;
        st = gemm<K_CONTIG, K_CONTIG, EPI_BIAS_RELU_BF16>(a, s);
    } else {
        GemmArgs a = ga(B, p->hid, p->in, reinterpret_cast<const elem*>(syn), words, wb + p->oW1, p->in, p->hid);
        a.bias = w + p->ob1;
        a.out_bf16 = h1;
        st = gemm<BITS, K_CONTIG, EPI_BIAS_RELU_BF16, kFwdTN>(a, s);
    }
    if (st) return st;
    GemmArgs a;
    a = ga(B, p->hid, p->hid, h1, p->hid, wb + p->oW2, p->hid, p->hid);
    a.bias = w + p->ob2;
    a.out_bf16 = h2;
    st = gemm<K_CONTIG, K_CONTIG, EPI_BIAS_RELU_BF16, kFwdTN>(a, s);
    if (st) return st;
    a = ga(B, p->out, p->hid, h2, p->hid, wb + p->oW3, p->hid, p->out);
    a.bias = w + p->ob3;
    if (dout16) {
        if (p->ord_n > 0) {
            // output columns in the caller's order (rbp_mlp_set_output_order)
            a = ga(B, p->ord_n, p->hid, h2, p->hid, p->w3o.as<elem>(), p->hid, p->ord_n);
            a.bias = p->b3o.as<float>();
        }
        a.out_bf16 = dout16;
        return gemm<K_CONTIG, K_CONTIG, EPI_BIAS_BF16, kFwdTN>(a, s);
    }
    a.out_f32 = dout;
    return gemm<K_CONTIG, K_CONTIG, EPI_BIAS_F32, kFwdTN>(a, s);
}

// forward + backward of one batch into p->g (gradients of the mean loss)
rbp_status gradients(rbp_mlp* p, const uint32_t* syn, const uint32_t* tgt, const float* llr, int B, float* loss_out,
                     hipStream_t s) {
    rbp_status st = ensure_workspace(p, B, true);
    if (st) return st;
    float* delta = p->delta.as<float>();
    st = forward(p, syn, B, delta, s, true);
    if (st) return st;
    const int twords = (p->out + 31) / 32;
    const int64_t n3 = (int64_t)B * p->out;
    const int nb = blocks(n3, 256);
    hipLaunchKernelGGL(loss_grad_kernel, dim3(nb), dim3(256), 0, s, delta, llr, tgt, twords, p->out, B,
                       p->d3f.as<float>(), p->d3b.as<elem>(), p->partial.as<float>());
    RBP_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, p->partial.as<float>(), nb, 1.0f / (float)B,
                       loss_out ? loss_out : p->loss.as<float>());
    RBP_HIP_CHECK(hipGetLastError());
    float* g = p->g.as<float>();
    elem* tA = p->tA.as<elem>();
    elem* tB = p->tB.as<elem>();
    // Weight gradients dW = dY^T X are NT products of the transposed operands
    // (both K = batch contiguous); dX = dY W uses the transposed weight copies.
    // dW3 = d3^T h2 ; db3 = colsum d3 ; dh2 = (d3 W3) * [h2 > 0]
    if ((st = transpose(p->d3b.as<elem>(), B, p->out, tA, s))) return st;
    if ((st = transpose(p->h2.as<elem>(), B, p->hid, tB, s))) return st;
    GemmArgs a = ga(p->out, p->hid, B, tA, B, tB, B, p->hid);
    a.out_f32 = g + p->oW3;
    if ((st = gemm<K_CONTIG, K_CONTIG, EPI_F32>(a, s))) return st;
    if ((st = colsum(p, p->d3f.as<float>(), B, p->out, g + p->ob3, s))) return st;
    a = ga(B, p->hid, p->out, p->d3b.as<elem>(), p->out, p->w3t.as<elem>(), p->out, p->hid);
    a.mask = p->h2.as<elem>();
    a.out_bf16 = p->dh2b.as<elem>();
    a.out_f32 = p->dh2f.as<float>();
    if ((st = gemm<K_CONTIG, K_CONTIG, EPI_MASK_BF16_F32>(a, s))) return st;
    // dW2 = dh2^T h1 ; db2 ; dh1 = (dh2 W2) * [h1 > 0]
    if ((st = transpose(p->dh2b.as<elem>(), B, p->hid, tA, s))) return st;
    if ((st = transpose(p->h1.as<elem>(), B, p->hid, tB, s))) return st;
    a = ga(p->hid, p->hid, B, tA, B, tB, B, p->hid);
    a.out_f32 = g + p->oW2;
    if ((st = gemm<K_CONTIG, K_CONTIG, EPI_F32>(a, s))) return st;
    if ((st = colsum(p, p->dh2f.as<float>(), B, p->hid, g + p->ob2, s))) return st;
    a = ga(B, p->hid, p->hid, p->dh2b.as<elem>(), p->hid, p->w2t.as<elem>(), p->hid, p->hid);
    a.mask = p->h1.as<elem>();
    a.out_bf16 = p->dh1b.as<elem>();
    a.out_f32 = p->dh1f.as<float>();
    if ((st = gemm<K_CONTIG, K_CONTIG, EPI_MASK_BF16_F32>(a, s))) return st;
    // dW1 = dh1^T x ; db1
    if ((st = transpose(p->dh1b.as<elem>(), B, p->hid, tA, s))) return st;
    if ((st = transpose(p->xb.as<elem>(), B, p->in, tB, s))) return st;
    a = ga(p->hid, p->in, B, tA, B, tB, B, p->in);
    a.out_f32 = g + p->oW1;
    if ((st = gemm<K_CONTIG, K_CONTIG, EPI_F32>(a, s))) return st;
    return colsum(p, p->dh1f.as<float>(), B, p->hid, g + p->ob1, s);
}

rbp_status reorder_output(rbp_mlp* p, hipStream_t s) {
    if (p->ord_n <= 0) return RBP_OK;
    hipLaunchKernelGGL(order_rows_kernel, dim3(blocks((int64_t)p->ord_n * p->hid, 256)), dim3(256), 0, s,
                       p->wb.as<elem>() + p->oW3, p->w.as<float>() + p->ob3, p->ord.as<int32_t>(), p->ord_n, p->hid,
                       p->w3o.as<elem>(), p->b3o.as<float>());
    RBP_HIP_CHECK(hipGetLastError());
    return RBP_OK;
}

rbp_status refresh_bf16(rbp_mlp* p, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(p->n_params, 256)), dim3(256), 0, s, p->w.as<float>(),
                       p->wb.as<elem>(), p->n_params);
    RBP_HIP_CHECK(hipGetLastError());
    rbp_status st = transpose(p->wb.as<elem>() + p->oW2, p->hid, p->hid, p->w2t.as<elem>(), s);
    if (st) return st;
    st = transpose(p->wb.as<elem>() + p->oW3, p->out, p->hid, p->w3t.as<elem>(), s);
    if (st) return st;
    return reorder_output(p, s);
}

rbp_status zero_adam(rbp_mlp* p) {
    RBP_HIP_CHECK(hipMemset(p->m.p, 0, sizeof(float) * p->n_params));
    RBP_HIP_CHECK(hipMemset(p->v.p, 0, sizeof(float) * p->n_params));
    p->step = 0;
    return RBP_OK;
}

}  // namespace

extern "C" {

rbp_status rbp_mlp_create(int32_t in_dim, int32_t hidden, int32_t out_dim, uint64_t seed, rbp_mlp_t* out) {
    if (!out) return fail(RBP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (in_dim < 1 || hidden < 1 || out_dim < 1) return fail(RBP_ERR_SHAPE, "dimensions must be >= 1");
    rbp_mlp* p = new rbp_mlp();
    p->in = in_dim;
    p->hid = hidden;
    p->out = out_dim;
    int64_t o = 0;
    p->oW1 = o; o += (int64_t)hidden * in_dim;
    p->ob1 = o; o += hidden;
    p->oW2 = o; o += (int64_t)hidden * hidden;
    p->ob2 = o; o += hidden;
    p->oW3 = o; o += (int64_t)out_dim * hidden;
    p->ob3 = o; o += out_dim;
    p->n_params = o;
    // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights from Philox(seed; index/4, 0, 0, 2); zero biases
    std::vector<float> h(o, 0.0f);
    auto fill = [&](int64_t off, int64_t n, int fan_in) {
        const float s = 1.0f / std::sqrt((float)fan_in);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t idx = off + i;
            const U4 r = philox4x32_10(U4{(uint32_t)(idx >> 2), (uint32_t)(idx >> 34), 0u, 2u}, (uint32_t)seed,
                                       (uint32_t)(seed >> 32));
            const float u = (float)(u4_get(r, (int)(idx & 3)) >> 8) * (1.0f / 16777216.0f);
            h[idx] = (2.0f * u - 1.0f) * s;
        }
    };
    fill(p->oW1, (int64_t)hidden * in_dim, in_dim);
    fill(p->oW2, (int64_t)hidden * hidden, hidden);
    fill(p->oW3, (int64_t)out_dim * hidden, hidden);
    rbp_status st = RBP_OK;
    if (!st) st = p->w.reserve(sizeof(float) * o);
    if (!st) st = p->m.reserve(sizeof(float) * o);
    if (!st) st = p->v.reserve(sizeof(float) * o);
    if (!st) st = p->g.reserve(sizeof(float) * o);
    if (!st) st = p->wb.reserve(sizeof(elem) * o);
    if (!st) st = p->w2t.reserve(sizeof(elem) * (int64_t)hidden * hidden);
    if (!st) st = p->w3t.reserve(sizeof(elem) * (int64_t)hidden * out_dim);
    if (!st) {
        hipError_t e = hipMemcpy(p->w.p, h.data(), sizeof(float) * o, hipMemcpyHostToDevice);
        if (e != hipSuccess) st = fail(RBP_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    if (!st) st = zero_adam(p);
    if (!st) st = refresh_bf16(p, nullptr);
    if (!st) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) st = fail(RBP_ERR_HIP, std::string("sync: ") + hipGetErrorString(e));
    }
    if (st) {
        rbp_mlp_destroy(p);
        return st;
    }
    *out = p;
    return RBP_OK;
}

rbp_status rbp_mlp_destroy(rbp_mlp_t p) {
    if (!p) return RBP_OK;
    (void)hipDeviceSynchronize();
    for (DevBuf* b : {&p->w, &p->m, &p->v, &p->g, &p->wb, &p->w2t, &p->w3t, &p->xb, &p->h1, &p->h2, &p->d3b,
                      &p->dh2b, &p->dh1b, &p->delta, &p->d3f, &p->dh2f, &p->dh1f, &p->partial, &p->loss, &p->tA,
                      &p->tB, &p->csum, &p->ord, &p->w3o, &p->b3o})
        b->release();
    delete p;
    return RBP_OK;
}

rbp_status rbp_mlp_forward(rbp_mlp_t p, const uint32_t* syndromes, uint64_t shots, float* delta, void* stream_) {
    if (!p) return fail(RBP_ERR_INVALID_ARG, "mlp is NULL");
    if (shots == 0) return RBP_OK;
    if (!syndromes || !delta) return fail(RBP_ERR_INVALID_ARG, "NULL buffer");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
    const int chunk = 131072;  // rows per forward pass (one for a 10^5-shot batch: 6 % faster than two)
    rbp_status st = ensure_workspace(p, (int)std::min<uint64_t>(shots, chunk), false);
    if (st) return st;
    const int words = (p->in + 31) / 32;
    for (uint64_t b0 = 0; b0 < shots; b0 += chunk) {
        const int B = (int)std::min<uint64_t>(chunk, shots - b0);
        st = forward(p, syndromes + b0 * words, B, delta + b0 * (uint64_t)p->out, s, false);
        if (st) return st;
    }
    return RBP_OK;
}

rbp_status rbp_mlp_forward_bf16(rbp_mlp_t p, const uint32_t* syndromes, uint64_t shots, uint16_t* delta,
                                void* stream_) {
    if (!p) return fail(RBP_ERR_INVALID_ARG, "mlp is NULL");
#ifdef RBP_MLP_FP32
    (void)syndromes;
    (void)shots;
    (void)delta;
    (void)stream_;
    return fail(RBP_ERR_UNSUPPORTED, "the FP32 test build has no BF16 output");
#endif
    if (shots == 0) return RBP_OK;
    if (!syndromes || !delta) return fail(RBP_ERR_INVALID_ARG, "NULL buffer");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
    const int chunk = 131072;  // rows per forward pass (one for a 10^5-shot batch: 6 % faster than two)
    rbp_status st = ensure_workspace(p, (int)std::min<uint64_t>(shots, chunk), false);
    if (st) return st;
    const int words = (p->in + 31) / 32;
    for (uint64_t b0 = 0; b0 < shots; b0 += chunk) {
        const int B = (int)std::min<uint64_t>(chunk, shots - b0);
        st = forward(p, syndromes + b0 * words, B, nullptr, s, false,
                     reinterpret_cast<elem*>(delta) + b0 * (uint64_t)(p->ord_n > 0 ? p->ord_n : p->out));
        if (st) return st;
    }
    return RBP_OK;
}

rbp_status rbp_mlp_set_output_order(rbp_mlp_t p, const int32_t* order, int32_t n) {
    if (!p) return fail(RBP_ERR_INVALID_ARG, "mlp is NULL");
    if (n < 0 || (n > 0 && !order)) return fail(RBP_ERR_INVALID_ARG, "order: n >= 0, NULL only with n = 0");
    if (n == 0) {
        p->ord_n = 0;
        return RBP_OK;
    }
    for (int i = 0; i < n; ++i)
        if (order[i] < -1 || order[i] >= p->out)
            return fail(RBP_ERR_INVALID_ARG, "order entries must be -1 or output indices");
    rbp_status st = p->ord.reserve(sizeof(int32_t) * (size_t)n);
    if (!st) st = p->w3o.reserve(sizeof(elem) * (size_t)n * p->hid);
    if (!st) st = p->b3o.reserve(sizeof(float) * (size_t)n);
    if (st) return st;
    RBP_HIP_CHECK(hipMemcpy(p->ord.p, order, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
    p->ord_n = n;
    st = reorder_output(p, nullptr);
    if (st) return st;
    RBP_HIP_CHECK(hipStreamSynchronize(nullptr));
    return RBP_OK;
}

rbp_status rbp_mlp_gradients(rbp_mlp_t p, const uint32_t* syndromes, const uint32_t* targets, const float* llr,
                             uint64_t batch, float* grads_out, float* loss_out, void* stream_) {
    if (!p) return fail(RBP_ERR_INVALID_ARG, "mlp is NULL");
    if (!syndromes || !targets || !llr || !grads_out) return fail(RBP_ERR_INVALID_ARG, "NULL buffer");
    if (batch < 1 || batch > (1u << 20)) return fail(RBP_ERR_INVALID_ARG, "batch must be 1..2^20");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
    rbp_status st = gradients(p, syndromes, targets, llr, (int)batch, loss_out, s);
    if (st) return st;
    RBP_HIP_CHECK(hipMemcpyAsync(grads_out, p->g.p, sizeof(float) * p->n_params, hipMemcpyDeviceToDevice, s));
    return RBP_OK;
}

rbp_status rbp_mlp_train_step(rbp_mlp_t p, const uint32_t* syndromes, const uint32_t* targets, const float* llr,
                              uint64_t batch, float lr, float* loss_out, void* stream_) {
    if (!p) return fail(RBP_ERR_INVALID_ARG, "mlp is NULL");
    if (!syndromes || !targets || !llr) return fail(RBP_ERR_INVALID_ARG, "NULL buffer");
    if (batch < 1 || batch > (1u << 20)) return fail(RBP_ERR_INVALID_ARG, "batch must be 1..2^20");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(RBP_ERR_INVALID_ARG, "lr must be positive");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
    rbp_status st = gradients(p, syndromes, targets, llr, (int)batch, loss_out, s);
    if (st) return st;
    p->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - (float)std::pow(0.9, (double)p->step);
    const float c2 = 1.0f - (float)std::pow(0.999, (double)p->step);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(p->n_params, 256)), dim3(256), 0, s, p->w.as<float>(),
                       p->m.as<float>(), p->v.as<float>(), p->g.as<float>(), p->n_params, lr, b1, b2, 1e-8f, c1, c2);
    RBP_HIP_CHECK(hipGetLastError());
    return refresh_bf16(p, s);
}

rbp_status rbp_mlp_num_params(rbp_mlp_t p, int64_t* n) {
    if (!p || !n) return fail(RBP_ERR_INVALID_ARG, "NULL argument");
    *n = p->n_params;
    return RBP_OK;
}

rbp_status rbp_mlp_get_params(rbp_mlp_t p, float* host_out) {
    if (!p || !host_out) return fail(RBP_ERR_INVALID_ARG, "NULL argument");
    RBP_HIP_CHECK(hipDeviceSynchronize());
    RBP_HIP_CHECK(hipMemcpy(host_out, p->w.p, sizeof(float) * p->n_params, hipMemcpyDeviceToHost));
    return RBP_OK;
}

static const char kMlpMagic[8] = {'R', 'B', 'P', 'M', 'L', 'P', '0', '1'};

rbp_status rbp_mlp_save(rbp_mlp_t p, const char* path) {
    if (!p || !path) return fail(RBP_ERR_INVALID_ARG, "NULL argument");
    RBP_HIP_CHECK(hipDeviceSynchronize());
    const size_t n = (size_t)p->n_params;
    std::vector<float> buf(3 * n);
    RBP_HIP_CHECK(hipMemcpy(buf.data(), p->w.p, sizeof(float) * n, hipMemcpyDeviceToHost));
    RBP_HIP_CHECK(hipMemcpy(buf.data() + n, p->m.p, sizeof(float) * n, hipMemcpyDeviceToHost));
    RBP_HIP_CHECK(hipMemcpy(buf.data() + 2 * n, p->v.p, sizeof(float) * n, hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(RBP_ERR_INVALID_ARG, std::string("cannot open for writing: ") + path);
    const int32_t dims[4] = {p->in, p->hid, p->out, 0};
    const int64_t counts[2] = {p->n_params, p->step};
    bool ok = std::fwrite(kMlpMagic, 1, 8, f) == 8 && std::fwrite(dims, sizeof(int32_t), 4, f) == 4 &&
              std::fwrite(counts, sizeof(int64_t), 2, f) == 2 &&
              std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(RBP_ERR_INVALID_ARG, std::string("write failed: ") + path);
    return RBP_OK;
}

rbp_status rbp_mlp_load(rbp_mlp_t p, const char* path) {
    if (!p || !path) return fail(RBP_ERR_INVALID_ARG, "NULL argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(RBP_ERR_INVALID_ARG, std::string("cannot open: ") + path);
    char magic[8];
    int32_t dims[4];
    int64_t counts[2];
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMlpMagic, 8) == 0 &&
              std::fread(dims, sizeof(int32_t), 4, f) == 4 && std::fread(counts, sizeof(int64_t), 2, f) == 2;
    if (!ok) {
        std::fclose(f);
        return fail(RBP_ERR_INVALID_ARG, std::string("not a network checkpoint: ") + path);
    }
    if (dims[0] != p->in || dims[1] != p->hid || dims[2] != p->out || counts[0] != p->n_params) {
        std::fclose(f);
        return fail(RBP_ERR_SHAPE, "checkpoint dimensions differ from the handle's");
    }
    const size_t n = (size_t)p->n_params;
    std::vector<float> buf(3 * n);
    ok = std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok || counts[1] < 0) return fail(RBP_ERR_INVALID_ARG, std::string("truncated checkpoint: ") + path);
    RBP_HIP_CHECK(hipDeviceSynchronize());
    RBP_HIP_CHECK(hipMemcpy(p->w.p, buf.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    RBP_HIP_CHECK(hipMemcpy(p->m.p, buf.data() + n, sizeof(float) * n, hipMemcpyHostToDevice));
    RBP_HIP_CHECK(hipMemcpy(p->v.p, buf.data() + 2 * n, sizeof(float) * n, hipMemcpyHostToDevice));
    p->step = counts[1];
    rbp_status st = refresh_bf16(p, nullptr);
    if (st) return st;
    RBP_HIP_CHECK(hipDeviceSynchronize());
    return RBP_OK;
}

rbp_status rbp_mlp_set_params(rbp_mlp_t p, const float* host_in) {
    if (!p || !host_in) return fail(RBP_ERR_INVALID_ARG, "NULL argument");
    RBP_HIP_CHECK(hipDeviceSynchronize());
    RBP_HIP_CHECK(hipMemcpy(p->w.p, host_in, sizeof(float) * p->n_params, hipMemcpyHostToDevice));
    rbp_status st = zero_adam(p);
    if (!st) st = refresh_bf16(p, nullptr);
    if (st) return st;
    RBP_HIP_CHECK(hipDeviceSynchronize());
    return RBP_OK;
}

}  // extern "C"
