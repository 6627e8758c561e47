// librbp: device ceilings measured on the running GPU, the denominators of the
// decoder's roofline fractions.
//
//  * lds_read_kernel   aggregate LDS read bandwidth: every wave reads 64
//                      consecutive cells of a 64 KB LDS buffer (no bank
//                      conflicts), four independent reads per step, two
//                      1024-thread workgroups per CU.
#include "rbp_common.h"

namespace rbp {
rbp_status fail(rbp_status st, const std::string& m);
}  // namespace rbp

using namespace rbp;

namespace {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef uint32_t v2u __attribute__((ext_vector_type(2)));

constexpr int kLdsCells = 4096;  // 16-byte cells: 64 KB per workgroup

template <int WIDTH>
struct Cell;
template <>
struct Cell<4> {
    typedef uint32_t T;
    static constexpr int n = 4 * kLdsCells;
};
template <>
struct Cell<8> {
    typedef v2u T;
    static constexpr int n = 2 * kLdsCells;
};
template <>
struct Cell<16> {
    typedef v4u T;
    static constexpr int n = kLdsCells;
};

__device__ __forceinline__ uint32_t fold(uint32_t v) { return v; }
__device__ __forceinline__ uint32_t fold(v2u v) { return v.x ^ v.y; }
__device__ __forceinline__ uint32_t fold(v4u v) { return v.x ^ v.y ^ v.z ^ v.w; }

// reps steps of four reads of WIDTH bytes per lane; the read address moves
// by one wave's span every step so no read can be hoisted out of the loop
template <int WIDTH>
__global__ void __launch_bounds__(1024) lds_read_kernel(uint32_t* out, int reps) {
    typedef typename Cell<WIDTH>::T T;
    constexpr int n = Cell<WIDTH>::n;
    __shared__ T buf[n];
    const int tid = threadIdx.x;
    for (int i = tid; i < n; i += 1024) {
        T v;
        if constexpr (WIDTH == 4) {
            v = (uint32_t)i;
        } else if constexpr (WIDTH == 8) {
            v.x = (uint32_t)i;
            v.y = (uint32_t)(3 * i);
        } else {
            v.x = (uint32_t)i;
            v.y = (uint32_t)(3 * i);
            v.z = (uint32_t)(5 * i);
            v.w = (uint32_t)(7 * i);
        }
        buf[i] = v;
    }
    __syncthreads();
    uint32_t acc = 0;
    int idx = tid;
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int k = 0; k < 4; ++k) acc ^= fold(buf[(idx + k * (n / 4)) & (n - 1)]);
        idx += 64;
    }
    out[blockIdx.x * 1024 + tid] = acc;
}

template <int WIDTH>
rbp_status measure(int cus, double* bps) {
    const int blocks = 2 * cus;
    const int reps = 4096;
    uint32_t* out = nullptr;
    RBP_HIP_CHECK(hipMalloc(&out, sizeof(uint32_t) * (size_t)blocks * 1024));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best_ms = 0.0f;
    for (int trial = 0; e == hipSuccess && trial < 4; ++trial) {
        e = hipEventRecord(e0, nullptr);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(lds_read_kernel<WIDTH>, dim3(blocks), dim3(1024), 0, nullptr, out, reps);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && trial > 0 && (best_ms == 0.0f || ms < best_ms)) best_ms = ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (e != hipSuccess) return fail(RBP_ERR_HIP, std::string("LDS probe: ") + hipGetErrorString(e));
    const double bytes = (double)blocks * 1024.0 * reps * 4.0 * WIDTH;
    *bps = bytes / (best_ms * 1e-3);
    return RBP_OK;
}

}  // namespace

extern "C" {

rbp_status rbp_measure_lds_bandwidth(int32_t width_bytes, double* bytes_per_s) {
    if (!bytes_per_s) return fail(RBP_ERR_INVALID_ARG, "bytes_per_s is NULL");
    int dev = 0, cus = 0;
    RBP_HIP_CHECK(hipGetDevice(&dev));
    RBP_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    RBP_HIP_CHECK(hipDeviceSynchronize());
    switch (width_bytes) {
        case 4: return measure<4>(cus, bytes_per_s);
        case 8: return measure<8>(cus, bytes_per_s);
        case 16: return measure<16>(cus, bytes_per_s);
        default: return fail(RBP_ERR_INVALID_ARG, "width_bytes must be 4, 8 or 16");
    }
}

}  // extern "C"
