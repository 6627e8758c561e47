// librbp: error reporting and device buffers shared by every source file.
#include <string>

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

}  // namespace rbp

extern "C" const char* rbp_last_error(void) { return rbp::g_err.c_str(); }
