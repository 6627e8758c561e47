// Learned-proposal network (placeholder until the kernels land).
#include "rbp_common.h"
using namespace rbp;
extern "C" {
rbp_status rbp_mlp_create(int32_t, int32_t, int32_t, uint64_t, rbp_mlp_t* out) {
    if (out) *out = nullptr;
    return fail(RBP_ERR_UNSUPPORTED, "mlp not built");
}
rbp_status rbp_mlp_destroy(rbp_mlp_t) { return RBP_OK; }
rbp_status rbp_mlp_forward(rbp_mlp_t, const uint32_t*, uint64_t, float*, void*) { return fail(RBP_ERR_UNSUPPORTED, "mlp not built"); }
rbp_status rbp_mlp_train_step(rbp_mlp_t, const uint32_t*, const uint32_t*, const float*, uint64_t, float, float*, void*) { return fail(RBP_ERR_UNSUPPORTED, "mlp not built"); }
rbp_status rbp_mlp_num_params(rbp_mlp_t, int64_t*) { return fail(RBP_ERR_UNSUPPORTED, "mlp not built"); }
rbp_status rbp_mlp_get_params(rbp_mlp_t, float*) { return fail(RBP_ERR_UNSUPPORTED, "mlp not built"); }
rbp_status rbp_mlp_set_params(rbp_mlp_t, const float*) { return fail(RBP_ERR_UNSUPPORTED, "mlp not built"); }
}
