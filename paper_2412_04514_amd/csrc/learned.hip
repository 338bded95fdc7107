// Learned-k form: placeholder until the network kernels land.
#include "internal.h"

struct votess_kmodel {
  votess_ctx* ctx;
};

namespace votess {
votess_status learned_first_pass(votess_ctx*, votess_kmodel*, double, const void*, int, const votess_grid&,
                                 const int32_t*, const ClipLaunch&, int32_t*, int32_t*, votess_stats&, hipStream_t) {
  return fail(VOTESS_EINVAL, "learned-k is not built yet");
}
}  // namespace votess

using votess::fail;
extern "C" {
votess_kmodel* votess_kmodel_create(votess_ctx*, uint64_t) { fail(VOTESS_EINVAL, "learned-k is not built yet"); return nullptr; }
void votess_kmodel_destroy(votess_kmodel*) {}
votess_status votess_kmodel_set_params(votess_kmodel*, const float*, const float*, const float*) { return fail(VOTESS_EINVAL, "n/a"); }
votess_status votess_kmodel_get_params(votess_kmodel*, float*, float*, float*) { return fail(VOTESS_EINVAL, "n/a"); }
votess_status votess_features(votess_ctx*, const void*, int64_t, const votess_grid*, const int32_t*, const int32_t*, int64_t, float*, void*) { return fail(VOTESS_EINVAL, "n/a"); }
votess_status votess_kmodel_forward(votess_kmodel*, const float*, int64_t, float*, void*) { return fail(VOTESS_EINVAL, "n/a"); }
votess_status votess_kmodel_grad(votess_kmodel*, const float*, const uint8_t*, int64_t, float*, float*, void*) { return fail(VOTESS_EINVAL, "n/a"); }
votess_status votess_kmodel_train_step(votess_kmodel*, const float*, const uint8_t*, int64_t, float, float*, void*) { return fail(VOTESS_EINVAL, "n/a"); }
votess_status votess_kmodel_choose(votess_kmodel*, const float*, int64_t, float, uint8_t*, void*) { return fail(VOTESS_EINVAL, "n/a"); }
}
