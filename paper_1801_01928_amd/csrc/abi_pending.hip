// Entry points whose kernels are not built yet: they validate nothing and
// report TT_ERR_UNSUPPORTED so that the exported symbol set is complete.
#include "common.h"

using namespace ttgfx;

extern "C" {
int tt_plan_create(const tt_batch *, const int32_t *, const float *, const int64_t *,
                   const tt_batch *, float *, tt_plan **plan) {
  if (plan) *plan = nullptr;
  return set_error(TT_ERR_UNSUPPORTED, "tt_plan_create: not available in this build");
}
int tt_plan_run(tt_plan *, void *) { return set_error(TT_ERR_UNSUPPORTED, "tt_plan_run: not available"); }
int tt_plan_capture(tt_plan *, void *) { return set_error(TT_ERR_UNSUPPORTED, "tt_plan_capture: not available"); }
int tt_plan_run_plain(tt_plan *, void *) { return set_error(TT_ERR_UNSUPPORTED, "tt_plan_run_plain: not available"); }
void tt_plan_destroy(tt_plan *) {}
int64_t tt_matmul_workspace(const tt_matrix *, int64_t, int) { return set_error(TT_ERR_UNSUPPORTED, "tt_matmul: not available"); }
int tt_matmul(const tt_matrix *, const void *, int64_t, float *, int, void *, size_t, void *) {
  return set_error(TT_ERR_UNSUPPORTED, "tt_matmul: not available");
}
int tt_matmul_backward(const tt_matrix *, const void *, int64_t, const void *, float *, float *, int,
                       void *, size_t, void *) {
  return set_error(TT_ERR_UNSUPPORTED, "tt_matmul_backward: not available");
}
}
