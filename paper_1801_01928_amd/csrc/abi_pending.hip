// Entry points whose kernels are not built yet: they validate nothing and
// report TT_ERR_UNSUPPORTED so that the exported symbol set is complete.
#include "common.h"

using namespace ttgfx;

extern "C" {
int64_t tt_matmul_workspace(const tt_matrix *, int64_t, int) { return set_error(TT_ERR_UNSUPPORTED, "tt_matmul: not available"); }
int tt_matmul(const tt_matrix *, const void *, int64_t, float *, int, void *, size_t, void *) {
  return set_error(TT_ERR_UNSUPPORTED, "tt_matmul: not available");
}
int tt_matmul_backward(const tt_matrix *, const void *, int64_t, const void *, float *, float *, int,
                       void *, size_t, void *) {
  return set_error(TT_ERR_UNSUPPORTED, "tt_matmul_backward: not available");
}
}
