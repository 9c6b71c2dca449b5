// Kernel selection for the gather, its adjoint and the fused MSE pass.
#include "kernels.h"

namespace ttgfx {

int gather_dispatch(const tt_tensor *X, const int32_t *idx, int64_t M, float *y, hipStream_t s) {
  return generic_gather(make_dev(X), max_rank_of(X), idx, M, y, s);
}

size_t adjoint_dispatch_ws(const tt_tensor *X, int64_t M) { return generic_adjoint_ws(X, M); }

int adjoint_dispatch(const tt_tensor *L, const tt_tensor *R, tt_tensor *O, const int32_t *idx,
                     int64_t M, const float *w, void *ws, size_t ws_bytes, hipStream_t s) {
  int mr = max_rank_of(L);
  if (max_rank_of(R) > mr) mr = max_rank_of(R);
  return generic_adjoint(make_dev(L), make_dev(R), make_dev(O), mr, idx, M, w, ws, ws_bytes, s);
}

size_t fused_mse_ws(const tt_tensor *X, int64_t M) {
  const size_t m = (size_t)(M > 0 ? M : 1);
  return arena_bytes<float>(m) * 2 + mse_ws(M) + adjoint_dispatch_ws(X, M);
}

int fused_mse_dispatch(const tt_tensor *X, const int32_t *idx, int64_t M, const float *t, float *y,
                       float *loss, tt_tensor *gX, void *ws, size_t ws_bytes, hipStream_t s) {
  const size_t m = (size_t)(M > 0 ? M : 1);
  Arena ar(ws, ws_bytes);
  float *ytmp = ar.take<float>(m);
  float *g = ar.take<float>(m);
  void *mws = ar.base + align_up(ar.used, 256);
  ar.used = align_up(ar.used, 256) + mse_ws(M);
  void *aws = ar.base + align_up(ar.used, 256);
  const size_t aws_bytes = adjoint_dispatch_ws(X, M);
  ar.used = align_up(ar.used, 256) + aws_bytes;
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "gather_mse_backward: workspace too small");
  float *yy = y ? y : ytmp;
  int rc = gather_dispatch(X, idx, M, yy, s);
  if (rc) return rc;
  if ((rc = mse_residual(yy, t, M, g, loss, mws, mse_ws(M), s))) return rc;
  return adjoint_dispatch(X, X, gX, idx, M, g, aws, aws_bytes, s);
}

}  // namespace ttgfx
