// C ABI of the TT-matrix layer.
#include "common.h"
#include "ttm.h"

using namespace ttgfx;

extern "C" {

int tt_matmul_set_path(int32_t path) {
  if (path < TTM_PATH_AUTO || path > TTM_PATH_DENSE)
    return set_error(TT_ERR_ARG, "tt_matmul_set_path: %d is not 0 (automatic), 1 (chain) or 2 (dense)", path);
  ttm_set_path(path);
  return TT_OK;
}

int32_t tt_matmul_path(const tt_matrix *W, int64_t B, int dtype) {
  TTMDims D;
  const int rc = ttm_validate(W, B, dtype, &D);
  if (rc) return rc;
  return ttm_path_of(D, B);
}

int64_t tt_matmul_workspace(const tt_matrix *W, int64_t B, int dtype) {
  TTMDims D;
  const int rc = ttm_validate(W, B, dtype, &D);
  if (rc) return rc;
  return (int64_t)ttm_ws(D, B, dtype, 1);
}

int tt_matmul(const tt_matrix *W, const void *X, int64_t B, float *Y, int dtype, void *ws, size_t ws_bytes,
              void *stream) {
  TTMDims D;
  int rc = ttm_validate(W, B, dtype, &D);
  if (rc) return rc;
  if (B > 0 && (!X || !Y)) return set_error(TT_ERR_ARG, "tt_matmul: null X or Y");
  if (B == 0) return TT_OK;
  const size_t need = ttm_ws(D, B, dtype, 0);
  if (!ws || ws_bytes < need)
    return set_error(TT_ERR_WORKSPACE, "tt_matmul: workspace of %zu bytes given, %zu required",
                     ws ? ws_bytes : (size_t)0, need);
  return ttm_forward(D, W->data, X, B, Y, dtype, ws, ws_bytes, (hipStream_t)stream);
}

int tt_matmul_backward(const tt_matrix *W, const void *X, int64_t B, const void *dY, float *dX, float *dWdata,
                       int dtype, void *ws, size_t ws_bytes, void *stream) {
  TTMDims D;
  int rc = ttm_validate(W, B, dtype, &D);
  if (rc) return rc;
  if (!dX && !dWdata) return TT_OK;
  if (B > 0 && !dY) return set_error(TT_ERR_ARG, "tt_matmul_backward: null dY");
  if (B > 0 && dWdata && !X) return set_error(TT_ERR_ARG, "tt_matmul_backward: null X with dW requested");
  const size_t need = ttm_ws(D, B, dtype, 1);
  if (!ws || ws_bytes < need)
    return set_error(TT_ERR_WORKSPACE, "tt_matmul_backward: workspace of %zu bytes given, %zu required",
                     ws ? ws_bytes : (size_t)0, need);
  return ttm_backward(D, W->data, X, B, dY, dX, dWdata, dtype, ws, ws_bytes, (hipStream_t)stream);
}

}  // extern "C"
