// Kernel selection for the gather, its adjoint and the fused MSE pass.
#include <stdlib.h>

#include "kernels.h"
#include "gather_mfma.h"

namespace ttgfx {

// The slice-grouped MFMA kernels serve ranks <= 32 (the gather alone up to
// 64) and small mode sizes; TTGFX_GENERIC=1 forces the generic
// one-lane-per-entry kernels.
static bool generic_forced() {
  static int forced = -1;
  if (forced < 0) {
    const char *e = getenv("TTGFX_GENERIC");
    forced = (e && e[0] == '1') ? 1 : 0;
  }
  return forced != 0;
}

static bool use_mfma(const tt_tensor *L, const tt_tensor *R) { return !generic_forced() && mfma_supported(L, R); }

// Deterministic mode: the adjoint must run on a slice-grouped kernel with a
// fixed-order accumulator (the generic kernels add with float atomics).
static int check_deterministic(const tt_tensor *L, const tt_tensor *R, int64_t M) {
  if (!mfma_deterministic()) return TT_OK;
  if (use_mfma(L, R) && mfma_deterministic_fits(R, mfma_rank_class(L, R), M)) return TT_OK;
  return set_error(TT_ERR_UNSUPPORTED,
                   "deterministic mode: this shape runs on kernels that add with float atomics "
                   "(ranks above 32, d outside 2..16, or mode sizes too large for the slice accumulator)");
}

// The gather alone also has a rank-64 class (0: generic kernel).
static int gather_class(const tt_tensor *X) { return generic_forced() ? 0 : mfma_gather_class(X); }

size_t gather_dispatch_ws(const tt_tensor *X, int64_t M) {
  const int rc = gather_class(X);
  return rc ? mfma_ws(X, rc, M, false) : 0;
}

int gather_dispatch(const tt_tensor *X, const int32_t *idx, int64_t M, float *y, void *ws,
                    size_t ws_bytes, hipStream_t s) {
  if (gather_class(X))
    return mfma_run(0, X, X, nullptr, idx, M, nullptr, nullptr, y, nullptr, nullptr, ws, ws_bytes, s);
  return generic_gather(make_dev(X), max_rank_of(X), idx, M, y, s);
}

size_t adjoint_dispatch_ws(const tt_tensor *X, int64_t M) {
  if (use_mfma(X, X)) return mfma_ws(X, mfma_rank_class(X, X), M, true);
  return generic_adjoint_ws(X, M);
}

size_t adjoint_dispatch_ws2(const tt_tensor *L, const tt_tensor *R, int64_t M) {
  if (use_mfma(L, R)) return mfma_ws(R, mfma_rank_class(L, R), M, true);
  return generic_adjoint_ws(R, M);
}

int adjoint_dispatch(const tt_tensor *L, const tt_tensor *R, tt_tensor *O, const int32_t *idx,
                     int64_t M, const float *w, void *ws, size_t ws_bytes, hipStream_t s) {
  int rc = check_deterministic(L, R, M);
  if (rc) return rc;
  if (use_mfma(L, R))
    return mfma_run(1, L, R, O, idx, M, nullptr, w, nullptr, nullptr, nullptr, ws, ws_bytes, s);
  int mr = max_rank_of(L);
  if (max_rank_of(R) > mr) mr = max_rank_of(R);
  return generic_adjoint(make_dev(L), make_dev(R), make_dev(O), mr, idx, M, w, ws, ws_bytes, s);
}

size_t fused_mse_ws(const tt_tensor *X, int64_t M) {
  if (use_mfma(X, X)) return mfma_ws(X, mfma_rank_class(X, X), M, true);
  const size_t m = (size_t)(M > 0 ? M : 1);
  return arena_bytes<float>(m) * 2 + mse_ws(M) + generic_adjoint_ws(X, M);
}

int fused_mse_dispatch(const tt_tensor *X, const int32_t *idx, int64_t M, const float *t, float *y,
                       float *g, float *loss, tt_tensor *gX, void *ws, size_t ws_bytes, hipStream_t s) {
  int rc0 = check_deterministic(X, X, M);
  if (rc0) return rc0;
  if (use_mfma(X, X))
    return mfma_run(2, X, X, gX, idx, M, t, nullptr, y, g, loss, ws, ws_bytes, s);
  const size_t m = (size_t)(M > 0 ? M : 1);
  Arena ar(ws, ws_bytes);
  float *ytmp = ar.take<float>(m);
  float *gtmp = ar.take<float>(m);
  if (!g) g = gtmp;
  void *mws = ar.base + align_up(ar.used, 256);
  ar.used = align_up(ar.used, 256) + mse_ws(M);
  void *aws = ar.base + align_up(ar.used, 256);
  const size_t aws_bytes = generic_adjoint_ws(X, M);
  ar.used = align_up(ar.used, 256) + aws_bytes;
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "gather_mse_backward: workspace too small");
  float *yy = y ? y : ytmp;
  int rc = generic_gather(make_dev(X), max_rank_of(X), idx, M, yy, s);
  if (rc) return rc;
  if ((rc = mse_residual(yy, t, M, g, loss, mws, mse_ws(M), s))) return rc;
  int mr = max_rank_of(X);
  return generic_adjoint(make_dev(X), make_dev(X), make_dev(gX), mr, idx, M, g, aws, aws_bytes, s);
}

}  // namespace ttgfx

using namespace ttgfx;

extern "C" {

int tt_set_suffix_depth(int32_t depth) {
  mfma_set_suffix_depth(depth);
  return TT_OK;
}

int tt_set_deterministic(int32_t on) {
  mfma_set_deterministic(on != 0);
  return TT_OK;
}

int32_t tt_deterministic(void) { return mfma_deterministic() ? 1 : 0; }

int32_t tt_suffix_depth(const tt_tensor *X, int64_t M) {
  int rc = validate_tt(X, "X", TT_MAX_RANK);
  if (rc) return rc;
  if (M < 0) return set_error(TT_ERR_ARG, "M = %lld is negative", (long long)M);
  if (!use_mfma(X, X)) return 0;
  return mfma_suffix_depth_of(X, mfma_rank_class(X, X), M);
}

}  // extern "C"
