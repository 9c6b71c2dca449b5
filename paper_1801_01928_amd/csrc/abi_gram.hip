// C ABI of the Gram matrix of two TT batches.
#include <stdio.h>

#include <vector>

#include "common.h"
#include "gram.h"

using namespace ttgfx;

namespace {

int validate_batch(const tt_batch *X, const tt_tensor *ref, const char *name) {
  if (!X || !X->tt || X->b < 1) return set_error(TT_ERR_ARG, "%s: empty or null batch", name);
  for (int j = 0; j < X->b; ++j) {
    char nm[64];
    snprintf(nm, sizeof nm, "%s[%d]", name, j);
    int rc = validate_tt(&X->tt[j], nm, GRAM_MAX_RANK);
    if (rc) return rc;
    if (!same_modes(&X->tt[j], ref)) return set_error(TT_ERR_SHAPE, "%s: mode sizes differ from A[0]", nm);
  }
  return TT_OK;
}

}  // namespace

extern "C" {

int64_t tt_gram_workspace(const tt_batch *A, const tt_batch *B) {
  if (!A || !A->tt || A->b < 1) return set_error(TT_ERR_ARG, "A: empty or null batch");
  int rc = validate_batch(A, &A->tt[0], "A");
  if (rc) return rc;
  if (B && (rc = validate_batch(B, &A->tt[0], "B"))) return rc;
  return (int64_t)gram_ws(A, B);
}

int tt_gram(const tt_batch *A, const tt_batch *B, float *G, void *ws, size_t ws_bytes, void *stream) {
  if (!A || !A->tt || A->b < 1) return set_error(TT_ERR_ARG, "A: empty or null batch");
  int rc = validate_batch(A, &A->tt[0], "A");
  if (rc) return rc;
  if (B && (rc = validate_batch(B, &A->tt[0], "B"))) return rc;
  if (!G) return set_error(TT_ERR_ARG, "null G");
  const size_t need = gram_ws(A, B);
  if (!ws || ws_bytes < need)
    return set_error(TT_ERR_WORKSPACE, "gram: workspace of %zu bytes given, %zu required",
                     ws ? ws_bytes : (size_t)0, need);
  return gram_run(A, B, G, ws, ws_bytes, (hipStream_t)stream);
}

namespace {

// Shape views of a float64 batch (validation and offsets read only the shape).
std::vector<tt_tensor> views_of(const tt_batch_f64 *X, std::vector<const double *> &data) {
  std::vector<tt_tensor> v;
  if (!X || !X->tt) return v;
  v.resize(X->b);
  data.resize(X->b);
  for (int j = 0; j < X->b; ++j) {
    const tt_tensor_f64 &x = X->tt[j];
    v[j] = tt_tensor{x.d, x.n, x.r, x.off, (float *)x.data};
    data[j] = x.data;
  }
  return v;
}

int validate_f64(const tt_batch_f64 *A, const tt_batch_f64 *B, std::vector<tt_tensor> &av, std::vector<tt_tensor> &bv,
                 std::vector<const double *> &ad, std::vector<const double *> &bd) {
  if (!A || !A->tt || A->b < 1) return set_error(TT_ERR_ARG, "A: empty or null batch");
  if (B && (!B->tt || B->b < 1)) return set_error(TT_ERR_ARG, "B: empty or null batch");
  av = views_of(A, ad);
  tt_batch ab = {A->b, av.data()};
  int rc = validate_batch(&ab, &av[0], "A");
  if (rc) return rc;
  if (B) {
    bv = views_of(B, bd);
    tt_batch bb = {B->b, bv.data()};
    if ((rc = validate_batch(&bb, &av[0], "B"))) return rc;
  }
  return TT_OK;
}

}  // namespace

int64_t tt_gram_f64_workspace(const tt_batch_f64 *A, const tt_batch_f64 *B) {
  std::vector<tt_tensor> av, bv;
  std::vector<const double *> ad, bd;
  int rc = validate_f64(A, B, av, bv, ad, bd);
  if (rc) return rc;
  return (int64_t)gram_ws_f64(av.data(), A->b, B ? bv.data() : nullptr, B ? B->b : 0);
}

int tt_gram_f64(const tt_batch_f64 *A, const tt_batch_f64 *B, double *G, void *ws, size_t ws_bytes, void *stream) {
  std::vector<tt_tensor> av, bv;
  std::vector<const double *> ad, bd;
  int rc = validate_f64(A, B, av, bv, ad, bd);
  if (rc) return rc;
  if (!G) return set_error(TT_ERR_ARG, "null G");
  const size_t need = gram_ws_f64(av.data(), A->b, B ? bv.data() : nullptr, B ? B->b : 0);
  if (!ws || ws_bytes < need)
    return set_error(TT_ERR_WORKSPACE, "gram: workspace of %zu bytes given, %zu required",
                     ws ? ws_bytes : (size_t)0, need);
  return gram_run_f64(av.data(), A->b, ad.data(), B ? bv.data() : nullptr, B ? B->b : 0, bd.data(), G, ws,
                      ws_bytes, (hipStream_t)stream);
}

}  // extern "C"
