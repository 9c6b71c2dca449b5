// C ABI of the Gram matrix of two TT batches.
#include <stdio.h>
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

}  // extern "C"
