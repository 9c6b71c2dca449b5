// C ABI of the Riemannian step: orthogonalization, sparse tangent projection
// and rounding.
#include "common.h"
#include "dense.h"
#include "kernels.h"

using namespace ttgfx;

namespace {

int check_dir(int dir) {
  if (dir != TT_LR && dir != TT_RL) return set_error(TT_ERR_ARG, "dir must be TT_LR or TT_RL");
  return TT_OK;
}

int check_ranks(const tt_tensor *O, const int32_t *want, const char *what) {
  for (int k = 0; k <= O->d; ++k)
    if (O->r[k] != want[k])
      return set_error(TT_ERR_SHAPE, "%s: output rank r[%d] = %d, expected %d", what, k, O->r[k], want[k]);
  return TT_OK;
}

int check_ws(void *ws, size_t bytes, size_t need, const char *what) {
  if (need && (!ws || bytes < need))
    return set_error(TT_ERR_WORKSPACE, "%s: workspace of %zu bytes given, %zu required", what,
                     ws ? bytes : (size_t)0, need);
  return TT_OK;
}

// Zhat shares U's mode sizes and ranks; it lives in the workspace.
size_t zhat_bytes(const tt_tensor *U) { return arena_bytes<float>((size_t)tt_elems(U)); }

}  // namespace

extern "C" {

int tt_orthogonalize_ranks(const tt_tensor *X, int dir, int32_t *out_r) {
  int rc = validate_tt(X, "X", DENSE_MAX_RANK);
  if (rc) return rc;
  if ((rc = check_dir(dir))) return rc;
  if (!out_r) return set_error(TT_ERR_ARG, "null out_r");
  return dense_orth_ranks(X, dir, out_r);
}

int64_t tt_orthogonalize_workspace(const tt_tensor *X, int dir) {
  int rc = validate_tt(X, "X", DENSE_MAX_RANK);
  if (rc) return rc;
  if ((rc = check_dir(dir))) return rc;
  return (int64_t)dense_ws(X);
}

int tt_orthogonalize(const tt_tensor *X, int dir, tt_tensor *out, void *ws, size_t ws_bytes,
                     void *stream) {
  int rc = validate_tt(X, "X", DENSE_MAX_RANK);
  if (rc) return rc;
  if ((rc = check_dir(dir))) return rc;
  if ((rc = validate_tt(out, "out", DENSE_MAX_RANK))) return rc;
  if (!same_modes(X, out)) return set_error(TT_ERR_SHAPE, "out must have X's mode sizes");
  int32_t want[TT_MAX_D + 1];
  dense_orth_ranks(X, dir, want);
  if ((rc = check_ranks(out, want, "orthogonalize"))) return rc;
  if ((rc = check_ws(ws, ws_bytes, dense_ws(X), "orthogonalize"))) return rc;
  return dense_orth(X, dir, out, ws, ws_bytes, (hipStream_t)stream);
}

int64_t tt_orthogonalize_both_workspace(const tt_tensor *X) {
  int rc = validate_tt(X, "X", DENSE_MAX_RANK);
  if (rc) return rc;
  return (int64_t)(2 * dense_ws(X));
}

int tt_orthogonalize_both(const tt_tensor *X, tt_tensor *U, tt_tensor *V, void *ws, size_t ws_bytes, void *stream) {
  int rc = validate_tt(X, "X", DENSE_MAX_RANK);
  if (rc) return rc;
  if ((rc = validate_tt(U, "U", DENSE_MAX_RANK))) return rc;
  if ((rc = validate_tt(V, "V", DENSE_MAX_RANK))) return rc;
  if (!same_modes(X, U) || !same_modes(X, V)) return set_error(TT_ERR_SHAPE, "U and V must have X's mode sizes");
  int32_t want[TT_MAX_D + 1];
  dense_orth_ranks(X, TT_LR, want);
  if ((rc = check_ranks(U, want, "orthogonalize_both (U)"))) return rc;
  dense_orth_ranks(X, TT_RL, want);
  if ((rc = check_ranks(V, want, "orthogonalize_both (V)"))) return rc;
  if ((rc = check_ws(ws, ws_bytes, 2 * dense_ws(X), "orthogonalize_both"))) return rc;
  return dense_orth_both(X, U, V, ws, ws_bytes, (hipStream_t)stream);
}

int64_t tt_project_sparse_workspace(const tt_tensor *U, int64_t M) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  if (M < 0) return set_error(TT_ERR_ARG, "M = %lld is negative", (long long)M);
  return (int64_t)(zhat_bytes(U) + adjoint_dispatch_ws2(U, U, M) + tangent_ws(U));
}

int tt_project_sparse(const tt_tensor *U, const tt_tensor *V, const int32_t *idx, int64_t M,
                      const float *z, float alpha, int add_x, tt_tensor *W, void *ws,
                      size_t ws_bytes, void *stream) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  if ((rc = validate_tt(V, "V", TT_MAX_RANK))) return rc;
  if ((rc = validate_tt(W, "W", 2 * TT_MAX_RANK))) return rc;
  if (U->d < 2) return set_error(TT_ERR_ARG, "project_sparse needs d >= 2");
  if (!same_shape(U, V))
    return set_error(TT_ERR_SHAPE, "U and V must have the same modes and ranks (X at feasible ranks)");
  if (!same_modes(U, W)) return set_error(TT_ERR_SHAPE, "W must have U's mode sizes");
  for (int k = 1; k < U->d; ++k)
    if (W->r[k] != 2 * U->r[k])
      return set_error(TT_ERR_SHAPE, "W rank r[%d] = %d, expected %d", k, W->r[k], 2 * U->r[k]);
  if (add_x != 0 && add_x != 1) return set_error(TT_ERR_ARG, "add_x must be 0 or 1");
  if (M < 0) return set_error(TT_ERR_ARG, "M = %lld is negative", (long long)M);
  if (M > 0 && (!idx || !z)) return set_error(TT_ERR_ARG, "null idx or z with M > 0");
  const size_t need = zhat_bytes(U) + adjoint_dispatch_ws2(U, V, M) + tangent_ws(U);
  if ((rc = check_ws(ws, ws_bytes, need, "project_sparse"))) return rc;
  hipStream_t s = (hipStream_t)stream;
  char *base = (char *)ws;
  tt_tensor Z = {U->d, U->n, U->r, nullptr, (float *)base};
  const size_t zb = zhat_bytes(U);
  const size_t ab = adjoint_dispatch_ws2(U, V, M);
  if ((rc = adjoint_dispatch(U, V, &Z, idx, M, z, base + zb, ab, s))) return rc;
  return tangent_assemble(U, V, &Z, W, alpha, add_x, base + zb + ab, ws_bytes - zb - ab, s);
}

int64_t tt_riemannian_grad_workspace(const tt_tensor *U) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  return (int64_t)tangent_ws(U);
}

int tt_riemannian_grad(const tt_tensor *U, const tt_tensor *V, const tt_tensor *Zhat, float alpha, int add_x,
                       tt_tensor *W, void *ws, size_t ws_bytes, void *stream) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  if ((rc = validate_tt(V, "V", TT_MAX_RANK))) return rc;
  if ((rc = validate_tt(Zhat, "Zhat", TT_MAX_RANK))) return rc;
  if ((rc = validate_tt(W, "W", 2 * TT_MAX_RANK))) return rc;
  if (U->d < 2) return set_error(TT_ERR_ARG, "riemannian_grad needs d >= 2");
  if (!same_shape(U, V))
    return set_error(TT_ERR_SHAPE, "U and V must have the same modes and ranks (X at feasible ranks)");
  if (!same_shape(U, Zhat)) return set_error(TT_ERR_SHAPE, "Zhat must have the shape of U (X's cores)");
  if (!same_modes(U, W)) return set_error(TT_ERR_SHAPE, "W must have U's mode sizes");
  for (int k = 1; k < U->d; ++k)
    if (W->r[k] != 2 * U->r[k])
      return set_error(TT_ERR_SHAPE, "W rank r[%d] = %d, expected %d", k, W->r[k], 2 * U->r[k]);
  if (add_x != 0 && add_x != 1) return set_error(TT_ERR_ARG, "add_x must be 0 or 1");
  if ((rc = check_ws(ws, ws_bytes, tangent_ws(U), "riemannian_grad"))) return rc;
  return tangent_assemble(U, V, Zhat, W, alpha, add_x, ws, ws_bytes, (hipStream_t)stream);
}

static int validate_project_tt(const tt_tensor *U, const tt_tensor *V, const tt_tensor *Y) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  if ((rc = validate_tt(V, "V", TT_MAX_RANK))) return rc;
  if ((rc = validate_tt(Y, "Y", DENSE_MAX_RANK))) return rc;
  if (U->d < 2) return set_error(TT_ERR_ARG, "project_tt needs d >= 2");
  if (!same_shape(U, V))
    return set_error(TT_ERR_SHAPE, "U and V must have the same modes and ranks (X at feasible ranks)");
  if (!same_modes(U, Y)) return set_error(TT_ERR_SHAPE, "Y must have X's mode sizes");
  return TT_OK;
}

int64_t tt_project_tt_workspace(const tt_tensor *U, const tt_tensor *Y) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  if ((rc = validate_tt(Y, "Y", DENSE_MAX_RANK))) return rc;
  if (!same_modes(U, Y)) return set_error(TT_ERR_SHAPE, "Y must have X's mode sizes");
  return (int64_t)project_tt_ws(U, Y);
}

int tt_project_tt(const tt_tensor *U, const tt_tensor *V, const tt_tensor *Y, float alpha, int add_x, tt_tensor *W,
                  void *ws, size_t ws_bytes, void *stream) {
  int rc = validate_project_tt(U, V, Y);
  if (rc) return rc;
  if ((rc = validate_tt(W, "W", 2 * TT_MAX_RANK))) return rc;
  if (!same_modes(U, W)) return set_error(TT_ERR_SHAPE, "W must have U's mode sizes");
  for (int k = 1; k < U->d; ++k)
    if (W->r[k] != 2 * U->r[k])
      return set_error(TT_ERR_SHAPE, "W rank r[%d] = %d, expected %d", k, W->r[k], 2 * U->r[k]);
  if (add_x != 0 && add_x != 1) return set_error(TT_ERR_ARG, "add_x must be 0 or 1");
  if ((rc = check_ws(ws, ws_bytes, project_tt_ws(U, Y), "project_tt"))) return rc;
  return project_tt(U, V, Y, alpha, add_x, W, ws, ws_bytes, (hipStream_t)stream);
}

static int validate_project_sum(const tt_tensor *U, const tt_tensor *V, const tt_batch *A, const float *c) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  if (V && (rc = validate_tt(V, "V", TT_MAX_RANK))) return rc;
  if (U->d < 2) return set_error(TT_ERR_ARG, "project_sum needs d >= 2");
  if (V && !same_shape(U, V))
    return set_error(TT_ERR_SHAPE, "U and V must have the same modes and ranks (X at feasible ranks)");
  if (!A || A->b < 1 || !A->tt) return set_error(TT_ERR_ARG, "project_sum: empty batch");
  for (int i = 0; i < A->b; ++i) {
    if ((rc = validate_tt(&A->tt[i], "A[i]", DENSE_MAX_RANK))) return rc;
    if (!same_modes(U, &A->tt[i])) return set_error(TT_ERR_SHAPE, "A[%d] must have X's mode sizes", i);
    if (!same_shape(&A->tt[0], &A->tt[i]))
      return set_error(TT_ERR_SHAPE, "A[%d] must have the ranks of A[0] (one shape per batch)", i);
    for (int k = 0; k < A->tt[i].d; ++k)
      if (core_off(&A->tt[i], k) != core_off(&A->tt[0], k))
        return set_error(TT_ERR_SHAPE, "A[%d] must have the core offsets of A[0]", i);
  }
  if (!c) return set_error(TT_ERR_ARG, "project_sum: null weights");
  return TT_OK;
}

int64_t tt_project_sum_workspace(const tt_tensor *U, const tt_batch *A) {
  int rc = validate_project_sum(U, nullptr, A, (const float *)1);
  if (rc) return rc;
  return (int64_t)project_sum_ws(U, &A->tt[0], A->b);
}

int tt_project_sum(const tt_tensor *U, const tt_tensor *V, const tt_batch *A, const float *c, float alpha,
                   int add_x, tt_tensor *W, void *ws, size_t ws_bytes, void *stream) {
  int rc = validate_project_sum(U, V, A, c);
  if (rc) return rc;
  if ((rc = validate_tt(W, "W", 2 * TT_MAX_RANK))) return rc;
  if (!same_modes(U, W)) return set_error(TT_ERR_SHAPE, "W must have U's mode sizes");
  for (int k = 1; k < U->d; ++k)
    if (W->r[k] != 2 * U->r[k])
      return set_error(TT_ERR_SHAPE, "W rank r[%d] = %d, expected %d", k, W->r[k], 2 * U->r[k]);
  if (add_x != 0 && add_x != 1) return set_error(TT_ERR_ARG, "add_x must be 0 or 1");
  if ((rc = check_ws(ws, ws_bytes, project_sum_ws(U, &A->tt[0], A->b), "project_sum"))) return rc;
  return project_sum(U, V, A->tt, A->b, c, alpha, add_x, W, ws, ws_bytes, (hipStream_t)stream);
}

int tt_tangent_combine(const tt_tensor *U, const tt_tensor *P, float alpha, int add_x, tt_tensor *W,
                       void *stream) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  if ((rc = validate_tt(P, "P", 2 * TT_MAX_RANK))) return rc;
  if ((rc = validate_tt(W, "W", 2 * TT_MAX_RANK))) return rc;
  if (U->d < 2) return set_error(TT_ERR_ARG, "tangent_combine needs d >= 2");
  if (!same_shape(P, W)) return set_error(TT_ERR_SHAPE, "W must have P's shape");
  if (!same_modes(U, P)) return set_error(TT_ERR_SHAPE, "P must have U's mode sizes");
  for (int k = 1; k < U->d; ++k)
    if (P->r[k] != 2 * U->r[k])
      return set_error(TT_ERR_SHAPE, "P rank r[%d] = %d, expected %d", k, P->r[k], 2 * U->r[k]);
  if (add_x != 0 && add_x != 1) return set_error(TT_ERR_ARG, "add_x must be 0 or 1");
  return tangent_combine(U, P, W, alpha, add_x, (hipStream_t)stream);
}

int tt_tangent_combine_dev(const tt_tensor *U, const tt_tensor *P, const float *alpha, float scale, int add_x,
                           tt_tensor *W, void *stream) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  if ((rc = validate_tt(P, "P", 2 * TT_MAX_RANK))) return rc;
  if ((rc = validate_tt(W, "W", 2 * TT_MAX_RANK))) return rc;
  if (U->d < 2) return set_error(TT_ERR_ARG, "tangent_combine_dev needs d >= 2");
  if (!alpha) return set_error(TT_ERR_ARG, "tangent_combine_dev: null alpha");
  if (!same_shape(P, W)) return set_error(TT_ERR_SHAPE, "W must have P's shape");
  if (!same_modes(U, P)) return set_error(TT_ERR_SHAPE, "P must have U's mode sizes");
  for (int k = 1; k < U->d; ++k)
    if (P->r[k] != 2 * U->r[k])
      return set_error(TT_ERR_SHAPE, "P rank r[%d] = %d, expected %d", k, P->r[k], 2 * U->r[k]);
  if (add_x != 0 && add_x != 1) return set_error(TT_ERR_ARG, "add_x must be 0 or 1");
  return tangent_combine_dev(U, P, W, alpha, scale, add_x, (hipStream_t)stream);
}

static int check_tangent(const tt_tensor *U, const tt_tensor *P, const char *name) {
  int rc = validate_tt(P, name, 2 * TT_MAX_RANK);
  if (rc) return rc;
  if (!same_modes(U, P)) return set_error(TT_ERR_SHAPE, "%s must have U's mode sizes", name);
  for (int k = 1; k < U->d; ++k)
    if (P->r[k] != 2 * U->r[k])
      return set_error(TT_ERR_SHAPE, "%s rank r[%d] = %d, expected %d", name, k, P->r[k], 2 * U->r[k]);
  return TT_OK;
}

int tt_tangent_inner(const tt_tensor *U, const tt_tensor *A, const tt_tensor *B, float *out, void *stream) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  if (U->d < 2) return set_error(TT_ERR_ARG, "tangent_inner needs d >= 2");
  if ((rc = check_tangent(U, A, "A")) || (rc = check_tangent(U, B, "B"))) return rc;
  if (!out) return set_error(TT_ERR_ARG, "tangent_inner: null out");
  return tangent_inner(U, A, B, out, (hipStream_t)stream);
}

int tt_tangent_axpby(const tt_tensor *U, float a, const tt_tensor *A, float b, const tt_tensor *B, tt_tensor *W,
                     void *stream) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  if (U->d < 2) return set_error(TT_ERR_ARG, "tangent_axpby needs d >= 2");
  if ((rc = check_tangent(U, A, "A")) || (rc = check_tangent(U, B, "B")) || (rc = check_tangent(U, W, "W")))
    return rc;
  return tangent_axpby(U, a, A, b, B, W, (hipStream_t)stream);
}

int tt_cg_direction(const tt_tensor *U, const tt_tensor *xi, const tt_tensor *Txi, const tt_tensor *Teta,
                    const float *prev_xi_sq, tt_tensor *eta, float *scalars, void *stream) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  if (U->d < 2) return set_error(TT_ERR_ARG, "cg_direction needs d >= 2");
  if ((rc = check_tangent(U, xi, "xi")) || (rc = check_tangent(U, eta, "eta"))) return rc;
  if (!same_shape(xi, eta)) return set_error(TT_ERR_SHAPE, "eta must have xi's shape");
  if (!scalars) return set_error(TT_ERR_ARG, "cg_direction: null scalars");
  if ((Txi == nullptr) != (Teta == nullptr))
    return set_error(TT_ERR_ARG, "cg_direction: Txi and Teta must both be given or both be NULL");
  if (Txi) {
    if ((rc = check_tangent(U, Txi, "Txi")) || (rc = check_tangent(U, Teta, "Teta"))) return rc;
    if (!same_shape(xi, Txi) || !same_shape(xi, Teta))
      return set_error(TT_ERR_SHAPE, "Txi and Teta must have xi's shape");
    if (!prev_xi_sq) return set_error(TT_ERR_ARG, "cg_direction: null prev_xi_sq");
    if (eta->data == Txi->data || eta->data == xi->data)
      return set_error(TT_ERR_ARG, "cg_direction: eta may alias Teta only");
  } else if (eta->data == xi->data) {
    return set_error(TT_ERR_ARG, "cg_direction: eta must not alias xi");
  }
  return cg_direction(U, xi, Txi, Teta, prev_xi_sq, eta, scalars, (hipStream_t)stream);
}

static int validate_tangent_gram(const tt_tensor *U, const tt_batch *A) {
  int rc = validate_tt(U, "U", TT_MAX_RANK);
  if (rc) return rc;
  if (U->d < 2) return set_error(TT_ERR_ARG, "tangent_gram needs d >= 2");
  if (!A || A->b < 1 || !A->tt) return set_error(TT_ERR_ARG, "tangent_gram: empty batch");
  for (int i = 0; i < A->b; ++i) {
    if ((rc = check_tangent(U, &A->tt[i], "A[i]"))) return rc;
    for (int k = 0; k < U->d; ++k)
      if (core_off(&A->tt[i], k) != core_off(&A->tt[0], k))
        return set_error(TT_ERR_SHAPE, "A[%d] must have the core offsets of A[0]", i);
  }
  return TT_OK;
}

int64_t tt_tangent_gram_workspace(const tt_tensor *U, const tt_batch *A) {
  int rc = validate_tangent_gram(U, A);
  if (rc) return rc;
  return (int64_t)tangent_gram_ws(U, A->b);
}

int tt_tangent_gram(const tt_tensor *U, const tt_batch *A, float *G, void *ws, size_t ws_bytes, void *stream) {
  int rc = validate_tangent_gram(U, A);
  if (rc) return rc;
  if (!G) return set_error(TT_ERR_ARG, "tangent_gram: null G");
  if ((rc = check_ws(ws, ws_bytes, tangent_gram_ws(U, A->b), "tangent_gram"))) return rc;
  return tangent_gram(U, A->tt, A->b, G, ws, ws_bytes, (hipStream_t)stream);
}

int tt_round_ranks(const tt_tensor *Y, int32_t max_rank, int32_t *out_r) {
  int rc = validate_tt(Y, "Y", DENSE_MAX_RANK);
  if (rc) return rc;
  if (max_rank < 1) return set_error(TT_ERR_ARG, "max_rank must be >= 1");
  if (!out_r) return set_error(TT_ERR_ARG, "null out_r");
  return dense_round_ranks(Y, max_rank, out_r);
}

int64_t tt_round_workspace(const tt_tensor *Y, int32_t max_rank) {
  int rc = validate_tt(Y, "Y", DENSE_MAX_RANK);
  if (rc) return rc;
  if (max_rank < 1) return set_error(TT_ERR_ARG, "max_rank must be >= 1");
  return (int64_t)dense_ws(Y);
}

int tt_round(const tt_tensor *Y, int32_t max_rank, tt_tensor *out, float *disc_sq, void *ws,
             size_t ws_bytes, void *stream) {
  return tt_round_status(Y, max_rank, out, disc_sq, nullptr, ws, ws_bytes, stream);
}

int tt_round_status(const tt_tensor *Y, int32_t max_rank, tt_tensor *out, float *disc_sq, int32_t *status,
                    void *ws, size_t ws_bytes, void *stream) {
  int rc = validate_tt(Y, "Y", DENSE_MAX_RANK);
  if (rc) return rc;
  if (max_rank < 1) return set_error(TT_ERR_ARG, "max_rank must be >= 1");
  if ((rc = validate_tt(out, "out", DENSE_MAX_RANK))) return rc;
  if (!same_modes(Y, out)) return set_error(TT_ERR_SHAPE, "out must have Y's mode sizes");
  int32_t want[TT_MAX_D + 1];
  dense_round_ranks(Y, max_rank, want);
  if ((rc = check_ranks(out, want, "round"))) return rc;
  if ((rc = check_ws(ws, ws_bytes, dense_ws(Y), "round"))) return rc;
  return dense_round(Y, max_rank, out, disc_sq, status, ws, ws_bytes, (hipStream_t)stream);
}

}  // extern "C"
