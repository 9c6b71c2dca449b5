/*
 * ttgfx.h -- C ABI of the MI355X (gfx950) TT-completion hot path.
 *
 * Operations follow the T3F paper (Novikov et al., arXiv 1801.01928):
 *   - the TT format and its entry formula (Introduction),
 *   - the library shape "one or two TT objects in, a TT or a number out" and
 *     batches of TT objects (Implementation Details, Batch Processing),
 *   - rounding t3f.round(x, max_tt_rank) (Implementation Details),
 *   - the tangent-space projection P_X, project_sum, the Gram matrix and
 *     Riemannian gradients (Riemannian Geometry Operations),
 *   - the TT-matrix layer t3f.matmul(tt_matrix, x) (Implementation Details).
 * Where the paper only names an operation, the standard algorithm of the TT
 * literature it cites is used (QR sweeps and TT-SVD rounding; tangent
 * parametrisation by left/right orthonormal cores with a gauge condition).
 *
 * Conventions for every entry point
 *   - Pointers marked (dev) are device memory owned by the CALLER; pointers
 *     marked (host) are host memory read during the call only.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the
 *     default stream), never synchronizes and never allocates device memory
 *     (scratch comes from the caller's workspace `ws` of `ws_bytes`; query
 *     its size with the matching *_workspace function).  Exceptions: the
 *     plan API (tt_plan_*) owns device memory allocated in tt_plan_create.
 *   - Return value: TT_OK (0) or a negative TT_ERR_* code; the message of the
 *     last failure of the calling thread is in tt_last_error().  Arguments are
 *     validated on the host before any HIP call; on a validation error no
 *     device work is queued and no output is touched.
 *   - M = 0 (no observed entries) is a successful no-op that still writes
 *     well-defined outputs (zero gradients, zero loss).
 *   - Indices outside [0, n_k) are undefined behaviour in every entry point
 *     except tt_check_indices, which finds them (checked mode).
 *   - Floating point is float32 on the device (the oracle is float64).
 */
#ifndef TTGFX_H
#define TTGFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TTGFX_VERSION 1
#define TT_MAX_D 32       /* modes per tensor */
#define TT_MAX_RANK 64    /* largest input bond rank (tt_matvec's outputs: products of two) */
#define TT_MAX_N 4096     /* largest mode size */

enum {
  TT_OK = 0,
  TT_ERR_ARG = -1,          /* null pointer, negative size, d out of range     */
  TT_ERR_SHAPE = -2,        /* rank or size mismatch between descriptors       */
  TT_ERR_UNSUPPORTED = -3,  /* rank/mode size beyond what the kernels support   */
  TT_ERR_WORKSPACE = -4,    /* workspace missing or smaller than required       */
  TT_ERR_HIP = -5,          /* HIP launch or runtime error                      */
  TT_ERR_INDEX = -6         /* out-of-range index (tt_check_indices, checked mode) */
};

enum { TT_LR = 0, TT_RL = 1 };  /* orthogonalization direction */

/*
 * A TT tensor (Introduction, TT format): d cores, core k of shape
 * r[k] x n[k] x r[k+1] with r[0] = r[d] = 1, stored row-major
 * ([r_k][n_k][r_{k+1}], the paper's index order G^k_{alpha_{k-1} i_k alpha_k})
 * at data + off[k] (off == NULL: cores packed back to back in mode order).
 * n, r, off are host arrays; data is (dev).  Entry (i_1..i_d) is the product
 * of the slices G^1[i_1] ... G^d[i_d].
 */
typedef struct {
  int32_t d;              /* 1 <= d <= TT_MAX_D                       */
  const int32_t *n;       /* (host) [d]   mode sizes, 1 <= n_k         */
  const int32_t *r;       /* (host) [d+1] bond ranks, r[0] = r[d] = 1  */
  const int64_t *off;     /* (host) [d]   element offsets or NULL      */
  float *data;            /* (dev) core storage                        */
} tt_tensor;

/* A batch of TT tensors with the same mode sizes; ranks may differ per
 * tensor (Batch Processing; uneven ranks are an extension). */
typedef struct {
  int32_t b;              /* number of tensors                          */
  const tt_tensor *tt;    /* (host) [b]                                 */
} tt_batch;

/* The same descriptors with float64 cores, for the double-precision
 * variants of Table 1's operations (the paper times them in double). */
typedef struct {
  int32_t d;
  const int32_t *n;
  const int32_t *r;
  const int64_t *off;
  double *data;           /* (dev) float64 core storage                 */
} tt_tensor_f64;
typedef struct {
  int32_t b;
  const tt_tensor_f64 *tt;
} tt_batch_f64;

/* ------------------------------------------------------------------ A1 */
/* Gather (Introduction, entry formula): y[m] = G^1[i_1^m] ... G^d[i_d^m].
 * idx: (dev) int32 structure-of-arrays [d][M] (mode k of entry m at
 * idx[k*M + m]); y: (dev) [M].  Ranks up to TT_MAX_RANK. */
int64_t tt_gather_workspace(const tt_tensor *X, int64_t M);
int tt_gather(const tt_tensor *X, const int32_t *idx, int64_t M, float *y,
              void *ws, size_t ws_bytes, void *stream);

/* --------------------------------------- gather by prefix/suffix tables */
/* The same values as tt_gather (the entry formula of the Introduction),
 * computed by regrouping the slice product: cut at bond `split`
 * (1 <= split <= d-1, 0-based modes 0..split-1 on the left), each entry is
 * the dot of its prefix product G^0[i_0]..G^{split-1}[i_{split-1}] and its
 * suffix product G^{split}[i_split]..G^{d-1}[i_{d-1}].  tt_halves_build
 * tabulates every prefix (prod_{k<split} n_k rows) and every suffix
 * (prod_{k>=split} n_k rows) of r[split] floats each; tt_halves_gather then
 * takes one r[split]-dot per entry.  This pays when M exceeds the table
 * rows; the tables depend only on X, so one build serves any number of
 * gathers until X changes.
 *   tt_halves_split: the split minimising the table size (d >= 2).
 *   tt_halves_bytes: bytes of the (dev) table buffer for that split, or a
 *     negative error (TT_ERR_UNSUPPORTED when a table level would exceed
 *     2^30 rows or reach 2^23 tiles of 64 x 64 outputs).
 *   tt_halves_build: fills `tables` (caller-owned, >= tt_halves_bytes).
 *   tt_halves_gather: y[m] as tt_gather, reading tables built for the same
 *     X shape and split; idx and y as for tt_gather.  An entry with an index
 *     outside [0, n_k) yields 0 (no out-of-bounds table read).
 * Summation differs from tt_gather only in order (float32 rounding). */
int32_t tt_halves_split(const tt_tensor *X);
int64_t tt_halves_bytes(const tt_tensor *X, int32_t split);
int tt_halves_build(const tt_tensor *X, int32_t split, void *tables, size_t bytes,
                    void *stream);
int tt_halves_gather(const tt_tensor *X, int32_t split, const void *tables,
                     size_t bytes, const int32_t *idx, int64_t M, float *y,
                     void *stream);

/* ------------------------------------------------------------------ A3 */
/* Adjoint of the gather (automatic differentiation, abstract): for every
 * core k, gX^k[:, i, :] = sum over m with i_k^m = i of
 *   gy[m] * (G^1[i_1]..G^{k-1}[i_{k-1}])^T (G^{k+1}[i_{k+1}]..G^d[i_d])^T.
 * gX must have X's shape; its cores are overwritten (not accumulated).
 * Repeated multi-indices contribute once per occurrence.  Summation over
 * entries is hierarchical (per-tile sums, per-workgroup sums, then a
 * fixed-order reduction over workgroups).  For ranks <= 32 the in-tile sums
 * have a fixed order; workgroups combine their tiles with float atomics, so
 * repeated calls may differ in the last bits (relative ~1e-7). */
int64_t tt_gather_backward_workspace(const tt_tensor *X, int64_t M);
int tt_gather_backward(const tt_tensor *X, const int32_t *idx, int64_t M,
                       const float *gy, tt_tensor *gX,
                       void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ A1+A2+A3 */
/* One fused completion-loss pass: y = gather(X), loss = mean((y - t)^2),
 * g = dloss/dy = 2 (y - t) / M, gX = gather_backward(X, g).  t: (dev) [M]
 * targets; y, g: (dev) [M] or NULL; loss: (dev) one float or NULL; gX
 * overwritten as above.  g is the value vector of the sparse Euclidean
 * gradient that tt_project_sparse projects. */
int64_t tt_gather_mse_workspace(const tt_tensor *X, int64_t M);
int tt_gather_mse_backward(const tt_tensor *X, const int32_t *idx, int64_t M,
                           const float *t, float *y, float *g, float *loss,
                           tt_tensor *gX, void *ws, size_t ws_bytes,
                           void *stream);

/* --------------------------------------------------- suffix tables */
/* The slice-grouped kernels of the gather, its adjoint and the fused pass
 * take the right partials rho of an entry's last l indices,
 * G^{d-l}[i_{d-l}] .. G^{d-1}[i_{d-1}] e_0, from a table holding one row per
 * value of those indices (n_{d-l} .. n_{d-1} rows), computed once per call
 * beside the padded slices: entries that share their last l indices share
 * these products (the entry formula of the Introduction, regrouped), so the
 * right sweep starts l modes later and the adjoint reads those partials
 * from the table instead of a per-entry stash.  Levels are taken while the
 * table stays within 2 MiB and the entries outnumber the deepest level's
 * rows 16 to 1; results differ from the table-free path only in rounding.
 *   tt_set_suffix_depth: process-wide policy for later calls: -1 automatic
 *     (the default), 0 never, k > 0 up to k levels whatever M is (within the
 *     size cap and d-1).  Workspace sizes depend on it: query them after.
 *   tt_suffix_depth: the levels a fused pass (tt_gather_mse_backward) over
 *     X with M entries takes under the current policy (0 on the generic
 *     kernels), or a negative error. */
int tt_set_suffix_depth(int32_t depth);
int32_t tt_suffix_depth(const tt_tensor *X, int64_t M);

/* ------------------------------------------------ reduction policy */
/* The adjoint sums, for each core slice, the outer products of every
 * entry whose index in that mode selects the slice (the gradient of the
 * entry formula of the Introduction with respect to one core).  The
 * slice-grouped kernels of rank classes 16 and 32 sum in a fixed order
 * (per-workgroup accumulators reduced in workgroup order), so their results
 * repeat bitwise.  The batched plan's persistent kernel, the generic
 * kernels (ranks above 32, d outside 2..16) and rank class 32 with mode
 * sizes whose slice accumulator does not fit the LDS add with float
 * atomics, so the last bits of their gradients may differ between runs.
 *   tt_set_deterministic(1): later adjoint, fused-pass, projection and plan
 *     calls sum in a fixed order: plans run tensor by tensor (tt_plan_run
 *     then equals tt_plan_run_plain; a graph captured under the other
 *     policy is not replayed), and shapes that only the atomic kernels
 *     serve fail with TT_ERR_UNSUPPORTED before any device work.
 *   tt_set_deterministic(0): the default.
 *   tt_deterministic: the current policy (0 or 1).
 * The policy is process-wide and not synchronised with calls in flight on
 * other host threads. */
int tt_set_deterministic(int32_t on);
int32_t tt_deterministic(void);

/* --------------------------------------- A1+A2+A3 without a workspace */
/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * fused pass above with the same arguments and results (the same kernels),
 * minus ws/ws_bytes.  Its workspace is a fixed device array of
 * tt_gather_mse_noalloc_limit() bytes (256 MiB) held by every GPU the
 * library runs on until the process ends; the first call on a device looks
 * up that device's copy.  Shapes whose tt_gather_mse_workspace exceeds the
 * limit fail with TT_ERR_WORKSPACE before any device work.  Calls share
 * the array: calls that overlap in time on one GPU (different streams or
 * host threads without ordering) race and give undefined results; calls
 * ordered on one stream are safe.  Nothing in the array needs to start at
 * zero (the kernels initialise what they accumulate into). */
int64_t tt_gather_mse_noalloc_limit(void);
int tt_gather_mse_backward_noalloc(const tt_tensor *X, const int32_t *idx,
                                   int64_t M, const float *t, float *y,
                                   float *g, float *loss, tt_tensor *gX,
                                   void *stream);

/* ---------------------------------------------- completion line search */
/* Terms of the exact line search of Riemannian tensor completion (the
 * completion use case of the Introduction with the Riemannian gradient of
 * the Riemannian Geometry Operations section; the step rule of Riemannian
 * TT completion in the cited literature).  P: a TT (normally the projected
 * gradient, rank 2r), y: (dev) [M] values of the current iterate at the
 * observed entries, t: (dev) [M] targets, idx as for tt_gather.
 * out: (dev) float [2], written asynchronously:
 *   out[0] = sum_m P(i^m)^2,   out[1] = sum_m (y_m - t_m) P(i^m);
 * the observed loss of the first-order model X - a P is smallest at
 * a = out[1] / out[0], which is written to out[2] (0 when out[0] = 0), so
 * that the step can feed tt_tangent_combine_dev without a host round trip.
 * out: (dev) float [3].  Sums are in a fixed order (deterministic).
 * M = 0 writes {0, 0, 0}. */
int64_t tt_line_search_workspace(const tt_tensor *P, int64_t M);
int tt_line_search(const tt_tensor *P, const int32_t *idx, int64_t M,
                   const float *y, const float *t, float *out,
                   void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------- checked mode */
/* Index check.  The entry formula (Introduction) is defined for
 * 0 <= i_k < n_k only, and the entry points above do not test their
 * indices; a caller that cannot trust them runs this first.
 * X: only d and n are read (data may be any non-null pointer).
 * idx: (dev) int32 [d][M] as above.  out: (dev) int64 [2], written
 * asynchronously: out[0] = number of entries m with some idx[k*M + m]
 * outside [0, n_k); out[1] = the smallest such m, or M when there is none.
 * M = 0 writes {0, 0}.  Reads idx once; no workspace; capturable.  The
 * caller turns a nonzero out[0] into TT_ERR_INDEX (the Python binding does
 * so before every call that takes indices when TTGFX_CHECKED=1). */
int tt_check_indices(const tt_tensor *X, const int32_t *idx, int64_t M,
                     int64_t *out, void *stream);

/* ------------------------------------------------------------------ A4 */
/* Orthogonalization sweep (QR sweeps of the TT literature the paper cites;
 * needed by rounding and the tangent projection).
 * TT_LR: for k = 1..d-1, Householder QR of reshape(G^k, r_{k-1} n_k x r_k)
 *   with diag(R) >= 0; out^k = Q (left-orthonormal), R pushed into G^{k+1}.
 * TT_RL: mirror, LQ of reshape(G^k, r_{k-1} x n_k r_k) with diag(L) >= 0,
 *   for k = d..2; out^k right-orthonormal, L pushed into G^{k-1}.
 * out ranks are min(r_{k-1} n_k, r_k) (LR) / min(r_k, n_k r_{k+1}) (RL)
 * chained along the sweep; compute them with tt_orthogonalize_ranks and
 * give `out` exactly those ranks.  The tensor represented is unchanged. */
int tt_orthogonalize_ranks(const tt_tensor *X, int dir, int32_t *out_r /*(host)[d+1]*/);
int64_t tt_orthogonalize_workspace(const tt_tensor *X, int dir);
int tt_orthogonalize(const tt_tensor *X, int dir, tt_tensor *out,
                     void *ws, size_t ws_bytes, void *stream);

/* Both sweeps of one X in a single launch (two workgroups, each with its
 * own half of the workspace): U receives the left-to-right result and V the
 * right-to-left result, exactly as two tt_orthogonalize calls would write
 * them (the same kernels; U and V at the ranks tt_orthogonalize_ranks gives
 * for TT_LR and TT_RL).  The tangent-space operations need both. */
int64_t tt_orthogonalize_both_workspace(const tt_tensor *X);
int tt_orthogonalize_both(const tt_tensor *X, tt_tensor *U, tt_tensor *V,
                          void *ws, size_t ws_bytes, void *stream);

/* --------------------------------------------------------------- A5+A6 */
/* Tangent projection of a sparse tensor (Riemannian Geometry Operations:
 * P_X Z, computed as project_sum of the M one-hot rank-1 tensors
 * z[m] e_{i^m}).  U: X after TT_LR (U^1..U^{d-1} left-orthonormal, U^d the
 * last core S_d); V: X after TT_RL (V^2..V^d right-orthonormal); both must
 * have the same ranks (X at feasible ranks).  Output W, a TT of ranks
 * (1, 2r_1, ..., 2r_{d-1}, 1), represents
 *     add_x * X + alpha * P_X(Z)          (add_x in {0, 1})
 * with cores W^1 = [alpha dG^1, U^1], W^k = [[V^k, 0], [alpha dG^k, U^k]],
 * W^d = [[V^d], [add_x S_d + alpha dG^d]], where dG are the gauge-fixed
 * tangent cores (U_k^L^T dG_k^L = 0 for k < d).  d >= 2. */
int64_t tt_project_sparse_workspace(const tt_tensor *U, int64_t M);
int tt_project_sparse(const tt_tensor *U, const tt_tensor *V,
                      const int32_t *idx, int64_t M, const float *z,
                      float alpha, int add_x, tt_tensor *W,
                      void *ws, size_t ws_bytes, void *stream);

/* Projection of a TT tensor onto the tangent space (Riemannian Geometry
 * Operations: P_B A with TT tensors A and B).  U, V: as for
 * tt_project_sparse (both sweeps of the point X, feasible ranks r); Y: any
 * TT with X's mode sizes and ranks <= 64.  W (ranks 2r, as for
 * tt_project_sparse) receives add_x X + alpha P_X(Y).  Interfaces
 * Psi_k = sum_i U^k[i]^T Psi_{k-1} Y^k[i] and
 * Phi_k = sum_i V^k[i] Phi_{k+1} Y^k[i]^T, core contractions
 * Psi_{k-1} Y^k[i] Phi_{k+1}^T, then the same gauge fix and assembly as the
 * sparse projection.  Used, e.g., to carry a tangent vector of one point
 * to the tangent space of the next. */
int64_t tt_project_tt_workspace(const tt_tensor *U, const tt_tensor *Y);
int tt_project_tt(const tt_tensor *U, const tt_tensor *V, const tt_tensor *Y,
                  float alpha, int add_x, tt_tensor *W,
                  void *ws, size_t ws_bytes, void *stream);

/* project_sum of a batch (Riemannian Geometry Operations):
 *   W = add_x X + alpha sum_i c[i] P_X(A_i),
 * one projection per batch member computed together.  The core
 * contractions are linear in A_i, so the weighted contractions are summed
 * (in batch order) before one gauge fix and assembly.  A: b >= 1 TTs with
 * X's mode sizes and one shape (equal ranks and core offsets; ranks up to
 * 64), cores anywhere in device memory; c: (host) [b] weights; U, V, W as
 * for tt_project_tt.  Launches process up to 64 members at a time. */
int64_t tt_project_sum_workspace(const tt_tensor *U, const tt_batch *A);
int tt_project_sum(const tt_tensor *U, const tt_tensor *V, const tt_batch *A,
                   const float *c, float alpha, int add_x, tt_tensor *W,
                   void *ws, size_t ws_bytes, void *stream);

/* Re-weighting of a tangent TT (Riemannian Geometry Operations: the
 * tangent vector is linear in its gauge-fixed cores).  P: the tangent TT
 * tt_project_sparse returned with alpha = 1, add_x = 0 for the point whose
 * left-orthonormal sweep is U; W (P's shape, may alias P) receives
 * add_x X + alpha P_X(Z), exactly as tt_project_sparse with these alpha
 * and add_x would return it, without repeating the sparse projection.
 * Needs no workspace. */
int tt_tangent_combine(const tt_tensor *U, const tt_tensor *P, float alpha,
                       int add_x, tt_tensor *W, void *stream);
/* The same with the coefficient read on the device: alpha = scale * (*alpha)
 * (alpha: (dev) one float, e.g. out + 2 of tt_line_search with scale = -1
 * for the completion step X - a P). */
int tt_tangent_combine_dev(const tt_tensor *U, const tt_tensor *P,
                           const float *alpha, float scale, int add_x,
                           tt_tensor *W, void *stream);

/* Tangent-space algebra for tangent vectors at one point X (Riemannian
 * Geometry Operations: elements of one tangent space add blockwise in the
 * gauge-fixed parametrisation, and the metric is that of the ambient
 * space).  A, B, W: tangent TTs in the block layout tt_project_sparse and
 * tt_project_tt produce with add_x = 0, for the point whose left-orthonormal
 * sweep is U (ranks 2 r_k of U's, same mode sizes).
 *   tt_tangent_inner: out (dev, one float) = <A, B> = sum_k <dG_k^A, dG_k^B>
 *     (exact under the gauge condition), summed in a fixed order.
 *   tt_tangent_axpby: W = a A + b B (dG blocks combined, the other blocks
 *     copied from A); W may alias A or B.
 * Used by Riemannian conjugate gradients (direction update and
 * Polak-Ribiere coefficient).  No workspace. */
int tt_tangent_inner(const tt_tensor *U, const tt_tensor *A,
                     const tt_tensor *B, float *out, void *stream);
int tt_tangent_axpby(const tt_tensor *U, float a, const tt_tensor *A, float b,
                     const tt_tensor *B, tt_tensor *W, void *stream);

/* Direction update of Riemannian conjugate gradients (the nonlinear CG of
 * Riemannian TT completion in the literature the paper cites, with the
 * Riemannian gradient of the Riemannian Geometry Operations section), all
 * scalars on the device.  xi: the projected gradient at X; Txi, Teta: the
 * previous step's gradient and direction transported to X (tt_project_tt),
 * or both NULL on the first step; prev_xi_sq: (dev) one float, <xi', xi'>
 * of the previous step (read only with Txi).  Writes eta (may alias Teta,
 * not xi or Txi) and scalars: (dev) float [5]:
 *   [0] <xi, xi>;
 *   [1] beta = max(0, (<xi, xi> - <xi, Txi>) / <xi', xi'>) (Polak-Ribiere+;
 *       0 on the first step or when <xi', xi'> <= 0);
 *   [2] 1 when eta = -xi + beta Teta was not a descent direction and was
 *       reset to -xi (beta then 0), else 0;
 *   [3] <xi, eta> before the reset;  [4] <xi, Txi> (scratch).
 * Tangent TTs as for tt_tangent_inner.  No workspace; sums in a fixed order. */
int tt_cg_direction(const tt_tensor *U, const tt_tensor *xi, const tt_tensor *Txi,
                    const tt_tensor *Teta, const float *prev_xi_sq,
                    tt_tensor *eta, float *scalars, void *stream);

/* Gram matrix of a batch of tangent vectors at one point X (Riemannian
 * Geometry Operations: the metric of the tangent space is that of the
 * ambient space; Table 1 lists the Gram matrix among the timed
 * operations).  A: b >= 1 tangent TTs in the block layout of
 * tt_tangent_inner, one shape and one set of core offsets for the whole
 * batch; U: the left-orthonormal sweep of X.  G (dev, b x b, row-major)
 * receives G[i][j] = <A_i, A_j> = sum_k <dG_k^i, dG_k^j>, exactly
 * symmetric, each entry summed in a fixed order.  The workspace holds the
 * b x S matrix of dG blocks (S = sum_k r_k n_k r_{k+1} over U's ranks). */
int64_t tt_tangent_gram_workspace(const tt_tensor *U, const tt_batch *A);
int tt_tangent_gram(const tt_tensor *U, const tt_batch *A, float *G,
                    void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------ Riemannian gradients */
/* Riemannian automatic differentiation in two bounded forms (Riemannian
 * Geometry Operations: the Riemannian gradient is the projection of the
 * Euclidean gradient onto the tangent space at X).
 *
 * tt_observed_loss: a per-entry loss over observed entries,
 * L = (1/M) sum_m phi(y_m, t_m), and g_m = phi'(y_m, t_m) / M, for
 *   TT_LOSS_SQUARED   phi = (y - t)^2;
 *   TT_LOSS_HUBER     r = y - t, phi = r^2 / 2 for |r| <= delta, else
 *                     delta (|r| - delta / 2)  (delta > 0);
 *   TT_LOSS_LOGISTIC  t in {-1, +1}, phi = log(1 + exp(-t y)).
 * y, t: (dev) [M]; g: (dev) [M] or NULL; loss: (dev) one float.  The loss
 * is summed in a fixed order.  The Riemannian gradient of L at X is
 * tt_project_sparse(U, V, idx, M, g, 1, 0, ...) with y = tt_gather(X).
 *
 * tt_riemannian_grad: the gauge-fixed tangent TT from per-core Euclidean
 * gradients Zhat_k of f in the tangent parametrisation
 * xi(dG) = sum_k U_<k dG_k V_>k at dG = 0 (what automatic differentiation
 * of f(X + xi(dG)) with respect to the dG_k returns): dG_k = Zhat_k -
 * U_k (U_k^T Zhat_k) for k < d, dG_d = Zhat_d, assembled as by
 * tt_project_sparse into W = add_x X + alpha P_X(grad f) (ranks 2 r_k).
 * Zhat: X's shape (U's ranks); U, V the two sweeps of X. */
enum { TT_LOSS_SQUARED = 0, TT_LOSS_HUBER = 1, TT_LOSS_LOGISTIC = 2 };
int64_t tt_observed_loss_workspace(int64_t M);
int tt_observed_loss(const float *y, const float *t, int64_t M, int kind,
                     float delta, float *g, float *loss, void *ws,
                     size_t ws_bytes, void *stream);
int64_t tt_riemannian_grad_workspace(const tt_tensor *U);
int tt_riemannian_grad(const tt_tensor *U, const tt_tensor *V,
                       const tt_tensor *Zhat, float alpha, int add_x,
                       tt_tensor *W, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ A7 */
/* TT rounding (t3f.round(x, max_tt_rank), Implementation Details): TT_RL
 * sweep, then left-to-right truncated SVDs of reshape(G^k, r_{k-1} n_k x r_k)
 * keeping min(max_rank, r_{k-1} n_k, r_k) leading triplets; each kept left
 * singular vector is sign-fixed (largest-magnitude component positive).
 * disc_sq: (dev) [d-1] sums of discarded squared singular values per bond,
 * or NULL.  Output ranks from tt_round_ranks. */
int tt_round_ranks(const tt_tensor *Y, int32_t max_rank, int32_t *out_r /*(host)[d+1]*/);
int64_t tt_round_workspace(const tt_tensor *Y, int32_t max_rank);
int tt_round(const tt_tensor *Y, int32_t max_rank, tt_tensor *out,
             float *disc_sq, void *ws, size_t ws_bytes, void *stream);
/* tt_round with a convergence report: status: (dev) int32 [1] or NULL,
 * receives the number of bonds whose one-sided Jacobi SVD did not converge
 * within its 40 sweeps (their factors are then used as they stand). */
int tt_round_status(const tt_tensor *Y, int32_t max_rank, tt_tensor *out,
                    float *disc_sq, int32_t *status, void *ws, size_t ws_bytes,
                    void *stream);

/* ------------------------------------------------------------------ A8 */
/* Gram matrix of two batches (Riemannian Geometry Operations; Table 1
 * 'gram'): G[a*bB + b] = <A_a, B_b> (Frobenius), B == NULL means B = A (the
 * result is then symmetric and computed once per unordered pair).
 * G: (dev) [bA][bB] row-major.  All tensors share mode sizes. */
int64_t tt_gram_workspace(const tt_batch *A, const tt_batch *B);
int tt_gram(const tt_batch *A, const tt_batch *B, float *G,
            void *ws, size_t ws_bytes, void *stream);
/* Float64 variant (Table 1 times the Gram matrix in double): the same
 * contraction on v_mfma_f64_16x16x4_f64, tt_batch_f64 members, G (dev)
 * double [bA][bB]; same rules and workspace query. */
int64_t tt_gram_f64_workspace(const tt_batch_f64 *A, const tt_batch_f64 *B);
int tt_gram_f64(const tt_batch_f64 *A, const tt_batch_f64 *B, double *G,
                void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ A9 */
/* Batched persistent gather + MSE + adjoint over many TT tensors of uneven
 * ranks (<= 32) and entry counts (Batch Processing).  X: the batch (same
 * mode sizes; 2 <= d <= 16); idx: (dev) int32, tensor j's entries are the
 * structure-of-arrays block [d][M_j] starting at element d*entry_off[j];
 * t: (dev) targets, tensor j's at t + entry_off[j]; entry_off: (host) [b+1]
 * prefix sums of M_j (entry_off[0] = 0); grads: output batch with X's shapes
 * (cores overwritten); loss: (dev) [b] per-tensor mean squared residual.
 * The pointers and shapes are bound into the plan; core VALUES may change
 * between runs.  The plan owns its device buffers (allocated here, freed by
 * tt_plan_destroy).  Gradients of one tensor are summed with float atomics
 * (run-to-run differences ~1e-7 relative).
 * tt_plan_run: padded-slice copies, zero fills (kernels), ONE persistent
 *   kernel over all tensors (work items = chunks of tiles, longest first,
 *   from an atomic queue), and the unpadding into grads.
 * tt_plan_capture: records that sequence into a hipGraph on `stream` (not
 *   the NULL stream); later tt_plan_run calls on the same stream replay it.
 *   Do not run tt_timer_start() across a capture.
 * tt_plan_run_plain: the same results by b plain tt_gather_mse_backward
 *   launch sequences (the reference that the batched form is compared with).
 * tt_plan_autotune: times every tile shape of the batched kernel (entries
 *   per tile of the rank-16 and rank-32 classes and threads per workgroup:
 *   1024/512/512, 512/512/512, 512/256/256, 1024/512/768) with every
 *   work-item chunk (1, 2, 4, 8, 16 tiles) and keeps the fastest pair;
 *   *chosen receives the chunk, tt_plan_config the whole choice.  With the
 *   environment variable TTGFX_TUNE_CACHE naming a file, choices are read
 *   from / appended to it, keyed by device architecture, CU count, d, mode
 *   sizes, tensors per rank class and the entry count's power-of-two
 *   bucket.  Drops a captured graph.
 * tt_plan_config: cfg (host) [4] = chunk, entries per tile at rank class
 *   16, at rank class 32, threads per workgroup of the plan's current
 *   launch.
 * tt_plan_set_config: sets that launch from cfg (host) [4] in the same
 *   order (the shape must be one of the four above; TT_ERR_UNSUPPORTED
 *   otherwise).  Rewrites the plan's work list with a synchronous copy:
 *   call it with no run of the plan in flight.  Drops a captured graph. */
typedef struct tt_plan tt_plan;
int tt_plan_create(const tt_batch *X, const int32_t *idx, const float *t,
                   const int64_t *entry_off, const tt_batch *grads, float *loss,
                   tt_plan **plan);
int tt_plan_run(tt_plan *plan, void *stream);
int tt_plan_capture(tt_plan *plan, void *stream);
int tt_plan_run_plain(tt_plan *plan, void *stream);
int tt_plan_autotune(tt_plan *plan, void *stream, int32_t *chosen);
int tt_plan_config(const tt_plan *plan, int32_t *cfg);
int tt_plan_set_config(tt_plan *plan, const int32_t *cfg);
void tt_plan_destroy(tt_plan *plan);

/* ----------------------------------------------------------------- A10 */
/* TT-matrix layer (t3f.matmul(tt_matrix, x), Implementation Details).
 * W (prod m_k x prod n_k) is a TT-matrix with cores of shape
 * r_k x m_k x n_k x r_{k+1} (row-major), W[(i_1..i_d),(j_1..j_d)] =
 * G^1[i_1,j_1]...G^d[i_d,j_d] with C-ordered row/column multi-indices.
 * Rows of X are input vectors: Y = X W^T, X (dev) [B][prod n], Y (dev)
 * [B][prod m].  dtype: 0 = float32 everywhere, 1 = bfloat16 inputs/cores
 * (X, cores, dY given as bf16 bit patterns) with float32 accumulation and
 * float32 outputs. */
typedef struct {
  int32_t d;
  const int32_t *m;       /* (host) [d] row (output) modes  */
  const int32_t *n;       /* (host) [d] column (input) modes */
  const int32_t *r;       /* (host) [d+1] ranks             */
  const int64_t *off;     /* (host) [d] element offsets or NULL */
  void *data;             /* (dev) cores (float32 or bf16)  */
} tt_matrix;
int64_t tt_matmul_workspace(const tt_matrix *W, int64_t B, int dtype);
int tt_matmul(const tt_matrix *W, const void *X, int64_t B, float *Y, int dtype,
              void *ws, size_t ws_bytes, void *stream);
/* dX = dY W (float32 [B][prod n]); dW cores (float32, W's shapes) =
 * gradient of <dY, X W^T>; either output may be NULL. */
int tt_matmul_backward(const tt_matrix *W, const void *X, int64_t B,
                       const void *dY, float *dX, float *dWdata, int dtype,
                       void *ws, size_t ws_bytes, void *stream);
/* Evaluation path of tt_matmul and tt_matmul_backward.  The chain contracts
 * one core per step against every row (intermediates B prod m_<k
 * prod n_>=k r_k); the dense path builds W from the left partial products
 * of the cores, runs Y = X W^T, dX = dY W and dW_dense = dY^T X on the
 * matrix cores, and takes dG^k from dW_dense by contracting it with the
 * partial products on either side of core k.  Both compute the same linear
 * map and its exact gradients (results differ in rounding; in bf16 the
 * dense path rounds W once where the chain rounds each intermediate).
 *   tt_matmul_set_path: 0 automatic (the default: dense when prod m prod n
 *     <= 2^28 and 2 B prod m prod n is below the chain's forward flops), 1
 *     chain, 2 dense (falls back to the chain when W exceeds 2^28
 *     elements).  Process-wide; workspace sizes follow it.
 *   tt_matmul_path: the path a call with this W and B takes now (1 or 2),
 *     or a negative error. */
int tt_matmul_set_path(int32_t path);
int32_t tt_matmul_path(const tt_matrix *W, int64_t B, int dtype);

/* TT-matrix by TT-vector product in the TT format (Implementation Details:
 * matrix-by-vector products of TT objects; Table 1 times it as matvec).
 * W: float32 TT-matrix, cores r_k x m_k x n_k x r_{k+1} (tt_matrix above;
 * no limit on prod m or prod n).  X: b >= 1 TT vectors of modes n_k, one
 * shape and one set of core offsets for the batch.  Y: b TT vectors (dev,
 * caller-owned) of modes m_k and ranks r_k s_k (s = X's ranks; up to
 * TT_MAX_RANK^2), receiving y_j = W x_j exactly (no rounding):
 *   Y_k[(a, b), i, (a', b')] = sum_j W_k[a, i, j, a'] X_k[b, j, b'],
 * with the bond index a s_k + b.  Every element is written; no workspace. */
int tt_matvec(const tt_matrix *W, const tt_batch *X, tt_batch *Y, void *stream);
/* TT-matrix by TT-matrix product C = A B in the TT format (Table 1's
 * matmul).  A: m_k x n_k modes, B: n_k x l_k modes (both float32, ranks up
 * to TT_MAX_RANK); C (dev, caller-owned, float32): modes m_k x l_k, ranks
 * r^A_k r^B_k, offsets from C->off or packed.  Exact:
 *   C_k[(a, b), i, l, (a', b')] = sum_j A_k[a, i, j, a'] B_k[b, j, l, b'],
 * bond index a r^B_k + b.  Every element is written; no workspace. */
int tt_matmat(const tt_matrix *A, const tt_matrix *B, tt_matrix *C, void *stream);
/* Frobenius norms of a batch of TT tensors (Table 1's norm): out (dev, [b])
 * receives ||A_j|| = sqrt(<A_j, A_j>), by the chain of r_k x r_k
 * interface matrices.  A: b >= 1 TTs of one shape and one set of core
 * offsets, ranks up to TT_MAX_RANK.  No workspace. */
int tt_norms(const tt_batch *A, float *out, void *stream);
/* Float64 variants of the three operations above, with the same layouts,
 * shapes and rules: W, A, B, C as tt_matrix with float64 cores (data is a
 * double pointer), TT vectors as tt_tensor_f64; arithmetic in float64. */
int tt_matvec_f64(const tt_matrix *W, const tt_batch_f64 *X, tt_batch_f64 *Y, void *stream);
int tt_matmat_f64(const tt_matrix *A, const tt_matrix *B, tt_matrix *C, void *stream);
int tt_norms_f64(const tt_batch_f64 *A, double *out, void *stream);

/* ---------------------------------------------------------------- misc */
/* ---------------------------------------------------------- measurement */
/* Microbenchmarks of the peaks that bound the kernels above, for reporting
 * fractions against measured as well as datasheet peaks.  kind: 0 fp32
 * matrix core (v_mfma_f32_16x16x4_f32), 1 bf16 matrix core
 * (v_mfma_f32_16x16x32_bf16), 2 fp32 vector FMA (unpacked), 3 LDS reads of
 * 16 bytes per lane, conflict-free.  tt_peak_launch queues one kernel of
 * `blocks` workgroups of 256 threads, each running `iters` iterations, on
 * `stream`; out: (dev) float [blocks * 256] (sink values).  tt_peak_work
 * returns the flop (kinds 0-2) or bytes (kind 3) of that launch, or a
 * negative value for an unknown kind. */
double tt_peak_work(int kind, int32_t blocks, int32_t iters);
int tt_peak_launch(int kind, int32_t blocks, int32_t iters, float *out, void *stream);

const char *tt_last_error(void);   /* thread-local message of the last failure */
int tt_version(void);              /* TTGFX_VERSION                            */

/* Kernel timer (measurement support, not part of any algorithm).  Between
 * tt_timer_start() and tt_timer_stop(), every entry point records a pair of
 * HIP events on its stream immediately around its dominant kernel (the
 * fused sweep kernel of the gather family, the sweep kernel of the dense
 * steps).  tt_timer_stop synchronizes those events and returns the summed
 * elapsed milliseconds and the number of timed launches.  At most 4096
 * launches are timed per start/stop pair; later ones are not recorded.
 * The events are created once and kept by the library. */
int tt_timer_start(void);
int tt_timer_stop(float *total_ms, int32_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* TTGFX_H */
