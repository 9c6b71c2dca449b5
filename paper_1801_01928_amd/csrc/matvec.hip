// TT-matrix by TT-vector product in the TT format (tt_matvec).
//
// For a TT-matrix W with cores W_k (r_k x m_k x n_k x r_{k+1}) and a TT
// vector x with cores x_k (s_k x n_k x s_{k+1}), y = W x is the TT vector
// with cores
//   y_k[(a, b), i, (a', b')] = sum_j W_k[a, i, j, a'] x_k[b, j, b'],
// of ranks r_k s_k (bond index a s_k + b) and modes m_k (Implementation
// Details: the TT-matrix by TT-vector product; Table 1 times it as matvec).
// No rounding: the product is exact and its ranks multiply.  Every output
// element is one n_k-term sum over W_k and x_k, which are small and stay in
// the caches; the bytes that must move are those of y.  This kernel gathers
// both factors per lane, which, not the bytes, limits it.
#include "common.h"

namespace ttgfx {
namespace {

constexpr int kMvBatch = 64;  // vectors per launch
constexpr int kMvThreads = 256;
constexpr int kMvPerThread = 8;  // fewer, fuller workgroups: dispatch is not the limit

struct MatDev {
  int d;
  int m[TT_MAX_D], n[TT_MAX_D], r[TT_MAX_D + 1];
  long long off[TT_MAX_D];
  const float *data;
};

struct MvIO {
  const float *x[kMvBatch];
  float *y[kMvBatch];
};

// grid (g, d, members), grid-stride over the elements of y_k for member
// blockIdx.z (g sized for about kMvPerThread elements per thread of the
// largest core): element e = (row m_k + i) R' + col, row = a s_k + b,
// col = a' s_{k+1} + b', R' = r_{k+1} s_{k+1}.
__global__ void __launch_bounds__(kMvThreads) matvec_kernel(MatDev W, TTDev X0, TTDev Y0, MvIO io) {
  const int k = blockIdx.y;
  const int r0 = W.r[k], r1 = W.r[k + 1], s0 = X0.r[k], s1 = X0.r[k + 1];
  const int mk = W.m[k], nk = W.n[k];
  // the host keeps every output core below 2^31 elements: 32-bit index
  // arithmetic
  const unsigned R1 = (unsigned)(r1 * s1);
  const unsigned cnt = (unsigned)r0 * s0 * mk * R1;
  const float *xm = io.x[blockIdx.z] + X0.off[k];
  float *yk = io.y[blockIdx.z] + Y0.off[k];
  for (unsigned e = blockIdx.x * kMvThreads + threadIdx.x; e < cnt; e += gridDim.x * kMvThreads) {
    const unsigned t = e / R1, col = e - t * R1;
    const unsigned row = t / mk, i = t - row * mk;
    const unsigned a = row / s0, b = row - a * s0, ap = col / s1, bp = col - ap * s1;
    const float *wk = W.data + W.off[k] + (((long long)a * mk + i) * nk) * r1 + ap;
    const float *xk = xm + (long long)b * nk * s1 + bp;
    float acc = 0.f;
    for (int j = 0; j < nk; ++j) acc = fmaf(wk[(long long)j * r1], xk[(long long)j * s1], acc);
    yk[e] = acc;
  }
}

int validate_matvec(const tt_matrix *W, const tt_batch *X, const tt_batch *Y, MatDev *md) {
  if (!W) return set_error(TT_ERR_ARG, "W: null descriptor");
  if (W->d < 1 || W->d > TT_MAX_D) return set_error(TT_ERR_ARG, "W: d = %d outside [1, %d]", W->d, TT_MAX_D);
  if (!W->m || !W->n || !W->r) return set_error(TT_ERR_ARG, "W: null m, n or r array");
  if (!W->data) return set_error(TT_ERR_ARG, "W: null data pointer");
  if (W->r[0] != 1 || W->r[W->d] != 1)
    return set_error(TT_ERR_SHAPE, "W: boundary ranks must be 1 (got %d, %d)", W->r[0], W->r[W->d]);
  md->d = W->d;
  md->data = (const float *)W->data;
  long long o = 0;
  for (int k = 0; k <= W->d; ++k) {
    if (W->r[k] < 1 || W->r[k] > TT_MAX_RANK)
      return set_error(TT_ERR_SHAPE, "W: r[%d] = %d outside [1, %d]", k, W->r[k], TT_MAX_RANK);
    md->r[k] = W->r[k];
  }
  for (int k = 0; k < W->d; ++k) {
    if (W->m[k] < 1 || W->n[k] < 1 || W->m[k] > TT_MAX_N || W->n[k] > TT_MAX_N)
      return set_error(TT_ERR_SHAPE, "W: mode sizes m[%d] = %d, n[%d] = %d outside [1, %d]", k, W->m[k], k,
                       W->n[k], TT_MAX_N);
    if (W->off && W->off[k] < 0) return set_error(TT_ERR_ARG, "W: negative offset for core %d", k);
    md->m[k] = W->m[k];
    md->n[k] = W->n[k];
    md->off[k] = W->off ? W->off[k] : o;
    o += (long long)W->r[k] * W->m[k] * W->n[k] * W->r[k + 1];
  }
  if (!X || X->b < 1 || !X->tt) return set_error(TT_ERR_ARG, "matvec: empty batch of vectors");
  if (!Y || Y->b != X->b || !Y->tt) return set_error(TT_ERR_ARG, "matvec: Y must hold as many TTs as X");
  int rc;
  const tt_tensor *x0 = &X->tt[0], *y0 = &Y->tt[0];
  for (int j = 0; j < X->b; ++j) {
    const tt_tensor *x = &X->tt[j], *y = &Y->tt[j];
    if ((rc = validate_tt(x, "X[j]", TT_MAX_RANK))) return rc;
    if ((rc = validate_tt(y, "Y[j]", TT_MAX_RANK * TT_MAX_RANK))) return rc;
    if (x->d != W->d || y->d != W->d) return set_error(TT_ERR_SHAPE, "X[%d], Y[%d] must have W's d", j, j);
    for (int k = 0; k < W->d; ++k) {
      if (x->n[k] != W->n[k]) return set_error(TT_ERR_SHAPE, "X[%d]: n[%d] must be W's column mode %d", j, k, W->n[k]);
      if (y->n[k] != W->m[k]) return set_error(TT_ERR_SHAPE, "Y[%d]: n[%d] must be W's row mode %d", j, k, W->m[k]);
      if (x->r[k + 1] != x0->r[k + 1]) return set_error(TT_ERR_SHAPE, "X[%d] must have the ranks of X[0]", j);
      if (y->r[k + 1] != W->r[k + 1] * x->r[k + 1])
        return set_error(TT_ERR_SHAPE, "Y[%d]: r[%d] = %d, expected %d", j, k + 1, y->r[k + 1],
                         W->r[k + 1] * x->r[k + 1]);
      if (core_off(x, k) != core_off(x0, k) || core_off(y, k) != core_off(y0, k))
        return set_error(TT_ERR_SHAPE, "X[%d], Y[%d] must have the core offsets of X[0], Y[0]", j, j);
    }
  }
  return TT_OK;
}

}  // namespace
}  // namespace ttgfx

using namespace ttgfx;

extern "C" int tt_matvec(const tt_matrix *W, const tt_batch *X, tt_batch *Y, void *stream) {
  MatDev md;
  int rc = validate_matvec(W, X, Y, &md);
  if (rc) return rc;
  const TTDev x0 = make_dev(&X->tt[0]), y0 = make_dev(&Y->tt[0]);
  long long maxcnt = 0;
  for (int k = 0; k < md.d; ++k) {
    const long long c = core_elems(&Y->tt[0], k);
    maxcnt = c > maxcnt ? c : maxcnt;
  }
  const long long gx = (maxcnt + (long long)kMvThreads * kMvPerThread - 1) / ((long long)kMvThreads * kMvPerThread);
  if (maxcnt >= (1LL << 31)) return set_error(TT_ERR_UNSUPPORTED, "matvec: an output core of 2^31 or more elements");
  for (int j0 = 0; j0 < X->b; j0 += kMvBatch) {
    const int m = (X->b - j0) < kMvBatch ? (X->b - j0) : kMvBatch;
    MvIO io{};
    for (int j = 0; j < m; ++j) {
      io.x[j] = X->tt[j0 + j].data;
      io.y[j] = Y->tt[j0 + j].data;
    }
    hipLaunchKernelGGL(matvec_kernel, dim3((unsigned)gx, (unsigned)md.d, (unsigned)m), dim3(kMvThreads), 0,
                       (hipStream_t)stream, md, x0, y0, io);
    if ((rc = launch_check("matvec"))) return rc;
  }
  return TT_OK;
}
