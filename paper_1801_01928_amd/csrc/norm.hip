// Frobenius norms of a batch of TT tensors (tt_norms; Table 1 times the norm).
//
// ||A||^2 = <A, A> is a chain of r_k x r_k matrices: M_0 = [1],
// M_{k+1} = sum_i G_k[i]^T M_k G_k[i], ||A|| = sqrt(M_d).  One workgroup per
// tensor keeps M, the products T_i = M_k G_k[i] of a group of slices and the
// next M in LDS.
#include <vector>

#include "common.h"

namespace ttgfx {
namespace {

constexpr int kNormBatch = 64;  // tensors per launch
constexpr int kNormThreads = 256;
constexpr int kNormRank = TT_MAX_RANK;

template <class T>
struct NormPtrs {
  const T *p[kNormBatch];
};

// T holds T_i for a group of slices at once: floor(TN / (r_k r_{k+1}))
// of them (at least 1 in float64, 2 in float32, since r_k r_{k+1} <= 4096),
// so a core costs two barriers per group instead of two per slice.
template <class T>
struct NormLds {
  static constexpr int TN = sizeof(T) == 4 ? 8192 : 4096;
};

template <class T>
__global__ void __launch_bounds__(kNormThreads) norm_kernel(TTDev A0, NormPtrs<T> np, int j0, T *__restrict__ out) {
  constexpr int TN = NormLds<T>::TN;
  __shared__ T M[kNormRank * kNormRank], N[kNormRank * kNormRank], Tq[TN], Gs[TN];
  const T *src = np.p[blockIdx.x];
  if (threadIdx.x == 0) M[0] = T(1);
  __syncthreads();
  for (int k = 0; k < A0.d; ++k) {
    const int r0 = A0.r[k], nk = A0.n[k], r1 = A0.r[k + 1];
    const int rr = r0 * r1, g = TN / rr;
    const T *G = src + A0.off[k];
    for (int e = threadIdx.x; e < r1 * r1; e += kNormThreads) N[e] = T(0);
    for (int i0 = 0; i0 < nk; i0 += g) {
      const int gi = (nk - i0) < g ? (nk - i0) : g;
      // the group's slices G_k[:, i0 .. i0 + gi, :] staged once (r0 runs of
      // gi r1 contiguous elements), Gs[(b gi + q) r1 + c]; both products
      // below then read LDS only
      const int run = gi * r1;
      for (int e = threadIdx.x; e < r0 * run; e += kNormThreads) {
        const int b = e / run, w = e - b * run;
        Gs[e] = G[((long long)b * nk + i0) * r1 + w];
      }
      __syncthreads();
      // T_q (r0 x r1) = M (r0 x r0) G_k[i0 + q] (r0 x r1)
      for (int e = threadIdx.x; e < gi * rr; e += kNormThreads) {
        const int q = e / rr, rem = e - q * rr, a = rem / r1, c = rem - a * r1;
        T acc = T(0);
        for (int b = 0; b < r0; ++b) acc = fma(M[a * r0 + b], Gs[(b * gi + q) * r1 + c], acc);
        Tq[e] = acc;
      }
      __syncthreads();
      // N (r1 x r1) += sum_q G_k[i0 + q]^T T_q, slices in order
      for (int e = threadIdx.x; e < r1 * r1; e += kNormThreads) {
        const int c = e / r1, f = e - c * r1;
        T acc = N[e];
        for (int q = 0; q < gi; ++q)
          for (int a = 0; a < r0; ++a) acc = fma(Gs[(a * gi + q) * r1 + c], Tq[q * rr + a * r1 + f], acc);
        N[e] = acc;
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < r1 * r1; e += kNormThreads) M[e] = N[e];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j0 + blockIdx.x] = sqrt(M[0] > T(0) ? M[0] : T(0));
}

// Validated batch of b TTs of one shape; data pointers of the members.
template <class T>
int run_norms(const tt_tensor *a0, int b, const T *const *data, T *out, hipStream_t s) {
  const TTDev d0 = make_dev(a0);
  for (int j0 = 0; j0 < b; j0 += kNormBatch) {
    const int m = (b - j0) < kNormBatch ? (b - j0) : kNormBatch;
    NormPtrs<T> np{};
    for (int j = 0; j < m; ++j) np.p[j] = data[j0 + j];
    hipLaunchKernelGGL(norm_kernel<T>, dim3((unsigned)m), dim3(kNormThreads), 0, s, d0, np, j0, out);
    int rc = launch_check("norms");
    if (rc) return rc;
  }
  return TT_OK;
}

int check_batch(const tt_tensor *ts, int b) {
  const tt_tensor *a0 = &ts[0];
  for (int j = 0; j < b; ++j) {
    const tt_tensor *a = &ts[j];
    int rc = validate_tt(a, "A[j]", kNormRank);
    if (rc) return rc;
    if (a->d != a0->d) return set_error(TT_ERR_SHAPE, "A[%d] must have the d of A[0]", j);
    for (int k = 0; k < a0->d; ++k)
      if (a->n[k] != a0->n[k] || a->r[k + 1] != a0->r[k + 1] || core_off(a, k) != core_off(a0, k))
        return set_error(TT_ERR_SHAPE, "A[%d] must have the modes, ranks and core offsets of A[0]", j);
  }
  return TT_OK;
}

}  // namespace
}  // namespace ttgfx

using namespace ttgfx;

extern "C" int tt_norms(const tt_batch *A, float *out, void *stream) {
  if (!A || A->b < 1 || !A->tt) return set_error(TT_ERR_ARG, "norms: empty batch");
  if (!out) return set_error(TT_ERR_ARG, "norms: null out");
  int rc = check_batch(A->tt, A->b);
  if (rc) return rc;
  std::vector<const float *> data(A->b);
  for (int j = 0; j < A->b; ++j) data[j] = A->tt[j].data;
  return run_norms<float>(&A->tt[0], A->b, data.data(), out, (hipStream_t)stream);
}

extern "C" int tt_norms_f64(const tt_batch_f64 *A, double *out, void *stream) {
  if (!A || A->b < 1 || !A->tt) return set_error(TT_ERR_ARG, "norms: empty batch");
  if (!out) return set_error(TT_ERR_ARG, "norms: null out");
  std::vector<tt_tensor> view(A->b);
  std::vector<const double *> data(A->b);
  for (int j = 0; j < A->b; ++j) {
    const tt_tensor_f64 &x = A->tt[j];
    view[j] = tt_tensor{x.d, x.n, x.r, x.off, (float *)x.data};  // shape view; data only tested for NULL
    data[j] = x.data;
  }
  int rc = check_batch(view.data(), A->b);
  if (rc) return rc;
  return run_norms<double>(&view[0], A->b, data.data(), out, (hipStream_t)stream);
}
