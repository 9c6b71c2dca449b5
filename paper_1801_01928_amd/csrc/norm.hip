// Frobenius norms of a batch of TT tensors (tt_norms; Table 1 times the norm).
//
// ||A||^2 = <A, A> is a chain of r_k x r_k matrices: M_0 = [1],
// M_{k+1} = sum_i G_k[i]^T M_k G_k[i], ||A|| = sqrt(M_d).  One workgroup per
// tensor keeps M, the products T_i = M_k G_k[i] of a group of slices and the
// next M in LDS.
#include "common.h"

namespace ttgfx {
namespace {

constexpr int kNormBatch = 64;  // tensors per launch
constexpr int kNormThreads = 256;
constexpr int kNormRank = TT_MAX_RANK;

struct NormPtrs {
  const float *p[kNormBatch];
};

// T holds T_i for a group of slices at once: floor(kNormT / (r_k r_{k+1}))
// of them (at least 2, since r_k r_{k+1} <= 4096), so a core costs two
// barriers per group instead of two per slice.
constexpr int kNormT = 8192;
__global__ void __launch_bounds__(kNormThreads) norm_kernel(TTDev A0, NormPtrs np, int j0, float *__restrict__ out) {
  __shared__ float M[kNormRank * kNormRank], N[kNormRank * kNormRank], T[kNormT];
  const float *src = np.p[blockIdx.x];
  if (threadIdx.x == 0) M[0] = 1.f;
  __syncthreads();
  for (int k = 0; k < A0.d; ++k) {
    const int r0 = A0.r[k], nk = A0.n[k], r1 = A0.r[k + 1];
    const int rr = r0 * r1, g = kNormT / rr;
    const float *G = src + A0.off[k];
    for (int e = threadIdx.x; e < r1 * r1; e += kNormThreads) N[e] = 0.f;
    for (int i0 = 0; i0 < nk; i0 += g) {
      const int gi = (nk - i0) < g ? (nk - i0) : g;
      // T_q (r0 x r1) = M (r0 x r0) G_k[i0 + q] (r0 x r1)
      for (int e = threadIdx.x; e < gi * rr; e += kNormThreads) {
        const int q = e / rr, rem = e - q * rr, a = rem / r1, c = rem - a * r1;
        float acc = 0.f;
        for (int b = 0; b < r0; ++b) acc = fmaf(M[a * r0 + b], G[((long long)b * nk + i0 + q) * r1 + c], acc);
        T[e] = acc;
      }
      __syncthreads();
      // N (r1 x r1) += sum_q G_k[i0 + q]^T T_q, slices in order
      for (int e = threadIdx.x; e < r1 * r1; e += kNormThreads) {
        const int c = e / r1, f = e - c * r1;
        float acc = N[e];
        for (int q = 0; q < gi; ++q)
          for (int a = 0; a < r0; ++a)
            acc = fmaf(G[((long long)a * nk + i0 + q) * r1 + c], T[q * rr + a * r1 + f], acc);
        N[e] = acc;
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < r1 * r1; e += kNormThreads) M[e] = N[e];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j0 + blockIdx.x] = sqrtf(fmaxf(M[0], 0.f));
}

}  // namespace
}  // namespace ttgfx

using namespace ttgfx;

extern "C" int tt_norms(const tt_batch *A, float *out, void *stream) {
  if (!A || A->b < 1 || !A->tt) return set_error(TT_ERR_ARG, "norms: empty batch");
  if (!out) return set_error(TT_ERR_ARG, "norms: null out");
  int rc;
  const tt_tensor *a0 = &A->tt[0];
  for (int j = 0; j < A->b; ++j) {
    const tt_tensor *a = &A->tt[j];
    if ((rc = validate_tt(a, "A[j]", kNormRank))) return rc;
    if (a->d != a0->d) return set_error(TT_ERR_SHAPE, "A[%d] must have the d of A[0]", j);
    for (int k = 0; k < a0->d; ++k)
      if (a->n[k] != a0->n[k] || a->r[k + 1] != a0->r[k + 1] || core_off(a, k) != core_off(a0, k))
        return set_error(TT_ERR_SHAPE, "A[%d] must have the modes, ranks and core offsets of A[0]", j);
  }
  const TTDev d0 = make_dev(a0);
  for (int j0 = 0; j0 < A->b; j0 += kNormBatch) {
    const int m = (A->b - j0) < kNormBatch ? (A->b - j0) : kNormBatch;
    NormPtrs np{};
    for (int j = 0; j < m; ++j) np.p[j] = A->tt[j0 + j].data;
    hipLaunchKernelGGL(norm_kernel, dim3((unsigned)m), dim3(kNormThreads), 0, (hipStream_t)stream, d0, np, j0, out);
    if ((rc = launch_check("norms"))) return rc;
  }
  return TT_OK;
}
