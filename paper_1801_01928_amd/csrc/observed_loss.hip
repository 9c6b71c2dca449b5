// Per-entry losses over the observed entries and their gradients: the
// completion use case of the Introduction with the squared residual or
// another per-entry loss phi.  L = (1/M) sum_m phi(y_m, t_m) and
// g_m = phi'(y_m, t_m) / M; the Riemannian gradient of L (Riemannian
// Geometry Operations) is then the sparse projection of g.
//   squared:  phi = (y - t)^2
//   Huber:    r = y - t, phi = r^2 / 2 for |r| <= delta, else delta (|r| - delta / 2)
//   logistic: labels t in {-1, +1}, phi = log(1 + exp(-t y))
// One thread per entry; per-block partial sums of phi, then one block sums
// the partials in a fixed order (deterministic).
#include "common.h"

namespace ttgfx {
namespace {

constexpr int kLossBlock = 256;

__device__ __forceinline__ float block_reduce(float v, float *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  float s = 0.f;
  for (int w = 0; w < kLossBlock / 64; ++w) s += red[w];
  return s;
}

// log(1 + exp(-z)) without overflow: for z < 0 it is -z + log(1 + exp(z)).
__device__ __forceinline__ float softplus_neg(float z) {
  return (z >= 0.f) ? log1pf(expf(-z)) : -z + log1pf(expf(z));
}

__global__ void __launch_bounds__(kLossBlock) observed_loss_kernel(const float *__restrict__ y,
                                                                   const float *__restrict__ t, long long M,
                                                                   int kind, float delta, float inv_m,
                                                                   float *__restrict__ g, float *__restrict__ part) {
  __shared__ float red[kLossBlock / 64];
  const long long m = (long long)blockIdx.x * kLossBlock + threadIdx.x;
  float phi = 0.f;
  if (m < M) {
    const float yv = y[m], tv = t[m];
    float dphi;
    if (kind == TT_LOSS_SQUARED) {
      const float r = yv - tv;
      phi = r * r;
      dphi = 2.f * r;
    } else if (kind == TT_LOSS_HUBER) {
      const float r = yv - tv, a = fabsf(r);
      if (a <= delta) {
        phi = 0.5f * r * r;
        dphi = r;
      } else {
        phi = delta * (a - 0.5f * delta);
        dphi = copysignf(delta, r);
      }
    } else {  // logistic
      const float z = tv * yv;
      phi = softplus_neg(z);
      // phi' = -t / (1 + exp(t y)), written to stay finite for large |z|
      const float e = expf(-fabsf(z));
      const float sig = (z >= 0.f) ? e / (1.f + e) : 1.f / (1.f + e);  // 1 / (1 + exp(z))
      dphi = -tv * sig;
    }
    if (g) g[m] = dphi * inv_m;
  }
  const float s = block_reduce(phi, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kLossBlock) observed_loss_final(const float *__restrict__ part, long long nb,
                                                                  float inv_m, float *__restrict__ loss) {
  __shared__ float red[kLossBlock / 64];
  float v = 0.f;
  for (long long i = threadIdx.x; i < nb; i += kLossBlock) v += part[i];
  const float s = block_reduce(v, red);
  if (threadIdx.x == 0) loss[0] = s * inv_m;
}

}  // namespace
}  // namespace ttgfx

using namespace ttgfx;

extern "C" {

int64_t tt_observed_loss_workspace(int64_t M) {
  if (M < 0) return set_error(TT_ERR_ARG, "M = %lld is negative", (long long)M);
  const long long nb = (M + kLossBlock - 1) / kLossBlock;
  return (int64_t)arena_bytes<float>((size_t)(nb > 0 ? nb : 1));
}

int tt_observed_loss(const float *y, const float *t, int64_t M, int kind, float delta, float *g, float *loss,
                     void *ws, size_t ws_bytes, void *stream) {
  if (M < 0) return set_error(TT_ERR_ARG, "M = %lld is negative", (long long)M);
  if (kind != TT_LOSS_SQUARED && kind != TT_LOSS_HUBER && kind != TT_LOSS_LOGISTIC)
    return set_error(TT_ERR_ARG, "observed_loss: unknown kind %d", kind);
  if (kind == TT_LOSS_HUBER && !(delta > 0.f)) return set_error(TT_ERR_ARG, "observed_loss: Huber delta must be > 0");
  if (M > 0 && (!y || !t)) return set_error(TT_ERR_ARG, "observed_loss: null y or t with M = %lld", (long long)M);
  if (!loss) return set_error(TT_ERR_ARG, "observed_loss: null loss");
  const int64_t need = tt_observed_loss_workspace(M);
  if (!ws || ws_bytes < (size_t)need)
    return set_error(TT_ERR_WORKSPACE, "observed_loss: workspace of %zu bytes, %lld needed", ws_bytes,
                     (long long)need);
  hipStream_t s = (hipStream_t)stream;
  const long long nb = (M + kLossBlock - 1) / kLossBlock;
  Arena ar(ws, ws_bytes);
  float *part = ar.take<float>((size_t)(nb > 0 ? nb : 1));
  const float inv_m = M > 0 ? 1.0f / (float)M : 0.f;
  if (nb > 0) {
    hipLaunchKernelGGL(observed_loss_kernel, dim3((unsigned)nb), dim3(kLossBlock), 0, s, y, t, (long long)M, kind,
                       delta, inv_m, g, part);
    int rc = launch_check("observed loss");
    if (rc) return rc;
  }
  hipLaunchKernelGGL(observed_loss_final, dim3(1), dim3(kLossBlock), 0, s, part, nb, inv_m, loss);
  return launch_check("observed loss sum");
}

}  // extern "C"
