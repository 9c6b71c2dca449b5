// Generic (any rank <= 64, any d <= 32) gather and adjoint kernels.
//
// One lane per observed entry.  The gather evaluates the entry formula of
// the TT format (Introduction): a row vector times one core slice per mode.
// The adjoint writes, for every mode k, the sum over entries of
// w_m * (left partial)^T (right partial)^T into slice i_k of core k; each
// (entry block, mode) pair is one workgroup that recomputes both partial
// products of its mode, accumulates in LDS (or in its private global partial
// when the slab is too large), and a fixed-order reduction over the
// per-block partials gives deterministic results.  These kernels back the
// shapes the specialised MFMA kernels do not cover.
#include "common.h"

namespace ttgfx {

namespace {

constexpr int kBlock = 256;
constexpr int kLdsSlabMax = 16384;  // floats (64 KiB)

struct Packed {
  long long po[TT_MAX_D + 1];  // packed element offsets of the output cores
};

// v (1 x r0) <- v * S  where S = core slice (r0 x r1), element (a, b) at
// base[a * stride + b].
template <int RM>
__device__ __forceinline__ void row_times_slice(float (&v)[RM], const float *__restrict__ base,
                                                long long stride, int r0, int r1) {
  float nv[RM];
#pragma unroll
  for (int b = 0; b < RM; ++b) nv[b] = 0.f;
#pragma unroll
  for (int a = 0; a < RM; ++a) {
    if (a < r0) {
      const float va = v[a];
      const float *row = base + a * stride;
#pragma unroll
      for (int b = 0; b < RM; ++b)
        if (b < r1) nv[b] = fmaf(va, row[b], nv[b]);
    }
  }
#pragma unroll
  for (int b = 0; b < RM; ++b) v[b] = nv[b];
}

// v (r0 x 1) <- S * v, S element (a, b) at base[a * stride + b], v has r1 rows.
template <int RM>
__device__ __forceinline__ void slice_times_col(float (&v)[RM], const float *__restrict__ base,
                                                long long stride, int r0, int r1) {
  float nv[RM];
#pragma unroll
  for (int a = 0; a < RM; ++a) {
    float acc = 0.f;
    if (a < r0) {
      const float *row = base + a * stride;
#pragma unroll
      for (int b = 0; b < RM; ++b)
        if (b < r1) acc = fmaf(row[b], v[b], acc);
    }
    nv[a] = acc;
  }
#pragma unroll
  for (int a = 0; a < RM; ++a) v[a] = nv[a];
}

template <int RM>
__global__ void __launch_bounds__(kBlock) gather_generic_kernel(TTDev X, const int32_t *__restrict__ idx,
                                                              long long M, float *__restrict__ y) {
  const long long m = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (m >= M) return;
  float v[RM];
#pragma unroll
  for (int a = 0; a < RM; ++a) v[a] = (a == 0) ? 1.f : 0.f;
  for (int k = 0; k < X.d; ++k) {
    const int i = idx[(long long)k * M + m];
    const int r0 = X.r[k], r1 = X.r[k + 1], n = X.n[k];
    const float *base = X.data + X.off[k] + (long long)i * r1;
    row_times_slice<RM>(v, base, (long long)n * r1, r0, r1);
  }
  y[m] = v[0];
}

template <int RM>
__global__ void __launch_bounds__(kBlock) adjoint_generic_kernel(TTDev L, TTDev R, TTDev O, Packed P,
                                                               const int32_t *__restrict__ idx,
                                                               long long M, const float *__restrict__ w,
                                                               float *__restrict__ partial,
                                                               long long part_stride, long long chunk,
                                                               int use_lds) {
  extern __shared__ float slab[];
  const int k = blockIdx.y;
  const int d = O.d;
  const int rl = O.r[k], rr = O.r[k + 1], nk = O.n[k];
  const int slab_elems = rl * nk * rr;
  float *mine = partial + (long long)blockIdx.x * part_stride + P.po[k];
  float *acc = use_lds ? slab : mine;
  if (use_lds) {
    for (int e = threadIdx.x; e < slab_elems; e += kBlock) slab[e] = 0.f;
    __syncthreads();
  }
  const long long m0 = (long long)blockIdx.x * chunk;
  const long long m1 = (m0 + chunk < M) ? m0 + chunk : M;
  for (long long m = m0 + threadIdx.x; m < m1; m += kBlock) {
    float lam[RM], rho[RM];
#pragma unroll
    for (int a = 0; a < RM; ++a) {
      lam[a] = (a == 0) ? 1.f : 0.f;
      rho[a] = (a == 0) ? 1.f : 0.f;
    }
    for (int j = 0; j < k; ++j) {
      const int i = idx[(long long)j * M + m];
      const int r0 = L.r[j], r1 = L.r[j + 1], n = L.n[j];
      row_times_slice<RM>(lam, L.data + L.off[j] + (long long)i * r1, (long long)n * r1, r0, r1);
    }
    for (int j = d - 1; j > k; --j) {
      const int i = idx[(long long)j * M + m];
      const int r0 = R.r[j], r1 = R.r[j + 1], n = R.n[j];
      slice_times_col<RM>(rho, R.data + R.off[j] + (long long)i * r1, (long long)n * r1, r0, r1);
    }
    const float wm = w[m];
    const int i = idx[(long long)k * M + m];
#pragma unroll
    for (int a = 0; a < RM; ++a) {
      if (a < rl) {
        const float la = wm * lam[a];
        float *row = acc + ((long long)a * nk + i) * rr;
#pragma unroll
        for (int b = 0; b < RM; ++b)
          if (b < rr) atomicAdd(row + b, la * rho[b]);
      }
    }
  }
  if (use_lds) {
    __syncthreads();
    for (int e = threadIdx.x; e < slab_elems; e += kBlock) mine[e] = slab[e];
  }
}

// out core k element e = sum over blocks b (in order) of partial[b][po[k] + e].
__global__ void reduce_partials_kernel(TTDev O, Packed P, const float *__restrict__ partial,
                                       long long part_stride, int nblk) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long total = P.po[O.d];
  if (e >= total) return;
  int k = 0;
  while (k + 1 < O.d && e >= P.po[k + 1]) ++k;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += partial[(long long)b * part_stride + e];
  O.data[O.off[k] + (e - P.po[k])] = s;
}

__global__ void fill_zero_kernel(float *p, long long count) {
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < count;
       e += (long long)gridDim.x * kBlock)
    p[e] = 0.f;
}

// Residual pass: g = 2 (y - t) / M and per-block sums of (y - t)^2.
__global__ void __launch_bounds__(kBlock) mse_kernel(const float *__restrict__ y,
                                                     const float *__restrict__ t, long long M,
                                                     float *__restrict__ g, float *__restrict__ part) {
  __shared__ float red[kBlock];
  const long long m = (long long)blockIdx.x * kBlock + threadIdx.x;
  float sq = 0.f;
  if (m < M) {
    const float rho = y[m] - t[m];
    g[m] = (2.0f / (float)M) * rho;
    sq = rho * rho;
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Single block: loss = (sum of block sums, pairwise by stride) / M.
__global__ void __launch_bounds__(kBlock) mse_final_kernel(const float *__restrict__ part, long long nb,
                                                           long long M, float *__restrict__ loss) {
  __shared__ float red[kBlock];
  float s = 0.f;
  for (long long b = threadIdx.x; b < nb; b += kBlock) s += part[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (M > 0) ? red[0] / (float)M : 0.f;
}

Packed packed_of(const TTDev &O) {
  Packed P;
  P.po[0] = 0;
  for (int k = 0; k < O.d; ++k) P.po[k + 1] = P.po[k] + (long long)O.r[k] * O.n[k] * O.r[k + 1];
  for (int k = O.d + 1; k <= TT_MAX_D; ++k) P.po[k] = P.po[O.d];
  return P;
}

int adjoint_blocks(int64_t M) {
  long long nb = (M + 4095) / 4096;
  if (nb < 1) nb = 1;
  if (nb > 96) nb = 96;
  return (int)nb;
}

}  // namespace

int fill_zero(float *p, long long count, hipStream_t s) {
  if (count <= 0) return TT_OK;
  long long nb = (count + kBlock - 1) / kBlock;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, p, count);
  return launch_check("fill_zero");
}

int generic_gather(const TTDev &X, int max_rank, const int32_t *idx, int64_t M, float *y,
                   hipStream_t s) {
  if (M == 0) return TT_OK;
  const dim3 grid((unsigned)((M + kBlock - 1) / kBlock));
  if (max_rank <= 8)
    hipLaunchKernelGGL(gather_generic_kernel<8>, grid, dim3(kBlock), 0, s, X, idx, (long long)M, y);
  else if (max_rank <= 16)
    hipLaunchKernelGGL(gather_generic_kernel<16>, grid, dim3(kBlock), 0, s, X, idx, (long long)M, y);
  else if (max_rank <= 32)
    hipLaunchKernelGGL(gather_generic_kernel<32>, grid, dim3(kBlock), 0, s, X, idx, (long long)M, y);
  else
    hipLaunchKernelGGL(gather_generic_kernel<64>, grid, dim3(kBlock), 0, s, X, idx, (long long)M, y);
  return launch_check("gather (generic)");
}

size_t generic_adjoint_ws(const tt_tensor *O, int64_t M) {
  const long long total = tt_elems(O);
  return arena_bytes<float>((size_t)adjoint_blocks(M) * total);
}

int generic_adjoint(const TTDev &L, const TTDev &R, const TTDev &O, int max_rank,
                    const int32_t *idx, int64_t M, const float *w,
                    void *ws, size_t ws_bytes, hipStream_t s) {
  const Packed P = packed_of(O);
  const long long total = P.po[O.d];
  const int nblk = adjoint_blocks(M);
  Arena ar(ws, ws_bytes);
  float *partial = ar.take<float>((size_t)nblk * total);
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "adjoint: workspace too small");
  int max_slab = 0;
  for (int k = 0; k < O.d; ++k) {
    const int sl = O.r[k] * O.n[k] * O.r[k + 1];
    if (sl > max_slab) max_slab = sl;
  }
  const int use_lds = max_slab <= kLdsSlabMax;
  if (!use_lds) {
    int rc = fill_zero(partial, (long long)nblk * total, s);
    if (rc) return rc;
  }
  const long long chunk = (M + nblk - 1) / nblk;
  const size_t shm = use_lds ? (size_t)max_slab * sizeof(float) : 0;
  const dim3 grid((unsigned)nblk, (unsigned)O.d);
  if (max_rank <= 8)
    hipLaunchKernelGGL(adjoint_generic_kernel<8>, grid, dim3(kBlock), shm, s, L, R, O, P, idx,
                       (long long)M, w, partial, total, chunk, use_lds);
  else if (max_rank <= 16)
    hipLaunchKernelGGL(adjoint_generic_kernel<16>, grid, dim3(kBlock), shm, s, L, R, O, P, idx,
                       (long long)M, w, partial, total, chunk, use_lds);
  else if (max_rank <= 32)
    hipLaunchKernelGGL(adjoint_generic_kernel<32>, grid, dim3(kBlock), shm, s, L, R, O, P, idx,
                       (long long)M, w, partial, total, chunk, use_lds);
  else
    hipLaunchKernelGGL(adjoint_generic_kernel<64>, grid, dim3(kBlock), shm, s, L, R, O, P, idx,
                       (long long)M, w, partial, total, chunk, use_lds);
  int rc = launch_check("gather_backward (generic)");
  if (rc) return rc;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((total + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, O, P, partial, total, nblk);
  return launch_check("gather_backward reduce");
}

size_t mse_ws(int64_t M) {
  const long long nb = (M + kBlock - 1) / kBlock;
  return arena_bytes<float>((size_t)(nb > 0 ? nb : 1));
}

int mse_residual(const float *y, const float *t, int64_t M, float *g, float *loss, void *ws,
                 size_t ws_bytes, hipStream_t s) {
  const long long nb = (M + kBlock - 1) / kBlock;
  Arena ar(ws, ws_bytes);
  float *part = ar.take<float>((size_t)(nb > 0 ? nb : 1));
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "mse: workspace too small");
  if (nb > 0) {
    hipLaunchKernelGGL(mse_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, y, t, (long long)M, g, part);
    int rc = launch_check("mse residual");
    if (rc) return rc;
  }
  if (loss) {
    hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(kBlock), 0, s, part, nb, (long long)M, loss);
    return launch_check("mse final");
  }
  return TT_OK;
}

}  // namespace ttgfx
