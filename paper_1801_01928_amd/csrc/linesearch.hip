// Terms of the exact line search of Riemannian tensor completion: for a
// tangent TT P (the projected gradient) the values p_m = P(i^m) at the
// observed entries come from the gather kernels, then
//   out[0] = sum_m p_m^2,   out[1] = sum_m (y_m - t_m) p_m,
// from which the minimiser of the linearised observed loss along -P is
// out[1] / out[0].  The values p_m come from the prefix/suffix-table gather
// when P's two tables have fewer rows than there are entries (and fit in
// 1 GiB), else from the chain gather.  Sums: per-thread partials over a
// fixed grid, wave and block sums, then one wave adds the block partials in
// a fixed order, so the result is deterministic.
#include "common.h"
#include "kernels.h"

namespace ttgfx {

namespace {

constexpr int kLsThreads = 256;
constexpr int kLsBlocks = 512;

__device__ __forceinline__ float wave_sum64(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ void __launch_bounds__(kLsThreads)
    ls_partial_kernel(const float *__restrict__ p, const float *__restrict__ y, const float *__restrict__ t,
                      long long M, float *__restrict__ part) {
  __shared__ float red[2][kLsThreads / 64];
  float pp = 0.f, rp = 0.f;
  for (long long m = (long long)blockIdx.x * kLsThreads + threadIdx.x; m < M;
       m += (long long)gridDim.x * kLsThreads) {
    const float v = p[m];
    pp = fmaf(v, v, pp);
    rp = fmaf(y[m] - t[m], v, rp);
  }
  pp = wave_sum64(pp);
  rp = wave_sum64(rp);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = pp;
    red[1][w] = rp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = 0.f, b = 0.f;
    for (int i = 0; i < kLsThreads / 64; ++i) {
      a += red[0][i];
      b += red[1][i];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

// One wave: out[c] = sum over blocks of part[2 b + c], lanes strided, then
// a fixed butterfly.
__global__ void ls_final_kernel(const float *__restrict__ part, int nblk, float *__restrict__ out) {
  const int lane = threadIdx.x;
  float a = 0.f, b = 0.f;
  for (int i = lane; i < nblk; i += 64) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  a = wave_sum64(a);
  b = wave_sum64(b);
  if (lane == 0) {
    out[0] = a;
    out[1] = b;
    out[2] = (a > 0.f) ? b / a : 0.f;  // minimiser of the linearised loss along -P
  }
}

int ls_blocks(long long M) {
  const long long want = (M + kLsThreads - 1) / kLsThreads;
  return (int)(want < kLsBlocks ? want : kLsBlocks);
}

// Table gather for P at M entries: split and table bytes, or false.
bool ls_halves(const tt_tensor *P, int64_t M, int &split, size_t &bytes) {
  if (P->d < 2) return false;
  split = halves_split_of(P);
  long long rows = 0;
  if (halves_bytes(P, split, &bytes, &rows) != TT_OK) return false;
  return rows < M && bytes <= ((size_t)1 << 30);
}

}  // namespace

size_t line_search_ws(const tt_tensor *P, int64_t M) {
  size_t b = arena_bytes<float>((size_t)M);
  b += arena_bytes<float>(2 * (size_t)kLsBlocks);
  int split = 0;
  size_t tb = 0;
  if (ls_halves(P, M, split, tb))
    b += arena_bytes<char>(tb);
  else
    b += gather_dispatch_ws(P, M) + 256;
  return b;
}

int line_search(const tt_tensor *P, const int32_t *idx, int64_t M, const float *y, const float *t, float *out,
                void *ws, size_t ws_bytes, hipStream_t s) {
  Arena ar(ws, ws_bytes);
  float *pv = ar.take<float>((size_t)M);
  float *part = ar.take<float>(2 * (size_t)kLsBlocks);
  int split = 0;
  size_t tb = 0;
  const bool tables = ls_halves(P, M, split, tb);
  const size_t gws = tables ? tb : gather_dispatch_ws(P, M);
  void *gw = ar.take<char>(gws);
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "line search: workspace too small");
  const int nblk = M > 0 ? ls_blocks(M) : 0;
  int rc = TT_OK;
  if (M > 0) {
    if (tables) {
      if ((rc = halves_build(P, split, gw, s))) return rc;
      if ((rc = halves_gather(P, split, gw, idx, M, pv, s))) return rc;
    } else if ((rc = gather_dispatch(P, idx, M, pv, gw, gws, s))) {
      return rc;
    }
    hipLaunchKernelGGL(ls_partial_kernel, dim3(nblk), dim3(kLsThreads), 0, s, pv, y, t, (long long)M, part);
    if ((rc = launch_check("line search partials"))) return rc;
  }
  hipLaunchKernelGGL(ls_final_kernel, dim3(1), dim3(64), 0, s, part, nblk, out);
  return launch_check("line search sum");
}

}  // namespace ttgfx
