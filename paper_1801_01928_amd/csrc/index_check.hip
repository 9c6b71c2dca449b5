// Device-side check of observed multi-indices against the mode sizes.  The
// entry formula (Introduction) is defined for 0 <= i_k < n_k only; the hot
// kernels do not test this, so a caller that cannot trust its indices runs
// this check first.  One pass over idx (4 d bytes per entry, HBM-bound).
#include "common.h"
#include "kernels.h"

namespace ttgfx {

namespace {

constexpr int kCheckThreads = 256;

struct IdxCheckArgs {
  int d;
  int n[TT_MAX_D];
};

// out[0] = 0 bad entries, out[1] = M (no bad entry yet).  A kernel, not a
// memset, so that the call can be captured into a graph.
__global__ void index_check_init(unsigned long long *out, long long M) {
  if (threadIdx.x == 0) {
    out[0] = 0ull;
    out[1] = (unsigned long long)M;
  }
}

__global__ void __launch_bounds__(kCheckThreads)
    index_check_kernel(IdxCheckArgs a, const int32_t *idx, long long M, unsigned long long *out) {
  unsigned long long bad = 0ull;
  unsigned long long first = (unsigned long long)M;
  const long long stride = (long long)gridDim.x * kCheckThreads;
  for (long long m = (long long)blockIdx.x * kCheckThreads + threadIdx.x; m < M; m += stride) {
    bool ok = true;
    for (int k = 0; k < a.d; ++k) ok &= (unsigned)idx[k * M + m] < (unsigned)a.n[k];
    if (!ok) {
      ++bad;
      first = (unsigned long long)m < first ? (unsigned long long)m : first;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    bad += __shfl_xor(bad, off);
    const unsigned long long f = __shfl_xor(first, off);
    first = f < first ? f : first;
  }
  // one lane per wave that saw a bad entry
  if ((threadIdx.x & 63) == 0 && bad) {
    atomicAdd(out, bad);
    atomicMin(out + 1, first);
  }
}

}  // namespace

int index_check(const tt_tensor *X, const int32_t *idx, long long M, int64_t *out, hipStream_t s) {
  unsigned long long *o = (unsigned long long *)out;
  hipLaunchKernelGGL(index_check_init, dim3(1), dim3(64), 0, s, o, M);
  int rc = launch_check("index check init");
  if (rc || M == 0) return rc;
  IdxCheckArgs a;
  a.d = X->d;
  for (int k = 0; k < TT_MAX_D; ++k) a.n[k] = k < X->d ? X->n[k] : 0;
  const long long want = (M + kCheckThreads - 1) / kCheckThreads;
  const int grid = (int)(want < 2048 ? want : 2048);
  hipLaunchKernelGGL(index_check_kernel, dim3(grid), dim3(kCheckThreads), 0, s, a, idx, M, o);
  return launch_check("index check");
}

}  // namespace ttgfx
