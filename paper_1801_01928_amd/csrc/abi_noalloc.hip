// The fused completion-loss pass without allocation: the same kernels as
// tt_gather_mse_backward, with their workspace taken from a file-scope
// device array instead of a caller buffer, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).
//
// The array lives in every GPU the library runs on, from the first use of
// the library's device code until the process ends.  Host code never passes
// the array's own name to a kernel (on the host it names a stand-in, not a
// device address): the first call on a device, with that device current,
// looks up the device address with hipGetSymbolAddress and keeps it per
// device.
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace ttgfx {
namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;  // covers d=10, n=10, r=16 at 2^20 entries
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

int scratch_of_current_device(void **out) {
  int dev = -1;
  int rc = hip_check(hipGetDevice(&dev), "gather_mse_backward_noalloc: current device");
  if (rc) return rc;
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(TT_ERR_UNSUPPORTED, "gather_mse_backward_noalloc: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "gather_mse_backward_noalloc: scratch address");
    if (rc) return rc;
    if (!p) return set_error(TT_ERR_HIP, "gather_mse_backward_noalloc: null scratch address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TT_OK;
}

}  // namespace
}  // namespace ttgfx

using namespace ttgfx;

extern "C" {

int64_t tt_gather_mse_noalloc_limit(void) { return (int64_t)kScratchBytes; }

int tt_gather_mse_backward_noalloc(const tt_tensor *X, const int32_t *idx, int64_t M, const float *t, float *y,
                                   float *g, float *loss, tt_tensor *gX, void *stream) {
  const int64_t need = tt_gather_mse_workspace(X, M);
  if (need < 0) return (int)need;  // descriptor or M rejected (message already set)
  if ((uint64_t)need > kScratchBytes)
    return set_error(TT_ERR_WORKSPACE,
                     "gather_mse_backward_noalloc: this shape needs %lld bytes of workspace, above the "
                     "fixed scratch of %zu bytes; use tt_gather_mse_backward with a caller workspace",
                     (long long)need, kScratchBytes);
  void *ws = nullptr;
  int rc = scratch_of_current_device(&ws);
  if (rc) return rc;
  return tt_gather_mse_backward(X, idx, M, t, y, g, loss, gX, ws, kScratchBytes, stream);
}

}  // extern "C"
