// Slice-grouped MFMA gather / adjoint (gather_mfma.hip).
#pragma once
#include "common.h"

namespace ttgfx {

#define MF_MAX_D 16

// Per rank class: entries per tile, largest mode size, permutation capacity.
template <int R>
struct MfTraits;
template <>
struct MfTraits<16> {
  static constexpr int T = 1024;
  static constexpr int THREADS = 512;
  static constexpr int MAX_N = 16;
  static constexpr int PERM_CAP = 16384;
};
template <>
struct MfTraits<32> {
  static constexpr int T = 512;
  static constexpr int THREADS = 256;
  static constexpr int MAX_N = 10;
  static constexpr int PERM_CAP = 7168;
};

// True when every descriptor fits the MFMA kernels (2 <= d <= 16, ranks <= 32,
// mode sizes within the rank class's limit).
bool mfma_supported(const tt_tensor *L, const tt_tensor *R);
int mfma_rank_class(const tt_tensor *L, const tt_tensor *R);
size_t mfma_ws(const tt_tensor *X, int R, int64_t M, bool adjoint);
// mode: 0 gather (y), 1 adjoint with weights gy, 2 fused MSE (t -> y, loss, O)
int mfma_run(int mode, const tt_tensor *L, const tt_tensor *R, tt_tensor *O, const int32_t *idx,
             int64_t M, const float *t, const float *gy, float *y, float *gout, float *loss, void *ws,
             size_t ws_bytes, hipStream_t s);

}  // namespace ttgfx
