// Slice-grouped MFMA gather / adjoint (gather_mfma.hip).
#pragma once
#include "common.h"

namespace ttgfx {

#define MF_MAX_D 16

// Per rank class: largest mode size (slice values per sort count row).
template <int R>
struct MfTraits;
template <>
struct MfTraits<16> {
  static constexpr int MAX_N = 16;
};
template <>
struct MfTraits<32> {
  static constexpr int MAX_N = 32;
};
// Gather only (no adjoint): ranks 33..64, e.g. tangent vectors of rank-32
// points.
template <>
struct MfTraits<64> {
  static constexpr int MAX_N = 16;
};

// One tensor of the slice-grouped kernels (kernel argument or batch table).
struct MfInst {
  int d;
  int n[MF_MAX_D];
  int sbase[MF_MAX_D];     // first padded slice of mode k
  long long M;
  const int32_t *idx;      // [d][M]
  const float *gp_right;   // padded slices (right sweep), MFMA operand order
  const float *gp_left;    // padded transposed slices (left sweep)
  const float *t;          // targets (fused MSE)
  const float *gy;         // given weights (adjoint)
  float *y;                // gather output or null
  float *gout;             // dloss/dy output or null
  float *grad;             // DIRECT accumulation target [slices][R][R] (zeroed)
  float *loss;             // batched: per-tensor loss (atomic target) or null
  float inv_m2;            // 2 / M
  float inv_m;             // 1 / M
  int rclass;              // 16 or 32
  // Suffix table: right partials rho_{d-l} of every value of the last l
  // indices, l = 1..suf_depth (level l at rows suf_row0[l-1] .., R floats a
  // row, row = C-ordered id of (i_{d-l}, .., i_{d-1})).  suf_depth = 0: none.
  const float *suf;
  int suf_depth;
  int suf_row0[MF_MAX_D];
  int suf_rows[MF_MAX_D];  // rows of level l: n_{d-l} * .. * n_{d-1}
};

// Tile shape of the batched kernel: entries per tile of rank classes 16
// and 32, threads per workgroup.
struct MfBatchShape {
  int t16, t32, threads;
};
#define MF_BATCH_SHAPES 4
#define MF_BATCH_MIN_T16 512  // smallest tiles over the shapes (work-list bound)
#define MF_BATCH_MIN_T32 256

// Work item of the batched kernel: `ntile` consecutive tiles of one tensor.
struct MfWorkItem {
  int inst;
  int tile0;
  int ntile;
  int rclass;
};

struct MfBatchArgs {
  const MfInst *table;
  const MfWorkItem *items;
  int nitems;
  int *counter;            // reset to 0 before every launch
  float *stash;            // per workgroup, stash_stride floats
  long long stash_stride;
  int nb16, nb32;          // blocks-per-mode capacities of the two classes
};

MfBatchShape mfma_batch_shape(int shape);
size_t mfma_batch_lds(int shape, int d, const int *n);  // dynamic LDS bytes of the batched kernel
int mfma_batch_wgs_per_cu(int shape, int d, const int *n);
int mfma_batch_prepare();
int mfma_batch_launch(const MfBatchArgs &a, int shape, int nwg, size_t lds, hipStream_t s);
int mfma_device_cus();
// Suffix table depth of the single-tensor kernels: -1 automatic, 0 off, k > 0
// at most k levels (within the table's byte cap and the LDS), whatever M is.
void mfma_set_suffix_depth(int depth);
// Deterministic mode: shapes whose adjoint would add with float atomics are
// refused; the batched plan runs tensor by tensor.
void mfma_set_deterministic(bool on);
bool mfma_deterministic();
// True when the adjoint of rank class R over X has a fixed-order accumulator
// (class 16 always; class 32 when the slice slab fits the LDS).
bool mfma_deterministic_fits(const tt_tensor *X, int R, int64_t M);
int mfma_suffix_depth_of(const tt_tensor *X, int R, int64_t M);

// True when every descriptor fits the MFMA kernels (2 <= d <= 16, ranks <= 32,
// mode sizes within the rank class's limit).
bool mfma_supported(const tt_tensor *L, const tt_tensor *R);
int mfma_rank_class(const tt_tensor *L, const tt_tensor *R);
bool mfma_class_fits(const tt_tensor *X, int R);
int mfma_gather_class(const tt_tensor *X);  // 16, 32 or 64 for the gather alone; 0 if none fits
size_t mfma_ws(const tt_tensor *X, int R, int64_t M, bool adjoint);
// padded slice copies (right: G, left: G^T of Lt or Rt) and the unpad copy
int mfma_pad(const tt_tensor *Rt, const tt_tensor *Lt, int R, float *gpr, float *gpl, hipStream_t s);
int mfma_unpad(const tt_tensor *O, int R, const float *padded, hipStream_t s);
// mode: 0 gather (y), 1 adjoint with weights gy, 2 fused MSE (t -> y, loss, O)
int mfma_run(int mode, const tt_tensor *L, const tt_tensor *R, tt_tensor *O, const int32_t *idx,
             int64_t M, const float *t, const float *gy, float *y, float *gout, float *loss, void *ws,
             size_t ws_bytes, hipStream_t s);

}  // namespace ttgfx
