// TT-matrix layer (ttm.hip).
#pragma once
#include "common.h"

namespace ttgfx {

// Every step contracts (mode, bond) pairs of at most this many values and
// produces at most this many: m_k r_k, m_k r_{k+1}, n_k r_k, n_k r_{k+1}.
#define TTM_MAX_FUSED 128

// Validated host copy of a tt_matrix descriptor.
struct TTMDims {
  int d;
  int m[TT_MAX_D], n[TT_MAX_D], r[TT_MAX_D + 1];
  long long off[TT_MAX_D];
  long long extent;  // elements spanned by the cores
  long long Mt, Nt;  // prod m, prod n
};

int ttm_validate(const tt_matrix *W, long long B, int dtype, TTMDims *D);
size_t ttm_ws(const TTMDims &D, long long B, int dtype, int backward);
int ttm_forward(const TTMDims &D, const void *cores, const void *X, long long B, float *Y, int dtype, void *ws,
                size_t bytes, hipStream_t s);
int ttm_backward(const TTMDims &D, const void *cores, const void *X, long long B, const void *dY, float *dX,
                 float *dW, int dtype, void *ws, size_t bytes, hipStream_t s);

}  // namespace ttgfx
