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

// Largest prod m * prod n the dense path builds W for (1 GiB in float32).
constexpr long long kTtmDenseMaxElems = 1LL << 28;

// Evaluation path of tt_matmul / tt_matmul_backward: 0 automatic (the dense
// path when W fits and its GEMM flops are below the core-by-core chain's),
// 1 the chain, 2 the dense matrix.
enum { TTM_PATH_AUTO = 0, TTM_PATH_CHAIN = 1, TTM_PATH_DENSE = 2 };
void ttm_set_path(int path);
int ttm_path_of(const TTMDims &D, long long B);  // TTM_PATH_CHAIN or TTM_PATH_DENSE
long long ttm_chain_flops(const TTMDims &D, long long B);

// The dense path (ttm_dense.hip).
bool ttm_dense_fits(const TTMDims &D);
long long ttm_dense_flops(const TTMDims &D, long long B);
size_t ttm_dense_ws(const TTMDims &D, long long B, int dtype, int backward);
int ttm_dense_forward(const TTMDims &D, const void *cores, const void *X, long long B, float *Y, int dtype, void *ws,
                      size_t bytes, hipStream_t s);
int ttm_dense_backward(const TTMDims &D, const void *cores, const void *X, long long B, const void *dY, float *dX,
                       float *dW, int dtype, void *ws, size_t bytes, hipStream_t s);

int ttm_validate(const tt_matrix *W, long long B, int dtype, TTMDims *D);
size_t ttm_ws(const TTMDims &D, long long B, int dtype, int backward);
int ttm_forward(const TTMDims &D, const void *cores, const void *X, long long B, float *Y, int dtype, void *ws,
                size_t bytes, hipStream_t s);
int ttm_backward(const TTMDims &D, const void *cores, const void *X, long long B, const void *dY, float *dX,
                 float *dW, int dtype, void *ws, size_t bytes, hipStream_t s);

}  // namespace ttgfx
