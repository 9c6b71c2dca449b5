// Gram matrix of TT batches (gram.hip).
#pragma once
#include "common.h"

namespace ttgfx {

#define GRAM_MAX_RANK 32

size_t gram_ws(const tt_batch *A, const tt_batch *B);
int gram_run(const tt_batch *A, const tt_batch *B, float *G, void *ws, size_t bytes, hipStream_t s);
// float64: A, B shape views of the members (B NULL: the symmetric Gram of A)
size_t gram_ws_f64(const tt_tensor *A, int na, const tt_tensor *B, int nb);
int gram_run_f64(const tt_tensor *A, int na, const double *const *adata, const tt_tensor *B, int nb,
                 const double *const *bdata, double *G, void *ws, size_t bytes, hipStream_t s);

}  // namespace ttgfx
