// Gram matrix of TT batches (gram.hip).
#pragma once
#include "common.h"

namespace ttgfx {

#define GRAM_MAX_RANK 32

size_t gram_ws(const tt_batch *A, const tt_batch *B);
int gram_run(const tt_batch *A, const tt_batch *B, float *G, void *ws, size_t bytes, hipStream_t s);

}  // namespace ttgfx
