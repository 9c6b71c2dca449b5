// Dispatch layer between the C ABI and the kernels: picks the specialised
// kernel for a shape when one exists, else the generic one.
#pragma once
#include "common.h"

namespace ttgfx {

size_t gather_dispatch_ws(const tt_tensor *X, int64_t M);
int gather_dispatch(const tt_tensor *X, const int32_t *idx, int64_t M, float *y, void *ws,
                    size_t ws_bytes, hipStream_t s);

// Adjoint with left cores L, right cores R, output O (all validated).
size_t adjoint_dispatch_ws(const tt_tensor *X, int64_t M);
size_t adjoint_dispatch_ws2(const tt_tensor *L, const tt_tensor *R, int64_t M);
int adjoint_dispatch(const tt_tensor *L, const tt_tensor *R, tt_tensor *O, const int32_t *idx,
                     int64_t M, const float *w, void *ws, size_t ws_bytes, hipStream_t s);

size_t fused_mse_ws(const tt_tensor *X, int64_t M);
int fused_mse_dispatch(const tt_tensor *X, const int32_t *idx, int64_t M, const float *t, float *y,
                       float *g, float *loss, tt_tensor *gX, void *ws, size_t ws_bytes, hipStream_t s);

// Line-search terms of Riemannian completion (linesearch.hip).
size_t line_search_ws(const tt_tensor *P, int64_t M);
int line_search(const tt_tensor *P, const int32_t *idx, int64_t M, const float *y, const float *t, float *out,
                void *ws, size_t ws_bytes, hipStream_t s);

// Gather by prefix/suffix tables (halves.hip); validated arguments, d >= 2,
// 1 <= split <= d-1.  halves_bytes: table buffer bytes and the rows of the
// two final tables.
int halves_split_of(const tt_tensor *X);
int halves_bytes(const tt_tensor *X, int split, size_t *bytes, long long *rows);
int halves_build(const tt_tensor *X, int split, void *tables, hipStream_t s);
int halves_gather(const tt_tensor *X, int split, const void *tables, const int32_t *idx, int64_t M, float *y,
                  hipStream_t s);

// Counts entries with an index outside [0, n_k) into out[0] and stores the
// smallest such entry (M if none) in out[1] (device int64 [2]).
int index_check(const tt_tensor *X, const int32_t *idx, long long M, int64_t *out, hipStream_t s);

}  // namespace ttgfx
