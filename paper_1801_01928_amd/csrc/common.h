// Internal declarations shared by the HIP translation units of libttgfx.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "ttgfx.h"

namespace ttgfx {

// Kernel-side view of a TT tensor (passed by value; host arrays copied in).
struct TTDev {
  int d;
  int n[TT_MAX_D];
  int r[TT_MAX_D + 1];
  long long off[TT_MAX_D];
  float *data;
};

// ---------------------------------------------------------------- host side
int set_error(int code, const char *fmt, ...);
int hip_check(hipError_t e, const char *what);
int launch_check(const char *what);

// Validates a descriptor (d, n, r, r[0]=r[d]=1, data) against limits.
int validate_tt(const tt_tensor *X, const char *name, int max_rank);
TTDev make_dev(const tt_tensor *X);
long long tt_elems(const tt_tensor *X);           // total core elements
long long core_elems(const tt_tensor *X, int k);  // elements of core k
long long core_off(const tt_tensor *X, int k);    // element offset of core k
int max_rank_of(const tt_tensor *X);
bool same_modes(const tt_tensor *A, const tt_tensor *B);
bool same_shape(const tt_tensor *A, const tt_tensor *B);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Simple bump allocator over the caller's workspace.
struct Arena {
  char *base;
  size_t cap;
  size_t used = 0;
  Arena(void *b, size_t c) : base((char *)b), cap(c) {}
  template <class T>
  T *take(size_t count) {
    size_t o = align_up(used, 256);
    used = o + count * sizeof(T);
    return (T *)(base + o);
  }
  bool ok() const { return used <= cap; }
};
template <class T>
inline size_t arena_bytes(size_t count) { return align_up(count * sizeof(T), 256) + 256; }

// --------------------------------------------------- generic gather/adjoint
// (gather_generic.hip)
int generic_gather(const TTDev &X, int max_rank, const int32_t *idx, int64_t M, float *y,
                   hipStream_t s);
// Workspace for the generic adjoint: per-block partial copies of the output.
size_t generic_adjoint_ws(const tt_tensor *out_shape, int64_t M);
// O.core[k][:, i, :] = sum_m w_m (L^1..L^{k-1})^T (R^{k+1}..R^d)^T over entries
// with i_k = i; every core of O is overwritten.  O's ranks are
// (1, L.r[1..k], ...) on the left and R's on the right.
int generic_adjoint(const TTDev &L, const TTDev &R, const TTDev &O, int max_rank,
                    const int32_t *idx, int64_t M, const float *w,
                    void *ws, size_t ws_bytes, hipStream_t s);
// g = 2 (y - t) / M and loss = mean((y - t)^2) (deterministic reduction).
size_t mse_ws(int64_t M);
int mse_residual(const float *y, const float *t, int64_t M, float *g, float *loss,
                 void *ws, size_t ws_bytes, hipStream_t s);
// Kernel timer hooks (abi.hip): no-ops unless tt_timer_start() is active.
void timer_before(hipStream_t s);
void timer_after(hipStream_t s);

// Zero-fill by a kernel (safe inside stream capture).
int fill_zero(float *p, long long count, hipStream_t s);

}  // namespace ttgfx
