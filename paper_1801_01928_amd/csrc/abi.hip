// C ABI of libttgfx: host-side validation, error reporting and dispatch to
// the kernels.  Every entry point validates its host metadata before the
// first HIP call and reports failures through tt_last_error().
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "common.h"
#include "kernels.h"

namespace ttgfx {

static thread_local std::string g_last_error;

int set_error(int code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return TT_OK;
  return set_error(TT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int launch_check(const char *what) { return hip_check(hipGetLastError(), what); }

int validate_tt(const tt_tensor *X, const char *name, int max_rank) {
  if (!X) return set_error(TT_ERR_ARG, "%s: null descriptor", name);
  if (X->d < 1 || X->d > TT_MAX_D)
    return set_error(TT_ERR_ARG, "%s: d = %d outside [1, %d]", name, X->d, TT_MAX_D);
  if (!X->n || !X->r) return set_error(TT_ERR_ARG, "%s: null n or r array", name);
  if (!X->data) return set_error(TT_ERR_ARG, "%s: null data pointer", name);
  if (X->r[0] != 1 || X->r[X->d] != 1)
    return set_error(TT_ERR_SHAPE, "%s: boundary ranks must be 1 (got %d, %d)", name, X->r[0],
                     X->r[X->d]);
  for (int k = 0; k < X->d; ++k) {
    if (X->n[k] < 1 || X->n[k] > TT_MAX_N)
      return set_error(TT_ERR_SHAPE, "%s: n[%d] = %d outside [1, %d]", name, k, X->n[k], TT_MAX_N);
  }
  for (int k = 0; k <= X->d; ++k) {
    if (X->r[k] < 1) return set_error(TT_ERR_SHAPE, "%s: r[%d] = %d < 1", name, k, X->r[k]);
    if (X->r[k] > max_rank)
      return set_error(TT_ERR_UNSUPPORTED, "%s: r[%d] = %d exceeds the supported maximum %d", name,
                       k, X->r[k], max_rank);
  }
  if (X->off) {
    for (int k = 0; k < X->d; ++k)
      if (X->off[k] < 0) return set_error(TT_ERR_ARG, "%s: negative offset for core %d", name, k);
  }
  return TT_OK;
}

long long core_elems(const tt_tensor *X, int k) {
  return (long long)X->r[k] * X->n[k] * X->r[k + 1];
}

long long core_off(const tt_tensor *X, int k) {
  if (X->off) return X->off[k];
  long long o = 0;
  for (int j = 0; j < k; ++j) o += core_elems(X, j);
  return o;
}

long long tt_elems(const tt_tensor *X) {
  long long t = 0;
  for (int k = 0; k < X->d; ++k) t += core_elems(X, k);
  return t;
}

int max_rank_of(const tt_tensor *X) {
  int m = 1;
  for (int k = 0; k <= X->d; ++k) m = X->r[k] > m ? X->r[k] : m;
  return m;
}

bool same_modes(const tt_tensor *A, const tt_tensor *B) {
  if (A->d != B->d) return false;
  for (int k = 0; k < A->d; ++k)
    if (A->n[k] != B->n[k]) return false;
  return true;
}

bool same_shape(const tt_tensor *A, const tt_tensor *B) {
  if (!same_modes(A, B)) return false;
  for (int k = 0; k <= A->d; ++k)
    if (A->r[k] != B->r[k]) return false;
  return true;
}

TTDev make_dev(const tt_tensor *X) {
  TTDev t;
  memset(&t, 0, sizeof t);
  t.d = X->d;
  for (int k = 0; k < X->d; ++k) {
    t.n[k] = X->n[k];
    t.off[k] = core_off(X, k);
  }
  for (int k = 0; k <= X->d; ++k) t.r[k] = X->r[k];
  t.data = X->data;
  return t;
}

// ------------------------------------------------------------ kernel timer
namespace {
constexpr int kTimerCap = 4096;
struct Timer {
  bool on = false;
  int n = 0;
  hipEvent_t ev[2 * kTimerCap];
  bool made[2 * kTimerCap] = {};
};
Timer g_timer;

hipEvent_t timer_event(int i) {
  if (!g_timer.made[i]) {
    if (hipEventCreate(&g_timer.ev[i]) != hipSuccess) return nullptr;
    g_timer.made[i] = true;
  }
  return g_timer.ev[i];
}
}  // namespace

void timer_before(hipStream_t s) {
  if (!g_timer.on || g_timer.n >= kTimerCap) return;
  hipEvent_t e = timer_event(2 * g_timer.n);
  if (e) (void)hipEventRecord(e, s);
}

void timer_after(hipStream_t s) {
  if (!g_timer.on || g_timer.n >= kTimerCap) return;
  hipEvent_t e = timer_event(2 * g_timer.n + 1);
  if (e) (void)hipEventRecord(e, s);
  ++g_timer.n;
}

static int check_entries(const int32_t *idx, int64_t M, const void *vals, const char *vname) {
  if (M < 0) return set_error(TT_ERR_ARG, "M = %lld is negative", (long long)M);
  if (M > 0 && !idx) return set_error(TT_ERR_ARG, "null index array with M = %lld", (long long)M);
  if (M > 0 && vname && !vals) return set_error(TT_ERR_ARG, "null %s array with M = %lld", vname, (long long)M);
  if (M > (int64_t)0x7fffffff) return set_error(TT_ERR_UNSUPPORTED, "M = %lld above 2^31-1", (long long)M);
  return TT_OK;
}

static int check_ws(void *ws, size_t ws_bytes, size_t need, const char *what) {
  if (need == 0) return TT_OK;
  if (!ws || ws_bytes < need)
    return set_error(TT_ERR_WORKSPACE, "%s: workspace of %zu bytes given, %zu required", what,
                     ws ? ws_bytes : (size_t)0, need);
  return TT_OK;
}

}  // namespace ttgfx

using namespace ttgfx;

extern "C" {

const char *tt_last_error(void) { return g_last_error.c_str(); }
int tt_version(void) { return TTGFX_VERSION; }

int tt_timer_start(void) {
  g_timer.on = true;
  g_timer.n = 0;
  return TT_OK;
}

int tt_timer_stop(float *total_ms, int32_t *launches) {
  g_timer.on = false;
  float tot = 0.f;
  for (int i = 0; i < g_timer.n; ++i) {
    int rc = hip_check(hipEventSynchronize(g_timer.ev[2 * i + 1]), "timer sync");
    if (rc) return rc;
    float ms = 0.f;
    rc = hip_check(hipEventElapsedTime(&ms, g_timer.ev[2 * i], g_timer.ev[2 * i + 1]), "timer read");
    if (rc) return rc;
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = g_timer.n;
  g_timer.n = 0;
  return TT_OK;
}

// ------------------------------------------------------------------ gather
int64_t tt_gather_workspace(const tt_tensor *X, int64_t M) {
  int rc = validate_tt(X, "X", TT_MAX_RANK);
  if (rc) return rc;
  if (M < 0) return set_error(TT_ERR_ARG, "M = %lld is negative", (long long)M);
  return (int64_t)gather_dispatch_ws(X, M);
}

int tt_gather(const tt_tensor *X, const int32_t *idx, int64_t M, float *y, void *ws,
              size_t ws_bytes, void *stream) {
  int rc = validate_tt(X, "X", TT_MAX_RANK);
  if (rc) return rc;
  if ((rc = check_entries(idx, M, y, "y"))) return rc;
  if (M == 0) return TT_OK;
  if ((rc = check_ws(ws, ws_bytes, gather_dispatch_ws(X, M), "gather"))) return rc;
  return gather_dispatch(X, idx, M, y, ws, ws_bytes, (hipStream_t)stream);
}

int64_t tt_gather_backward_workspace(const tt_tensor *X, int64_t M) {
  int rc = validate_tt(X, "X", TT_MAX_RANK);
  if (rc) return rc;
  if (M < 0) return set_error(TT_ERR_ARG, "M = %lld is negative", (long long)M);
  return (int64_t)adjoint_dispatch_ws(X, M);
}

int tt_gather_backward(const tt_tensor *X, const int32_t *idx, int64_t M, const float *gy,
                       tt_tensor *gX, void *ws, size_t ws_bytes, void *stream) {
  int rc = validate_tt(X, "X", TT_MAX_RANK);
  if (rc) return rc;
  if ((rc = validate_tt(gX, "gX", TT_MAX_RANK))) return rc;
  if (!same_shape(X, gX)) return set_error(TT_ERR_SHAPE, "gX must have the shape of X");
  if ((rc = check_entries(idx, M, gy, "gy"))) return rc;
  if ((rc = check_ws(ws, ws_bytes, adjoint_dispatch_ws(X, M), "gather_backward"))) return rc;
  return adjoint_dispatch(X, X, gX, idx, M, gy, ws, ws_bytes, (hipStream_t)stream);
}

// ------------------------------------------------------- fused MSE pass
int64_t tt_gather_mse_workspace(const tt_tensor *X, int64_t M) {
  int rc = validate_tt(X, "X", TT_MAX_RANK);
  if (rc) return rc;
  if (M < 0) return set_error(TT_ERR_ARG, "M = %lld is negative", (long long)M);
  return (int64_t)fused_mse_ws(X, M);
}

int tt_gather_mse_backward(const tt_tensor *X, const int32_t *idx, int64_t M, const float *t,
                           float *y, float *g, float *loss, tt_tensor *gX, void *ws, size_t ws_bytes,
                           void *stream) {
  int rc = validate_tt(X, "X", TT_MAX_RANK);
  if (rc) return rc;
  if ((rc = validate_tt(gX, "gX", TT_MAX_RANK))) return rc;
  if (!same_shape(X, gX)) return set_error(TT_ERR_SHAPE, "gX must have the shape of X");
  if ((rc = check_entries(idx, M, t, "t"))) return rc;
  if ((rc = check_ws(ws, ws_bytes, fused_mse_ws(X, M), "gather_mse_backward"))) return rc;
  return fused_mse_dispatch(X, idx, M, t, y, g, loss, gX, ws, ws_bytes, (hipStream_t)stream);
}

// ------------------------------------------------------------ line search
int64_t tt_line_search_workspace(const tt_tensor *P, int64_t M) {
  int rc = validate_tt(P, "P", TT_MAX_RANK);
  if (rc) return rc;
  if (M < 0) return set_error(TT_ERR_ARG, "M = %lld is negative", (long long)M);
  return (int64_t)line_search_ws(P, M);
}

int tt_line_search(const tt_tensor *P, const int32_t *idx, int64_t M, const float *y, const float *t,
                   float *out, void *ws, size_t ws_bytes, void *stream) {
  int rc = validate_tt(P, "P", TT_MAX_RANK);
  if (rc) return rc;
  if (!out) return set_error(TT_ERR_ARG, "line_search: null out");
  if ((rc = check_entries(idx, M, y, "y"))) return rc;
  if (M > 0 && !t) return set_error(TT_ERR_ARG, "null t array with M = %lld", (long long)M);
  if ((rc = check_ws(ws, ws_bytes, line_search_ws(P, M), "line_search"))) return rc;
  return line_search(P, idx, M, y, t, out, ws, ws_bytes, (hipStream_t)stream);
}

// ------------------------------------------------------------ index check
int tt_check_indices(const tt_tensor *X, const int32_t *idx, int64_t M, int64_t *out, void *stream) {
  int rc = validate_tt(X, "X", TT_MAX_RANK);
  if (rc) return rc;
  if (!out) return set_error(TT_ERR_ARG, "check_indices: null out");
  if ((rc = check_entries(idx, M, nullptr, nullptr))) return rc;
  return index_check(X, idx, M, out, (hipStream_t)stream);
}

}  // extern "C"
