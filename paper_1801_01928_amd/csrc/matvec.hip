// TT-matrix by TT-vector product in the TT format (tt_matvec).
//
// For a TT-matrix W with cores W_k (r_k x m_k x n_k x r_{k+1}) and a TT
// vector x with cores x_k (s_k x n_k x s_{k+1}), y = W x is the TT vector
// with cores
//   y_k[(a, b), i, (a', b')] = sum_j W_k[a, i, j, a'] x_k[b, j, b'],
// of ranks r_k s_k (bond index a s_k + b) and modes m_k (Implementation
// Details: the TT-matrix by TT-vector product; Table 1 times it as matvec).
// No rounding: the product is exact and its ranks multiply.  Every output
// element is one n_k-term sum over W_k and x_k, which are small and stay in
// the caches; the bytes that must move are those of y.  The LDS path stages
// both factors' slices per workgroup; the grid-stride fallback gathers them
// per lane.
#include <type_traits>
#include <vector>

#include "common.h"

namespace ttgfx {
namespace {

constexpr int kMvBatch = 64;  // vectors per launch
constexpr int kMvThreads = 256;
constexpr int kMvPerThread = 8;  // fewer, fuller workgroups: dispatch is not the limit

template <class T>
struct MatDev {
  int d;
  int m[TT_MAX_D], n[TT_MAX_D], r[TT_MAX_D + 1];
  long long off[TT_MAX_D];
  const T *data;
};

// The right factor: a TT vector (L_k = 1) or a TT-matrix with cores
// s_k x n_k x L_k x s_{k+1}; and the output's core offsets.
struct RightDev {
  int r[TT_MAX_D + 1], L[TT_MAX_D];
  long long off[TT_MAX_D];
};
struct OutDev {
  long long off[TT_MAX_D];
};

template <class T>
struct MvIO {
  const T *x[kMvBatch];
  T *y[kMvBatch];
};

// grid (g, d, members), grid-stride over the elements of y_k for member
// blockIdx.z (g sized for about kMvPerThread elements per thread of the
// largest core): element e = ((row m_k + i) L_k + l) R' + col, with
// row = a s_k + b, col = a' s_{k+1} + b', R' = r_{k+1} s_{k+1}.
template <class T>
__global__ void __launch_bounds__(kMvThreads) matvec_kernel(MatDev<T> W, RightDev X0, OutDev Y0, MvIO<T> io) {
  const int k = blockIdx.y;
  const int r0 = W.r[k], r1 = W.r[k + 1], s0 = X0.r[k], s1 = X0.r[k + 1];
  const int mk = W.m[k], nk = W.n[k], lk = X0.L[k];
  // the host keeps every output core below 2^31 elements: 32-bit index
  // arithmetic
  const unsigned R1 = (unsigned)(r1 * s1);
  const unsigned cnt = (unsigned)r0 * s0 * mk * lk * R1;
  const T *xm = io.x[blockIdx.z] + X0.off[k];
  T *yk = io.y[blockIdx.z] + Y0.off[k];
  const long long xs = (long long)lk * s1;  // x stride along j
  for (unsigned e = blockIdx.x * kMvThreads + threadIdx.x; e < cnt; e += gridDim.x * kMvThreads) {
    const unsigned t = e / R1, col = e - t * R1;
    const unsigned t2 = t / lk, l = t - t2 * lk;
    const unsigned row = t2 / mk, i = t2 - row * mk;
    const unsigned a = row / s0, b = row - a * s0, ap = col / s1, bp = col - ap * s1;
    const T *wk = W.data + W.off[k] + (((long long)a * mk + i) * nk) * r1 + ap;
    const T *xk = xm + ((long long)b * nk * lk + l) * s1 + bp;
    T acc = T(0);
    for (int j = 0; j < nk; ++j) acc = fma(wk[(long long)j * r1], xk[j * xs], acc);
    yk[e] = acc;
  }
}

// LDS path: one workgroup per (a, i, l) of core k and member blockIdx.z.
// W_k[a, i, :, :] (n_k x r_{k+1}) and the l-slice of the right factor's
// core (s_k x n_k x s_{k+1}) are staged in LDS once; the workgroup then
// writes the s_k rows (a, b) at (i, l), each a contiguous run of
// r_{k+1} s_{k+1} elements.  The host takes this path when some core's
// output rows are longer than a workgroup's threads (the row-block path's
// limit) and both slices fit in kMvLdsBytes for every core; cores with
// shorter rows use fixed output columns per thread as the row-block path
// does.
constexpr int kMvLdsBytes = 65536;  // 64 KB of dynamic LDS
constexpr long long kMvMinRowBlocks = 2048;  // about eight workgroups per CU of a 256-CU device
constexpr int kMvMaxN = 16;  // row-block path: W columns of up to this many n_k held in registers

// Stages the l-slice of a right-factor core, s_k n_k runs of s_{k+1}
// elements (run u = b n_k + j starts at (u L_k + l) s_{k+1}), into xs: each
// thread keeps one position in the run, so no division per element.
// Up to kMvStage loads per thread are issued before their LDS stores, so a
// workgroup waits for one round trip to memory per kMvStage elements.
constexpr int kMvStage = 8;
template <class T>
__device__ __forceinline__ void stage_x_slice(T *xs, const T *xm, int runs, int s1, int lk, int l) {
  if (s1 <= kMvThreads) {
    const int rpp = kMvThreads / s1;  // runs per pass
    const int u0 = threadIdx.x / s1, bp = threadIdx.x - u0 * s1;
    if (u0 < rpp)
      for (int ub = u0; ub < runs; ub += rpp * kMvStage) {
        T v[kMvStage];
#pragma unroll
        for (int q = 0; q < kMvStage; ++q) {
          const int u = ub + q * rpp;
          v[q] = (u < runs) ? xm[((long long)u * lk + l) * s1 + bp] : T(0);
        }
#pragma unroll
        for (int q = 0; q < kMvStage; ++q) {
          const int u = ub + q * rpp;
          if (u < runs) xs[u * s1 + bp] = v[q];
        }
      }
  } else {
    for (int u = 0; u < runs; ++u)
      for (int bp = threadIdx.x; bp < s1; bp += kMvThreads) xs[u * s1 + bp] = xm[((long long)u * lk + l) * s1 + bp];
  }
}

// The thread's W column w[j * r1], j < N = n_k, and its n_k-term sum with
// an x column, N a compile-time constant (every n_k up to kMvMaxN has its
// own copy): all loads are issued before the first use, with no branch
// between them.
template <int N, class T>
__device__ __forceinline__ void load_wcol(T (&wcol)[N], const T *w, int r1) {
#pragma unroll
  for (int j = 0; j < N; ++j) wcol[j] = w[j * r1];
}

template <int N, class T>
__device__ __forceinline__ T dot_wcol(const T (&wcol)[N], const T *x, int s1) {
  T xv[N];
#pragma unroll
  for (int j = 0; j < N; ++j) xv[j] = x[j * s1];
  T acc = T(0);
#pragma unroll
  for (int j = 0; j < N; ++j) acc = fma(wcol[j], xv[j], acc);
  return acc;
}

// Calls f(std::integral_constant<int, n_k>) for 1 <= n_k <= kMvMaxN.
template <class F>
__device__ __forceinline__ void with_nk(int nk, F &&f) {
  static_assert(kMvMaxN == 16, "one case per n_k up to kMvMaxN");
  switch (nk) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 10: f(std::integral_constant<int, 10>{}); break;
    case 11: f(std::integral_constant<int, 11>{}); break;
    case 12: f(std::integral_constant<int, 12>{}); break;
    case 13: f(std::integral_constant<int, 13>{}); break;
    case 14: f(std::integral_constant<int, 14>{}); break;
    case 15: f(std::integral_constant<int, 15>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: break;
  }
}

// Contiguous staging of n elements (W slices), kMvStage loads in flight.
template <class T>
__device__ __forceinline__ void stage_run(T *dst, const T *src, int n) {
  for (int eb = threadIdx.x; eb < n; eb += kMvThreads * kMvStage) {
    T v[kMvStage];
#pragma unroll
    for (int q = 0; q < kMvStage; ++q) {
      const int e = eb + q * kMvThreads;
      v[q] = (e < n) ? src[e] : T(0);
    }
#pragma unroll
    for (int q = 0; q < kMvStage; ++q) {
      const int e = eb + q * kMvThreads;
      if (e < n) dst[e] = v[q];
    }
  }
}

template <class T>
__global__ void __launch_bounds__(kMvThreads) matvec_lds_kernel(MatDev<T> W, RightDev X0, OutDev Y0, MvIO<T> io) {
  extern __shared__ __align__(16) char lds_raw[];
  T *lds = (T *)lds_raw;
  const int k = blockIdx.y;
  const int r0 = W.r[k], r1 = W.r[k + 1], s0 = X0.r[k], s1 = X0.r[k + 1];
  const int mk = W.m[k], nk = W.n[k], lk = X0.L[k];
  const unsigned pairs = (unsigned)r0 * mk * lk;
  if (blockIdx.x >= pairs) return;  // uniform over the workgroup, before any barrier
  const unsigned t = blockIdx.x / lk, l = blockIdx.x - t * lk;
  const unsigned a = t / mk, i = t - a * mk;
  T *ws = lds, *xs = lds + nk * r1;
  const T *wsrc = W.data + W.off[k] + ((long long)a * mk + i) * nk * r1;
  stage_run(ws, wsrc, nk * r1);
  stage_x_slice(xs, io.x[blockIdx.z] + X0.off[k], s0 * nk, s1, lk, (int)l);
  __syncthreads();
  const int R1 = r1 * s1;
  // row b of this (a, i, l) starts at ((((a s_k + b) m_k + i) L_k + l) R'
  const long long rstride = (long long)mk * lk * R1;
  T *yb0 = io.y[blockIdx.z] + Y0.off[k] + (((long long)a * s0 * mk + i) * lk + l) * R1;
  if (R1 <= kMvThreads && nk <= kMvMaxN) {
    // fixed output column per thread: its W column sits in registers and
    // serves rows b = q0, q0 + per, ...
    const int per = kMvThreads / R1;
    const int col = threadIdx.x % R1, q0 = threadIdx.x / R1;
    if (q0 >= per) return;  // after the only barrier
    const int ap = col / s1, bp = col - ap * s1;
    with_nk(nk, [&](auto nc) __attribute__((always_inline)) {
      constexpr int N = decltype(nc)::value;
      T wcol[N];
      load_wcol<N>(wcol, ws + ap, r1);
      for (int b = q0; b < s0; b += per) yb0[b * rstride + col] = dot_wcol<N>(wcol, xs + b * nk * s1 + bp, s1);
    });
    return;
  }
  for (int o = threadIdx.x; o < s0 * R1; o += kMvThreads) {
    const int b = o / R1, col = o - b * R1;
    const int ap = col / s1, bp = col - ap * s1;
    const T *xb = xs + b * nk * s1 + bp;
    T acc = T(0);
    for (int j = 0; j < nk; ++j) acc = fma(ws[j * r1 + ap], xb[j * s1], acc);
    yb0[b * rstride + col] = acc;
  }
}

// Row-block LDS path: one workgroup per (core, member, a, l, chunk of ib
// row modes i) stages W_k[a, i0 : i0 + ib, :, :] and the l-slice of x_k
// once and writes the ib s_k output rows (i, b) of that (a, l), each a
// contiguous run of r_{k+1} s_{k+1} elements.  With ib = m_k (launches that
// fill the chip that way, such as Table 1's batch of matvecs) a tenth of
// the workgroups of one per (a, i) at Table 1's shape, and one staging of
// the x slice per m_k rows; a single product takes smaller chunks.
// Threads take fixed output columns (col = t mod R', computed once) and
// walk the rows.
template <class T>
__global__ void __launch_bounds__(kMvThreads) matvec_rows_kernel(MatDev<T> W, RightDev X0, OutDev Y0, MvIO<T> io,
                                                                  int ib, int nchunk) {
  extern __shared__ __align__(16) char lds_raw[];
  T *lds = (T *)lds_raw;
  const int k = blockIdx.y;
  const int r0 = W.r[k], r1 = W.r[k + 1], s0 = X0.r[k], s1 = X0.r[k + 1];
  const int mk0 = W.m[k], nk = W.n[k], lk = X0.L[k];
  const unsigned groups = (unsigned)r0 * lk;
  const unsigned g = blockIdx.x / (unsigned)nchunk;
  const int i0 = (int)(blockIdx.x - g * (unsigned)nchunk) * ib;
  if (g >= groups || i0 >= mk0) return;  // uniform over the workgroup, before any barrier
  const int mk = (mk0 - i0) < ib ? (mk0 - i0) : ib;  // rows i0 .. i0 + mk - 1 of this workgroup
  const unsigned a = g / lk, l = g - a * lk;
  const int wn = mk * nk * r1;
  T *ws = lds, *xs = lds + wn;
  const T *wsrc = W.data + W.off[k] + ((long long)a * mk0 + i0) * nk * r1;
  stage_run(ws, wsrc, wn);
  stage_x_slice(xs, io.x[blockIdx.z] + X0.off[k], s0 * nk, s1, lk, (int)l);
  __syncthreads();
  const int R1 = r1 * s1;
  const int per = kMvThreads / R1;  // row offsets per pass (R1 <= kMvThreads on this path)
  const int t = threadIdx.x;
  const int col = t % R1, q0 = t / R1;
  if (q0 >= per) return;  // after the only barrier
  const int ap = col / s1, bp = col - ap * s1;
  T *yk = io.y[blockIdx.z] + Y0.off[k];
  if (nk <= kMvMaxN) {
    // rows by i, then b = q0, q0 + per, ...: the thread's W column of each
    // i sits in registers and serves all of its rows b
    with_nk(nk, [&](auto nc) __attribute__((always_inline)) {
      constexpr int N = decltype(nc)::value;
      for (int i = 0; i < mk; ++i) {
        T wcol[N];
        load_wcol<N>(wcol, ws + i * nk * r1 + ap, r1);
        for (int b = q0; b < s0; b += per) {
          const long long row = (long long)a * s0 + b;
          yk[((row * mk0 + i0 + i) * lk + l) * R1 + col] = dot_wcol<N>(wcol, xs + b * nk * s1 + bp, s1);
        }
      }
    });
    return;
  }
  for (int ix = q0; ix < mk * s0; ix += per) {
    const int i = ix / s0, b = ix - i * s0;
    const T *wi = ws + i * nk * r1 + ap;
    const T *xb = xs + b * nk * s1 + bp;
    T acc = T(0);
    for (int j = 0; j < nk; ++j) acc = fma(wi[j * r1], xb[j * s1], acc);
    const long long row = (long long)a * s0 + b;
    yk[((row * mk0 + i0 + i) * lk + l) * R1 + col] = acc;
  }
}

// Launches the product kernels for `members` right factors: the row-block
// LDS path when every core's output rows fit a workgroup's threads and its
// staged slices fit (at some chunk of row modes), else the per-(a, i) LDS
// path when its two slices fit, else the grid-stride kernel.
template <class T>
int launch_products(const MatDev<T> &md, const RightDev &x0, const OutDev &y0, const MvIO<T> &io, int members,
                    hipStream_t s) {
  long long maxcnt = 0, maxpairs = 0, maxlds = 0, maxgroups = 0, maxR1 = 0;
  for (int k = 0; k < md.d; ++k) {
    const long long r0 = md.r[k], r1 = md.r[k + 1], s0 = x0.r[k], s1 = x0.r[k + 1];
    const long long c = r0 * s0 * md.m[k] * x0.L[k] * r1 * s1;
    const long long p = r0 * md.m[k] * x0.L[k];
    const long long f = (long long)md.n[k] * r1 + s0 * md.n[k] * s1;
    const long long g = r0 * x0.L[k];
    maxcnt = c > maxcnt ? c : maxcnt;
    maxpairs = p > maxpairs ? p : maxpairs;
    maxlds = f > maxlds ? f : maxlds;
    maxgroups = g > maxgroups ? g : maxgroups;
    maxR1 = r1 * s1 > maxR1 ? r1 * s1 : maxR1;
  }
  if (maxcnt >= (1LL << 31)) return set_error(TT_ERR_UNSUPPORTED, "product: an output core of 2^31 or more elements");
  // Row-block chunk: the whole row mode when that grid fills the chip, else
  // smaller chunks (down to one i per workgroup) until it does and the
  // staged slices fit the LDS.
  int maxmk = 1;
  for (int k = 0; k < md.d; ++k) maxmk = md.m[k] > maxmk ? md.m[k] : maxmk;
  auto rows_lds = [&](int ib) {
    long long mx = 0;
    for (int k = 0; k < md.d; ++k) {
      const long long mi = md.m[k] < ib ? md.m[k] : ib;
      const long long fr = mi * md.n[k] * md.r[k + 1] + (long long)x0.r[k] * md.n[k] * x0.r[k + 1];
      mx = fr > mx ? fr : mx;
    }
    return mx;
  };
  int ib = maxmk, nchunk = 1;
  while (ib > 1 && (maxgroups * nchunk * md.d * members < kMvMinRowBlocks ||
                    rows_lds(ib) * (long long)sizeof(T) > kMvLdsBytes)) {
    --ib;
    nchunk = (maxmk + ib - 1) / ib;
  }
  const long long rowlds = rows_lds(ib);
  if (maxR1 <= kMvThreads && rowlds * (long long)sizeof(T) <= kMvLdsBytes && maxgroups * nchunk <= 0x7fffffffLL) {
    hipLaunchKernelGGL(matvec_rows_kernel<T>, dim3((unsigned)(maxgroups * nchunk), (unsigned)md.d, (unsigned)members),
                       dim3(kMvThreads), (size_t)rowlds * sizeof(T), s, md, x0, y0, io, ib, nchunk);
  } else if (maxlds * (long long)sizeof(T) <= kMvLdsBytes && maxpairs <= 0x7fffffffLL) {
    hipLaunchKernelGGL(matvec_lds_kernel<T>, dim3((unsigned)maxpairs, (unsigned)md.d, (unsigned)members),
                       dim3(kMvThreads), (size_t)maxlds * sizeof(T), s, md, x0, y0, io);
  } else {
    const long long gx = (maxcnt + (long long)kMvThreads * kMvPerThread - 1) / ((long long)kMvThreads * kMvPerThread);
    hipLaunchKernelGGL(matvec_kernel<T>, dim3((unsigned)gx, (unsigned)md.d, (unsigned)members), dim3(kMvThreads), 0,
                       s, md, x0, y0, io);
  }
  return launch_check("TT-matrix product");
}

template <class T>
int validate_matrix(const tt_matrix *W, MatDev<T> *md) {
  if (!W) return set_error(TT_ERR_ARG, "W: null descriptor");
  if (W->d < 1 || W->d > TT_MAX_D) return set_error(TT_ERR_ARG, "W: d = %d outside [1, %d]", W->d, TT_MAX_D);
  if (!W->m || !W->n || !W->r) return set_error(TT_ERR_ARG, "W: null m, n or r array");
  if (!W->data) return set_error(TT_ERR_ARG, "W: null data pointer");
  if (W->r[0] != 1 || W->r[W->d] != 1)
    return set_error(TT_ERR_SHAPE, "W: boundary ranks must be 1 (got %d, %d)", W->r[0], W->r[W->d]);
  md->d = W->d;
  md->data = (const T *)W->data;
  long long o = 0;
  for (int k = 0; k <= W->d; ++k) {
    if (W->r[k] < 1 || W->r[k] > TT_MAX_RANK)
      return set_error(TT_ERR_SHAPE, "W: r[%d] = %d outside [1, %d]", k, W->r[k], TT_MAX_RANK);
    md->r[k] = W->r[k];
  }
  for (int k = 0; k < W->d; ++k) {
    if (W->m[k] < 1 || W->n[k] < 1 || W->m[k] > TT_MAX_N || W->n[k] > TT_MAX_N)
      return set_error(TT_ERR_SHAPE, "W: mode sizes m[%d] = %d, n[%d] = %d outside [1, %d]", k, W->m[k], k,
                       W->n[k], TT_MAX_N);
    if (W->off && W->off[k] < 0) return set_error(TT_ERR_ARG, "W: negative offset for core %d", k);
    md->m[k] = W->m[k];
    md->n[k] = W->n[k];
    md->off[k] = W->off ? W->off[k] : o;
    o += (long long)W->r[k] * W->m[k] * W->n[k] * W->r[k + 1];
  }
  return TT_OK;
}

// X, Y: shape views of the b vectors and products (data only tested for NULL).
template <class T>
int validate_matvec(const tt_matrix *W, const tt_tensor *X, const tt_tensor *Y, int b, MatDev<T> *md) {
  int rc = validate_matrix(W, md);
  if (rc) return rc;
  if (b < 1 || !X) return set_error(TT_ERR_ARG, "matvec: empty batch of vectors");
  if (!Y) return set_error(TT_ERR_ARG, "matvec: Y must hold as many TTs as X");
  const tt_tensor *x0 = &X[0], *y0 = &Y[0];
  for (int j = 0; j < b; ++j) {
    const tt_tensor *x = &X[j], *y = &Y[j];
    if ((rc = validate_tt(x, "X[j]", TT_MAX_RANK))) return rc;
    if ((rc = validate_tt(y, "Y[j]", TT_MAX_RANK * TT_MAX_RANK))) return rc;
    if (x->d != W->d || y->d != W->d) return set_error(TT_ERR_SHAPE, "X[%d], Y[%d] must have W's d", j, j);
    for (int k = 0; k < W->d; ++k) {
      if (x->n[k] != W->n[k]) return set_error(TT_ERR_SHAPE, "X[%d]: n[%d] must be W's column mode %d", j, k, W->n[k]);
      if (y->n[k] != W->m[k]) return set_error(TT_ERR_SHAPE, "Y[%d]: n[%d] must be W's row mode %d", j, k, W->m[k]);
      if (x->r[k + 1] != x0->r[k + 1]) return set_error(TT_ERR_SHAPE, "X[%d] must have the ranks of X[0]", j);
      if (y->r[k + 1] != W->r[k + 1] * x->r[k + 1])
        return set_error(TT_ERR_SHAPE, "Y[%d]: r[%d] = %d, expected %d", j, k + 1, y->r[k + 1],
                         W->r[k + 1] * x->r[k + 1]);
      if (core_off(x, k) != core_off(x0, k) || core_off(y, k) != core_off(y0, k))
        return set_error(TT_ERR_SHAPE, "X[%d], Y[%d] must have the core offsets of X[0], Y[0]", j, j);
    }
  }
  return TT_OK;
}

template <class T>
int run_matvec(const tt_matrix *W, const tt_tensor *X, const tt_tensor *Y, const T *const *xdata, T *const *ydata,
               int b, hipStream_t s) {
  MatDev<T> md;
  int rc = validate_matvec(W, X, Y, b, &md);
  if (rc) return rc;
  RightDev x0{};
  OutDev y0{};
  for (int k = 0; k < md.d; ++k) {
    x0.r[k] = X[0].r[k];
    x0.L[k] = 1;
    x0.off[k] = core_off(&X[0], k);
    y0.off[k] = core_off(&Y[0], k);
  }
  x0.r[md.d] = 1;
  for (int j0 = 0; j0 < b; j0 += kMvBatch) {
    const int m = (b - j0) < kMvBatch ? (b - j0) : kMvBatch;
    MvIO<T> io{};
    for (int j = 0; j < m; ++j) {
      io.x[j] = xdata[j0 + j];
      io.y[j] = ydata[j0 + j];
    }
    if ((rc = launch_products(md, x0, y0, io, m, s))) return rc;
  }
  return TT_OK;
}

// C = A B for two TT-matrices (A: m x n modes, B: n x l modes): the cores
// C_k[(a, b), i, l, (a', b')] = sum_j A_k[a, i, j, a'] B_k[b, j, l, b'].
template <class T>
int run_matmat(const tt_matrix *A, const tt_matrix *B, tt_matrix *Cm, hipStream_t s) {
  MatDev<T> ma, mb;
  int rc;
  if ((rc = validate_matrix(A, &ma)) || (rc = validate_matrix(B, &mb))) return rc;
  if (!Cm) return set_error(TT_ERR_ARG, "C: null descriptor");
  if (!Cm->m || !Cm->n || !Cm->r || !Cm->data) return set_error(TT_ERR_ARG, "C: null array or data pointer");
  if (B->d != A->d || Cm->d != A->d) return set_error(TT_ERR_SHAPE, "A, B and C must have the same d");
  for (int k = 0; k < A->d; ++k) {
    if (B->m[k] != A->n[k]) return set_error(TT_ERR_SHAPE, "B: row mode %d = %d, expected A's column mode %d", k, B->m[k], A->n[k]);
    if (Cm->m[k] != A->m[k] || Cm->n[k] != B->n[k])
      return set_error(TT_ERR_SHAPE, "C: modes of core %d must be A's rows and B's columns", k);
  }
  for (int k = 0; k <= A->d; ++k)
    if (Cm->r[k] != A->r[k] * B->r[k])
      return set_error(TT_ERR_SHAPE, "C: r[%d] = %d, expected %d", k, Cm->r[k], A->r[k] * B->r[k]);
  RightDev x0{};
  OutDev y0{};
  long long oc = 0;
  for (int k = 0; k < A->d; ++k) {
    if (Cm->off && Cm->off[k] < 0) return set_error(TT_ERR_ARG, "C: negative offset for core %d", k);
    x0.r[k] = B->r[k];
    x0.L[k] = B->n[k];
    x0.off[k] = mb.off[k];
    y0.off[k] = Cm->off ? Cm->off[k] : oc;
    const long long c = (long long)Cm->r[k] * Cm->m[k] * Cm->n[k] * Cm->r[k + 1];
    oc += c;
  }
  x0.r[A->d] = 1;
  MvIO<T> io{};
  io.x[0] = mb.data;
  io.y[0] = (T *)Cm->data;
  return launch_products(ma, x0, y0, io, 1, s);
}

}  // namespace
}  // namespace ttgfx

using namespace ttgfx;

extern "C" int tt_matvec(const tt_matrix *W, const tt_batch *X, tt_batch *Y, void *stream) {
  if (!X || X->b < 1 || !X->tt) return set_error(TT_ERR_ARG, "matvec: empty batch of vectors");
  if (!Y || Y->b != X->b || !Y->tt) return set_error(TT_ERR_ARG, "matvec: Y must hold as many TTs as X");
  std::vector<const float *> xd(X->b);
  std::vector<float *> yd(X->b);
  for (int j = 0; j < X->b; ++j) {
    xd[j] = X->tt[j].data;
    yd[j] = Y->tt[j].data;
  }
  return run_matvec<float>(W, X->tt, Y->tt, xd.data(), yd.data(), X->b, (hipStream_t)stream);
}

extern "C" int tt_matvec_f64(const tt_matrix *W, const tt_batch_f64 *X, tt_batch_f64 *Y, void *stream) {
  if (!X || X->b < 1 || !X->tt) return set_error(TT_ERR_ARG, "matvec: empty batch of vectors");
  if (!Y || Y->b != X->b || !Y->tt) return set_error(TT_ERR_ARG, "matvec: Y must hold as many TTs as X");
  std::vector<tt_tensor> xv(X->b), yv(X->b);
  std::vector<const double *> xd(X->b);
  std::vector<double *> yd(X->b);
  for (int j = 0; j < X->b; ++j) {
    const tt_tensor_f64 &x = X->tt[j], &y = Y->tt[j];
    xv[j] = tt_tensor{x.d, x.n, x.r, x.off, (float *)x.data};  // shape views
    yv[j] = tt_tensor{y.d, y.n, y.r, y.off, (float *)y.data};
    xd[j] = x.data;
    yd[j] = y.data;
  }
  return run_matvec<double>(W, xv.data(), yv.data(), xd.data(), yd.data(), X->b, (hipStream_t)stream);
}

extern "C" int tt_matmat(const tt_matrix *A, const tt_matrix *B, tt_matrix *Cm, void *stream) {
  return run_matmat<float>(A, B, Cm, (hipStream_t)stream);
}

extern "C" int tt_matmat_f64(const tt_matrix *A, const tt_matrix *B, tt_matrix *Cm, void *stream) {
  return run_matmat<double>(A, B, Cm, (hipStream_t)stream);
}
