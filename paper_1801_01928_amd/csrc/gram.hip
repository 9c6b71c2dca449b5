// Gram matrix of two batches of TT tensors (Riemannian Geometry Operations:
// Gram matrices of batches; Table 1 'gram'): G[a][b] = <A_a, B_b>.
//
// For one pair the inner product is the bond-by-bond contraction
//   Phi_0 = 1,  Phi_k = sum_i A^k[i]^T Phi_{k-1} B^k[i],  <A, B> = Phi_d.
// Ranks are zero-padded to R = 32 (padding leaves every value unchanged).
// A workgroup owns a 4 x 4 tile of (a, b) pairs, one wave per pair; the
// slices of its 8 tensors for the current (mode, slice) are staged in LDS.
// Each wave keeps Psi = Phi^T in registers in MFMA D layout and per slice
// computes  Y = Phi B_i  and  Psi_next += Y^T A_i  with
// v_mfma_f32_16x16x4_f32: in this orientation both products take their
// register operand straight from the previous result (no transposes), and
// both slices are read in the same operand layout.
#include <string.h>

#include <vector>

#include "common.h"
#include "gram.h"

namespace ttgfx {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

// Per scalar type: the 16 x 16 x 4 matrix-core product (the float64 one
// has the float32 one's operand and result layout), 4-element accumulator
// and 16-byte load vectors, and the pair tile (a float64 slice takes twice
// the LDS, so its tiles are 2 x 2).
template <class T>
struct GramT;
// Result layout (lane c + 16 q, register v): the float32 product holds row
// 4 q + v, the float64 one row q + 4 v (measured).  A result used as the
// next product's A operand therefore brings K chunk v as the K indices
// {v, 4 + v, 8 + v, 12 + v} in float32 and {4 v .. 4 v + 3} in float64, and
// the packed slices (the B operands) follow the same order (KCONTIG).
template <>
struct GramT<float> {
  typedef v4f acc4;
  typedef v4f vec16;
  static constexpr int TILE = 4;
  static constexpr bool KCONTIG = false;
  __device__ static acc4 mfma(float a, float b, acc4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <>
struct GramT<double> {
  typedef v4d acc4;
  typedef v2d vec16;
  static constexpr int TILE = 2;
  static constexpr bool KCONTIG = true;
  __device__ static acc4 mfma(double a, double b, acc4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

constexpr int R = 32;
constexpr int SLICE = R * R;                 // elements per padded slice

// Per-instance metadata on the device.
struct InstMeta {
  const void *data;  // float or double cores
  long long off[TT_MAX_D];
  int r[TT_MAX_D + 1];
};

struct Modes {
  int d;
  int n[TT_MAX_D];
  int total;  // sum of n
};

// Padded slice (k, i) of an instance in operand order: for lane (q, c),
// comp tiles (ti, tc) and v < 4, the element at ((ti*2 + tc)*64 + lane)*4 + v
// holds S[16 ti + 4 q + v][16 tc + c] (float32) or S[16 ti + q + 4 v][16 tc + c]
// (float64), the K order of the matching result layout.
template <class T>
__global__ void gram_pack_kernel(const InstMeta *__restrict__ meta, Modes md, T *__restrict__ out) {
  const int inst = blockIdx.y;
  const int slice = blockIdx.x;
  if (slice >= md.total) return;
  int k = 0, base = 0;
  while (k < md.d && slice >= base + md.n[k]) {
    base += md.n[k];
    ++k;
  }
  const int s = slice - base;
  const InstMeta &m = meta[inst];
  const T *src = (const T *)m.data;
  const int r0 = m.r[k], r1 = m.r[k + 1], nk = md.n[k];
  T *dst = out + ((long long)inst * md.total + slice) * SLICE;
  for (int e = threadIdx.x; e < SLICE; e += blockDim.x) {
    const int v = e & 3, lane = (e >> 2) & 63, tile = e >> 8;
    const int ti = tile >> 1, tc = tile & 1;
    const int q = lane >> 4;
    const int row = 16 * ti + (GramT<T>::KCONTIG ? q + 4 * v : 4 * q + v), col = 16 * tc + (lane & 15);
    T x = T(0);
    if (row < r0 && col < r1) x = src[m.off[k] + ((long long)row * nk + s) * r1 + col];
    dst[e] = x;
  }
}

// Grid: one workgroup per pair tile (ta, tb), given by the tile list.
template <class T>
__global__ void __launch_bounds__(GramT<T>::TILE * GramT<T>::TILE * 64)
    gram_kernel(const T *__restrict__ pa, const T *__restrict__ pb, int na, int nb, Modes md, int sym,
                const int2 *__restrict__ tiles, T *__restrict__ G) {
  constexpr int TILE = GramT<T>::TILE;
  constexpr int THREADS = TILE * TILE * 64;  // one wave per pair
  typedef typename GramT<T>::acc4 acc4;
  typedef typename GramT<T>::vec16 vec16;
  constexpr int VL = 16 / sizeof(T);        // elements per 16-byte vector
  __shared__ __align__(16) T sa[2][TILE][SLICE];
  __shared__ __align__(16) T sb[2][TILE][SLICE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wa = wave / TILE, wb = wave % TILE;
  const int2 tp = tiles[blockIdx.x];
  const int ta = tp.x, tb = tp.y;
  const int a = ta * TILE + wa, b = tb * TILE + wb;

  // one slice of the TILE + TILE tensors: loaded into registers (kPer
  // vectors per thread) while the current slice is multiplied, stored to
  // the other LDS buffer after the products
  constexpr int kPer = 2 * TILE * SLICE / VL / THREADS;
  static_assert(kPer * THREADS == 2 * TILE * SLICE / VL, "whole vectors per thread");
  vec16 pre[kPer];
  auto load = [&](int sl) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + u * THREADS;
      const int side = e / (TILE * SLICE / VL);
      const int rem = e % (TILE * SLICE / VL);
      const int which = rem / (SLICE / VL), off = rem % (SLICE / VL);
      pre[u] = vec16{};
      if (side == 0) {
        const int ia = ta * TILE + which;
        if (ia < na) pre[u] = ((const vec16 *)(pa + ((long long)ia * md.total + sl) * SLICE))[off];
      } else {
        const int ib = tb * TILE + which;
        if (ib < nb) pre[u] = ((const vec16 *)(pb + ((long long)ib * md.total + sl) * SLICE))[off];
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + u * THREADS;
      const int side = e / (TILE * SLICE / VL);
      const int rem = e % (TILE * SLICE / VL);
      const int which = rem / (SLICE / VL), off = rem % (SLICE / VL);
      if (side == 0) ((vec16 *)sa[buf][which])[off] = pre[u];
      else ((vec16 *)sb[buf][which])[off] = pre[u];
    }
  };

  // Psi = Phi_0^T = e_0 e_0^T in D layout (tile (0,0), lane 0, v 0)
  acc4 psi[4], nxt[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    psi[x] = acc4{};
    nxt[x] = acc4{};
  }
  if (lane == 0) psi[0][0] = T(1);

  int sl = 0, buf = 0;
  load(0);
  store(0);
  __syncthreads();
  for (int k = 0; k < md.d; ++k) {
    for (int i = 0; i < md.n[k]; ++i, ++sl) {
      const bool more = sl + 1 < md.total;
      if (more) load(sl + 1);  // in flight during this slice's products
      acc4 bo[4], ao[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        bo[x] = ((const acc4 *)sb[buf][wb])[x * 64 + lane];
        ao[x] = ((const acc4 *)sa[buf][wa])[x * 64 + lane];
      }
      // Y = Phi B_i; A operand Phi[16 to + c][16 ti + K(q, v)] = Psi tile (ti, to), with
      // K(q, v) = 4q + v (float32) or q + 4v (float64)
      acc4 y[4];
#pragma unroll
      for (int to = 0; to < 2; ++to)
#pragma unroll
        for (int tc = 0; tc < 2; ++tc) {
          acc4 acc = acc4{};
#pragma unroll
          for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc = GramT<T>::mfma(psi[ti * 2 + to][v], bo[ti * 2 + tc][v], acc);
          y[to * 2 + tc] = acc;
        }
      // Psi_next += Y^T A_i; A operand Y^T[16 to + c][16 ti + K(q, v)] = Y tile (ti, to)
#pragma unroll
      for (int to = 0; to < 2; ++to)
#pragma unroll
        for (int tc = 0; tc < 2; ++tc) {
          acc4 acc = nxt[to * 2 + tc];
#pragma unroll
          for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc = GramT<T>::mfma(y[ti * 2 + to][v], ao[ti * 2 + tc][v], acc);
          nxt[to * 2 + tc] = acc;
        }
      if (more) store(buf ^ 1);
      __syncthreads();  // the next slice's buffer is complete; this one may be overwritten
      buf ^= 1;
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      psi[x] = nxt[x];
      nxt[x] = acc4{};
    }
  }
  // <A_a, B_b> = Phi_d[0][0] = Psi[0][0]
  // symmetric case: in diagonal tiles only the pairs with a <= b write, so
  // that G is exactly symmetric
  if (lane == 0 && a < na && b < nb && !(sym && a > b)) {
    const T g = psi[0][0];
    G[(long long)a * nb + b] = g;
    if (sym && a != b) G[(long long)b * nb + a] = g;
  }
}

template <class T>
int ntiles_of(int b) {
  return (b + GramT<T>::TILE - 1) / GramT<T>::TILE;
}

}  // namespace

template <class T>
size_t gram_ws_t(const tt_tensor *A, int na, const tt_tensor *B, int nb_in) {
  const tt_tensor &t0 = A[0];
  long total = 0;
  for (int k = 0; k < t0.d; ++k) total += t0.n[k];
  const int sym = (B == nullptr);
  const int nb = sym ? na : nb_in;
  const long nta = ntiles_of<T>(na), ntb = ntiles_of<T>(nb);
  size_t bytes = arena_bytes<InstMeta>((size_t)na + (sym ? 0 : nb));
  bytes += arena_bytes<T>((size_t)na * total * SLICE);
  if (!sym) bytes += arena_bytes<T>((size_t)nb * total * SLICE);
  bytes += arena_bytes<int2>((size_t)nta * ntb);
  return bytes;
}

// A, B: shape views of the members; adata, bdata their core pointers.
template <class T>
int gram_run_t(const tt_tensor *A, int na, const T *const *adata, const tt_tensor *B, int nb_in,
               const T *const *bdata, T *G, void *ws, size_t bytes, hipStream_t s) {
  const int sym = (B == nullptr);
  const int nbb = sym ? na : nb_in;
  const tt_tensor &t0 = A[0];
  Modes md = {};
  md.d = t0.d;
  md.total = 0;
  for (int k = 0; k < t0.d; ++k) {
    md.n[k] = t0.n[k];
    md.total += t0.n[k];
  }
  Arena ar(ws, bytes);
  InstMeta *dmeta = ar.take<InstMeta>((size_t)na + (sym ? 0 : nbb));
  T *packA = ar.take<T>((size_t)na * md.total * SLICE);
  T *packB = sym ? packA : ar.take<T>((size_t)nbb * md.total * SLICE);
  const int nta = ntiles_of<T>(na), ntb = ntiles_of<T>(nbb);
  int2 *dtiles = ar.take<int2>((size_t)nta * ntb);
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "gram: workspace too small");

  // host tables: instance metadata and the list of pair tiles (kept in
  // per-thread buffers that only grow)
  static thread_local std::vector<InstMeta> hmeta_buf;
  static thread_local std::vector<int2> htile_buf;
  const int nmeta = na + (sym ? 0 : nbb);
  if ((int)hmeta_buf.size() < nmeta) hmeta_buf.resize(nmeta);
  if (htile_buf.size() < (size_t)nta * ntb) htile_buf.resize((size_t)nta * ntb);
  InstMeta *hmeta = hmeta_buf.data();
  for (int j = 0; j < nmeta; ++j) {
    const tt_tensor *X = (j < na) ? &A[j] : &B[j - na];
    InstMeta &m = hmeta[j];
    memset(&m, 0, sizeof m);
    m.data = (j < na) ? (const void *)adata[j] : (const void *)bdata[j - na];
    for (int k = 0; k < X->d; ++k) m.off[k] = core_off(X, k);
    for (int k = 0; k <= X->d; ++k) m.r[k] = X->r[k];
  }
  int ntile = 0;
  int2 *htiles = htile_buf.data();
  for (int i = 0; i < nta; ++i)
    for (int j = sym ? i : 0; j < ntb; ++j) htiles[ntile++] = make_int2(i, j);
  int rc = hip_check(hipMemcpyAsync(dmeta, hmeta, sizeof(InstMeta) * nmeta, hipMemcpyHostToDevice, s),
                     "gram metadata copy");
  if (!rc)
    rc = hip_check(hipMemcpyAsync(dtiles, htiles, sizeof(int2) * ntile, hipMemcpyHostToDevice, s),
                   "gram tile copy");
  if (rc) return rc;
  hipLaunchKernelGGL(gram_pack_kernel<T>, dim3(md.total, na), dim3(256), 0, s, dmeta, md, packA);
  if ((rc = launch_check("gram pack"))) return rc;
  if (!sym) {
    hipLaunchKernelGGL(gram_pack_kernel<T>, dim3(md.total, nbb), dim3(256), 0, s, dmeta + na, md, packB);
    if ((rc = launch_check("gram pack"))) return rc;
  }
  constexpr int THREADS = GramT<T>::TILE * GramT<T>::TILE * 64;
  timer_before(s);
  hipLaunchKernelGGL(gram_kernel<T>, dim3(ntile), dim3(THREADS), 0, s, packA, packB, na, nbb, md, sym, dtiles, G);
  timer_after(s);
  return launch_check("gram");
}

size_t gram_ws(const tt_batch *A, const tt_batch *B) {
  return gram_ws_t<float>(A->tt, A->b, B ? B->tt : nullptr, B ? B->b : 0);
}

int gram_run(const tt_batch *A, const tt_batch *B, float *G, void *ws, size_t bytes, hipStream_t s) {
  std::vector<const float *> ad(A->b), bd(B ? B->b : 0);
  for (int j = 0; j < A->b; ++j) ad[j] = A->tt[j].data;
  for (int j = 0; B && j < B->b; ++j) bd[j] = B->tt[j].data;
  return gram_run_t<float>(A->tt, A->b, ad.data(), B ? B->tt : nullptr, B ? B->b : 0, bd.data(), G, ws, bytes, s);
}

size_t gram_ws_f64(const tt_tensor *A, int na, const tt_tensor *B, int nb) { return gram_ws_t<double>(A, na, B, nb); }

int gram_run_f64(const tt_tensor *A, int na, const double *const *adata, const tt_tensor *B, int nb,
                 const double *const *bdata, double *G, void *ws, size_t bytes, hipStream_t s) {
  return gram_run_t<double>(A, na, adata, B, nb, bdata, G, ws, bytes, s);
}

}  // namespace ttgfx
