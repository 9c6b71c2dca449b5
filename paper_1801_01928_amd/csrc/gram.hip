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

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int R = 32;
constexpr int TILE = 4;                      // instances per side of a pair tile
constexpr int THREADS = TILE * TILE * 64;    // one wave per pair
constexpr int SLICE = R * R;                 // floats per padded slice

// Per-instance metadata on the device.
struct InstMeta {
  const float *data;
  long long off[TT_MAX_D];
  int r[TT_MAX_D + 1];
};

struct Modes {
  int d;
  int n[TT_MAX_D];
  int total;  // sum of n
};

// Padded slice (k, i) of an instance in operand order: for lane (q, c),
// comp tiles (ti, tc) and v < 4, the float at ((ti*2 + tc)*64 + lane)*4 + v
// holds S[16 ti + 4 q + v][16 tc + c].
__global__ void gram_pack_kernel(const InstMeta *__restrict__ meta, Modes md,
                                 float *__restrict__ out) {
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
  const int r0 = m.r[k], r1 = m.r[k + 1], nk = md.n[k];
  float *dst = out + ((long long)inst * md.total + slice) * SLICE;
  for (int e = threadIdx.x; e < SLICE; e += blockDim.x) {
    const int v = e & 3, lane = (e >> 2) & 63, tile = e >> 8;
    const int ti = tile >> 1, tc = tile & 1;
    const int row = 16 * ti + 4 * (lane >> 4) + v, col = 16 * tc + (lane & 15);
    float x = 0.f;
    if (row < r0 && col < r1) x = m.data[m.off[k] + ((long long)row * nk + s) * r1 + col];
    dst[e] = x;
  }
}

// Grid: one workgroup per pair tile (ta, tb), given by the tile list.
__global__ void __launch_bounds__(THREADS) gram_kernel(const float *__restrict__ pa,
                                                       const float *__restrict__ pb, int na, int nb,
                                                       Modes md, int sym,
                                                       const int2 *__restrict__ tiles,
                                                       float *__restrict__ G) {
  __shared__ __align__(16) float sa[2][TILE][SLICE];
  __shared__ __align__(16) float sb[2][TILE][SLICE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wa = wave / TILE, wb = wave % TILE;
  const int2 tp = tiles[blockIdx.x];
  const int ta = tp.x, tb = tp.y;
  const int a = ta * TILE + wa, b = tb * TILE + wb;

  // one slice of the 4 + 4 tensors: loaded into registers (kPer vectors
  // per thread) while the current slice is multiplied, stored to the other
  // LDS buffer after the products
  constexpr int kPer = 2 * TILE * SLICE / 4 / THREADS;
  static_assert(kPer * THREADS == 2 * TILE * SLICE / 4, "whole vectors per thread");
  v4f pre[kPer];
  auto load = [&](int sl) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + u * THREADS;
      const int side = e / (TILE * SLICE / 4);
      const int rem = e % (TILE * SLICE / 4);
      const int which = rem / (SLICE / 4), off = rem % (SLICE / 4);
      pre[u] = v4f{0.f, 0.f, 0.f, 0.f};
      if (side == 0) {
        const int ia = ta * TILE + which;
        if (ia < na) pre[u] = ((const v4f *)(pa + ((long long)ia * md.total + sl) * SLICE))[off];
      } else {
        const int ib = tb * TILE + which;
        if (ib < nb) pre[u] = ((const v4f *)(pb + ((long long)ib * md.total + sl) * SLICE))[off];
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + u * THREADS;
      const int side = e / (TILE * SLICE / 4);
      const int rem = e % (TILE * SLICE / 4);
      const int which = rem / (SLICE / 4), off = rem % (SLICE / 4);
      if (side == 0) ((v4f *)sa[buf][which])[off] = pre[u];
      else ((v4f *)sb[buf][which])[off] = pre[u];
    }
  };

  // Psi = Phi_0^T = e_0 e_0^T in D layout (tile (0,0), lane 0, v 0)
  v4f psi[4], nxt[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    psi[x] = v4f{0.f, 0.f, 0.f, 0.f};
    nxt[x] = v4f{0.f, 0.f, 0.f, 0.f};
  }
  if (lane == 0) psi[0][0] = 1.f;

  int sl = 0, buf = 0;
  load(0);
  store(0);
  __syncthreads();
  for (int k = 0; k < md.d; ++k) {
    for (int i = 0; i < md.n[k]; ++i, ++sl) {
      const bool more = sl + 1 < md.total;
      if (more) load(sl + 1);  // in flight during this slice's products
      v4f bo[4], ao[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        bo[x] = ((const v4f *)sb[buf][wb])[x * 64 + lane];
        ao[x] = ((const v4f *)sa[buf][wa])[x * 64 + lane];
      }
      // Y = Phi B_i; A operand Phi[16 to + c][16 ti + 4q + v] = Psi tile (ti, to)
      v4f y[4];
#pragma unroll
      for (int to = 0; to < 2; ++to)
#pragma unroll
        for (int tc = 0; tc < 2; ++tc) {
          v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc = mfma4(psi[ti * 2 + to][v], bo[ti * 2 + tc][v], acc);
          y[to * 2 + tc] = acc;
        }
      // Psi_next += Y^T A_i; A operand Y^T[16 to + c][16 ti + 4q + v] = Y tile (ti, to)
#pragma unroll
      for (int to = 0; to < 2; ++to)
#pragma unroll
        for (int tc = 0; tc < 2; ++tc) {
          v4f acc = nxt[to * 2 + tc];
#pragma unroll
          for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc = mfma4(y[ti * 2 + to][v], ao[ti * 2 + tc][v], acc);
          nxt[to * 2 + tc] = acc;
        }
      if (more) store(buf ^ 1);
      __syncthreads();  // the next slice's buffer is complete; this one may be overwritten
      buf ^= 1;
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      psi[x] = nxt[x];
      nxt[x] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  }
  // <A_a, B_b> = Phi_d[0][0] = Psi[0][0]
  // symmetric case: in diagonal tiles only the pairs with a <= b write, so
  // that G is exactly symmetric
  if (lane == 0 && a < na && b < nb && !(sym && a > b)) {
    const float g = psi[0][0];
    G[(long long)a * nb + b] = g;
    if (sym && a != b) G[(long long)b * nb + a] = g;
  }
}

int pack(const tt_batch *X, const InstMeta *dmeta, const Modes &md, float *out, hipStream_t s) {
  hipLaunchKernelGGL(gram_pack_kernel, dim3(md.total, X->b), dim3(256), 0, s, dmeta, md, out);
  return launch_check("gram pack");
}

int ntiles_of(int b) { return (b + TILE - 1) / TILE; }

}  // namespace

size_t gram_ws(const tt_batch *A, const tt_batch *B) {
  const tt_tensor &t0 = A->tt[0];
  long total = 0;
  for (int k = 0; k < t0.d; ++k) total += t0.n[k];
  const int sym = (B == nullptr);
  const int nb = sym ? A->b : B->b;
  const long nta = ntiles_of(A->b), ntb = ntiles_of(nb);
  size_t bytes = arena_bytes<InstMeta>((size_t)A->b + (sym ? 0 : nb));
  bytes += arena_bytes<float>((size_t)A->b * total * SLICE);
  if (!sym) bytes += arena_bytes<float>((size_t)nb * total * SLICE);
  bytes += arena_bytes<int2>((size_t)nta * ntb);
  return bytes;
}

int gram_run(const tt_batch *A, const tt_batch *B, float *G, void *ws, size_t bytes, hipStream_t s) {
  const int sym = (B == nullptr);
  const tt_batch *Bb = sym ? A : B;
  const tt_tensor &t0 = A->tt[0];
  Modes md = {};
  md.d = t0.d;
  md.total = 0;
  for (int k = 0; k < t0.d; ++k) {
    md.n[k] = t0.n[k];
    md.total += t0.n[k];
  }
  Arena ar(ws, bytes);
  InstMeta *dmeta = ar.take<InstMeta>((size_t)A->b + (sym ? 0 : Bb->b));
  float *packA = ar.take<float>((size_t)A->b * md.total * SLICE);
  float *packB = sym ? packA : ar.take<float>((size_t)Bb->b * md.total * SLICE);
  const int nta = ntiles_of(A->b), ntb = ntiles_of(Bb->b);
  int2 *dtiles = ar.take<int2>((size_t)nta * ntb);
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "gram: workspace too small");

  // host tables: instance metadata and the list of pair tiles (kept in
  // per-thread buffers that only grow)
  static thread_local std::vector<InstMeta> hmeta_buf;
  static thread_local std::vector<int2> htile_buf;
  const int nmeta = A->b + (sym ? 0 : Bb->b);
  if ((int)hmeta_buf.size() < nmeta) hmeta_buf.resize(nmeta);
  if (htile_buf.size() < (size_t)nta * ntb) htile_buf.resize((size_t)nta * ntb);
  InstMeta *hmeta = hmeta_buf.data();
  for (int j = 0; j < nmeta; ++j) {
    const tt_tensor *X = (j < A->b) ? &A->tt[j] : &Bb->tt[j - A->b];
    InstMeta &m = hmeta[j];
    memset(&m, 0, sizeof m);
    m.data = X->data;
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
  if ((rc = pack(A, dmeta, md, packA, s))) return rc;
  if (!sym && (rc = pack(Bb, dmeta + A->b, md, packB, s))) return rc;
  timer_before(s);
  hipLaunchKernelGGL(gram_kernel, dim3(ntile), dim3(THREADS), 0, s, packA, packB, A->b, Bb->b, md, sym,
                     dtiles, G);
  timer_after(s);
  return launch_check("gram");
}

}  // namespace ttgfx
