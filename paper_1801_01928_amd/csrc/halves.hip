// Gather by shared prefix and suffix products.
//
// The entry formula of the TT format (Introduction) multiplies one slice per
// mode.  Cut the modes at bond s (0-based modes 0..s-1 on the left, s..d-1 on
// the right): every entry is the dot of a prefix G^0[i_0]..G^{s-1}[i_{s-1}]
// (1 x r_s) and a suffix G^s[i_s]..G^{d-1}[i_{d-1}] (r_s x 1).  The prefixes
// of all index tuples of the left modes are the rows of the left
// half-unfolding of the tensor, the suffixes those of the right one.  When
// the observed entries outnumber the rows of the two tables, building the
// tables once and taking one r_s-dot per entry does far less work than the
// per-entry chain of slice products.
//
// Tables (row-major, r_s floats per row):
//   left   Lt[row_L], row_L = (..(i_0 n_1 + i_1) n_2 + ..) n_{s-1} + i_{s-1}
//   right  Rt[row_R], row_R = i_s + n_s (i_{s+1} + n_{s+1} (.. i_{d-1}))
// Each is built level by level from the 1 x 1 table [1], one GEMM per mode:
//   left   T_j (P n_{j-1} x r_j)  = T_{j-1} (P x r_{j-1}) * G^{j-1} viewed as
//          (r_{j-1} x n_{j-1} r_j) row-major (its natural layout);
//   right  U_j (Q n_j x r_j)      = U_{j+1} (Q x r_{j+1}) * B_j,
//          B_j[b][i r_j + a] = G^j[a][i][b];
// the row-major GEMM output is the next table with the new index fastest.
// Every level is kept in the caller's table buffer (the levels shrink
// geometrically, so the earlier ones add little).
#include "common.h"
#include "kernels.h"

namespace ttgfx {

namespace {

constexpr int kHalvesThreads = 256;
constexpr int kTile = 64;   // GEMM output tile (rows and columns)
constexpr int kKc = 32;     // GEMM K chunk staged in LDS

// One level: C (P x N) = A (P x K) * B, A row-major (A == nullptr: the 1 x 1
// table [1]), B(l, j) read from core `g` of shape (rl x n x rr):
//   left  (right = 0): K = rl, N = n rr, B(l, j) = g[l N + j];
//   right (right = 1): K = rr, N = n rl, B(l, i rl + a) = g[a n rr + i rr + l].
struct LevelJob {
  const float *A;
  const float *g;
  float *C;
  long long P;
  int rl, n, rr, right;
  int tiles_p, tiles_j;  // 64-row and 64-column tiles of C
};

// One step of both chains in one launch: workgroups [0, job0 tiles) take
// job 0, the rest job 1 (count 0 when a chain has no step left).  256
// threads; thread (ty, tx) = (t / 16, t % 16) owns rows ty + 16u and
// columns tx + 16v of a 64 x 64 tile (u, v < 4); K is staged in LDS in
// chunks of 32.
__global__ void __launch_bounds__(kHalvesThreads) halves_level_kernel(LevelJob j0b, LevelJob j1b) {
  const bool second = (int)blockIdx.x >= j0b.tiles_p * j0b.tiles_j;
  const LevelJob &jb = second ? j1b : j0b;
  const int b = second ? (int)blockIdx.x - j0b.tiles_p * j0b.tiles_j : (int)blockIdx.x;
  const int K = jb.right ? jb.rr : jb.rl;
  const int N = jb.right ? jb.n * jb.rl : jb.n * jb.rr;
  const float *__restrict__ A = jb.A;
  const float *__restrict__ g = jb.g;
  __shared__ float As[kTile][kKc + 1];
  __shared__ float Bs[kKc][kTile + 1];
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  const long long p0 = (long long)(b / jb.tiles_j) * kTile;
  const int j0 = (b % jb.tiles_j) * kTile;
  float acc[4][4] = {};
  for (int l0 = 0; l0 < K; l0 += kKc) {
    for (int e = t; e < kTile * kKc; e += kHalvesThreads) {
      const int i = e / kKc, l = e % kKc;
      const long long p = p0 + i;
      float v = 0.f;
      if (p < jb.P && l0 + l < K) v = A ? A[p * K + l0 + l] : 1.f;
      As[i][l] = v;
    }
    for (int e = t; e < kKc * kTile; e += kHalvesThreads) {
      const int l = e / kTile, j = e % kTile;
      const int gl = l0 + l, gj = j0 + j;
      float v = 0.f;
      if (gl < K && gj < N) {
        if (jb.right) {
          const int i = gj / jb.rl, a = gj - i * jb.rl;
          v = g[((long long)a * jb.n + i) * jb.rr + gl];
        } else {
          v = g[(long long)gl * N + gj];
        }
      }
      Bs[l][j] = v;
    }
    __syncthreads();
    const int kc = (K - l0) < kKc ? (K - l0) : kKc;
    for (int l = 0; l < kc; ++l) {
      float a[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = As[ty + 16 * u][l];
#pragma unroll
      for (int v = 0; v < 4; ++v) bv[v] = Bs[l][tx + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(a[u], bv[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const long long p = p0 + ty + 16 * u;
    if (p >= jb.P) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = j0 + tx + 16 * v;
      if (j < N) jb.C[p * N + j] = acc[u][v];
    }
  }
}

struct HalvesArgs {
  int d, s, rs;
  int n[TT_MAX_D];
  const float *lt;
  const float *rt;
};

// Row numbers of entry m in the two tables (0 and ok = false when an index
// is outside [0, n_k)).  The index loads come first (unrolled up to MAXD
// modes), all issued before the first use.
template <int MAXD>
__device__ __forceinline__ void halves_rows(const HalvesArgs &a, const int32_t *__restrict__ idx, long long M,
                                            long long m, int &rl, int &rr, bool &ok) {
  int iv[MAXD];
#pragma unroll
  for (int k = 0; k < MAXD; ++k) iv[k] = (k < a.d) ? idx[(long long)k * M + m] : 0;
  ok = true;
  long long l = 0, r = 0;
#pragma unroll
  for (int k = 0; k < MAXD; ++k) {
    if (k < a.s) {
      ok = ok && (unsigned)iv[k] < (unsigned)a.n[k];
      l = l * a.n[k] + iv[k];
    }
  }
#pragma unroll
  for (int k = MAXD - 1; k >= 0; --k) {
    if (k >= a.s && k < a.d) {
      ok = ok && (unsigned)iv[k] < (unsigned)a.n[k];
      r = r * a.n[k] + iv[k];
    }
  }
  rl = ok ? (int)l : 0;
  rr = ok ? (int)r : 0;
}

// y[m] = Lt[row_L(m)] . Rt[row_R(m)].
// LPE > 0 (rs = 4 LPE): each lane finds the rows of one entry (64 entries
// per wave, coalesced index loads); then in LPE rounds, groups of LPE lanes
// take one entry each (rows passed by shuffles), every lane reading 4
// consecutive components of both rows (16-byte loads, rows 16-byte
// aligned), and a butterfly over the group sums them.  The loads of up to
// 8 rounds are issued before their first sum.
// LPE = 0: one lane per entry, scalar loop over rs.
// Grid-stride over M padded to whole blocks, so every lane of a wave runs
// the same iterations (the shuffles need all of them); lanes past M repeat
// entry M - 1 and store nothing.
template <int LPE, int MAXD>
__global__ void __launch_bounds__(kHalvesThreads)
    halves_gather_kernel(HalvesArgs a, const int32_t *__restrict__ idx, long long M, float *__restrict__ y) {
  const long long lanes = (M + kHalvesThreads - 1) / kHalvesThreads * kHalvesThreads;
  const long long stride = (long long)gridDim.x * kHalvesThreads;
  const int lane = threadIdx.x & 63;
  for (long long tid = (long long)blockIdx.x * kHalvesThreads + threadIdx.x; tid < lanes; tid += stride) {
    const long long m = tid < M ? tid : M - 1;
    int rl, rr;
    bool ok;
    halves_rows<MAXD>(a, idx, M, m, rl, rr, ok);
    if constexpr (LPE > 0) {
      typedef float v4 __attribute__((ext_vector_type(4)));
      constexpr int EPR = 64 / LPE;  // entries per round
      const int part = lane % LPE;
      const long long wbase = tid - lane;  // entry of lane 0
      constexpr int QG = LPE < 8 ? LPE : 8;  // rounds whose loads are in flight together
      const int okw = ok ? 1 : 0;
#pragma unroll
      for (int q0 = 0; q0 < LPE; q0 += QG) {
        v4 lv[QG], rv[QG];
#pragma unroll
        for (int u = 0; u < QG; ++u) {
          const int src = (q0 + u) * EPR + lane / LPE;
          const int ql = __shfl(rl, src), qr = __shfl(rr, src);
          lv[u] = *(const v4 *)(a.lt + (long long)ql * a.rs + 4 * part);
          rv[u] = *(const v4 *)(a.rt + (long long)qr * a.rs + 4 * part);
        }
#pragma unroll
        for (int u = 0; u < QG; ++u) {
          const int src = (q0 + u) * EPR + lane / LPE;
          float v = lv[u].x * rv[u].x;
          v = fmaf(lv[u].y, rv[u].y, v);
          v = fmaf(lv[u].z, rv[u].z, v);
          v = fmaf(lv[u].w, rv[u].w, v);
#pragma unroll
          for (int off = LPE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
          const int qok = __shfl(okw, src);
          const long long e = wbase + src;
          if (part == 0 && e < M) y[e] = qok ? v : 0.f;
        }
      }
    } else {
      const float *lp = a.lt + (long long)rl * a.rs;
      const float *rp = a.rt + (long long)rr * a.rs;
      float v = 0.f;
      for (int c = 0; c < a.rs; ++c) v = fmaf(lp[c], rp[c], v);
      if (tid < M) y[tid] = ok ? v : 0.f;
    }
  }
}

// Table layout inside the caller's buffer: left levels 1..s, then right
// levels d-1 down to s, each 256-byte aligned; the last level of each side
// (left level s, right level s) is the table the gather reads.  Left level
// j has prod_{k<j} n_k rows of r_j floats, right level j prod_{k>=j} n_k rows
// of r_j floats.
struct HalvesLayout {
  long long lrows[TT_MAX_D + 1], rrows[TT_MAX_D + 1];
  size_t loff[TT_MAX_D + 1], roff[TT_MAX_D + 1];
  size_t total;
};

// Limits: at most 2^30 rows per level, and fewer than 2^23 output tiles per
// level, so that one launch of two levels (256 lanes per tile) stays below
// 2^32 lanes.
constexpr long long kMaxRows = 1ll << 30;
constexpr long long kMaxTiles = 1ll << 23;

long long level_tiles(long long prev_rows, int n, int r) {
  return (prev_rows + kTile - 1) / kTile * (((long long)n * r + kTile - 1) / kTile);
}

int halves_layout(const tt_tensor *X, int s, HalvesLayout &L) {
  const int d = X->d;
  size_t at = 0;
  long long P = 1;
  for (int j = 1; j <= s; ++j) {
    if (level_tiles(P, X->n[j - 1], X->r[j]) >= kMaxTiles)
      return set_error(TT_ERR_UNSUPPORTED, "halves: left level %d has over 2^23 tiles", j);
    P *= X->n[j - 1];
    if (P > kMaxRows) return set_error(TT_ERR_UNSUPPORTED, "halves: left level %d has over 2^30 rows", j);
    L.lrows[j] = P;
    L.loff[j] = at;
    at += align_up((size_t)P * X->r[j] * sizeof(float), 256);
  }
  long long Q = 1;
  for (int j = d - 1; j >= s; --j) {
    if (level_tiles(Q, X->n[j], X->r[j]) >= kMaxTiles)
      return set_error(TT_ERR_UNSUPPORTED, "halves: right level %d has over 2^23 tiles", j);
    Q *= X->n[j];
    if (Q > kMaxRows) return set_error(TT_ERR_UNSUPPORTED, "halves: right level %d has over 2^30 rows", j);
    L.rrows[j] = Q;
    L.roff[j] = at;
    at += align_up((size_t)Q * X->r[j] * sizeof(float), 256);
  }
  L.total = at;
  return TT_OK;
}

int halves_check(const tt_tensor *X, int split) {
  int rc = validate_tt(X, "X", TT_MAX_RANK);
  if (rc) return rc;
  if (X->d < 2) return set_error(TT_ERR_UNSUPPORTED, "halves: needs d >= 2 (d = %d)", X->d);
  if (split < 1 || split >= X->d)
    return set_error(TT_ERR_ARG, "halves: split %d outside [1, %d]", split, X->d - 1);
  return TT_OK;
}

// Split minimising the table floats (left rows + right rows) * r_s.
int halves_auto_split(const tt_tensor *X) {
  const int d = X->d;
  int best = 1;
  double bestv = -1.0;
  for (int s = 1; s < d; ++s) {
    double pl = 1.0, pr = 1.0;
    for (int k = 0; k < s; ++k) pl *= X->n[k];
    for (int k = s; k < d; ++k) pr *= X->n[k];
    const double v = (pl + pr) * X->r[s];
    if (bestv < 0.0 || v < bestv) {
      bestv = v;
      best = s;
    }
  }
  return best;
}

template <int LPE>
void launch_gather_lpe(const HalvesArgs &a, const int32_t *idx, long long M, float *y, hipStream_t st) {
  long long blocks = (M + kHalvesThreads - 1) / kHalvesThreads;
  if (blocks > 65536) blocks = 65536;
  if (a.d <= 8)
    hipLaunchKernelGGL((halves_gather_kernel<LPE, 8>), dim3((unsigned)blocks), dim3(kHalvesThreads), 0, st, a,
                       idx, M, y);
  else if (a.d <= 16)
    hipLaunchKernelGGL((halves_gather_kernel<LPE, 16>), dim3((unsigned)blocks), dim3(kHalvesThreads), 0, st, a,
                       idx, M, y);
  else
    hipLaunchKernelGGL((halves_gather_kernel<LPE, TT_MAX_D>), dim3((unsigned)blocks), dim3(kHalvesThreads), 0,
                       st, a, idx, M, y);
}

}  // namespace

// Internal entry points (arguments validated by the caller).
int halves_bytes(const tt_tensor *X, int split, size_t *bytes, long long *rows) {
  HalvesLayout L;
  int rc = halves_layout(X, split, L);
  if (rc) return rc;
  if (bytes) *bytes = L.total;
  if (rows) *rows = L.lrows[split] + L.rrows[split];
  return TT_OK;
}

int halves_build(const tt_tensor *X, int split, void *tables, hipStream_t st) {
  HalvesLayout L;
  int rc = halves_layout(X, split, L);
  if (rc) return rc;
  char *base = (char *)tables;
  const int d = X->d, s = split;
  // step t of both chains in one launch: left level t (from level t-1,
  // level 0 being [1]) and right level d-t (from level d-t+1, level d
  // being [1])
  auto left_job = [&](int j) {
    LevelJob jb;
    jb.A = (j == 1) ? nullptr : (const float *)(base + L.loff[j - 1]);
    jb.g = X->data + core_off(X, j - 1);
    jb.C = (float *)(base + L.loff[j]);
    jb.P = (j == 1) ? 1 : L.lrows[j - 1];
    jb.rl = X->r[j - 1];
    jb.n = X->n[j - 1];
    jb.rr = X->r[j];
    jb.right = 0;
    jb.tiles_p = (int)((jb.P + kTile - 1) / kTile);
    jb.tiles_j = (jb.n * jb.rr + kTile - 1) / kTile;
    return jb;
  };
  auto right_job = [&](int j) {
    LevelJob jb;
    jb.A = (j == d - 1) ? nullptr : (const float *)(base + L.roff[j + 1]);
    jb.g = X->data + core_off(X, j);
    jb.C = (float *)(base + L.roff[j]);
    jb.P = (j == d - 1) ? 1 : L.rrows[j + 1];
    jb.rl = X->r[j];
    jb.n = X->n[j];
    jb.rr = X->r[j + 1];
    jb.right = 1;
    jb.tiles_p = (int)((jb.P + kTile - 1) / kTile);
    jb.tiles_j = (jb.n * jb.rl + kTile - 1) / kTile;
    return jb;
  };
  const int steps = s > d - s ? s : d - s;
  for (int t = 1; t <= steps; ++t) {
    LevelJob a = {}, b = {};
    if (t <= s) a = left_job(t);
    if (t <= d - s) b = right_job(d - t);
    const long long blocks = (long long)a.tiles_p * a.tiles_j + (long long)b.tiles_p * b.tiles_j;
    timer_before(st);
    hipLaunchKernelGGL(halves_level_kernel, dim3((unsigned)blocks), dim3(kHalvesThreads), 0, st, a, b);
    timer_after(st);
    if ((rc = launch_check("halves level"))) return rc;
  }
  return TT_OK;
}

int halves_gather(const tt_tensor *X, int split, const void *tables, const int32_t *idx, int64_t M, float *y,
                  hipStream_t st) {
  if (M == 0) return TT_OK;
  HalvesLayout L;
  int rc = halves_layout(X, split, L);
  if (rc) return rc;
  HalvesArgs a;
  a.d = X->d;
  a.s = split;
  a.rs = X->r[split];
  for (int k = 0; k < TT_MAX_D; ++k) a.n[k] = k < X->d ? X->n[k] : 1;
  a.lt = (const float *)((const char *)tables + L.loff[split]);
  a.rt = (const float *)((const char *)tables + L.roff[split]);
  timer_before(st);
  switch (a.rs) {
    case 4: launch_gather_lpe<1>(a, idx, M, y, st); break;
    case 8: launch_gather_lpe<2>(a, idx, M, y, st); break;
    case 16: launch_gather_lpe<4>(a, idx, M, y, st); break;
    case 32: launch_gather_lpe<8>(a, idx, M, y, st); break;
    case 64: launch_gather_lpe<16>(a, idx, M, y, st); break;
    default: launch_gather_lpe<0>(a, idx, M, y, st); break;
  }
  timer_after(st);
  return launch_check("halves gather");
}

int halves_split_of(const tt_tensor *X) { return halves_auto_split(X); }

}  // namespace ttgfx

using namespace ttgfx;

extern "C" {

int32_t tt_halves_split(const tt_tensor *X) {
  int rc = validate_tt(X, "X", TT_MAX_RANK);
  if (rc) return rc;
  if (X->d < 2) return set_error(TT_ERR_UNSUPPORTED, "halves: needs d >= 2 (d = %d)", X->d);
  return halves_auto_split(X);
}

int64_t tt_halves_bytes(const tt_tensor *X, int32_t split) {
  int rc = halves_check(X, split);
  if (rc) return rc;
  size_t b = 0;
  if ((rc = halves_bytes(X, split, &b, nullptr))) return rc;
  return (int64_t)b;
}

int tt_halves_build(const tt_tensor *X, int32_t split, void *tables, size_t bytes, void *stream) {
  int rc = halves_check(X, split);
  if (rc) return rc;
  size_t need = 0;
  if ((rc = halves_bytes(X, split, &need, nullptr))) return rc;
  if (!tables || bytes < need)
    return set_error(TT_ERR_WORKSPACE, "halves_build: table buffer of %zu bytes given, %zu required",
                     tables ? bytes : (size_t)0, need);
  return halves_build(X, split, tables, (hipStream_t)stream);
}

int tt_halves_gather(const tt_tensor *X, int32_t split, const void *tables, size_t bytes, const int32_t *idx,
                     int64_t M, float *y, void *stream) {
  int rc = halves_check(X, split);
  if (rc) return rc;
  if (M < 0) return set_error(TT_ERR_ARG, "M = %lld is negative", (long long)M);
  if (M > 0 && (!idx || !y)) return set_error(TT_ERR_ARG, "halves_gather: null idx or y with M = %lld", (long long)M);
  if (M > (int64_t)0x7fffffff) return set_error(TT_ERR_UNSUPPORTED, "M = %lld above 2^31-1", (long long)M);
  size_t need = 0;
  if ((rc = halves_bytes(X, split, &need, nullptr))) return rc;
  if (!tables || bytes < need)
    return set_error(TT_ERR_WORKSPACE, "halves_gather: table buffer of %zu bytes given, %zu required",
                     tables ? bytes : (size_t)0, need);
  return halves_gather(X, split, tables, idx, M, y, (hipStream_t)stream);
}

}  // extern "C"
