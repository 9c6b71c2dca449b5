// Dense steps of the Riemannian update: QR orthogonalization sweeps, the
// tangent-space core assembly and TT-SVD rounding.
//
// The paper names rounding (t3f.round with max_tt_rank) and the tangent
// projection P_X; the algorithms are the standard ones of the TT literature
// it cites.  Each sweep is sequential over the cores, so one workgroup runs a
// whole sweep; the factorizations inside it are block-parallel:
//   * Householder QR (Golub & Van Loan, Alg. 5.1.1 / 5.2.1) with the sign
//     chosen so that diag(R) >= 0, thin Q by backward accumulation;
//   * SVD of the small R factor by one-sided (Hestenes) Jacobi rotations in
//     round-robin order, one wave per column pair;
//   * small GEMMs (one factor at most 64 x 64) on the fp32 matrix cores.
// Matrices live in a global workspace (they stay in L2); the Jacobi state
// lives in LDS.  All arithmetic is float32.
#include "common.h"
#include "dense.h"

namespace ttgfx {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;

// Elementwise work over a row-major rows x cols block with no 64-bit
// index division: at 64 columns or more, rows by wave (a wave-uniform
// index) and columns by lane; below, each wave takes 64 / cols rows at a
// time, every lane a fixed (row offset, column) pair computed once.
template <class F>
__device__ __forceinline__ void for_rows(int rows, int cols, F f) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (cols >= 64) {
    for (int row = wave; row < rows; row += kWaves)
      for (int c = lane; c < cols; c += 64) f(row, c);
  } else if (cols > 0) {
    const int rpw = 64 / cols;  // rows per wave and step
    const int sub = lane / cols, c = lane - sub * cols;
    if (sub < rpw)
      for (int row = wave * rpw + sub; row < rows; row += kWaves * rpw) f(row, c);
  }
}
constexpr int kJac = DENSE_MAX_RANK;  // Jacobi matrices are at most 64 x 64
constexpr int kProjBatch = 64;        // tensors per launch of a batched projection

struct Shared {
  float red[kWaves];
  float bval[4];
  int ival[4];
  __attribute__((aligned(16))) float jb[kJac * kJac];  // Jacobi working matrix B (column-major, ld = kJac)
  __attribute__((aligned(16))) float jv[kJac * kJac];  // accumulated rotations V (column-major, ld = kJac)
  float sig[kJac];
  int perm[kJac];
  int rotated;
  int wide;                 // Jacobi: some pair of the sweep had cos^2 above 1e-8
  float hv[2][64 * 10];     // register QR: broadcast Householder vector (double-buffered)
  float stg[64 * 65];       // staging chunk of the large GEMM operand
  float sm[64 * 65];        // the small GEMM factor, staged (row stride 65)
  float hb[kJac];           // register QR: reflector coefficients
};

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over the 64 lanes (all lanes active), returned wave-uniform: DPP
// butterflies inside each row of 16 (quad swaps, half-row and row
// mirrors), two row broadcasts that gather the four row sums in lane 63,
// and one read of that lane as a scalar.  VALU only, no LDS round trips.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<0xB1>(v);   // quad_perm(1,0,3,2)
  v += dpp_f<0x4E>(v);   // quad_perm(2,3,0,1)
  v += dpp_f<0x141>(v);  // row_half_mirror
  v += dpp_f<0x140>(v);  // row_mirror: every lane holds its row's sum
  v += dpp_f<0x142>(v);  // row_bcast:15: rows 1 and 3 add rows 0 and 2
  v += dpp_f<0x143>(v);  // row_bcast:31: row 3 adds lane 31 (rows 0 + 1)
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Sum over the block; every thread gets the result.
__device__ float block_sum(float v, Shared &sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh.red[wave] = v;
  __syncthreads();
  float s = 0.f;
  for (int w = 0; w < kWaves; ++w) s += sh.red[w];
  return s;
}

// In-place Householder QR of the column-major m x c matrix W (ld = m).
// On return the upper triangle holds R (diag >= 0) and column j below the
// diagonal holds v_j (v_j[j] = 1 implied); tau[j] = beta_j.
__device__ void blk_qr(float *W, int m, int c, float *tau, Shared &sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = m < c ? m : c;
  for (int j = 0; j < p; ++j) {
    float *col = W + (long)j * m;
    float part = 0.f;
#pragma unroll 8
    for (int i = j + 1 + threadIdx.x; i < m; i += kThreads) part = fmaf(col[i], col[i], part);
    const float sigma = block_sum(part, sh);
    if (threadIdx.x == 0) {
      const float x0 = col[j];
      float beta, v0, rjj;
      if (sigma == 0.f) {
        v0 = 1.f;
        beta = (x0 >= 0.f) ? 0.f : 2.f;
        rjj = fabsf(x0);
      } else {
        const float mu = sqrtf(x0 * x0 + sigma);
        v0 = (x0 <= 0.f) ? x0 - mu : -sigma / (x0 + mu);
        beta = 2.f * v0 * v0 / (sigma + v0 * v0);
        rjj = mu;
      }
      sh.bval[0] = v0;
      sh.bval[1] = beta;
      sh.bval[2] = rjj;
      tau[j] = beta;
    }
    __syncthreads();
    const float v0 = sh.bval[0], beta = sh.bval[1];
    if (sigma != 0.f) {
      const float inv = 1.f / v0;
      for (int i = j + 1 + threadIdx.x; i < m; i += kThreads) col[i] *= inv;
    }
    __syncthreads();
    // apply H_j to the trailing columns, one wave per column
    for (int l = j + 1 + wave; l < c; l += kWaves) {
      float *cl = W + (long)l * m;
      float s = 0.f;
#pragma unroll 8
      for (int i = j + 1 + lane; i < m; i += 64) s = fmaf(col[i], cl[i], s);
      s = wave_sum(s) + cl[j];
      const float w = beta * s;
      if (lane == 0) cl[j] -= w;
#pragma unroll 8
      for (int i = j + 1 + lane; i < m; i += 64) cl[i] = fmaf(-w, col[i], cl[i]);
    }
    if (threadIdx.x == 0) col[j] = sh.bval[2];
    __syncthreads();
  }
}

// Thin Q (m x p, column-major, ld = m) from the reflectors stored in W.
__device__ void blk_form_q(const float *W, int m, int c, const float *tau, float *Q, Shared &sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = m < c ? m : c;
  for (long e = threadIdx.x; e < (long)m * p; e += kThreads) {
    const int i = (int)(e % m), j = (int)(e / m);
    Q[e] = (i == j) ? 1.f : 0.f;
  }
  __syncthreads();
  for (int j = p - 1; j >= 0; --j) {
    const float *v = W + (long)j * m;
    const float beta = tau[j];
    for (int l = j + wave; l < p; l += kWaves) {
      float *ql = Q + (long)l * m;
      float s = 0.f;
#pragma unroll 8
      for (int i = j + 1 + lane; i < m; i += 64) s = fmaf(v[i], ql[i], s);
      s = wave_sum(s) + ql[j];
      const float w = beta * s;
      if (lane == 0) ql[j] -= w;
#pragma unroll 8
      for (int i = j + 1 + lane; i < m; i += 64) ql[i] = fmaf(-w, v[i], ql[i]);
    }
    __syncthreads();
  }
}

// Sum over the 16 lanes of a DPP row; every lane of the row gets it.
__device__ __forceinline__ float row16_sum(float v) {
  v += dpp_f<0xB1>(v);   // quad_perm(1,0,3,2)
  v += dpp_f<0x4E>(v);   // quad_perm(2,3,0,1)
  v += dpp_f<0x141>(v);  // row_half_mirror
  v += dpp_f<0x140>(v);  // row_mirror
  return v;
}

// Three row sums at once, their steps interleaved so that no DPP read waits
// on the add just before it.
__device__ __forceinline__ void row16_sum3(float &x, float &y, float &z) {
  x += dpp_f<0xB1>(x);
  y += dpp_f<0xB1>(y);
  z += dpp_f<0xB1>(z);
  x += dpp_f<0x4E>(x);
  y += dpp_f<0x4E>(y);
  z += dpp_f<0x4E>(z);
  x += dpp_f<0x141>(x);
  y += dpp_f<0x141>(y);
  z += dpp_f<0x141>(z);
  x += dpp_f<0x140>(x);
  y += dpp_f<0x140>(y);
  z += dpp_f<0x140>(z);
}

// Sums over the 64 lanes of N values at once, returned wave-uniform: each
// butterfly stage of wave_sum runs on all N values before the next, so the
// N dependent chains overlap instead of running back to back.
template <int N>
__device__ __forceinline__ void wave_sum_n(float (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_f<0xB1>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_f<0x4E>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_f<0x141>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_f<0x140>(v[i]);
  // every lane of a row now holds the row's sum: row_bcast:15 adds row 0's
  // into row 1 and row 2's into row 3, row_bcast:31 then adds lane 31
  // (rows 0 + 1) into row 3, and lane 63 holds the total (rows 0 and 2,
  // whatever they receive, are not read)
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_f<0x142>(v[i]);  // row_bcast:15
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_f<0x143>(v[i]);  // row_bcast:31
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[i]), 63));
}

// Householder QR plus thin Q of an m x c matrix (m <= 64 RR, c <= 64) held
// in registers: wave w owns columns w, w + 8, ..., lane l rows l, l + 64, ...
// Element (i, j) is read through load(i, j).  For each column the owner
// wave forms the reflector and broadcasts it through LDS (double-buffered,
// one barrier per column); every wave applies it to its own trailing
// columns, with the dot products of all its columns reduced together.  Q is
// then accumulated backwards, each column on its own (it is
// H_0 .. H_{p-1} e_col) with no barriers, the reflectors read back from Wm.
// On return Wm (column-major, ld = m) holds R in its upper triangle and the
// reflectors below it, and Q (m x p) went through storeq(i, j, value).  Same
// arithmetic as blk_qr / blk_form_q (diag(R) >= 0); only the data placement
// and the summation order differ.
constexpr int kRegRows = 10;               // rows per lane at the largest size (m <= 640)
constexpr int kRegCols = kJac / kWaves;    // columns per wave
static_assert(kRegCols * kWaves == kJac, "columns must split over the waves");

__device__ bool reg_qr_fits(int m, int c) { return m <= 64 * kRegRows && c <= kJac; }

// wave_sum_n over the eight column sums of a wave; either half is skipped
// when none of its columns is still live (first_live, second_live false;
// the second half has no columns at all when the matrix has at most 32).
__device__ __forceinline__ void reduce_live(float (&sp)[kRegCols], bool first_live, bool second_live) {
  float lo[kRegCols / 2], hi[kRegCols / 2];
#pragma unroll
  for (int i = 0; i < kRegCols / 2; ++i) {
    lo[i] = sp[i];
    hi[i] = sp[kRegCols / 2 + i];
  }
  if (first_live) wave_sum_n<kRegCols / 2>(lo);
  if (second_live) wave_sum_n<kRegCols / 2>(hi);
#pragma unroll
  for (int i = 0; i < kRegCols / 2; ++i) {
    sp[i] = lo[i];
    sp[kRegCols / 2 + i] = hi[i];
  }
}

template <int C, int RR>
__device__ __forceinline__ void take_col(const float (&x)[kRegCols][RR], float (&y)[RR]) {
  static_assert(C < kRegCols, "column slot out of range");
#pragma unroll
  for (int rr = 0; rr < RR; ++rr) y[rr] = x[C][rr];
}

template <int RR, class Load, class StoreQ>
__device__ void reg_qr(Load load, int m, int c, float *Wm, StoreQ storeq, Shared &sh) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int p = m < c ? m : c;
  float x[kRegCols][RR];
#pragma unroll
  for (int cc = 0; cc < kRegCols; ++cc)
#pragma unroll
    for (int rr = 0; rr < RR; ++rr) {
      const int col = wave + kWaves * cc, row = lane + 64 * rr;
      x[cc][rr] = (col < c && row < m) ? load(row, col) : 0.f;
    }
  // ---- factorization
  for (int j = 0; j < p; ++j) {
    const int owner = j % kWaves, cj = j / kWaves;
    float *hv = sh.hv[j & 1];
    if (wave == owner) {
      float y[RR];  // column j: a uniform branch on cj, constant register indices
      switch (cj) {
        case 0: take_col<0>(x, y); break;
        case 1: take_col<1>(x, y); break;
        case 2: take_col<2>(x, y); break;
        case 3: take_col<3>(x, y); break;
        case 4: take_col<4>(x, y); break;
        case 5: take_col<5>(x, y); break;
        case 6: take_col<6>(x, y); break;
        default: take_col<7>(x, y); break;
      }
      float sx[2] = {0.f, 0.f};  // sigma = |x(j+1:)|^2, x0 = x(j)
#pragma unroll
      for (int rr = 0; rr < RR; ++rr) {
        const int row = lane + 64 * rr;
        if (row > j && row < m) sx[0] = fmaf(y[rr], y[rr], sx[0]);
        if (row == j) sx[1] = y[rr];
      }
      wave_sum_n<2>(sx);
      const float sigma = sx[0], x0 = sx[1];
      float beta, v0, rjj;
      if (sigma == 0.f) {
        v0 = 1.f;
        beta = (x0 >= 0.f) ? 0.f : 2.f;
        rjj = fabsf(x0);
      } else {
        // sigma > 0, so x0 + mu > 0 when x0 > 0, v0 < 0 and sigma + v0^2 > 0:
        // the hardware reciprocal (about 1 ulp) is safe for all three
        // quotients on this wave's serial path
        const float mu = sqrtf(x0 * x0 + sigma);
        v0 = (x0 <= 0.f) ? x0 - mu : -sigma * __builtin_amdgcn_rcpf(x0 + mu);
        beta = 2.f * v0 * v0 * __builtin_amdgcn_rcpf(sigma + v0 * v0);
        rjj = mu;
      }
      const float inv = (sigma != 0.f) ? __builtin_amdgcn_rcpf(v0) : 1.f;
#pragma unroll
      for (int rr = 0; rr < RR; ++rr) {
        const int row = lane + 64 * rr;
        float v = 0.f;
        if (row > j) {
          y[rr] *= inv;  // reflector below the diagonal
          v = y[rr];
        } else if (row == j) {
          y[rr] = rjj;   // R(j, j)
          v = 1.f;
        }
        if (row < m) hv[row] = v;
      }
#pragma unroll
      for (int cc = 0; cc < kRegCols; ++cc)
        if (cc == cj) {
#pragma unroll
          for (int rr = 0; rr < RR; ++rr) x[cc][rr] = y[rr];
        }
      if (lane == 0) sh.hb[j] = beta;
    }
    __syncthreads();
    const float beta = sh.hb[j];
    float v[RR];
#pragma unroll
    for (int rr = 0; rr < RR; ++rr) {
      const int row = lane + 64 * rr;
      v[rr] = (row < m) ? hv[row] : 0.f;
    }
    // trailing columns of this wave: col > j, col < c (a wave-uniform
    // range); finished columns take no dot products, and a half of the
    // columns with none left takes no reduction
    float sp[kRegCols];
#pragma unroll
    for (int cc = 0; cc < kRegCols; ++cc) {
      sp[cc] = 0.f;
      const int col = wave + kWaves * cc;
      if (col <= j || col >= c) continue;
#pragma unroll
      for (int rr = 0; rr < RR; ++rr) sp[cc] = fmaf(v[rr], x[cc][rr], sp[cc]);
    }
    reduce_live(sp, wave + kWaves * (kRegCols / 2 - 1) > j,
                wave + kWaves * (kRegCols / 2) < c && wave + kWaves * (kRegCols - 1) > j);
#pragma unroll
    for (int cc = 0; cc < kRegCols; ++cc) {
      const int col = wave + kWaves * cc;
      if (col <= j || col >= c) continue;
      const float w = beta * sp[cc];
#pragma unroll
      for (int rr = 0; rr < RR; ++rr) x[cc][rr] = fmaf(-w, v[rr], x[cc][rr]);
    }
  }
  // R (upper triangle) and the reflectors (below it) to Wm; the register
  // tile is dead from here on, which leaves its registers to Q
#pragma unroll
  for (int cc = 0; cc < kRegCols; ++cc)
#pragma unroll
    for (int rr = 0; rr < RR; ++rr) {
      const int col = wave + kWaves * cc, row = lane + 64 * rr;
      if (col < c && row < m) Wm[(long)col * m + row] = x[cc][rr];
    }
  // ---- thin Q by backward accumulation (no barriers: each column of Q
  // is H_0 .. H_{p-1} e_col on its own); the next reflector is loaded from
  // Wm while the current one is applied
  float q[kRegCols][RR];
#pragma unroll
  for (int cc = 0; cc < kRegCols; ++cc)
#pragma unroll
    for (int rr = 0; rr < RR; ++rr) {
      const int col = wave + kWaves * cc, row = lane + 64 * rr;
      q[cc][rr] = (row == col) ? 1.f : 0.f;
    }
  __syncthreads();  // Wm's reflectors are visible to every wave
  // Reflector j from Wm through global-memory loads (a flat load would also
  // hold up the LDS counter), every lane loading unconditionally (rows past
  // m read row m - 1, rows at or above j are replaced), so that the
  // compiler's memory-counter waits stay exact: two register sets used in
  // turn, each loaded one step before its use.
  const __attribute__((address_space(1))) float *Wg = (const __attribute__((address_space(1))) float *)Wm;
  auto fetch = [&](int j, float(&dst)[RR]) __attribute__((always_inline)) {
    const __attribute__((address_space(1))) float *wc = Wg + (long)j * m;
#pragma unroll
    for (int rr = 0; rr < RR; ++rr) {
      const int row = lane + 64 * rr;
      const float t = wc[row < m ? row : m - 1];
      dst[rr] = (row > j && row < m) ? t : (row == j ? 1.f : 0.f);
    }
  };
  auto apply = [&](int j, const float(&v)[RR]) __attribute__((always_inline)) {
    const float beta = sh.hb[j];
    float sp[kRegCols];
#pragma unroll
    for (int cc = 0; cc < kRegCols; ++cc) {
      sp[cc] = 0.f;
      const int col = wave + kWaves * cc;
      if (col < j || col >= p) continue;
#pragma unroll
      for (int rr = 0; rr < RR; ++rr) sp[cc] = fmaf(v[rr], q[cc][rr], sp[cc]);
    }
    reduce_live(sp, wave + kWaves * (kRegCols / 2 - 1) >= j,
                wave + kWaves * (kRegCols / 2) < p && wave + kWaves * (kRegCols - 1) >= j);
#pragma unroll
    for (int cc = 0; cc < kRegCols; ++cc) {
      const int col = wave + kWaves * cc;
      if (col < j || col >= p) continue;
      const float w = beta * sp[cc];
#pragma unroll
      for (int rr = 0; rr < RR; ++rr) q[cc][rr] = fmaf(-w, v[rr], q[cc][rr]);
    }
  };
  float va[RR], vb[RR];
  fetch(p - 1, va);
  int j = p - 1;
  for (; j >= 1; j -= 2) {
    fetch(j - 1, vb);
    apply(j, va);
    fetch(j >= 2 ? j - 2 : 0, va);  // j = 1: a spare load of reflector 0
    apply(j - 1, vb);
  }
  if (j == 0) apply(0, va);
  __syncthreads();  // every load and LDS read precedes the stores below
#pragma unroll
  for (int cc = 0; cc < kRegCols; ++cc)
#pragma unroll
    for (int rr = 0; rr < RR; ++rr) {
      const int col = wave + kWaves * cc, row = lane + 64 * rr;
      if (col < p && row < m) storeq(row, col, q[cc][rr]);
    }
  __syncthreads();
}

// QR with thin Q of the m x c matrix read through load(i, j): registers
// when the matrix fits, else the global-memory kernels on a column-major
// copy in Wm (ld = m) with Q built in Qg.  On return R is in Wm's upper
// triangle and Q went through storeq(i, j, value) (which may write over the
// source that load reads).
template <class Load, class StoreQ>
__device__ void qr_thin(Load load, int m, int c, float *Wm, float *tau, float *Qg, StoreQ storeq, Shared &sh) {
  if (reg_qr_fits(m, c)) {
    // rows per lane: the smallest of 2, 5 and 10 that holds the m rows
    if (m <= 128) reg_qr<2>(load, m, c, Wm, storeq, sh);
    else if (m <= 320) reg_qr<5>(load, m, c, Wm, storeq, sh);
    else reg_qr<kRegRows>(load, m, c, Wm, storeq, sh);
    return;
  }
  const int p = m < c ? m : c;
  for (long e = threadIdx.x; e < (long)m * c; e += kThreads) Wm[e] = load((int)(e % m), (int)(e / m));
  __syncthreads();
  blk_qr(Wm, m, c, tau, sh);
  blk_form_q(Wm, m, c, tau, Qg, sh);
  __syncthreads();
  for (long e = threadIdx.x; e < (long)m * p; e += kThreads) storeq((int)(e % m), (int)(e / m), Qg[e]);
  __syncthreads();
}

// One-sided Jacobi on the columns of sh.jb (rows x cols, ld = kJac); sh.jv
// accumulates the rotations (cols x cols).  On return the columns of jb are
// mutually orthogonal (jb = B V) and V is orthogonal.  Block-cyclic order:
// the columns form nb blocks of 4 (nb even).  In each of a sweep's nb - 1
// super-rounds a round-robin tournament hands wave w one pair of blocks, and
// the wave rotates the 16 column pairs between them in 4 rounds of 4
// disjoint pairs (in the first super-round also the 6 pairs inside each of
// its two blocks, in 3 more rounds).  A row of 16 lanes takes one pair, with
// 4 matrix rows per lane (jb and jv are zero beyond rows and cols, so whole
// columns of 64 are rotated).  Inside a super-round no other wave touches
// the wave's blocks and a wave's LDS accesses complete in issue order, so
// only the super-rounds end with a workgroup barrier: nb - 1 barriers per
// sweep instead of one per round.
__device__ int blk_jacobi(int rows, int cols, Shared &sh) {
  (void)rows;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < kJac * kJac; e += kThreads) {
    const int i = e % kJac, j = e / kJac;
    sh.jv[e] = (i == j) ? 1.f : 0.f;
  }
  __syncthreads();
  int nb = (cols + 3) >> 2;
  nb += nb & 1;  // at most kJac / 4 = 2 kWaves blocks
  const int slot = lane >> 4, c4 = 4 * (lane & 15);
  const bool live = wave < nb / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (threadIdx.x == 0) {
      sh.rotated = 0;
      sh.wide = 0;
    }
    bool wide = false;  // this row met a pair with ga^2 > 1e-8 al be in the sweep
    __syncthreads();
    // block position ba = w pairs with bb = nb-1-w; every position other
    // than 0 advances by one block per super-round
    int ba = wave, bb = nb - 1 - wave;
    for (int sr = 0; sr < nb - 1; ++sr) {
      if (live) {
        const int nloc = sr == 0 ? 7 : 4;
        for (int t = 0; t < nloc; ++t) {
          int pa, pb;
          if (sr == 0 && t < 3) {
            // inside a block: rows 0, 1 of lanes in block ba, rows 2, 3 in
            // bb; pairs (0,1)(2,3), then (0,2)(1,3), then (0,3)(1,2)
            const int blk = slot < 2 ? ba : bb, h = slot & 1;
            const int i = t == 0 ? 2 * h : h;
            const int j = t == 0 ? 2 * h + 1 : (t == 1 ? h + 2 : 3 - h);
            pa = 4 * blk + i;
            pb = 4 * blk + j;
          } else {
            const int sh4 = sr == 0 ? t - 3 : t;
            pa = 4 * ba + slot;
            pb = 4 * bb + ((slot + sh4) & 3);
          }
          const bool on = pa < cols && pb < cols;
          const v4f xa = *(const v4f *)(sh.jb + pa * kJac + c4);
          const v4f xb = *(const v4f *)(sh.jb + pb * kJac + c4);
          const v4f ya = *(const v4f *)(sh.jv + pa * kJac + c4);
          const v4f yb = *(const v4f *)(sh.jv + pb * kJac + c4);
          float al = 0.f, be = 0.f, ga = 0.f;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            al = fmaf(xa[v], xa[v], al);
            be = fmaf(xb[v], xb[v], be);
            ga = fmaf(xa[v], xb[v], ga);
          }
          // the rotation's V columns were read with the B columns; this
          // empty use keeps the compiler from sinking those reads into the
          // branch below, which would add a second LDS round trip
          asm volatile("" ::"v"(ya), "v"(yb));
          row16_sum3(al, be, ga);
          // every lane of the row takes the same decision
          // |ga| > 1e-6 sqrt(al be), compared squared; the rotation uses the
          // hardware reciprocal, square root and reciprocal square root
          // (about 1 ulp each, so cs^2 + sn^2 = 1 to a few ulp), which
          // shortens the dependent chain of every round.  A rotating pair
          // has ga^2 > 0, so 1 / (2 ga) is finite and zeta is never 0 * inf.
          wide |= on && ga * ga > 1e-8f * (al * be);
          if (on && ga * ga > 1e-12f * (al * be) && ga != 0.f) {
            const float zeta = (be - al) * __builtin_amdgcn_rcpf(2.f * ga);
            const float tn = copysignf(1.f, zeta) *
                             __builtin_amdgcn_rcpf(fabsf(zeta) + __builtin_amdgcn_sqrtf(fmaf(zeta, zeta, 1.f)));
            const float cs = __builtin_amdgcn_rsqf(fmaf(tn, tn, 1.f));
            const float sn = cs * tn;
            v4f na, nb4, ma, mb;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              na[v] = cs * xa[v] - sn * xb[v];
              nb4[v] = sn * xa[v] + cs * xb[v];
              ma[v] = cs * ya[v] - sn * yb[v];
              mb[v] = sn * ya[v] + cs * yb[v];
            }
            *(v4f *)(sh.jb + pa * kJac + c4) = na;
            *(v4f *)(sh.jb + pb * kJac + c4) = nb4;
            *(v4f *)(sh.jv + pa * kJac + c4) = ma;
            *(v4f *)(sh.jv + pb * kJac + c4) = mb;
            if ((lane & 15) == 0) sh.rotated = 1;
          }
          // the next round reads columns that other rows of this wave just
          // wrote: keep the compiler from moving LDS accesses across rounds
          asm volatile("" ::: "memory");
        }
      }
      if (ba != 0) ba = (ba == nb - 1) ? 1 : ba + 1;
      bb = (bb == nb - 1) ? 1 : bb + 1;
      __syncthreads();
    }
    if ((lane & 15) == 0 && wide) sh.wide = 1;
    __syncthreads();
    const int any = sh.rotated, w = sh.wide;
    __syncthreads();
    if (!any) return sweep + 1;
    // Cyclic Jacobi converges quadratically: after a sweep whose pairs were
    // all within |cos| <= 1e-4 of orthogonal, the next sweep's pairs are
    // within about 1e-8, below the 1e-6 rotation threshold, so that sweep
    // would only confirm convergence.
    if (!w) return sweep + 1;
  }
  return -1;  // not converged within 40 sweeps
}

// The two GEMM helpers below run on the fp32 matrix cores
// (v_mfma_f32_16x16x4f32).  Each 64 x 64 block of C is 16 tiles of 16 x 16;
// wave w takes row tile w % 4 and column tiles w / 4 and w / 4 + 2.  MFMA
// operands, lane (q4, c16) = (lane / 16, lane % 16): A(row c16, k q4),
// B(k q4, column c16); the result lane holds C(rows 4 q4 .. 4 q4 + 3,
// column c16).  Both factors sit in LDS as zero-padded 64 x 64 tables of
// row stride 65: the small one (read through its accessor) in sh.sm, the
// large one (staged from global memory in 64-row or 64-column chunks) in
// sh.stg.

// One 64 x 64 block: C(i, j) = sum_l A(i, l) B(l, j) for l < K, with A at
// ta[i * 65 + l] and B at tb[l * 65 + j]; K rounded up to 4 (the tables are
// zero past K).  out(i, j, value) stores the block's elements.
template <class Out>
__device__ __forceinline__ void mfma_block(const float *ta, const float *tb, int K, Out out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c16 = lane & 15, q4 = lane >> 4;
  const int rt = wave & 3, ct0 = wave >> 2;
  v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 4) {
    const float av = ta[(16 * rt + c16) * 65 + k0 + q4];
    const float b0 = tb[(k0 + q4) * 65 + 16 * ct0 + c16];
    const float b1 = tb[(k0 + q4) * 65 + 16 * (ct0 + 2) + c16];
    acc0 = mfma4(av, b0, acc0);
    acc1 = mfma4(av, b1, acc1);
  }
  __syncthreads();  // every read of the staged tables precedes the stores
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    out(16 * rt + 4 * q4 + v, 16 * ct0 + c16, acc0[v]);
    out(16 * rt + 4 * q4 + v, 16 * (ct0 + 2) + c16, acc1[v]);
  }
}

// C (M x N) = A (M x K) * B (K x N) for K <= 64, the small factor A read
// through aop(i, l) (consecutive l on consecutive lanes when staged), B in
// global memory (element (l, j) at B[l*br + j*bc]), staged in chunks of 64
// columns; each thread loads its part of the next chunk into registers
// while the current one is multiplied.  C may alias B: a chunk's columns
// are written only after the whole chunk was staged, and the next chunk's
// columns were read before (element (i, j) of C at C[i*cr + j*cc]).
template <class AOp>
__device__ void gemm_lds_a(int M, int N, int K, AOp aop, const float *B, long br, long bc, float *C, long cr,
                           long cc, Shared &sh) {
  constexpr int PER = 64 * 64 / kThreads;
  auto fetch = [&](int j0, float (&r)[PER]) {
    const int nc = (N - j0) < 64 ? (N - j0) : 64;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * kThreads;
      const int l = e >> 6, jj = e & 63;
      r[u] = (jj < nc && l < K) ? B[(long)l * br + (long)(j0 + jj) * bc] : 0.f;
    }
  };
  for (int i0 = 0; i0 < M; i0 += 64) {
    const int mr = (M - i0) < 64 ? (M - i0) : 64;
    for (int e = threadIdx.x; e < 64 * 64; e += kThreads) {
      const int i = e >> 6, l = e & 63;
      sh.sm[i * 65 + l] = (i < mr && l < K) ? aop(i0 + i, l) : 0.f;
    }
    float cur[PER];
    fetch(0, cur);
    for (int j0 = 0; j0 < N; j0 += 64) {
      const int nc = (N - j0) < 64 ? (N - j0) : 64;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * kThreads;
        sh.stg[(e >> 6) * 65 + (e & 63)] = cur[u];
      }
      __syncthreads();
      if (j0 + 64 < N) fetch(j0 + 64, cur);
      mfma_block(sh.sm, sh.stg, K, [&](int i, int jj, float v) {
        if (i < mr && jj < nc) C[(long)(i0 + i) * cr + (long)(j0 + jj) * cc] = v;
      });
    }
    __syncthreads();
  }
}

// C (M x N) = A (M x K) * B (K x N) for K <= 64 and N <= 64, A in global
// memory (element (i, l) at A[i*ar + l*ac]) staged in chunks of 64 rows
// (the next chunk loaded into registers while the current one is
// multiplied), the small factor B read through bop(l, j).  ROWS_ON_LANES:
// bop is read with consecutive l on consecutive lanes (for factors whose
// elements of one row l are 64 floats apart), else with consecutive j.  C
// may alias A when row i of C (C[i*ldc + j]) never reaches past row i of
// A, i.e. ldc <= A's row stride: a chunk's rows are written after the chunk
// and the next one were read.
template <bool ROWS_ON_LANES = false, class BOp>
__device__ void gemm_lds_b(int M, int N, int K, const float *A, long ar, long ac, BOp bop, float *C, long ldc,
                           Shared &sh) {
  constexpr int PER = 64 * 64 / kThreads;
  for (int e = threadIdx.x; e < 64 * 64; e += kThreads) {
    const int l = ROWS_ON_LANES ? (e & 63) : (e >> 6), j = ROWS_ON_LANES ? (e >> 6) : (e & 63);
    sh.sm[l * 65 + j] = (l < K && j < N) ? bop(l, j) : 0.f;
  }
  // consecutive threads walk the unit-stride index of A (coalesced loads)
  auto fetch = [&](int i0, float (&r)[PER]) {
    const int mr = (M - i0) < 64 ? (M - i0) : 64;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * kThreads;
      const int ii = (ar == 1) ? (e & 63) : (e >> 6), l = (ar == 1) ? (e >> 6) : (e & 63);
      r[u] = (ii < mr && l < K) ? A[(long)(i0 + ii) * ar + (long)l * ac] : 0.f;
    }
  };
  float cur[PER];
  fetch(0, cur);
  for (int i0 = 0; i0 < M; i0 += 64) {
    const int mr = (M - i0) < 64 ? (M - i0) : 64;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * kThreads;
      const int ii = (ar == 1) ? (e & 63) : (e >> 6), l = (ar == 1) ? (e >> 6) : (e & 63);
      sh.stg[ii * 65 + l] = cur[u];
    }
    __syncthreads();
    if (i0 + 64 < M) fetch(i0 + 64, cur);
    mfma_block(sh.stg, sh.sm, K, [&](int ii, int j, float v) {
      if (ii < mr && j < N) C[(long)(i0 + ii) * ldc + j] = v;
    });
  }
  __syncthreads();
}

// Cores of the working TT in the workspace: each core has its own slot of
// `slot` floats; shape (r[k], n[k], r[k+1]) row-major.
struct WorkTT {
  float *data;
  long slot;
  __device__ float *core(int k) const { return data + (long)k * slot; }
};

__device__ void copy_in(const TTDev &X, WorkTT &w) {
  for (int k = 0; k < X.d; ++k) {
    const long n = (long)X.r[k] * X.n[k] * X.r[k + 1];
    const float *src = X.data + X.off[k];
    float *dst = w.core(k);
    for (long e = threadIdx.x; e < n; e += kThreads) dst[e] = src[e];
  }
  __syncthreads();
}

// Left-to-right QR sweep over the working TT; ranks r[] updated in place.
// Core k becomes left-orthonormal; the last core carries the tensor.
__device__ void sweep_lr(WorkTT &w, int d, const int *n, int *r, float *Wm, float *Q, float *tau,
                         Shared &sh) {
  for (int k = 0; k + 1 < d; ++k) {
    const int m = r[k] * n[k], c = r[k + 1];
    const int p = m < c ? m : c;
    float *G = w.core(k);
    // QR of the left unfolding (row-major m x c); core k <- Q (row-major
    // m x p), written over the unfolding once it was read
    qr_thin([&](int i, int j) { return G[(long)i * c + j]; }, m, c, Wm, tau, Q,
            [&](int i, int j, float v) { G[(long)i * p + j] = v; }, sh);
    // next core <- R (p x c, upper triangle of Wm) * next (c x n r'), in place
    const int nn = n[k + 1] * r[k + 2];
    float *Gn = w.core(k + 1);
    for (int e = threadIdx.x; e < kJac * kJac; e += kThreads) {
      const int i = e / kJac, l = e % kJac;
      sh.jb[e] = (i < p && l < c && l >= i) ? Wm[(long)l * m + i] : 0.f;
    }
    __syncthreads();
    gemm_lds_a(p, nn, c, [&](int i, int l) { return sh.jb[i * kJac + l]; }, Gn, nn, 1, Gn, nn, 1, sh);
    if (threadIdx.x == 0) r[k + 1] = p;
    __syncthreads();
  }
}

// Right-to-left LQ sweep; core k becomes right-orthonormal, the first core
// carries the tensor.
__device__ void sweep_rl(WorkTT &w, int d, const int *n, int *r, float *Wm, float *Q, float *tau,
                         Shared &sh) {
  for (int k = d - 1; k >= 1; --k) {
    const int rows = r[k], mm = n[k] * r[k + 1];  // unfolding rows x mm; QR of its transpose
    const int p = mm < rows ? mm : rows;
    float *G = w.core(k);
    // QR of the transposed right unfolding (mm x rows; the row-major core
    // holds it column-major); core k <- Q^T (p x mm row-major = Q
    // column-major), written over the core once it was read
    qr_thin([&](int i, int j) { return G[(long)j * mm + i]; }, mm, rows, Wm, tau, Q,
            [&](int i, int j, float v) { G[(long)j * mm + i] = v; }, sh);
    // previous core (r[k-1] n[k-1] x rows) <- prev * L, L = R^T (rows x p),
    // in place (the output row stride p does not exceed rows)
    const int mp = r[k - 1] * n[k - 1];
    float *Gp = w.core(k - 1);
    for (int e = threadIdx.x; e < kJac * kJac; e += kThreads) {
      const int l = e / kJac, j = e % kJac;  // L[l][j] = R[j][l], nonzero for l >= j
      sh.jb[e] = (l < rows && j < p && l >= j) ? Wm[(long)l * mm + j] : 0.f;
    }
    __syncthreads();
    gemm_lds_b(mp, p, rows, Gp, rows, 1, [&](int l, int j) { return sh.jb[l * kJac + j]; }, Gp, p, sh);
    if (threadIdx.x == 0) r[k] = p;
    __syncthreads();
  }
}

__device__ void copy_out(const WorkTT &w, int d, const int *n, const int *r, const TTDev &O) {
  for (int k = 0; k < d; ++k) {
    const long cnt = (long)r[k] * n[k] * r[k + 1];
    const float *src = w.core(k);
    float *dst = O.data + O.off[k];
    for (long e = threadIdx.x; e < cnt; e += kThreads) dst[e] = src[e];
  }
}

struct DenseBufs {
  float *work;    // working TT cores
  long slot;      // floats per core slot
  float *wm;      // m x c matrix
  float *q;       // m x p matrix
  float *tau;     // reflector coefficients
};

__global__ void __launch_bounds__(kThreads) orth_kernel(TTDev X, TTDev O, int dir, DenseBufs b) {
  __shared__ Shared sh;
  __shared__ int n[TT_MAX_D], r[TT_MAX_D + 1];
  for (int k = threadIdx.x; k < X.d; k += kThreads) n[k] = X.n[k];
  for (int k = threadIdx.x; k <= X.d; k += kThreads) r[k] = X.r[k];
  WorkTT w{b.work, b.slot};
  copy_in(X, w);
  if (dir == TT_LR) sweep_lr(w, X.d, n, r, b.wm, b.q, b.tau, sh);
  else sweep_rl(w, X.d, n, r, b.wm, b.q, b.tau, sh);
  copy_out(w, X.d, n, r, O);
}

// Both sweeps at once: workgroup 0 runs the left-to-right sweep into OL,
// workgroup 1 the right-to-left sweep into OR, each on its own buffers.
__global__ void __launch_bounds__(kThreads) orth_both_kernel(TTDev X, TTDev OL, TTDev OR, DenseBufs bl,
                                                             DenseBufs br) {
  __shared__ Shared sh;
  __shared__ int n[TT_MAX_D], r[TT_MAX_D + 1];
  for (int k = threadIdx.x; k < X.d; k += kThreads) n[k] = X.n[k];
  for (int k = threadIdx.x; k <= X.d; k += kThreads) r[k] = X.r[k];
  // Branch on the workgroup rather than select between the by-value
  // parameters: a selected reference would force them into private memory.
  if (blockIdx.x == 0) {
    WorkTT w{bl.work, bl.slot};
    copy_in(X, w);
    sweep_lr(w, X.d, n, r, bl.wm, bl.q, bl.tau, sh);
    copy_out(w, X.d, n, r, OL);
  } else {
    WorkTT w{br.work, br.slot};
    copy_in(X, w);
    sweep_rl(w, X.d, n, r, br.wm, br.q, br.tau, sh);
    copy_out(w, X.d, n, r, OR);
  }
}

// TT rounding: right-to-left LQ sweep, then left-to-right truncated SVDs.
__global__ void __launch_bounds__(kThreads) round_kernel(TTDev Y, TTDev O, int max_rank,
                                                         float *disc, int *status, DenseBufs b) {
  __shared__ Shared sh;
  __shared__ int n[TT_MAX_D], r[TT_MAX_D + 1];
  const int d = Y.d;
  int unconverged = 0;  // bonds whose Jacobi SVD hit the sweep limit (thread 0's count)
  for (int k = threadIdx.x; k < d; k += kThreads) n[k] = Y.n[k];
  for (int k = threadIdx.x; k <= d; k += kThreads) r[k] = Y.r[k];
  WorkTT w{b.work, b.slot};
  copy_in(Y, w);
  sweep_rl(w, d, n, r, b.wm, b.q, b.tau, sh);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = 0; k + 1 < d; ++k) {
    const int m = r[k] * n[k], c = r[k + 1];
    const int p = m < c ? m : c;
    float *G = w.core(k);
    float *bq = b.q;
    qr_thin([&](int i, int j) { return G[(long)i * c + j]; }, m, c, b.wm, b.tau, bq,
            [&](int i, int j, float v) { bq[(long)j * m + i] = v; }, sh);
    // Jacobi on B = R^T (c x p): jb[row l][col j] = R[j][l]
    for (int e = threadIdx.x; e < kJac * kJac; e += kThreads) {
      const int l = e % kJac, j = e / kJac;
      sh.jb[e] = (l < c && j < p && l >= j) ? b.wm[(long)l * m + j] : 0.f;
    }
    __syncthreads();
    if (blk_jacobi(c, p, sh) < 0) ++unconverged;
    // singular values (column norms of B V) and their descending order
    for (int j = wave; j < p; j += kWaves) {
      const float x = lane < c ? sh.jb[j * kJac + lane] : 0.f;
      const float s2 = wave_sum(x * x);
      if (lane == 0) sh.sig[j] = sqrtf(s2);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < p; j += kThreads) {
      int rank = 0;
      for (int l = 0; l < p; ++l)
        rank += (sh.sig[l] > sh.sig[j]) || (sh.sig[l] == sh.sig[j] && l < j);
      sh.perm[rank] = j;
    }
    __syncthreads();
    const int keep = max_rank < p ? max_rank : p;
    if (threadIdx.x == 0 && disc) {
      float s = 0.f;
      for (int l = keep; l < p; ++l) s += sh.sig[sh.perm[l]] * sh.sig[sh.perm[l]];
      disc[k] = s;
    }
    // U = Q (m x p) * V[:, perm[j]] for j < keep -> core k (row-major m x keep)
    // (columns of V are kJac floats apart: one LDS bank for a fixed l)
    gemm_lds_b<true>(m, keep, p, b.q, 1, m, [&](int l, int j) { return sh.jv[sh.perm[j] * kJac + l]; }, G, keep,
                     sh);
    // sign fix: the largest-magnitude component of each kept column is positive
    for (int j = wave; j < keep; j += kWaves) {
      float best = -1.f, val = 0.f;
      int bi = 1 << 30;
      for (int i = lane; i < m; i += 64) {
        const float x = G[(long)i * keep + j];
        if (fabsf(x) > best) {
          best = fabsf(x);
          val = x;
          bi = i;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const float ob = __shfl_xor(best, off), ov = __shfl_xor(val, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          val = ov;
          bi = oi;
        }
      }
      if (lane == 0) sh.sig[j] = (val < 0.f) ? -1.f : 1.f;  // reuse as the sign of column j
    }
    __syncthreads();
    {
      const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
      for (int i = wv; i < m; i += kWaves)
        for (int j = lane; j < keep; j += 64) G[(long)i * keep + j] *= sh.sig[j];
    }
    // next core <- (Sigma V^T)[kept] (keep x c) * next (c x n r'');
    // (Sigma V^T) row j = sign_j * column perm[j] of B V, transposed
    const int nn = n[k + 1] * r[k + 2];
    float *Gn = w.core(k + 1);
    gemm_lds_a(keep, nn, c, [&](int i, int l) { return sh.sig[i] * sh.jb[sh.perm[i] * kJac + l]; }, Gn, nn, 1,
               Gn, nn, 1, sh);
    if (threadIdx.x == 0) r[k + 1] = keep;
    __syncthreads();
  }
  copy_out(w, d, n, r, O);
  if (status && threadIdx.x == 0) status[0] = unconverged;
}

// Tangent cores and the rank-2r tangent TT (one workgroup per mode):
// dG_k = Zhat_k - U_k (U_k^L^T Zhat_k^L) for k < d-1, dG_{d-1} = Zhat_{d-1};
// W_1 = [a dG_1, U_1], W_k = [[V_k, 0], [a dG_k, U_k]],
// W_d = [[V_d], [x S_d + a dG_d]].
__global__ void __launch_bounds__(kThreads) tangent_kernel(TTDev U, TTDev V, TTDev Z, TTDev W,
                                                           float alpha, float addx, float *scratch,
                                                           long scratch_stride) {
  __shared__ Shared sh;
  const int k = blockIdx.x, d = U.d;
  const int r0 = U.r[k], nk = U.n[k], r1 = U.r[k + 1];
  const int m = r0 * nk;
  const float *Uk = U.data + U.off[k];
  const float *Zk = Z.data + Z.off[k];
  float *dG = scratch + (long)k * scratch_stride;   // m x r1 (row-major)
  float *C = dG + (long)m * r1;                     // r1 x r1
  if (k < d - 1) {
    // C = U^T Z (r1 x r1), K = m, on the matrix cores: wave w takes the
    // 16 x 16 output tiles w, w + 8, ...; operand lane (q4, c16) reads
    // U[k0 + q4][16 ti + c16] and Z[k0 + q4][16 tj + c16] (rows of r1
    // floats, 16 consecutive per quarter-wave)
    {
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      const int c16 = lane & 15, q4 = lane >> 4;
      const int nt = (r1 + 15) / 16;
      for (int tile = wave; tile < nt * nt; tile += kWaves) {
        const int ti = tile / nt, tj = tile % nt;
        const int ci = 16 * ti + c16, cj = 16 * tj + c16;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        // eight k-steps' operands are loaded before their products, so the
        // loads of a group are in flight together
        for (int k0 = 0; k0 < m; k0 += 32) {
          float av[8], bv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int kr = k0 + 4 * u + q4;
            av[u] = (kr < m && ci < r1) ? Uk[(long)kr * r1 + ci] : 0.f;
            bv[u] = (kr < m && cj < r1) ? Zk[(long)kr * r1 + cj] : 0.f;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) acc = mfma4(av[u], bv[u], acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * ti + 4 * q4 + v;
          if (row < r1 && cj < r1) C[row * r1 + cj] = acc[v];
        }
      }
    }
    __syncthreads();
    // dG = Z - U C: U C on the matrix cores, then the difference
    gemm_lds_b(m, r1, r1, Uk, r1, 1, [&](int l, int j) { return C[l * r1 + j]; }, dG, r1, sh);
    for (long e = threadIdx.x; e < (long)m * r1; e += kThreads) dG[e] = Zk[e] - dG[e];
  } else {
    for (long e = threadIdx.x; e < (long)m * r1; e += kThreads) dG[e] = Zk[e];
  }
  __syncthreads();
  float *Wk = W.data + W.off[k];
  const int w0 = W.r[k], w1 = W.r[k + 1];
  const float *Vk = V.data + V.off[k];
  for_rows(w0 * nk, w1, [&](int row, int b) {
    const int a = row / nk, s = row - a * nk;
    const long e = (long)row * w1 + b;
    float v = 0.f;
    if (k == 0) {  // [alpha dG, U]
      v = (b < r1) ? alpha * dG[(long)s * r1 + b] : Uk[(long)s * r1 + (b - r1)];
    } else if (k == d - 1) {  // [[V], [addx S + alpha dG]]
      if (a < r0) v = Vk[((long)a * nk + s) * r1 + b];
      else v = addx * Uk[((long)(a - r0) * nk + s) * r1 + b] + alpha * dG[((long)(a - r0) * nk + s) * r1 + b];
    } else {  // [[V, 0], [alpha dG, U]]
      if (a < r0) v = (b < r1) ? Vk[((long)a * nk + s) * r1 + b] : 0.f;
      else if (b < r1) v = alpha * dG[((long)(a - r0) * nk + s) * r1 + b];
      else v = Uk[((long)(a - r0) * nk + s) * r1 + (b - r1)];
    }
    Wk[e] = v;
  });
}

// add_x X + alpha P_X(Z) from the tangent TT P = P_X(Z) that
// tangent_kernel assembled with alpha = 1, add_x = 0 (same block layout):
// the dG blocks are scaled by alpha and add_x S (S = the last core of the
// left-orthonormal U) is added to the lower block of the last core.  One
// workgroup per core; W may alias P (each element is read, then written, by
// one thread).
__global__ void __launch_bounds__(kThreads) tangent_combine_kernel(TTDev U, TTDev P, TTDev W, float alpha,
                                                                   const float *alpha_dev, float addx) {
  const int k = blockIdx.x, d = U.d;
  if (alpha_dev) alpha *= alpha_dev[0];  // coefficient computed on the device (the line-search step)
  const int r0 = U.r[k], nk = U.n[k], r1 = U.r[k + 1];
  const float *Uk = U.data + U.off[k];
  const float *Pk = P.data + P.off[k];
  float *Wk = W.data + W.off[k];
  const int w0 = W.r[k], w1 = W.r[k + 1];
  for_rows(w0 * nk, w1, [&](int row, int b) {
    const int a = row / nk, s = row - a * nk;
    const long e = (long)row * w1 + b;
    float v = Pk[e];
    if (k == 0) {  // [dG, U]
      if (b < r1) v *= alpha;
    } else if (k == d - 1) {  // [[V], [dG]]
      if (a >= r0) v = addx * Uk[((long)(a - r0) * nk + s) * r1 + b] + alpha * v;
    } else {  // [[V, 0], [dG, U]]
      if (a >= r0 && b < r1) v *= alpha;
    }
    Wk[e] = v;
  });
}

// z[e] = (acc ? z[e] : 0) + sum_{i < nb} c[i] zp[i * stride + e], in order.
struct ZWeights {
  float c[kProjBatch];
};
__global__ void __launch_bounds__(256) zsum_kernel(const float *__restrict__ zp, long long stride, int nb, ZWeights w,
                                                   long long cnt, int acc, float *__restrict__ z) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= cnt) return;
  float v = acc ? z[e] : 0.f;
  for (int i = 0; i < nb; ++i) v = fmaf(w.c[i], zp[(long long)i * stride + e], v);
  z[e] = v;
}

// Offset, in core k of a tangent TT in the assembly's block layout, of the
// dG block's element (a, s, b) (a < r_k, s < n_k, b < r_{k+1} of X): the
// block sits at columns 0..r_{k+1} of the first core, at rows r_k.. of the
// others (w1 = the tangent TT's rank r[k+1]).
__device__ __forceinline__ long dg_offset(int k, int r0, int nk, int w1, int a, int s, int b) {
  const int row = (k == 0) ? a : a + r0;
  return ((long)row * nk + s) * w1 + b;
}

// <A, B> for two tangent vectors at the same point, both in the block
// layout with add_x = 0.  Under the gauge condition the terms
// U_<k dG_k V_>k are mutually orthogonal and the interfaces orthonormal, so
// the inner product is sum_k <dG_k^A, dG_k^B> (tangent-space metric of the
// Riemannian Geometry Operations section).  One workgroup; each thread
// sums a fixed set of elements, then a fixed-order block sum.
__global__ void __launch_bounds__(kThreads) tangent_inner_kernel(TTDev U, TTDev A, TTDev B, float *out) {
  __shared__ Shared sh;
  float acc = 0.f;
  for (int k = 0; k < U.d; ++k) {
    const int r0 = U.r[k], nk = U.n[k], r1 = U.r[k + 1], w1 = A.r[k + 1];
    const float *Ak = A.data + A.off[k];
    const float *Bk = B.data + B.off[k];
    for_rows(r0 * nk, r1, [&](int row, int b) {
      const int a = row / nk, sl = row - a * nk;
      const long o = dg_offset(k, r0, nk, w1, a, sl, b);
      acc = fmaf(Ak[o], Bk[o], acc);
    });
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = acc;
}

// W = a A + b B for two tangent vectors at the same point in the block
// layout with add_x = 0 (their V and U blocks are the same): the dG blocks
// combine, the other blocks are copied from A.  One workgroup per core; W
// may alias A or B (each element is read, then written, by one thread).
__global__ void __launch_bounds__(kThreads) tangent_axpby_kernel(TTDev U, TTDev A, TTDev B, TTDev W, float ca,
                                                                 float cb) {
  const int k = blockIdx.x, d = U.d;
  const int r0 = U.r[k], nk = U.n[k], r1 = U.r[k + 1];
  const float *Ak = A.data + A.off[k];
  const float *Bk = B.data + B.off[k];
  float *Wk = W.data + W.off[k];
  const int w0 = W.r[k], w1 = W.r[k + 1];
  for_rows(w0 * nk, w1, [&](int row, int b) {
    const int a = row / nk;
    const long e = (long)row * w1 + b;
    bool dg;
    if (k == 0)
      dg = b < r1;
    else if (k == d - 1)
      dg = a >= r0;
    else
      dg = a >= r0 && b < r1;
    const float va = Ak[e];
    Wk[e] = dg ? fmaf(ca, va, cb * Bk[e]) : va;
  });
}

// Nonlinear conjugate gradients on tangent vectors (the Riemannian CG of
// the TT-completion literature the paper cites), with every scalar kept on
// the device in sc[]: sc[0] = <xi, xi>, sc[1] = beta, sc[2] = 1 when the
// direction was reset to -xi, sc[3] = <xi, eta>, sc[4] = <xi, T xi'>.
// Polak-Ribiere+: beta = max(0, (<xi, xi> - <xi, T xi'>) / <xi', xi'>),
// 0 on the first step or when <xi', xi'> is not positive.
__global__ void cg_beta_kernel(const float *prev_sq, float *sc) {
  if (threadIdx.x != 0) return;
  float beta = 0.f;
  if (prev_sq) {
    const float q = prev_sq[0];
    if (q > 0.f) beta = fmaxf(0.f, (sc[0] - sc[4]) / q);
  }
  sc[1] = beta;
  sc[2] = 0.f;
}

// eta = -xi + sc[0] * T (dG blocks; the V and U blocks are xi's); one
// workgroup per core.  T may be xi itself (first step, coefficient 0).
__global__ void __launch_bounds__(kThreads) cg_axpby_kernel(TTDev U, TTDev A, TTDev T, TTDev W, const float *cb) {
  const int k = blockIdx.x, d = U.d;
  const int r0 = U.r[k], nk = U.n[k], r1 = U.r[k + 1];
  const float b = cb[0];
  const float *Ak = A.data + A.off[k];
  const float *Tk = T.data + T.off[k];
  float *Wk = W.data + W.off[k];
  const int w0 = W.r[k], w1 = W.r[k + 1];
  for_rows(w0 * nk, w1, [&](int row, int bb) {
    const int a = row / nk;
    const long e = (long)row * w1 + bb;
    bool dg;
    if (k == 0)
      dg = bb < r1;
    else if (k == d - 1)
      dg = a >= r0;
    else
      dg = a >= r0 && bb < r1;
    const float va = Ak[e];
    Wk[e] = dg ? fmaf(-1.f, va, b * Tk[e]) : va;
  });
}

// When eta is not a descent direction (<xi, eta> >= 0), reset it to -xi:
// beta = 0, sc[2] = 1.  Every workgroup reads the same sc[3]; workgroup 0
// writes the scalars.
__global__ void __launch_bounds__(kThreads) cg_restart_kernel(TTDev U, TTDev A, TTDev W, float *sc) {
  if (!(sc[3] >= 0.f)) return;
  const int k = blockIdx.x, d = U.d;
  const int r0 = U.r[k], nk = U.n[k], r1 = U.r[k + 1];
  const float *Ak = A.data + A.off[k];
  float *Wk = W.data + W.off[k];
  const int w0 = W.r[k], w1 = W.r[k + 1];
  for_rows(w0 * nk, w1, [&](int row, int bb) {
    const int a = row / nk;
    const long e = (long)row * w1 + bb;
    bool dg;
    if (k == 0)
      dg = bb < r1;
    else if (k == d - 1)
      dg = a >= r0;
    else
      dg = a >= r0 && bb < r1;
    const float va = Ak[e];
    Wk[e] = dg ? -va : va;
  });
  if (k == 0 && threadIdx.x == 0) {
    sc[1] = 0.f;
    sc[2] = 1.f;
  }
}

// Gram matrix of a batch of tangent vectors at one point.  Under the gauge
// condition <A, B> = sum_k <dG_k^A, dG_k^B>, so the Gram matrix is D D^T
// for the matrix D whose row j lists member j's dG blocks (S elements:
// sum_k r_k n_k r_{k+1} over X's ranks).  A pack launch copies the blocks of
// up to 64 members into rows of D; the Gram launch forms 8 x 8 tiles of
// D D^T.
constexpr int kGramTile = 8;
struct MemberPtrs {
  const float *p[kProjBatch];
};

// grid (ceil(S / 256), members); row i0 + blockIdx.y of D receives the dG
// blocks of member blockIdx.y (core offsets and ranks of A0, shared by the
// batch) in core order, each block in (a, s, b) order.
__global__ void __launch_bounds__(256) tangent_pack_kernel(TTDev U, TTDev A0, MemberPtrs mp, int i0, long long S,
                                                           float *__restrict__ D) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= S) return;
  const float *src = mp.p[blockIdx.y];
  long long base = 0;
  int k = 0;
  for (; k + 1 < U.d; ++k) {
    const long long sz = (long long)U.r[k] * U.n[k] * U.r[k + 1];
    if (e < base + sz) break;
    base += sz;
  }
  const int r0 = U.r[k], nk = U.n[k], r1 = U.r[k + 1];
  const int l = (int)(e - base);  // within one core
  const int b = l % r1, sl = (l / r1) % nk, a = l / (r1 * nk);
  D[(long long)(i0 + blockIdx.y) * S + e] = src[A0.off[k] + dg_offset(k, r0, nk, A0.r[k + 1], a, sl, b)];
}

// One workgroup per tile pair (ta <= tb) of 8 x 8 members: each thread sums
// its strided share of the S columns for all 64 pairs, then a fixed-order
// reduction (waves, then the four wave sums in order).  The tile (tb, ta)
// is the transpose, written from the same sums, so G is exactly symmetric.
__global__ void __launch_bounds__(256) tangent_gram_kernel(const float *__restrict__ D, int nb, long long S,
                                                           float *__restrict__ G) {
  __shared__ float red[4][kGramTile * kGramTile];
  int t = blockIdx.x, tb = 0;
  while (t > tb) {
    t -= tb + 1;
    ++tb;
  }
  const int ta = t;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float *Da[kGramTile], *Db[kGramTile];
#pragma unroll
  for (int i = 0; i < kGramTile; ++i) {
    const int ra = ta * kGramTile + i, rb = tb * kGramTile + i;
    Da[i] = D + (long long)(ra < nb ? ra : 0) * S;
    Db[i] = D + (long long)(rb < nb ? rb : 0) * S;
  }
  float acc[kGramTile][kGramTile];
#pragma unroll
  for (int i = 0; i < kGramTile; ++i)
#pragma unroll
    for (int j = 0; j < kGramTile; ++j) acc[i][j] = 0.f;
  for (long long e = threadIdx.x; e < S; e += 256) {
    float xa[kGramTile], xb[kGramTile];
#pragma unroll
    for (int i = 0; i < kGramTile; ++i) {
      xa[i] = Da[i][e];
      xb[i] = Db[i][e];
    }
#pragma unroll
    for (int i = 0; i < kGramTile; ++i)
#pragma unroll
      for (int j = 0; j < kGramTile; ++j) acc[i][j] = fmaf(xa[i], xb[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < kGramTile; ++i)
#pragma unroll
    for (int j = 0; j < kGramTile; ++j) {
      const float v = wave_sum(acc[i][j]);
      if (lane == 0) red[wave][i * kGramTile + j] = v;
    }
  __syncthreads();
  if (threadIdx.x < kGramTile * kGramTile) {
    const int i = threadIdx.x / kGramTile, j = threadIdx.x % kGramTile;
    const int ra = ta * kGramTile + i, rb = tb * kGramTile + j;
    if (ra < nb && rb < nb) {
      const float v = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
      G[(long long)ra * nb + rb] = v;
      if (ta != tb) G[(long long)rb * nb + ra] = v;
    }
  }
}

// Projection of a TT tensor Y onto the tangent space at X (U left- and V
// right-orthonormal cores of X).  Interfaces: Psi_0 = 1,
// Psi_{k+1} = sum_i U_k[i]^T Psi_k Y_k[i] (left), Phi_d = 1,
// Phi_k = sum_i V_k[i] Phi_{k+1} Y_k[i]^T (right); then one workgroup per
// core forms Zhat_k[i] = Psi_k Y_k[i] Phi_{k+1}^T.
struct ProjBufs {
  float *psi, *phi, *tmp;
  long pslot, tslot;
};

// One step of both interface sweeps, launch t of d: the left side handles
// k = t, the right side k = d-1-t.  A side's input interface (Psi_k, or
// Phi_{k+1}) is [1] at the chain's start, else the sum, in slice order, of
// the previous launch's per-slice partials; workgroup 0 of the side writes
// it to its slot.  Then, unless the chain ends here, workgroup i forms the
// slice-i term of the next interface:
//   left  U_k[i]^T (Psi_k Y_k[i])          (r_{k+1} x s_{k+1}),
//   right V_k[i] (Phi_{k+1} Y_k[i]^T)      (r_k x s_k),
// both products in LDS.  Workgroups [0, lw) are left, the rest right.
struct ProjStep {
  int lk, rk;               // left k, right k
  int lw;                   // left workgroups
  const float *lin, *rin;   // previous partials ([n][pslot]) or null for [1]
  int lnin, rnin;           // number of previous partials
  float *lout, *rout;       // this step's partials
};

constexpr int kPs = kJac + 1;  // LDS row stride of the step's 64 x 64 tiles

// A batch of TTs of one shape projected at once (project_sum): tensor
// blockIdx.y has its cores at ydata[blockIdx.y] (offsets of the shared
// shape) and its own interface, partial, scratch and Zhat blocks, `stride`
// floats apart for each kind.  A single projection is the batch of one.
struct ProjBatch {
  const float *ydata[kProjBatch];
  long long psi_stride, part_stride, tmp_stride, z_stride;
};

__global__ void __launch_bounds__(kThreads) proj_step_kernel(TTDev U, TTDev V, TTDev Y, ProjBufs b, ProjStep st,
                                                             ProjBatch pb) {
  __shared__ float ta[kJac * kPs], tb[kJac * kPs], tc[kJac * kPs];
  // this tensor's blocks (locals: the by-value arguments stay unmodified,
  // so they are read from the argument segment, not copied to scratch)
  const int bi = blockIdx.y;
  const float *ydat = pb.ydata[bi];
  float *psi = b.psi + bi * pb.psi_stride, *phi = b.phi + bi * pb.psi_stride;
  const float *lin = st.lin ? st.lin + bi * pb.part_stride : nullptr;
  const float *rin = st.rin ? st.rin + bi * pb.part_stride : nullptr;
  float *lout = st.lout + bi * pb.part_stride, *rout = st.rout + bi * pb.part_stride;
  const int d = U.d;
  const bool left = (int)blockIdx.x < st.lw;
  const int i = left ? (int)blockIdx.x : (int)blockIdx.x - st.lw;
  const int k = left ? st.lk : st.rk;
  // input interface: rows x cols, into ta
  const int ir = left ? U.r[k] : V.r[k + 1], ic = left ? Y.r[k] : Y.r[k + 1];
  const float *in = left ? lin : rin;
  const int nin = left ? st.lnin : st.rnin;
  for (int e = threadIdx.x; e < ir * ic; e += kThreads) {
    float v = 1.f;  // the 1 x 1 start of a chain
    if (in) {
      v = 0.f;
      for (int j = 0; j < nin; ++j) v += in[(long)j * b.pslot + e];
    }
    ta[(e / ic) * kPs + e % ic] = v;
    if (i == 0) (left ? psi + (long)k * b.pslot : phi + (long)(k + 1) * b.pslot)[e] = v;
  }
  const bool more = left ? (k + 1 < d) : (k >= 1);
  if (!more) return;
  const int r0 = U.r[k], r1 = U.r[k + 1], n = U.n[k], s0 = Y.r[k], s1 = Y.r[k + 1];
  // Y_k[i] (s0 x s1) into tb
  const float *Yk = ydat + Y.off[k];
  for (int e = threadIdx.x; e < s0 * s1; e += kThreads) {
    const int bb = e / s1, ee = e % s1;
    tb[bb * kPs + ee] = Yk[((long)bb * n + i) * s1 + ee];
  }
  __syncthreads();
  if (left) {
    // tc = Psi_k Y_k[i] (r0 x s1)
    for (int e = threadIdx.x; e < r0 * s1; e += kThreads) {
      const int a = e / s1, ee = e % s1;
      float acc = 0.f;
      for (int l = 0; l < s0; ++l) acc = fmaf(ta[a * kPs + l], tb[l * kPs + ee], acc);
      tc[a * kPs + ee] = acc;
    }
  } else {
    // tc = Phi_{k+1} Y_k[i]^T (r1 x s0)
    for (int e = threadIdx.x; e < r1 * s0; e += kThreads) {
      const int c = e / s0, bb = e % s0;
      float acc = 0.f;
      for (int l = 0; l < s1; ++l) acc = fmaf(ta[c * kPs + l], tb[bb * kPs + l], acc);
      tc[c * kPs + bb] = acc;
    }
  }
  __syncthreads();
  // U_k[i] or V_k[i] (r0 x r1) into ta
  const float *Gk = left ? U.data + U.off[k] : V.data + V.off[k];
  for (int e = threadIdx.x; e < r0 * r1; e += kThreads) {
    const int a = e / r1, c = e % r1;
    ta[a * kPs + c] = Gk[((long)a * n + i) * r1 + c];
  }
  __syncthreads();
  if (left) {
    // partial of Psi_{k+1} (r1 x s1) = U_k[i]^T tc
    float *out = lout + (long)i * b.pslot;
    for (int e = threadIdx.x; e < r1 * s1; e += kThreads) {
      const int c = e / s1, ee = e % s1;
      float acc = 0.f;
      for (int a = 0; a < r0; ++a) acc = fmaf(ta[a * kPs + c], tc[a * kPs + ee], acc);
      out[e] = acc;
    }
  } else {
    // partial of Phi_k (r0 x s0) = V_k[i] tc
    float *out = rout + (long)i * b.pslot;
    for (int e = threadIdx.x; e < r0 * s0; e += kThreads) {
      const int a = e / s0, bb = e % s0;
      float acc = 0.f;
      for (int c = 0; c < r1; ++c) acc = fmaf(ta[a * kPs + c], tc[c * kPs + bb], acc);
      out[e] = acc;
    }
  }
}

__global__ void __launch_bounds__(kThreads) proj_cores_kernel(TTDev U, TTDev Y, TTDev Z, ProjBufs b, ProjBatch pb) {
  __shared__ Shared sh;
  const int k = blockIdx.x;
  const int bi = blockIdx.y;
  const float *ydat = pb.ydata[bi];
  const float *psi = b.psi + bi * pb.psi_stride, *phi = b.phi + bi * pb.psi_stride;
  float *tmp = b.tmp + bi * pb.tmp_stride, *zdat = Z.data + bi * pb.z_stride;
  const int r0 = U.r[k], r1 = U.r[k + 1], n = U.n[k], s0 = Y.r[k], s1 = Y.r[k + 1];
  const long ns1 = (long)n * s1;
  float *T = tmp + (2 + k) * b.tslot;
  // T (r0 x n s1) = Psi_k Y_k
  const float *Pk = psi + k * b.pslot;
  gemm_lds_a(r0, (int)ns1, s0, [&](int i, int l) { return Pk[i * s0 + l]; }, ydat + Y.off[k], ns1, 1, T, ns1, 1,
             sh);
  __syncthreads();
  // Zhat_k ((r0 n) x r1) = T ((r0 n) x s1) Phi_{k+1}^T (s1 x r1)
  const float *Fk = phi + (k + 1) * b.pslot;
  gemm_lds_b<true>(r0 * n, r1, s1, T, s1, 1, [&](int l, int j) { return Fk[j * s1 + l]; }, zdat + Z.off[k], r1,
                   sh);
}

long slot_of(const int *n, const int *r, int d) {
  long s = 1;
  for (int k = 0; k < d; ++k) {
    const long c = (long)r[k] * n[k] * r[k + 1];
    s = c > s ? c : s;
  }
  return s;
}

long mat_of(const int *n, const int *r, int d) {
  long s = 1;
  for (int k = 0; k < d; ++k) {
    const long a = (long)r[k] * n[k] * r[k + 1];
    s = a > s ? a : s;
  }
  return s;
}

}  // namespace

// ----------------------------------------------------------------- host side
int dense_orth_ranks(const tt_tensor *X, int dir, int32_t *out) {
  const int d = X->d;
  for (int k = 0; k <= d; ++k) out[k] = X->r[k];
  if (dir == TT_LR) {
    for (int k = 0; k + 1 < d; ++k) {
      const long m = (long)out[k] * X->n[k];
      out[k + 1] = (int32_t)(m < out[k + 1] ? m : out[k + 1]);
    }
  } else {
    for (int k = d - 1; k >= 1; --k) {
      const long mm = (long)X->n[k] * out[k + 1];
      out[k] = (int32_t)(mm < out[k] ? mm : out[k]);
    }
  }
  return TT_OK;
}

int dense_round_ranks(const tt_tensor *Y, int max_rank, int32_t *out) {
  dense_orth_ranks(Y, TT_RL, out);
  for (int k = 0; k + 1 < Y->d; ++k) {
    long t = (long)out[k] * Y->n[k];
    if (out[k + 1] < t) t = out[k + 1];
    if (max_rank < t) t = max_rank;
    out[k + 1] = (int32_t)t;
  }
  return TT_OK;
}

size_t dense_ws(const tt_tensor *X) {
  const long slot = slot_of(X->n, X->r, X->d);
  const long mat = mat_of(X->n, X->r, X->d);
  return arena_bytes<float>((size_t)slot * X->d) + 2 * arena_bytes<float>((size_t)mat) +
         arena_bytes<float>(DENSE_MAX_RANK + 64);
}

static int dense_bufs(const tt_tensor *X, void *ws, size_t bytes, DenseBufs &b) {
  const long slot = slot_of(X->n, X->r, X->d);
  const long mat = mat_of(X->n, X->r, X->d);
  Arena ar(ws, bytes);
  b.work = ar.take<float>((size_t)slot * X->d);
  b.slot = slot;
  b.wm = ar.take<float>((size_t)mat);
  b.q = ar.take<float>((size_t)mat);
  b.tau = ar.take<float>(DENSE_MAX_RANK + 64);
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "dense sweep: workspace too small");
  return TT_OK;
}

int dense_orth(const tt_tensor *X, int dir, tt_tensor *O, void *ws, size_t bytes, hipStream_t s) {
  DenseBufs b;
  int rc = dense_bufs(X, ws, bytes, b);
  if (rc) return rc;
  timer_before(s);
  hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(kThreads), 0, s, make_dev(X), make_dev(O), dir, b);
  timer_after(s);
  return launch_check("orthogonalize");
}

int dense_orth_both(const tt_tensor *X, tt_tensor *OL, tt_tensor *OR, void *ws, size_t bytes, hipStream_t s) {
  const size_t half = dense_ws(X);
  if (bytes < 2 * half) return set_error(TT_ERR_WORKSPACE, "orthogonalize_both: workspace too small");
  DenseBufs bl, br;
  int rc = dense_bufs(X, ws, half, bl);
  if (rc) return rc;
  if ((rc = dense_bufs(X, (char *)ws + half, half, br))) return rc;
  timer_before(s);
  hipLaunchKernelGGL(orth_both_kernel, dim3(2), dim3(kThreads), 0, s, make_dev(X), make_dev(OL), make_dev(OR), bl,
                     br);
  timer_after(s);
  return launch_check("orthogonalize both");
}

int dense_round(const tt_tensor *Y, int max_rank, tt_tensor *O, float *disc, int *status, void *ws, size_t bytes,
                hipStream_t s) {
  DenseBufs b;
  int rc = dense_bufs(Y, ws, bytes, b);
  if (rc) return rc;
  timer_before(s);
  hipLaunchKernelGGL(round_kernel, dim3(1), dim3(kThreads), 0, s, make_dev(Y), make_dev(O), max_rank,
                     disc, status, b);
  timer_after(s);
  return launch_check("round");
}

size_t tangent_ws(const tt_tensor *U) {
  long stride = 0;
  for (int k = 0; k < U->d; ++k) {
    const long m = (long)U->r[k] * U->n[k];
    const long need = m * U->r[k + 1] + (long)U->r[k + 1] * U->r[k + 1];
    stride = need > stride ? need : stride;
  }
  return arena_bytes<float>((size_t)stride * U->d);
}

int tangent_assemble(const tt_tensor *U, const tt_tensor *V, const tt_tensor *Z, tt_tensor *W,
                     float alpha, int add_x, void *ws, size_t bytes, hipStream_t s) {
  long stride = 0;
  for (int k = 0; k < U->d; ++k) {
    const long m = (long)U->r[k] * U->n[k];
    const long need = m * U->r[k + 1] + (long)U->r[k + 1] * U->r[k + 1];
    stride = need > stride ? need : stride;
  }
  Arena ar(ws, bytes);
  float *scratch = ar.take<float>((size_t)stride * U->d);
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "tangent assembly: workspace too small");
  hipLaunchKernelGGL(tangent_kernel, dim3(U->d), dim3(kThreads), 0, s, make_dev(U), make_dev(V),
                     make_dev(Z), make_dev(W), alpha, add_x ? 1.f : 0.f, scratch, stride);
  return launch_check("tangent assembly");
}

// Scratch of the TT projection: interface slots (r x s) and product slots
// (r n x s) over all cores.
static void proj_slots(const tt_tensor *U, const tt_tensor *Y, long *pslot, long *tslot) {
  long ps = 1, ts = 1;
  for (int k = 0; k <= U->d; ++k) {
    const long a = (long)U->r[k] * Y->r[k];
    ps = a > ps ? a : ps;
  }
  for (int k = 0; k < U->d; ++k) {
    const long a = (long)U->r[k] * U->n[k] * Y->r[k + 1];
    ts = a > ts ? a : ts;
  }
  *pslot = ps;
  *tslot = ts;
}

// Workspace of `nb` projections of TTs of Y's shape run together: per tensor
// the interfaces, the step partials (two ping-pong pairs), the core-step
// scratch and its Zhat.
struct ProjWs {
  ProjBufs b;
  float *lpart[2], *rpart[2], *zpart;
  ProjBatch pb;
};

static long proj_zel(const tt_tensor *U) {
  long zel = 0;
  for (int k = 0; k < U->d; ++k) zel += (long)U->r[k] * U->n[k] * U->r[k + 1];
  return zel;
}

static int proj_nmax(const tt_tensor *U) {
  int nmax = 1;
  for (int k = 0; k < U->d; ++k) nmax = U->n[k] > nmax ? U->n[k] : nmax;
  return nmax;
}

static size_t proj_batch_bytes(const tt_tensor *U, const tt_tensor *Y, int nb) {
  long ps, ts;
  proj_slots(U, Y, &ps, &ts);
  size_t b = 2 * arena_bytes<float>((size_t)nb * (U->d + 1) * ps);
  b += 4 * arena_bytes<float>((size_t)nb * proj_nmax(U) * ps);
  b += arena_bytes<float>((size_t)nb * (U->d + 2) * ts);
  b += arena_bytes<float>((size_t)nb * proj_zel(U));
  return b;
}

static void proj_batch_take(Arena &ar, const tt_tensor *U, const tt_tensor *Y, int nb, ProjWs &w) {
  long ps, ts;
  proj_slots(U, Y, &ps, &ts);
  const long nmax = proj_nmax(U), zel = proj_zel(U);
  w.b.psi = ar.take<float>((size_t)nb * (U->d + 1) * ps);
  w.b.phi = ar.take<float>((size_t)nb * (U->d + 1) * ps);
  for (int i = 0; i < 2; ++i) w.lpart[i] = ar.take<float>((size_t)nb * nmax * ps);
  for (int i = 0; i < 2; ++i) w.rpart[i] = ar.take<float>((size_t)nb * nmax * ps);
  w.b.tmp = ar.take<float>((size_t)nb * (U->d + 2) * ts);
  w.b.pslot = ps;
  w.b.tslot = ts;
  w.zpart = ar.take<float>((size_t)nb * zel);
  w.pb.psi_stride = (long long)(U->d + 1) * ps;
  w.pb.part_stride = (long long)nmax * ps;
  w.pb.tmp_stride = (long long)(U->d + 2) * ts;
  w.pb.z_stride = zel;
}

// Zhat of each of the nb tensors (cores at ydata[i], Y's shape) into
// w.zpart + i * zel: d interface launches (left step t and right step
// d-1-t, a workgroup per slice and tensor), then the core step.
static int proj_batch_run(const tt_tensor *U, const tt_tensor *V, const tt_tensor *Y, const float *const *ydata,
                          int nb, ProjWs &w, hipStream_t s) {
  const int d = U->d;
  for (int i = 0; i < nb; ++i) w.pb.ydata[i] = ydata[i];
  const TTDev Ud = make_dev(U), Vd = make_dev(V), Yd = make_dev(Y);
  int rc = TT_OK;
  for (int t = 0; t < d; ++t) {
    ProjStep st;
    st.lk = t;
    st.rk = d - 1 - t;
    st.lw = (st.lk + 1 < d) ? U->n[st.lk] : 1;
    const int rw = (st.rk >= 1) ? U->n[st.rk] : 1;
    st.lin = t == 0 ? nullptr : w.lpart[(t - 1) & 1];
    st.lnin = t == 0 ? 0 : U->n[st.lk - 1];
    st.rin = t == 0 ? nullptr : w.rpart[(t - 1) & 1];
    st.rnin = t == 0 ? 0 : U->n[st.rk + 1];
    st.lout = w.lpart[t & 1];
    st.rout = w.rpart[t & 1];
    hipLaunchKernelGGL(proj_step_kernel, dim3(st.lw + rw, nb), dim3(kThreads), 0, s, Ud, Vd, Yd, w.b, st, w.pb);
    if ((rc = launch_check("TT projection interface step"))) return rc;
  }
  tt_tensor Z = {U->d, U->n, U->r, nullptr, w.zpart};
  hipLaunchKernelGGL(proj_cores_kernel, dim3(U->d, nb), dim3(kThreads), 0, s, Ud, Yd, make_dev(&Z), w.b, w.pb);
  return launch_check("TT projection cores");
}

size_t project_tt_ws(const tt_tensor *U, const tt_tensor *Y) {
  return proj_batch_bytes(U, Y, 1) + tangent_ws(U) + 256;
}

int project_tt(const tt_tensor *U, const tt_tensor *V, const tt_tensor *Y, float alpha, int add_x, tt_tensor *W,
               void *ws, size_t bytes, hipStream_t s) {
  Arena ar(ws, bytes);
  ProjWs w;
  proj_batch_take(ar, U, Y, 1, w);
  const size_t tws = tangent_ws(U);
  void *tw = ar.take<char>(tws);
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "project_tt: workspace too small");
  const float *yd = Y->data;
  int rc = proj_batch_run(U, V, Y, &yd, 1, w, s);
  if (rc) return rc;
  tt_tensor Z = {U->d, U->n, U->r, nullptr, w.zpart};
  return tangent_assemble(U, V, &Z, W, alpha, add_x, tw, tws, s);
}

size_t project_sum_ws(const tt_tensor *U, const tt_tensor *A0, int nb) {
  const int chunk = nb < kProjBatch ? nb : kProjBatch;
  return proj_batch_bytes(U, A0, chunk) + arena_bytes<float>((size_t)proj_zel(U)) + tangent_ws(U) + 256;
}

int project_sum(const tt_tensor *U, const tt_tensor *V, const tt_tensor *A, int nb, const float *c, float alpha,
                int add_x, tt_tensor *W, void *ws, size_t bytes, hipStream_t s) {
  const int chunk = nb < kProjBatch ? nb : kProjBatch;
  Arena ar(ws, bytes);
  ProjWs w;
  proj_batch_take(ar, U, &A[0], chunk, w);
  const long zel = proj_zel(U);
  float *zsum = ar.take<float>((size_t)zel);
  const size_t tws = tangent_ws(U);
  void *tw = ar.take<char>(tws);
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "project_sum: workspace too small");
  int rc = TT_OK;
  for (int i0 = 0; i0 < nb; i0 += chunk) {
    const int m = (nb - i0) < chunk ? (nb - i0) : chunk;
    const float *yd[kProjBatch];
    ZWeights zw;
    for (int i = 0; i < m; ++i) {
      yd[i] = A[i0 + i].data;
      zw.c[i] = c[i0 + i];
    }
    if ((rc = proj_batch_run(U, V, &A[0], yd, m, w, s))) return rc;
    hipLaunchKernelGGL(zsum_kernel, dim3((unsigned)((zel + 255) / 256)), dim3(256), 0, s, w.zpart,
                       (long long)zel, m, zw, (long long)zel, i0 > 0 ? 1 : 0, zsum);
    if ((rc = launch_check("project_sum weighted sum"))) return rc;
  }
  tt_tensor Z = {U->d, U->n, U->r, nullptr, zsum};
  return tangent_assemble(U, V, &Z, W, alpha, add_x, tw, tws, s);
}

int tangent_inner(const tt_tensor *U, const tt_tensor *A, const tt_tensor *B, float *out, hipStream_t s) {
  hipLaunchKernelGGL(tangent_inner_kernel, dim3(1), dim3(kThreads), 0, s, make_dev(U), make_dev(A), make_dev(B),
                     out);
  return launch_check("tangent inner product");
}

static long long tangent_dg_count(const tt_tensor *U) {
  long long S = 0;
  for (int k = 0; k < U->d; ++k) S += (long long)U->r[k] * U->n[k] * U->r[k + 1];
  return S;
}

size_t tangent_gram_ws(const tt_tensor *U, int nb) {
  return arena_bytes<float>((size_t)nb * (size_t)tangent_dg_count(U));
}

int tangent_gram(const tt_tensor *U, const tt_tensor *A, int nb, float *G, void *ws, size_t bytes, hipStream_t s) {
  const long long S = tangent_dg_count(U);
  Arena ar(ws, bytes);
  float *D = ar.take<float>((size_t)nb * (size_t)S);
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "tangent_gram: workspace too small");
  const TTDev ud = make_dev(U), a0 = make_dev(&A[0]);
  const unsigned gx = (unsigned)((S + 255) / 256);
  for (int i0 = 0; i0 < nb; i0 += kProjBatch) {
    const int m = (nb - i0) < kProjBatch ? (nb - i0) : kProjBatch;
    MemberPtrs mp{};
    for (int i = 0; i < m; ++i) mp.p[i] = A[i0 + i].data;
    hipLaunchKernelGGL(tangent_pack_kernel, dim3(gx, (unsigned)m), dim3(256), 0, s, ud, a0, mp, i0, S, D);
    int rc = launch_check("tangent gram pack");
    if (rc) return rc;
  }
  const long long nt = (nb + kGramTile - 1) / kGramTile;
  hipLaunchKernelGGL(tangent_gram_kernel, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, s, D, nb, S, G);
  return launch_check("tangent gram");
}

int tangent_axpby(const tt_tensor *U, float a, const tt_tensor *A, float b, const tt_tensor *B, tt_tensor *W,
                  hipStream_t s) {
  hipLaunchKernelGGL(tangent_axpby_kernel, dim3(U->d), dim3(kThreads), 0, s, make_dev(U), make_dev(A),
                     make_dev(B), make_dev(W), a, b);
  return launch_check("tangent axpby");
}

int tangent_combine(const tt_tensor *U, const tt_tensor *P, tt_tensor *W, float alpha, int add_x,
                    hipStream_t s) {
  hipLaunchKernelGGL(tangent_combine_kernel, dim3(U->d), dim3(kThreads), 0, s, make_dev(U), make_dev(P),
                     make_dev(W), alpha, (const float *)nullptr, add_x ? 1.f : 0.f);
  return launch_check("tangent combine");
}

int tangent_combine_dev(const tt_tensor *U, const tt_tensor *P, tt_tensor *W, const float *alpha, float scale,
                        int add_x, hipStream_t s) {
  hipLaunchKernelGGL(tangent_combine_kernel, dim3(U->d), dim3(kThreads), 0, s, make_dev(U), make_dev(P),
                     make_dev(W), scale, alpha, add_x ? 1.f : 0.f);
  return launch_check("tangent combine (device coefficient)");
}

int cg_direction(const tt_tensor *U, const tt_tensor *xi, const tt_tensor *txi, const tt_tensor *teta,
                 const float *prev_sq, tt_tensor *eta, float *sc, hipStream_t s) {
  const TTDev ud = make_dev(U), xd = make_dev(xi), ed = make_dev(eta);
  hipLaunchKernelGGL(tangent_inner_kernel, dim3(1), dim3(kThreads), 0, s, ud, xd, xd, sc + 0);
  int rc = launch_check("cg: <xi, xi>");
  if (rc) return rc;
  const bool first = (txi == nullptr);
  if (!first) {
    hipLaunchKernelGGL(tangent_inner_kernel, dim3(1), dim3(kThreads), 0, s, ud, xd, make_dev(txi), sc + 4);
    if ((rc = launch_check("cg: <xi, T xi'>"))) return rc;
  }
  hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(64), 0, s, first ? nullptr : prev_sq, sc);
  if ((rc = launch_check("cg: beta"))) return rc;
  // eta = -xi + beta T eta' (first step: -xi)
  const TTDev td = first ? xd : make_dev(teta);
  hipLaunchKernelGGL(cg_axpby_kernel, dim3(U->d), dim3(kThreads), 0, s, ud, xd, td, ed, sc + 1);
  if ((rc = launch_check("cg: direction"))) return rc;
  hipLaunchKernelGGL(tangent_inner_kernel, dim3(1), dim3(kThreads), 0, s, ud, xd, ed, sc + 3);
  if ((rc = launch_check("cg: <xi, eta>"))) return rc;
  hipLaunchKernelGGL(cg_restart_kernel, dim3(U->d), dim3(kThreads), 0, s, ud, xd, ed, sc);
  return launch_check("cg: restart");
}

}  // namespace ttgfx
