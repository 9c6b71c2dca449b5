// TT-matrix layer through the dense matrix (t3f.matmul(tt_matrix, x),
// Implementation Details).
//
// Y = X W^T with W[(i_1..i_d), (j_1..j_d)] = G^1[i_1, j_1] ... G^d[i_d, j_d]
// is a linear map; when prod m * prod n is small beside the batch, building
// W once and running one GEMM costs far fewer flops than contracting the
// cores one step at a time against every row (at 4096 x 1024 with modes 4^5
// and rank 32: 8.6 against 105 GFLOP forward).  This path
//   * builds the left partial products P_k[(i_1..i_k)][(j_1..j_k)][b] of the
//     first k cores (P_d = W) with one small contraction kernel per core;
//   * runs Y = X W^T, dX = dY W and dW_dense = dY^T X on the matrix cores
//     (one GEMM kernel whose operands are read either k-contiguous or
//     row-contiguous, so no transposes are materialised);
//   * takes the core gradients from dW_dense: the right partial sums
//     Z_k[(i_1..i_k)][(j_1..j_k)][b] = sum over the later indices of
//     dW_dense times the cores after k (a sweep from Z_{d-1} = dW_dense), then
//     dG^k[a, i, j, b] = sum_{I<, J<} P_k[I<][J<][a] Z_k[(I<, i)][(J<, j)][b],
//     split over the contracted range with a fixed-order reduction.
// bf16: the cores, X and dY are bf16; W is accumulated in float32 and
// rounded to bf16 once for the two GEMMs that read it; every product
// accumulates in float32.
#include <type_traits>

#include "common.h"
#include "ttm.h"

namespace ttgfx {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));  // 16 raw bytes

__device__ __forceinline__ float bf_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
// Round to nearest, ties to even (NaN stays NaN).
__device__ __forceinline__ uint16_t f_to_bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <int BF16>
__device__ __forceinline__ float ld_el(const void *p, long long i) {
  if (BF16) return bf_to_f(((const uint16_t *)p)[i]);
  return ((const float *)p)[i];
}

constexpr int kBlk = 256;

// out[e] = sum_c part[c][e] in chunk order (the loads of eight chunks are
// issued together; the additions keep the order).
__global__ void __launch_bounds__(kBlk) dg_reduce_kernel(const float *__restrict__ part, int nchunk, long long cnt,
                                                         float *__restrict__ out) {
  const long long e = (long long)blockIdx.x * kBlk + threadIdx.x;
  if (e >= cnt) return;
  float s = 0.f;
  int c = 0;
  for (; c + 8 <= nchunk; c += 8) {
    float v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = part[(long long)(c + t) * cnt + e];
#pragma unroll
    for (int t = 0; t < 8; ++t) s += v[t];
  }
  for (; c < nchunk; ++c) s += part[(long long)c * cnt + e];
  out[e] = s;
}

__global__ void __launch_bounds__(kBlk) to_bf16_kernel(const float *__restrict__ x, uint16_t *__restrict__ y,
                                                       long long n) {
  for (long long e = (long long)blockIdx.x * kBlk + threadIdx.x; e < n; e += (long long)gridDim.x * kBlk)
    y[e] = f_to_bf(x[e]);
}

__global__ void set_one_kernel(float *p) { *p = 1.f; }

// ------------------------------------------------------------------ GEMM
// C(m, n) = sum_k A(m, k) B(n, k) in float32.  AK: A(m, k) at A[m lda + k]
// (k-contiguous), else at A[k lda + m] (row-contiguous); likewise BK for B.
// Workgroups of 4 waves own 128 x 128 tiles of C (each wave 64 x 64, 4 x 4
// MFMA tiles of 16 x 16); the k range goes in chunks of 32 staged in LDS,
// k-contiguous operands as [row][k], row-contiguous ones as [k][row], so
// both are written with 16-byte stores and read by the MFMA lanes without
// bank conflicts; the next chunk is loaded into registers while the
// current one is multiplied.  float32: v_mfma_f32_16x16x4_f32; bf16:
// v_mfma_f32_16x16x16_bf16 with bf16 kept in LDS.  gridDim.z splits the k
// range (each slice writes its own partial C, cstride floats apart).  The
// epilogue places C(m, n) through a CMap.  FULL: every tile and chunk lies
// inside the matrices and rows are 16-byte aligned (vector loads, no
// guards).
// The epilogue places C(row, col) at f(row) + g(col), each a mixed-radix
// remap: the index is split into up to three digits (innermost radix
// first) and a remainder, and the digits are weighted.  Used for plain row-major
// output and for the interleaved layouts of the partial products.
struct Remap {
  unsigned radix[3];    // digits 0..2 (a 0 radix ends the digits); the rest is digit 3
  long long weight[4];
};

__device__ __forceinline__ long long remap(const Remap &m, int x) {
  unsigned u = (unsigned)x;
  long long a = 0;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const unsigned R = m.radix[t];
    if (R == 0) break;
    a += (long long)(u % R) * m.weight[t];
    u /= R;
  }
  return a + (long long)u * m.weight[3];
}

struct CMap {
  Remap row, col;
};

struct GemmArgs {
  const void *A, *B;
  float *C;
  int M, N, K;
  int kslice;           // k per z slice (a multiple of TK)
  long long lda, ldb;
  long long cstride;    // floats between the partial C of consecutive slices
  CMap map;
};

constexpr int TM = 128, TN = 128, TK = 32;
constexpr int kGemmThreads = 256;

template <int BF16>
struct GemmE {
  using E = typename std::conditional<BF16, uint16_t, float>::type;
};

// LDS row stride (elements) of a staged operand: [row][k] (KC) or [k][row].
template <int BF16, int KC>
constexpr int lds_ld() {
  return KC ? (BF16 ? TK + 8 : TK + 4) : TM + 16;
}

// One operand tile (128 rows x 32 k) into registers: VEC elements (16
// bytes) per load, PER loads per thread, held as raw 16-byte words.
template <int BF16, int KC, int FULL>
struct Stage {
  static constexpr int VEC = BF16 ? 8 : 4;
  static constexpr int PER = TM * TK / VEC / kGemmThreads;  // 4 (fp32) or 2 (bf16)
  using E = typename GemmE<BF16>::E;
  v4u r[PER];

  __device__ __forceinline__ void load(const void *base, long long ld, int row0, int rows, int k0, int kend) {
    const E *p = (const E *)base;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = threadIdx.x + kGemmThreads * u;
      const int row = KC ? idx / (TK / VEC) : (idx % (TM / VEC)) * VEC;
      const int kk = KC ? (idx % (TK / VEC)) * VEC : idx / (TM / VEC);
      const long long off = KC ? (long long)(row0 + row) * ld + k0 + kk : (long long)(k0 + kk) * ld + row0 + row;
      if (FULL) {
        r[u] = *(const v4u *)(p + off);
      } else {
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const bool in = KC ? (row0 + row < rows && k0 + kk + e < kend) : (row0 + row + e < rows && k0 + kk < kend);
          if (BF16) {
            const uint32_t h = in ? (uint32_t)((const uint16_t *)p)[off + e] : 0u;
            w[e / 2] |= h << (16 * (e % 2));
          } else {
            w[e] = in ? __float_as_uint(((const float *)p)[off + e]) : 0u;
          }
        }
        r[u] = v4u{w[0], w[1], w[2], w[3]};
      }
    }
  }

  __device__ __forceinline__ void store(E *lds) const {
    constexpr int LD = lds_ld<BF16, KC>();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = threadIdx.x + kGemmThreads * u;
      const int row = KC ? idx / (TK / VEC) : (idx % (TM / VEC)) * VEC;
      const int kk = KC ? (idx % (TK / VEC)) * VEC : idx / (TM / VEC);
      *(v4u *)(lds + (KC ? row * LD + kk : kk * LD + row)) = r[u];
    }
  }
};

// MFMA operands from a staged tile: fp32 one value (row, k); bf16 four
// values (row, k .. k + 3).
template <int KC>
__device__ __forceinline__ float frag_f32(const float *lds, int row, int k) {
  constexpr int LD = lds_ld<0, KC>();
  return KC ? lds[row * LD + k] : lds[k * LD + row];
}
template <int KC>
__device__ __forceinline__ v4s frag_bf16(const uint16_t *lds, int row, int k) {
  constexpr int LD = lds_ld<1, KC>();
  if (KC) return *(const v4s *)(lds + row * LD + k);
  v4s v;
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = (short)lds[(k + e) * LD + row];
  return v;
}

template <int BF16, int AK, int BK, int FULL>
__global__ void __launch_bounds__(kGemmThreads) gemm_kernel(GemmArgs g) {
  using E = typename GemmE<BF16>::E;
  constexpr int SA = AK ? TM * lds_ld<BF16, 1>() : TK * lds_ld<BF16, 0>();
  constexpr int SB = BK ? TN * lds_ld<BF16, 1>() : TK * lds_ld<BF16, 0>();
  __shared__ __attribute__((aligned(16))) E As[SA];
  __shared__ __attribute__((aligned(16))) E Bs[SB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c16 = lane & 15, q4 = lane >> 4;
  const int wm = wave >> 1, wn = wave & 1;
  const int bm = blockIdx.y * TM, bn = blockIdx.x * TN;
  const int kbeg = blockIdx.z * g.kslice;
  const int kend = min(g.K, kbeg + g.kslice);
  v4f acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  Stage<BF16, AK, FULL> sa;
  Stage<BF16, BK, FULL> sb;
  const int nk = (kend - kbeg + TK - 1) / TK;
  if (nk > 0) {
    sa.load(g.A, g.lda, bm, g.M, kbeg, kend);
    sb.load(g.B, g.ldb, bn, g.N, kbeg, kend);
  }
  for (int kc = 0; kc < nk; ++kc) {
    sa.store(As);
    sb.store(Bs);
    __syncthreads();
    if (kc + 1 < nk) {
      sa.load(g.A, g.lda, bm, g.M, kbeg + (kc + 1) * TK, kend);
      sb.load(g.B, g.ldb, bn, g.N, kbeg + (kc + 1) * TK, kend);
    }
    if (BF16) {
#pragma unroll
      for (int ks = 0; ks < TK; ks += 16) {
        v4s av[4], bv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          av[t] = frag_bf16<AK>((const uint16_t *)As, wm * 64 + t * 16 + c16, ks + 4 * q4);
          bv[t] = frag_bf16<BK>((const uint16_t *)Bs, wn * 64 + t * 16 + c16, ks + 4 * q4);
        }
#pragma unroll
        for (int ta = 0; ta < 4; ++ta)
#pragma unroll
          for (int tb = 0; tb < 4; ++tb)
            acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[ta], bv[tb], acc[ta][tb], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < TK; ks += 4) {
        float av[4], bv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          av[t] = frag_f32<AK>((const float *)As, wm * 64 + t * 16 + c16, ks + q4);
          bv[t] = frag_f32<BK>((const float *)Bs, wn * 64 + t * 16 + c16, ks + q4);
        }
#pragma unroll
        for (int ta = 0; ta < 4; ++ta)
#pragma unroll
          for (int tb = 0; tb < 4; ++tb)
            acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ta], bv[tb], acc[ta][tb], 0, 0, 0);
      }
    }
    __syncthreads();  // every read of this chunk precedes the next stores
  }
  // lane holds C(rows 4 q4 .. 4 q4 + 3, column c16) of each 16 x 16 tile
  float *C = g.C + (long long)blockIdx.z * g.cstride;
  long long fr[4][4], fc[4];
#pragma unroll
  for (int tb = 0; tb < 4; ++tb) fc[tb] = remap(g.map.col, bn + wn * 64 + tb * 16 + c16);
#pragma unroll
  for (int ta = 0; ta < 4; ++ta)
#pragma unroll
    for (int v = 0; v < 4; ++v) fr[ta][v] = remap(g.map.row, bm + wm * 64 + ta * 16 + 4 * q4 + v);
#pragma unroll
  for (int ta = 0; ta < 4; ++ta)
#pragma unroll
    for (int tb = 0; tb < 4; ++tb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = bm + wm * 64 + ta * 16 + 4 * q4 + v, col = bn + wn * 64 + tb * 16 + c16;
        if (FULL || (row < g.M && col < g.N)) C[fr[ta][v] + fc[tb]] = acc[ta][tb][v];
      }
}

template <int BF16, int AK, int BK>
int gemm_launch(const GemmArgs &g, int splits, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return TT_OK;
  const int vec = BF16 ? 8 : 4;
  const bool full = g.M % TM == 0 && g.N % TN == 0 && g.K % TK == 0 && g.kslice % TK == 0 && g.lda % vec == 0 &&
                    g.ldb % vec == 0 && (uintptr_t)g.A % 16 == 0 && (uintptr_t)g.B % 16 == 0 && g.K > 0;
  const dim3 grid((unsigned)((g.N + TN - 1) / TN), (unsigned)((g.M + TM - 1) / TM), (unsigned)splits),
      blk(kGemmThreads);
  if (full) hipLaunchKernelGGL((gemm_kernel<BF16, AK, BK, 1>), grid, blk, 0, s, g);
  else hipLaunchKernelGGL((gemm_kernel<BF16, AK, BK, 0>), grid, blk, 0, s, g);
  return launch_check("ttm dense GEMM");
}

// C = A B^T with operand layouts AK, BK; splits > 1 writes `splits` partial
// results cstride floats apart (k slices of kslice).
template <int AK, int BK>
int gemm(int bf16, const void *A, long long lda, const void *B, long long ldb, float *C, const CMap &map, int M,
         int N, int K, hipStream_t s, int splits = 1, int kslice = 0, long long cstride = 0) {
  GemmArgs g{A, B, C, M, N, K, splits > 1 ? kslice : ((K + TK - 1) / TK) * TK, lda, ldb, cstride, map};
  return bf16 ? gemm_launch<1, AK, BK>(g, splits, s) : gemm_launch<0, AK, BK>(g, splits, s);
}

// Remap of one digit-free index: x w.
Remap lin(long long w) { return Remap{{0, 0, 0}, {0, 0, 0, w}}; }

CMap plain(long long ldc) { return CMap{lin(ldc), lin(1)}; }

// Left partial products: rows (u, v) = u V + v, columns (i, j, b) =
// (i nn + j) r + b -> ((u mm + i) (V nn) + v nn + j) r + b.
CMap map_left(long long V, int mm, int nn, int r) {
  return CMap{Remap{{(unsigned)V, 0, 0}, {(long long)nn * r, 0, 0, (long long)mm * V * nn * r}},
              Remap{{(unsigned)r, (unsigned)nn, 0}, {1, r, 0, V * nn * r}}};
}

// dW_dense by output blocks: rows I = U mm + i, columns J = V nn + j ->
// ((U Vb + V) mm + i) nn + j with Vb = columns / nn.
CMap map_blocks(long long Vb, int mm, int nn) {
  return CMap{Remap{{(unsigned)mm, 0, 0}, {nn, 0, 0, Vb * mm * nn}},
              Remap{{(unsigned)nn, 0, 0}, {1, 0, 0, (long long)mm * nn}}};
}

// Right partial sums: rows (u', v') = u' V + v' with u' = u mm + i and
// v' = v nn + j, columns b -> (((u (V / nn) + v) mm + i) nn + j) r + b.
CMap map_right(long long V, int mm, int nn, int r) {
  const long long Vb = V / nn;
  return CMap{Remap{{(unsigned)nn, (unsigned)Vb, (unsigned)mm},
                    {r, (long long)mm * nn * r, (long long)nn * r, Vb * mm * nn * r}},
              lin(1)};
}

long long prodl(const int *a, int lo, int hi) {
  long long p = 1;
  for (int k = lo; k < hi; ++k) p *= a[k];
  return p;
}

// Elements of P_k (U_k x V_k x r_k, U_k = prod m_<k, V_k = prod n_<k).
long long p_elems(const TTMDims &D, int k) { return prodl(D.m, 0, k) * prodl(D.n, 0, k) * D.r[k]; }
// Elements of Z_k (U_{k+1} x V_{k+1} x r_{k+1}).
long long z_elems(const TTMDims &D, int k) { return prodl(D.m, 0, k + 1) * prodl(D.n, 0, k + 1) * D.r[k + 1]; }
long long core_elems(const TTMDims &D, int k) { return (long long)D.r[k] * D.m[k] * D.n[k] * D.r[k + 1]; }

// k slices of a core gradient: about 256 workgroups over the output tiles.
void dg_split(const TTMDims &D, int k, int *splits, int *kslice) {
  const long long K = prodl(D.m, 0, k) * prodl(D.n, 0, k);
  const long long tiles = ((D.r[k] + TM - 1) / TM) * (((long long)D.m[k] * D.n[k] * D.r[k + 1] + TN - 1) / TN);
  long long sp = 256 / tiles;
  const long long maxsp = (K + 4 * TK - 1) / (4 * TK);  // at least 4 chunks per slice
  sp = sp < 1 ? 1 : (sp > maxsp ? maxsp : sp);
  long long ks = (K + sp - 1) / sp;
  ks = (ks + TK - 1) / TK * TK;
  *splits = (int)((K + ks - 1) / ks);
  *kslice = (int)ks;
}

// Batch slices of dW_dense = dY^T X: enough workgroups for the chip (about
// 256 over the 128 x 128 output tiles), each slice at least 8 chunks long.
void dw_split(const TTMDims &D, long long B, int *splits, int *kslice) {
  if (B < 8 * TK) {
    *splits = 1;
    *kslice = (int)((B + TK - 1) / TK * TK + TK);
    return;
  }
  const long long tiles = ((D.Mt + TM - 1) / TM) * ((D.Nt + TN - 1) / TN);
  long long sp = 256 / tiles;
  const long long maxsp = B / (8 * TK);
  sp = sp < 1 ? 1 : (sp > maxsp ? maxsp : sp);
  if (sp > 8) sp = 8;
  if (sp < 1) sp = 1;
  long long ks = (B + sp - 1) / sp;
  ks = (ks + TK - 1) / TK * TK;
  *splits = (int)((B + ks - 1) / ks);
  *kslice = (int)ks;
}

unsigned grid_of(long long n) {
  long long g = (n + kBlk - 1) / kBlk;
  return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// P_1 .. P_d into P[1..d] (P[0] is the scalar 1 held in one):
// P_{k+1}[(u, i)][(v, j)][b] = sum_a P_k[(u, v)][a] G^k[a][(i, j, b)], a GEMM
// with rows (u, v), k = a and columns (i, j, b) placed through CMap 1.
int densify(const TTMDims &D, const void *cores, int bf16, float *const *P, float *one, hipStream_t s) {
  const size_t es = bf16 ? 2 : 4;
  for (int k = 0; k < D.d; ++k) {
    const float *in = k ? P[k] : one;
    const void *G = (const char *)cores + es * D.off[k];
    const long long U = prodl(D.m, 0, k), V = prodl(D.n, 0, k);
    const int ncol = D.m[k] * D.n[k] * D.r[k + 1];
    const CMap map = map_left(V, D.m[k], D.n[k], D.r[k + 1]);
    // the partial products stay float32: A is read as float32, B (the
    // core) in its own precision through a float32 copy when bf16
    const int rc = gemm<1, 0>(0, in, D.r[k], G, ncol, P[k + 1], map, (int)(U * V), ncol, D.r[k], s);
    if (rc) return rc;
  }
  return TT_OK;
}

struct DenseBufs {
  float *P[TT_MAX_D + 1];
  float *one;
  float *cf;      // float32 copy of the cores (bf16 inputs)
  uint16_t *wbf;  // W rounded to bf16
  float *dWd;     // dW_dense by output blocks (map_blocks)
  float *dwp;     // batch-slice partials of dW_dense
  float *Z[TT_MAX_D];
  float *part;
};

bool take_bufs(const TTMDims &D, long long B, int bf16, int backward, Arena &ar, DenseBufs &b) {
  b = DenseBufs{};
  b.one = ar.take<float>(1);
  for (int k = 1; k <= D.d; ++k) b.P[k] = ar.take<float>((size_t)p_elems(D, k));
  const size_t MN = (size_t)(D.Mt * D.Nt);
  if (bf16) {
    b.cf = ar.take<float>((size_t)D.extent);
    b.wbf = ar.take<uint16_t>(MN);
  }
  if (backward) {
    b.dWd = ar.take<float>(MN);
    int sp, ks;
    dw_split(D, B, &sp, &ks);
    if (sp > 1) b.dwp = ar.take<float>(MN * (size_t)sp);
    for (int k = 0; k + 1 < D.d; ++k) b.Z[k] = ar.take<float>((size_t)z_elems(D, k));
    size_t mp = 1;
    for (int k = 0; k < D.d; ++k) {
      int sp, ks;
      dg_split(D, k, &sp, &ks);
      const size_t c = (size_t)sp * (size_t)core_elems(D, k);
      mp = c > mp ? c : mp;
    }
    b.part = ar.take<float>(mp);
  }
  return ar.ok();
}

__global__ void __launch_bounds__(kBlk) bf16_to_f32_kernel(const uint16_t *__restrict__ x, float *__restrict__ y,
                                                           long long n) {
  for (long long e = (long long)blockIdx.x * kBlk + threadIdx.x; e < n; e += (long long)gridDim.x * kBlk)
    y[e] = bf_to_f(x[e]);
}

// W (float32 in P[d], bf16 rounded copy in wbf when bf16) from the cores.
int build_w(const TTMDims &D, const void *cores, int dtype, DenseBufs &b, const void **Wm, const void **cf,
            hipStream_t s) {
  hipLaunchKernelGGL(set_one_kernel, dim3(1), dim3(1), 0, s, b.one);
  int rc = launch_check("ttm one");
  if (rc) return rc;
  *cf = cores;
  if (dtype) {
    hipLaunchKernelGGL(bf16_to_f32_kernel, dim3(grid_of(D.extent)), dim3(kBlk), 0, s, (const uint16_t *)cores, b.cf,
                       D.extent);
    if ((rc = launch_check("ttm cores to float32"))) return rc;
    *cf = b.cf;
  }
  if ((rc = densify(D, *cf, 0, b.P, b.one, s))) return rc;
  *Wm = b.P[D.d];
  if (dtype) {
    const long long MN = D.Mt * D.Nt;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_of(MN)), dim3(kBlk), 0, s, b.P[D.d], b.wbf, MN);
    if ((rc = launch_check("ttm W to bf16"))) return rc;
    *Wm = b.wbf;
  }
  return TT_OK;
}

}  // namespace

bool ttm_dense_fits(const TTMDims &D) { return D.Mt * D.Nt <= kTtmDenseMaxElems; }

long long ttm_dense_flops(const TTMDims &D, long long B) { return 2 * B * D.Mt * D.Nt; }

size_t ttm_dense_ws(const TTMDims &D, long long B, int dtype, int backward) {
  // sizes only: a null-based arena counts the bytes (plus slack for an
  // unaligned workspace)
  Arena ar(nullptr, ~(size_t)0);
  DenseBufs b;
  take_bufs(D, B, dtype, backward, ar, b);
  return ar.used + 256;
}

int ttm_dense_forward(const TTMDims &D, const void *cores, const void *X, long long B, float *Y, int dtype, void *ws,
                      size_t bytes, hipStream_t s) {
  Arena ar(ws, bytes);
  DenseBufs b;
  if (!take_bufs(D, B, dtype, 0, ar, b)) return set_error(TT_ERR_WORKSPACE, "tt_matmul: workspace too small");
  timer_before(s);
  const void *Wm, *cf;
  int rc = build_w(D, cores, dtype, b, &Wm, &cf, s);
  if (rc) return rc;
  // Y[b][i] = sum_j X[b][j] W[i][j]
  rc = gemm<1, 1>(dtype, X, D.Nt, Wm, D.Nt, Y, plain(D.Mt), (int)B, (int)D.Mt, (int)D.Nt, s);
  timer_after(s);
  return rc;
}

int ttm_dense_backward(const TTMDims &D, const void *cores, const void *X, long long B, const void *dY, float *dX,
                       float *dW, int dtype, void *ws, size_t bytes, hipStream_t s) {
  Arena ar(ws, bytes);
  DenseBufs b;
  if (!take_bufs(D, B, dtype, 1, ar, b)) return set_error(TT_ERR_WORKSPACE, "tt_matmul_backward: workspace too small");
  const int d = D.d;
  timer_before(s);
  const void *Wm, *cf;
  int rc = build_w(D, cores, dtype, b, &Wm, &cf, s);
  if (rc) return rc;
  // dX[b][j] = sum_i dY[b][i] W[i][j]  (W read row-contiguous)
  if (dX && (rc = gemm<1, 0>(dtype, dY, D.Mt, Wm, D.Nt, dX, plain(D.Nt), (int)B, (int)D.Nt, (int)D.Mt, s))) return rc;
  if (dW) {
    // Z_{d-1} = dW_dense[i][j] = sum_b dY[b][i] X[b][j] (both operands
    // row-contiguous), stored as [(I<, J<)][(i_{d-1}, j_{d-1})] (CMap 2)
    const CMap mdw = map_blocks(D.Nt / D.n[d - 1], D.m[d - 1], D.n[d - 1]);
    const long long MN = D.Mt * D.Nt;
    int sp, ks;
    dw_split(D, B, &sp, &ks);
    if (sp > 1) {
      // too few output tiles to fill the chip: slices of the batch into
      // partial matrices, summed in slice order
      if ((rc = gemm<0, 0>(dtype, dY, D.Mt, X, D.Nt, b.dwp, mdw, (int)D.Mt, (int)D.Nt, (int)B, s, sp, ks, MN)))
        return rc;
      hipLaunchKernelGGL(dg_reduce_kernel, dim3(grid_of(MN)), dim3(kBlk), 0, s, b.dwp, sp, MN, b.dWd);
      if ((rc = launch_check("ttm dW slices"))) return rc;
    } else if ((rc = gemm<0, 0>(dtype, dY, D.Mt, X, D.Nt, b.dWd, mdw, (int)D.Mt, (int)D.Nt, (int)B, s))) {
      return rc;
    }
    // Z_k[(u', v')][b] = sum_{(i, j, b')} Z_{k+1}[(u', v')][(i, j, b')] G^{k+1}[b][(i, j, b')],
    // stored as [(u, v)][(i_k, j_k)][b] (CMap 3) for the next step
    for (int k = d - 2; k >= 0; --k) {
      const float *Zn = (k == d - 2) ? b.dWd : b.Z[k + 1];
      const float *G = (const float *)cf + D.off[k + 1];
      const long long U = prodl(D.m, 0, k + 1), V = prodl(D.n, 0, k + 1);
      const int kk = D.m[k + 1] * D.n[k + 1] * D.r[k + 2];
      const CMap mz = map_right(V, D.m[k], D.n[k], D.r[k + 1]);
      if ((rc = gemm<1, 1>(0, Zn, kk, G, kk, b.Z[k], mz, (int)(U * V), D.r[k + 1], kk, s))) return rc;
    }
    // dG^k[a][(i, j, b)] = sum_{(u, v)} P_k[(u, v)][a] Z_k[(u, v)][(i, j, b)]:
    // both operands row-contiguous, the k range split over workgroups and
    // the slices summed in order
    for (int k = 0; k < d; ++k) {
      const float *Pk = k ? b.P[k] : b.one;
      const float *Zk = (k == d - 1) ? b.dWd : b.Z[k];
      const long long K = prodl(D.m, 0, k) * prodl(D.n, 0, k);
      const int ncol = D.m[k] * D.n[k] * D.r[k + 1];
      const long long cnt = core_elems(D, k);
      int sp, ks;
      dg_split(D, k, &sp, &ks);
      if ((rc = gemm<0, 0>(0, Pk, D.r[k], Zk, ncol, b.part, plain(ncol), D.r[k], ncol, (int)K, s, sp, ks, cnt)))
        return rc;
      hipLaunchKernelGGL(dg_reduce_kernel, dim3((unsigned)((cnt + kBlk - 1) / kBlk)), dim3(kBlk), 0, s, b.part, sp,
                         cnt, dW + D.off[k]);
      if ((rc = launch_check("ttm core gradient reduce"))) return rc;
    }
  }
  timer_after(s);
  return TT_OK;
}

}  // namespace ttgfx
