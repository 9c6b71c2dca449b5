// TT-matrix layer (t3f.matmul(tt_matrix, x), Implementation Details):
// Y = X W^T with W[(i_1..i_d), (j_1..j_d)] = G^1[i_1, j_1] ... G^d[i_d, j_d]
// (cores r_k x m_k x n_k x r_{k+1}), and its adjoint dX = dY W, dG^k.
//
// All sweeps are built from one contraction step over an intermediate laid
// out as IN[p][j][q][a] (p = batch row and modes already produced, j = the
// mode being contracted, q = modes still to come, a = bond index):
//     OUT[p][i][q][b] = sum_{j, a} IN[p][j][q][a] * core(a, j -> i, b)
// evaluated as a GEMM with rows (p, q), K = (j, a), N = (i, b) on
// v_mfma_f32_16x16x4_f32, or v_mfma_f32_16x16x16_bf16 with float32
// accumulation.  The core element is addressed through four strides, so the
// same kernel runs the forward sweep (contract j_k, produce i_k), dX
// (contract i_k, produce j_k) and the right-to-left sweep of dY that the core
// gradient needs.  The gradient of core k is
//     dG^k[a, i, j, b] = sum_{p, q} T_k[p][j][q][a] * V_{k+1}[p][i][q][b]
// (forward intermediate against backward intermediate), a GEMM whose K = (p, q)
// is split across workgroups; the per-workgroup partial tiles are summed in a
// fixed order, so the gradient is deterministic.
#include "common.h"
#include "ttm.h"

namespace ttgfx {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma_f32(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma_bf16(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
// Round to nearest, ties to even (NaN stays NaN).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <int BF16>
__device__ __forceinline__ float load_el(const void *p, long long i) {
  if (BF16) return bf16_to_f32(((const uint16_t *)p)[i]);
  return ((const float *)p)[i];
}


// Eight consecutive bfloat16 elements at element offset i (a multiple of
// 8), widened to float.
__device__ __forceinline__ void load8_bf16(const void *p, long long i, float (&o)[8]) {
  const uint4 u = *(const uint4 *)((const uint16_t *)p + i);
  const unsigned w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    o[2 * x] = __uint_as_float(w[x] << 16);
    o[2 * x + 1] = __uint_as_float(w[x] & 0xffff0000u);
  }
}

constexpr int kThreads = 256;  // 4 waves
// The step kernel stages the whole core in LDS (64 KB in fp32 at the
// largest fused sizes), so its workgroups are 8 waves: two of them per CU
// still give 4 waves per SIMD.
constexpr int kStepThreads = 512;
constexpr int kStepRows = 16 * (kStepThreads / 64);
constexpr int kMaxTiles = TTM_MAX_FUSED / 16;

struct Step {
  long long P, Q;   // outer and trailing counts
  int nin, rin;     // contracted mode size, bond of IN
  int mout, rout;   // produced mode size, bond of OUT
  const void *in;
  void *out;
  const void *core;
  long long sa, sj, si, sb;  // core element (a, j, i, b) at a*sa + j*sj + i*si + b*sb
};

// One workgroup stages the whole core in B-operand order (in its own
// precision) and the offsets of the K indices (j, a) inside an IN row, then
// walks row blocks of 64 (p, q) rows; every wave owns 16 rows and all N
// tiles.  Row and column offsets are computed once per block and per lane,
// so the inner loop has no integer division.  VEC: the bond of IN is a
// multiple of 4, so the 4 K values of a lane are contiguous and load as
// one vector.
template <int BF16, int VEC>
__global__ void __launch_bounds__(kStepThreads) ttm_step_kernel(Step s, int out_f32) {
  extern __shared__ __align__(16) char smem[];
  const int K = s.nin * s.rin, N = s.mout * s.rout;
  const int KC = (K + 15) / 16, NT = (N + 15) / 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c16 = lane & 15, q4 = lane >> 4;
  long long *koff = (long long *)smem;  // [KC * 16], -1 past K
  char *bsm = smem + 16 * ((KC * 16 * 8 + 15) / 16);
  const long long jstride = s.Q * s.rin;
  for (int kk = tid; kk < KC * 16; kk += kStepThreads) koff[kk] = kk < K ? (kk / s.rin) * jstride + kk % s.rin : -1;
  // chunk x (16 K values), tile t: lane (q4, c16) holds B[16x + 4q4 + v][16t + c16]
  for (int e = tid; e < KC * NT * 256; e += kStepThreads) {
    const int v = e & 3, ln = (e >> 2) & 63, xt = e >> 8;
    const int x = xt / NT, t = xt % NT;
    const int kk = 16 * x + 4 * (ln >> 4) + v, nn = 16 * t + (ln & 15);
    const long long ci = (kk < K && nn < N)
                             ? (kk / s.rin) * s.sj + (kk % s.rin) * s.sa + (nn / s.rout) * s.si + (nn % s.rout) * s.sb
                             : -1;
    if (BF16) ((uint16_t *)bsm)[e] = ci >= 0 ? ((const uint16_t *)s.core)[ci] : (uint16_t)0;
    else ((float *)bsm)[e] = ci >= 0 ? ((const float *)s.core)[ci] : 0.f;
  }
  // per-lane output column offsets
  long long coff[kMaxTiles];
#pragma unroll
  for (int t = 0; t < kMaxTiles; ++t) {
    const int nn = 16 * t + c16;
    coff[t] = (t < NT && nn < N) ? (long long)(nn / s.rout) * s.Q * s.rout + nn % s.rout : -1;
  }
  __syncthreads();
  const long long rows = s.P * s.Q;
  for (long long r0 = (long long)blockIdx.x * kStepRows; r0 < rows; r0 += (long long)gridDim.x * kStepRows) {
    const long long row = r0 + wave * 16 + c16;  // A-operand row of this lane
    const bool rvalid = row < rows;
    const long long p = rvalid ? row / s.Q : 0, q = rvalid ? row % s.Q : 0;
    const long long abase = (p * s.nin * s.Q + q) * s.rin;
    v4f acc[kMaxTiles];
#pragma unroll
    for (int t = 0; t < kMaxTiles; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    // A operand of K chunk x: the lane's 4 K values of its row (fp32), or
    // the same 4 as bfloat16; the next chunk's load is in flight while this
    // chunk's products run
    auto load_a = [&](int x, v4f &af, v4s &ab) {
      const int kb = 16 * x + 4 * q4;
      if (BF16) {
        if (VEC) {
          const long long o = koff[kb];
          ab = (rvalid && o >= 0) ? *(const v4s *)((const uint16_t *)s.in + abase + o) : v4s{0, 0, 0, 0};
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const long long o = koff[kb + v];
            ab[v] = (rvalid && o >= 0) ? (short)((const uint16_t *)s.in)[abase + o] : (short)0;
          }
        }
      } else {
        if (VEC) {
          const long long o = koff[kb];
          af = (rvalid && o >= 0) ? *(const v4f *)((const float *)s.in + abase + o) : v4f{0.f, 0.f, 0.f, 0.f};
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const long long o = koff[kb + v];
            af[v] = (rvalid && o >= 0) ? ((const float *)s.in)[abase + o] : 0.f;
          }
        }
      }
    };
    v4f afn = {0.f, 0.f, 0.f, 0.f};
    v4s abn = {0, 0, 0, 0};
    load_a(0, afn, abn);
    for (int x = 0; x < KC; ++x) {
      const v4f av = afn;
      const v4s a4 = abn;
      if (x + 1 < KC) load_a(x + 1, afn, abn);
      if (BF16) {
#pragma unroll
        for (int t = 0; t < kMaxTiles; ++t)
          if (t < NT) acc[t] = mfma_bf16(a4, ((const v4s *)bsm)[(x * NT + t) * 64 + lane], acc[t]);
      } else {
#pragma unroll
        for (int t = 0; t < kMaxTiles; ++t) {
          if (t < NT) {
            const v4f bv = ((const v4f *)bsm)[(x * NT + t) * 64 + lane];
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t] = mfma_f32(av[v], bv[v], acc[t]);
          }
        }
      }
    }
    // D tile t: lane (q4, c16) value v is row r0 + 16 wave + 4 q4 + v, column 16 t + c16
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long long orow = r0 + wave * 16 + 4 * q4 + v;
      if (orow >= rows) continue;
      const long long op = orow / s.Q, oq = orow % s.Q;
      const long long rbase = op * s.mout * s.Q * s.rout + oq * s.rout;
#pragma unroll
      for (int t = 0; t < kMaxTiles; ++t) {
        if (coff[t] < 0) continue;
        const long long off = rbase + coff[t];
        if (BF16 && !out_f32) ((uint16_t *)s.out)[off] = f32_to_bf16(acc[t][v]);
        else ((float *)s.out)[off] = acc[t][v];
      }
    }
  }
}

struct GradArgs {
  long long P, Q;
  int n, m, rT, rV;
  const void *T;     // [P][n][Q][rT]
  const void *V;     // [P][m][Q][rV]
  float *part;       // [gridDim.x][rT * m * n * rV], core order
  long long kchunk;  // (p, q) pairs per workgroup, a multiple of 4
};

// Partial core gradient over this workgroup's (p, q) range.  Rows of the
// product are (j, a) with a fastest, columns (i, b) with b fastest.  Slabs
// of kSlab consecutive (p, q) pairs of T and V are staged in LDS (coalesced
// loads through precomputed row/column offsets, no division in the loop),
// then every wave multiplies its row tiles against all column tiles.
constexpr int kSlab = 32;
constexpr int kLd = TTM_MAX_FUSED + 4;

// VT, VV: the rank of T (of V) is a multiple of 4 (8 for bfloat16), so that
// operand's elements (a, or b, fastest) load 16 bytes at a time.
template <int BF16, int VT, int VV>
__global__ void __launch_bounds__(kThreads) ttm_grad_kernel(GradArgs g) {
  __shared__ float ts[kSlab][kLd];
  __shared__ float vs[kSlab][kLd];
  // bfloat16 slabs reuse the same memory as [row][k] tables
  constexpr int kLdb = kSlab + 4;
  static_assert(TTM_MAX_FUSED * kLdb * 2 <= kSlab * kLd * 4, "bf16 slab fits");
  uint16_t *tsb = (uint16_t *)&ts[0][0];
  uint16_t *vsb = (uint16_t *)&vs[0][0];
  __shared__ long long roff[TTM_MAX_FUSED], coffs[TTM_MAX_FUSED];
  const int ROWS = g.rT * g.n, COLS = g.m * g.rV;
  const int RT = (ROWS + 15) / 16, CT = (COLS + 15) / 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c16 = lane & 15, q4 = lane >> 4;
  for (int i = tid; i < ROWS; i += kThreads) roff[i] = (long long)(i / g.rT) * g.Q * g.rT + i % g.rT;
  for (int i = tid; i < COLS; i += kThreads) coffs[i] = (long long)(i / g.rV) * g.Q * g.rV + i % g.rV;
  // rows and columns past the product are zero (their outputs are discarded)
  for (int e = tid; e < kSlab * kLd; e += kThreads) {
    (&ts[0][0])[e] = 0.f;
    (&vs[0][0])[e] = 0.f;
  }
  const long long K = g.P * g.Q;
  const long long k0 = (long long)blockIdx.x * g.kchunk;
  const long long k1 = (k0 + g.kchunk < K) ? k0 + g.kchunk : K;
  constexpr int RPW = kMaxTiles / (kThreads / 64);  // row tiles per wave
  v4f acc[RPW][kMaxTiles];
#pragma unroll
  for (int u = 0; u < RPW; ++u)
#pragma unroll
    for (int t = 0; t < kMaxTiles; ++t) acc[u][t] = v4f{0.f, 0.f, 0.f, 0.f};
  // slab loads go through registers: the next slab is fetched while the
  // current one is multiplied.  Per-slab (p, q) base offsets are computed
  // one slab ahead by kSlab threads into a double-buffered table.
  __shared__ long long tb[2][kSlab], vb[2][kSlab];
  constexpr int EW = BF16 ? 8 : 4;                   // elements in 16 bytes
  constexpr int ET = VT ? EW : 1, EV = VV ? EW : 1;  // elements per load
  constexpr int kPerT = kSlab * TTM_MAX_FUSED / kThreads / ET, kPerV = kSlab * TTM_MAX_FUSED / kThreads / EV;
  float tr[kPerT][ET], vr[kPerV][EV];
  auto bases = [&](long long kb, int buf) {
    if (tid < kSlab) {
      const long long kk = kb + tid;
      const long long p = kk / g.Q, q = kk % g.Q;
      tb[buf][tid] = kk < k1 ? (p * g.n * g.Q + q) * g.rT : -1;
      vb[buf][tid] = kk < k1 ? (p * g.m * g.Q + q) * g.rV : -1;
    }
  };
  auto fetch = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kPerT; ++u) {
      const int e = ET * (tid + u * kThreads);  // first of this load's elements
#pragma unroll
      for (int x = 0; x < ET; ++x) tr[u][x] = 0.f;
      if (e < kSlab * ROWS) {
        const long long base = tb[buf][e / ROWS];
        if (base >= 0) {
          if constexpr (VT && BF16) {
            load8_bf16(g.T, base + roff[e % ROWS], tr[u]);
          } else if constexpr (VT) {
            const v4f w = *(const v4f *)((const float *)g.T + base + roff[e % ROWS]);
#pragma unroll
            for (int x = 0; x < ET; ++x) tr[u][x] = w[x];
          } else {
            tr[u][0] = load_el<BF16>(g.T, base + roff[e % ROWS]);
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kPerV; ++u) {
      const int e = EV * (tid + u * kThreads);
#pragma unroll
      for (int x = 0; x < EV; ++x) vr[u][x] = 0.f;
      if (e < kSlab * COLS) {
        const long long base = vb[buf][e / COLS];
        if (base >= 0) {
          if constexpr (VV && BF16) {
            load8_bf16(g.V, base + coffs[e % COLS], vr[u]);
          } else if constexpr (VV) {
            const v4f w = *(const v4f *)((const float *)g.V + base + coffs[e % COLS]);
#pragma unroll
            for (int x = 0; x < EV; ++x) vr[u][x] = w[x];
          } else {
            vr[u][0] = load_el<BF16>(g.V, base + coffs[e % COLS]);
          }
        }
      }
    }
  };
  bases(k0, 0);
  __syncthreads();  // offsets and the first bases ready
  if (k0 < k1) fetch(0);
  int sl = 0;
  for (long long kb = k0; kb < k1; kb += kSlab, ++sl) {
    __syncthreads();  // the previous slab is consumed
    if constexpr (BF16) {
      // bfloat16 slabs, K fastest: tsb[row][k], vsb[col][k] (the values
      // came from bfloat16, so the conversion back is exact)
#pragma unroll
      for (int u = 0; u < kPerT; ++u) {
        const int e = ET * (tid + u * kThreads);
#pragma unroll
        for (int x = 0; x < ET; ++x)
          if (e < kSlab * ROWS) tsb[(e % ROWS + x) * kLdb + e / ROWS] = f32_to_bf16(tr[u][x]);
      }
#pragma unroll
      for (int u = 0; u < kPerV; ++u) {
        const int e = EV * (tid + u * kThreads);
#pragma unroll
        for (int x = 0; x < EV; ++x)
          if (e < kSlab * COLS) vsb[(e % COLS + x) * kLdb + e / COLS] = f32_to_bf16(vr[u][x]);
      }
    } else {
#pragma unroll
      for (int u = 0; u < kPerT; ++u) {
        const int e = ET * (tid + u * kThreads);
#pragma unroll
        for (int x = 0; x < ET; ++x)
          if (e < kSlab * ROWS) ts[e / ROWS][e % ROWS + x] = tr[u][x];
      }
#pragma unroll
      for (int u = 0; u < kPerV; ++u) {
        const int e = EV * (tid + u * kThreads);
#pragma unroll
        for (int x = 0; x < EV; ++x)
          if (e < kSlab * COLS) vs[e / COLS][e % COLS + x] = vr[u][x];
      }
    }
    bases(kb + kSlab, (sl + 1) & 1);
    __syncthreads();
    if (kb + kSlab < k1) fetch((sl + 1) & 1);
    if constexpr (BF16) {
      // bfloat16 MFMA, 16 K values per product: lane (q4, c16) holds K
      // values 4 q4 .. 4 q4 + 3 of its row (A) and of its column (B), one
      // 8-byte LDS read each; the D layout is that of the fp32 product
#pragma unroll
      for (int kg = 0; kg < kSlab / 16; ++kg) {
        const int kl = 16 * kg + 4 * q4;
        v4s a4[RPW];
#pragma unroll
        for (int u = 0; u < RPW; ++u) a4[u] = *(const v4s *)(tsb + (16 * (wave + 4 * u) + c16) * kLdb + kl);
#pragma unroll
        for (int t = 0; t < kMaxTiles; ++t) {
          if (t >= CT) continue;
          const v4s b4 = *(const v4s *)(vsb + (16 * t + c16) * kLdb + kl);
#pragma unroll
          for (int u = 0; u < RPW; ++u)
            if (wave + 4 * u < RT) acc[u][t] = mfma_bf16(a4[u], b4, acc[u][t]);
        }
      }
      continue;
    }
#pragma unroll
    for (int ks = 0; ks < kSlab / 4; ++ks) {
      const int kl = 4 * ks + q4;  // K slot q4 of this lane
      float av[RPW];
#pragma unroll
      for (int u = 0; u < RPW; ++u) av[u] = ts[kl][16 * (wave + 4 * u) + c16];
#pragma unroll
      for (int t = 0; t < kMaxTiles; ++t) {
        if (t >= CT) continue;
        const float bv = vs[kl][16 * t + c16];
#pragma unroll
        for (int u = 0; u < RPW; ++u)
          if (wave + 4 * u < RT) acc[u][t] = mfma_f32(av[u], bv, acc[u][t]);
      }
    }
  }
  float *part = g.part + (long long)blockIdx.x * ROWS * COLS;
#pragma unroll
  for (int u = 0; u < RPW; ++u) {
    const int rt = wave + 4 * u;
    if (rt >= RT) continue;
#pragma unroll
    for (int t = 0; t < kMaxTiles; ++t) {
      const int col = 16 * t + c16;
      if (t >= CT || col >= COLS) continue;
      const int i = col / g.rV, b = col % g.rV;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * rt + 4 * q4 + v;
        if (row >= ROWS) continue;
        const int j = row / g.rT, a = row % g.rT;
        part[(((long long)a * g.m + i) * g.n + j) * g.rV + b] = acc[u][t][v];
      }
    }
  }
}

// out[e] = sum_w part[w][e] in a fixed order (4 interleaved partial sums).
__global__ void __launch_bounds__(256) ttm_grad_reduce_kernel(const float *__restrict__ part, int nwg,
                                                             long long cnt, float *__restrict__ out) {
  __shared__ float red[4][64];
  const int el = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const long long e = (long long)blockIdx.x * 64 + el;
  float s = 0.f;
  if (e < cnt)
    for (int w = grp; w < nwg; w += 4) s += part[(long long)w * cnt + e];
  red[grp][el] = s;
  __syncthreads();
  if (grp == 0 && e < cnt) out[e] = (red[0][el] + red[1][el]) + (red[2][el] + red[3][el]);
}

constexpr int kMaxGradWG = 512;

size_t step_lds(int K, int N, int bf16) {
  const size_t kc = (K + 15) / 16, nt = (N + 15) / 16;
  return 16 * ((kc * 16 * 8 + 15) / 16) + (bf16 ? 2 : 4) * 256 * kc * nt;
}

int set_step_attrs() {
  const int lds = (int)step_lds(TTM_MAX_FUSED, TTM_MAX_FUSED, 0);
  const void *fns[4] = {(const void *)ttm_step_kernel<0, 0>, (const void *)ttm_step_kernel<0, 1>,
                        (const void *)ttm_step_kernel<1, 0>, (const void *)ttm_step_kernel<1, 1>};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 4 && e == hipSuccess; ++i)
    e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  return hip_check(e, "ttm step LDS attribute");
}

int launch_step(const Step &s, int bf16, int out_f32, hipStream_t st) {
  static const int attr_rc = set_step_attrs();
  if (attr_rc) return attr_rc;
  const size_t shm = step_lds(s.nin * s.rin, s.mout * s.rout, bf16);
  const long long rows = s.P * s.Q;
  // enough workgroups to fill the chip a few times over; each one stages the
  // core once and then walks many row blocks
  long long nb = (rows + kStepRows - 1) / kStepRows;
  nb = nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
  // vector loads need the 4 K values of a lane contiguous: a bond of IN
  // that is a multiple of 4 and an IN pointer aligned to 4 elements
  const size_t esize = bf16 ? 2 : 4;
  const bool vec = (s.rin % 4 == 0) && ((uintptr_t)s.in % (4 * esize) == 0);
  const dim3 g((unsigned)nb), blk(kStepThreads);
  if (bf16 && vec) hipLaunchKernelGGL((ttm_step_kernel<1, 1>), g, blk, shm, st, s, out_f32);
  else if (bf16) hipLaunchKernelGGL((ttm_step_kernel<1, 0>), g, blk, shm, st, s, out_f32);
  else if (vec) hipLaunchKernelGGL((ttm_step_kernel<0, 1>), g, blk, shm, st, s, out_f32);
  else hipLaunchKernelGGL((ttm_step_kernel<0, 0>), g, blk, shm, st, s, out_f32);
  return launch_check("ttm step");
}

long long prod(const int *a, int lo, int hi) {
  long long p = 1;
  for (int k = lo; k < hi; ++k) p *= a[k];
  return p;
}

size_t esz(int bf16) { return bf16 ? 2 : 4; }
long long core_cnt(const TTMDims &D, int k) { return (long long)D.r[k] * D.m[k] * D.n[k] * D.r[k + 1]; }

// Forward intermediate after k steps (also the size of the dY-sweep
// intermediate V_k): B * prod m_<k * prod n_>=k * r_k elements.
long long fwd_elems(const TTMDims &D, long long B, int k) {
  return B * prod(D.m, 0, k) * prod(D.n, k, D.d) * D.r[k];
}
// dX-sweep intermediate after k steps: B * prod n_<k * prod m_>=k * r_k.
long long adj_elems(const TTMDims &D, long long B, int k) {
  return B * prod(D.n, 0, k) * prod(D.m, k, D.d) * D.r[k];
}

long long max_pingpong(const TTMDims &D, long long B, int backward) {
  long long mx = 1;
  for (int k = 1; k < D.d; ++k) {
    mx = fwd_elems(D, B, k) > mx ? fwd_elems(D, B, k) : mx;
    if (backward) mx = adj_elems(D, B, k) > mx ? adj_elems(D, B, k) : mx;
  }
  return mx;
}

// Step k of the forward sweep: contract (j_k, left bond), produce (i_k, right bond).
Step forward_step(const TTMDims &D, const void *cores, int bf16, long long B, int k, const void *in, void *out) {
  Step s;
  s.P = B * prod(D.m, 0, k);
  s.Q = prod(D.n, k + 1, D.d);
  s.nin = D.n[k];
  s.rin = D.r[k];
  s.mout = D.m[k];
  s.rout = D.r[k + 1];
  s.in = in;
  s.out = out;
  s.core = (const char *)cores + esz(bf16) * D.off[k];
  s.sa = (long long)D.m[k] * D.n[k] * D.r[k + 1];
  s.si = (long long)D.n[k] * D.r[k + 1];
  s.sj = D.r[k + 1];
  s.sb = 1;
  return s;
}

}  // namespace

int ttm_validate(const tt_matrix *W, long long B, int dtype, TTMDims *D) {
  if (!W) return set_error(TT_ERR_ARG, "W: null descriptor");
  if (W->d < 1 || W->d > TT_MAX_D) return set_error(TT_ERR_ARG, "W: d = %d outside [1, %d]", W->d, TT_MAX_D);
  if (!W->m || !W->n || !W->r) return set_error(TT_ERR_ARG, "W: null m, n or r array");
  if (!W->data) return set_error(TT_ERR_ARG, "W: null data pointer");
  if (dtype != 0 && dtype != 1) return set_error(TT_ERR_ARG, "dtype %d is neither 0 (float32) nor 1 (bf16)", dtype);
  if (B < 0) return set_error(TT_ERR_ARG, "negative batch %lld", B);
  if (B > (1LL << 24)) return set_error(TT_ERR_UNSUPPORTED, "batch %lld above 2^24", B);
  if (W->r[0] != 1 || W->r[W->d] != 1)
    return set_error(TT_ERR_SHAPE, "W: boundary ranks must be 1 (got %d, %d)", W->r[0], W->r[W->d]);
  D->d = W->d;
  for (int k = 0; k <= W->d; ++k) {
    if (W->r[k] < 1 || W->r[k] > TT_MAX_RANK)
      return set_error(TT_ERR_SHAPE, "W: r[%d] = %d outside [1, %d]", k, W->r[k], TT_MAX_RANK);
    D->r[k] = W->r[k];
  }
  D->Mt = D->Nt = 1;
  D->extent = 0;
  long long o = 0;
  for (int k = 0; k < W->d; ++k) {
    if (W->m[k] < 1 || W->n[k] < 1 || W->m[k] > TT_MAX_N || W->n[k] > TT_MAX_N)
      return set_error(TT_ERR_SHAPE, "W: mode sizes m[%d] = %d, n[%d] = %d outside [1, %d]", k, W->m[k], k,
                       W->n[k], TT_MAX_N);
    D->m[k] = W->m[k];
    D->n[k] = W->n[k];
    const int lim = TTM_MAX_FUSED;
    if (W->m[k] * W->r[k] > lim || W->m[k] * W->r[k + 1] > lim || W->n[k] * W->r[k] > lim ||
        W->n[k] * W->r[k + 1] > lim)
      return set_error(TT_ERR_UNSUPPORTED, "W: core %d (%d x %d x %d x %d): a mode size times a rank exceeds %d",
                       k, W->r[k], W->m[k], W->n[k], W->r[k + 1], lim);
    D->Mt *= W->m[k];
    D->Nt *= W->n[k];
    if (D->Mt > (1LL << 31) || D->Nt > (1LL << 31))
      return set_error(TT_ERR_UNSUPPORTED, "W: more than 2^31 rows or columns");
    if (W->off && W->off[k] < 0) return set_error(TT_ERR_ARG, "W: negative offset for core %d", k);
    D->off[k] = W->off ? W->off[k] : o;
    o += core_cnt(*D, k);
    const long long end = D->off[k] + core_cnt(*D, k);
    D->extent = end > D->extent ? end : D->extent;
  }
  return TT_OK;
}

static size_t chain_ws(const TTMDims &D, long long B, int dtype, int backward) {
  const size_t e = esz(dtype);
  size_t bytes = 2 * arena_bytes<char>(e * (size_t)max_pingpong(D, B, backward));
  if (backward) {
    for (int k = 1; k < D.d; ++k) bytes += arena_bytes<char>(e * (size_t)fwd_elems(D, B, k));
    long long mc = 1;
    for (int k = 0; k < D.d; ++k) mc = core_cnt(D, k) > mc ? core_cnt(D, k) : mc;
    bytes += arena_bytes<float>((size_t)kMaxGradWG * mc);
  }
  return bytes;
}

static int chain_forward(const TTMDims &D, const void *cores, const void *X, long long B, float *Y, int dtype,
                         void *ws, size_t bytes, hipStream_t st) {
  Arena ar(ws, bytes);
  const size_t pp = esz(dtype) * (size_t)max_pingpong(D, B, 0);
  void *buf[2] = {ar.take<char>(pp), ar.take<char>(pp)};
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "tt_matmul: workspace too small");
  timer_before(st);
  const void *in = X;
  for (int k = 0; k < D.d; ++k) {
    const bool last = (k == D.d - 1);
    const Step s = forward_step(D, cores, dtype, B, k, in, last ? (void *)Y : buf[k & 1]);
    const int rc = launch_step(s, dtype, last ? 1 : 0, st);
    if (rc) return rc;
    in = s.out;
  }
  timer_after(st);
  return TT_OK;
}

static int chain_backward(const TTMDims &D, const void *cores, const void *X, long long B, const void *dY,
                          float *dX, float *dW, int dtype, void *ws, size_t bytes, hipStream_t st) {
  const size_t e = esz(dtype);
  const int d = D.d;
  Arena ar(ws, bytes);
  const size_t pp = e * (size_t)max_pingpong(D, B, 1);
  void *buf[2] = {ar.take<char>(pp), ar.take<char>(pp)};
  void *V[TT_MAX_D + 1] = {};  // V[k]: dY with cores k..d-1 contracted, k = 1..d-1
  for (int k = 1; k < d; ++k) V[k] = ar.take<char>(e * (size_t)fwd_elems(D, B, k));
  long long mc = 1;
  for (int k = 0; k < d; ++k) mc = core_cnt(D, k) > mc ? core_cnt(D, k) : mc;
  float *part = ar.take<float>((size_t)kMaxGradWG * mc);
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "tt_matmul_backward: workspace too small");
  const char *cb = (const char *)cores;
  int rc;
  timer_before(st);
  // dX = dY W: contract (i_k, left bond), produce (j_k, right bond), left to right
  if (dX) {
    const void *in = dY;
    for (int k = 0; k < d; ++k) {
      const bool last = (k == d - 1);
      Step s;
      s.P = B * prod(D.n, 0, k);
      s.Q = prod(D.m, k + 1, d);
      s.nin = D.m[k];
      s.rin = D.r[k];
      s.mout = D.n[k];
      s.rout = D.r[k + 1];
      s.in = in;
      s.out = last ? (void *)dX : buf[k & 1];
      s.core = cb + e * D.off[k];
      s.sa = (long long)D.m[k] * D.n[k] * D.r[k + 1];
      s.sj = (long long)D.n[k] * D.r[k + 1];  // contracted i_k
      s.si = D.r[k + 1];                      // produced j_k
      s.sb = 1;
      if ((rc = launch_step(s, dtype, last ? 1 : 0, st))) return rc;
      in = s.out;
    }
  }
  if (dW) {
    // V_k from V_{k+1} (V_d = dY), k = d-1 .. 1.  V_{k+1} is laid out as
    // [B prod m_<k][m_k][prod n_>k][r_{k+1}]; contracting (i_k, right bond)
    // and producing (j_k, left bond) gives V_k as [B prod m_<k][n_k][prod n_>k][r_k].
    for (int k = d - 1; k >= 1; --k) {
      Step s;
      s.P = B * prod(D.m, 0, k);
      s.Q = prod(D.n, k + 1, d);
      s.nin = D.m[k];
      s.rin = D.r[k + 1];
      s.mout = D.n[k];
      s.rout = D.r[k];
      s.in = (k == d - 1) ? dY : V[k + 1];
      s.out = V[k];
      s.core = cb + e * D.off[k];
      s.sa = 1;                                        // right bond (contracted)
      s.sj = (long long)D.n[k] * D.r[k + 1];           // i_k (contracted)
      s.si = D.r[k + 1];                               // j_k (produced)
      s.sb = (long long)D.m[k] * D.n[k] * D.r[k + 1];  // left bond (produced)
      if ((rc = launch_step(s, dtype, 0, st))) return rc;
    }
    // forward sweep T_0 = X, T_{k+1} = step_k(T_k), with dG^k from T_k and V_{k+1}:
    // T_k is [B prod m_<k][n_k][prod n_>k][r_k], V_{k+1} is [B prod m_<k][m_k][prod n_>k][r_{k+1}]
    const void *T = X;
    for (int k = 0; k < d; ++k) {
      GradArgs g;
      g.P = B * prod(D.m, 0, k);
      g.Q = prod(D.n, k + 1, d);
      g.n = D.n[k];
      g.m = D.m[k];
      g.rT = D.r[k];
      g.rV = D.r[k + 1];
      g.T = T;
      g.V = (k == d - 1) ? dY : V[k + 1];
      g.part = part;
      const long long K = g.P * g.Q;
      long long nwg = (K + 1023) / 1024;
      nwg = nwg < 1 ? 1 : (nwg > kMaxGradWG ? kMaxGradWG : nwg);
      g.kchunk = ((K + nwg - 1) / nwg + 3) / 4 * 4;
      if (g.kchunk < 4) g.kchunk = 4;
      nwg = (K + g.kchunk - 1) / g.kchunk;
      if (nwg < 1) nwg = 1;
      // 16-byte loads need the operand's rank to fill them and its base
      // 16-byte aligned
      const int ew = dtype ? 8 : 4;
      const int vt = g.rT % ew == 0 && (uintptr_t)g.T % 16 == 0;
      const int vv = g.rV % ew == 0 && (uintptr_t)g.V % 16 == 0;
      typedef void (*GradFn)(GradArgs);
      static const GradFn fns[2][2][2] = {
          {{ttm_grad_kernel<0, 0, 0>, ttm_grad_kernel<0, 0, 1>}, {ttm_grad_kernel<0, 1, 0>, ttm_grad_kernel<0, 1, 1>}},
          {{ttm_grad_kernel<1, 0, 0>, ttm_grad_kernel<1, 0, 1>}, {ttm_grad_kernel<1, 1, 0>, ttm_grad_kernel<1, 1, 1>}}};
      hipLaunchKernelGGL(fns[dtype ? 1 : 0][vt][vv], dim3((unsigned)nwg), dim3(kThreads), 0, st, g);
      if ((rc = launch_check("ttm core gradient"))) return rc;
      const long long cnt = core_cnt(D, k);
      hipLaunchKernelGGL(ttm_grad_reduce_kernel, dim3((unsigned)((cnt + 63) / 64)), dim3(256), 0, st,
                         (const float *)part, (int)nwg, cnt, dW + D.off[k]);
      if ((rc = launch_check("ttm gradient reduce"))) return rc;
      if (k + 1 < d) {
        const Step s = forward_step(D, cores, dtype, B, k, T, buf[k & 1]);
        if ((rc = launch_step(s, dtype, 0, st))) return rc;
        T = s.out;
      }
    }
  }
  timer_after(st);
  return TT_OK;
}

// ---------------------------------------------------------------- dispatch

static int g_ttm_path = TTM_PATH_AUTO;

void ttm_set_path(int path) { g_ttm_path = path; }

// Flops of the core-by-core forward chain: step k contracts (j_k, r_k) and
// produces (i_k, r_{k+1}) for B prod m_<k prod n_>k rows.
long long ttm_chain_flops(const TTMDims &D, long long B) {
  long long f = 0;
  for (int k = 0; k < D.d; ++k)
    f += 2 * B * prod(D.m, 0, k) * prod(D.n, k + 1, D.d) * D.n[k] * D.r[k] * D.m[k] * D.r[k + 1];
  return f;
}

int ttm_path_of(const TTMDims &D, long long B) {
  if (g_ttm_path == TTM_PATH_CHAIN) return TTM_PATH_CHAIN;
  if (!ttm_dense_fits(D)) return TTM_PATH_CHAIN;
  if (g_ttm_path == TTM_PATH_DENSE) return TTM_PATH_DENSE;
  return ttm_dense_flops(D, B) < ttm_chain_flops(D, B) ? TTM_PATH_DENSE : TTM_PATH_CHAIN;
}

size_t ttm_ws(const TTMDims &D, long long B, int dtype, int backward) {
  return ttm_path_of(D, B) == TTM_PATH_DENSE ? ttm_dense_ws(D, B, dtype, backward) : chain_ws(D, B, dtype, backward);
}

int ttm_forward(const TTMDims &D, const void *cores, const void *X, long long B, float *Y, int dtype, void *ws,
                size_t bytes, hipStream_t st) {
  if (ttm_path_of(D, B) == TTM_PATH_DENSE) return ttm_dense_forward(D, cores, X, B, Y, dtype, ws, bytes, st);
  return chain_forward(D, cores, X, B, Y, dtype, ws, bytes, st);
}

int ttm_backward(const TTMDims &D, const void *cores, const void *X, long long B, const void *dY, float *dX,
                 float *dW, int dtype, void *ws, size_t bytes, hipStream_t st) {
  if (ttm_path_of(D, B) == TTM_PATH_DENSE) return ttm_dense_backward(D, cores, X, B, dY, dX, dW, dtype, ws, bytes, st);
  return chain_backward(D, cores, X, B, dY, dX, dW, dtype, ws, bytes, st);
}

}  // namespace ttgfx
