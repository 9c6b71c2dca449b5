// Slice-grouped MFMA kernels for the gather, its adjoint and the fused MSE
// pass (bond ranks <= 32).
//
// The entry formula of the TT format (Introduction) multiplies, for every
// observed entry, one core slice per mode.  A tile of T entries is sorted
// by the slice index of each mode (a stable counting sort in LDS); entries
// that use the same slice are packed into 16-entry blocks, so that one mode
// step of a block is a dense product  (R x R slice) x (R x 16 entries)
// evaluated with v_mfma_f32_16x16x4_f32.  Ranks are zero-padded to R.
//
// Right sweep (modes d..1):  rho_k = G^k[i_k] rho_{k+1},  rho_{d+1} = e_0,
// so rho_1 = y (the gather).  Left sweep (modes 1..d):
// lambda_{k+1}^T = G^k[i_k]^T lambda_k^T with lambda_1 = e_0; at every mode
// the adjoint adds  sum_e w_e lambda_k,e (x) rho_{k+1},e  into slice i_k,
// which for one block is again an MFMA product with K = entries.  Right
// partials are stashed (in MFMA operand layout) in a per-workgroup global
// buffer between the sweeps; left partials are recomputed by the left sweep.
//
// Suffix table: entries that share their last l indices share rho_{d-l+1}
// (1-based).  When the entries outnumber the distinct suffixes, the rho of
// every suffix of length l = 1..depth is computed once per call (beside the
// padded slices) into a small table that stays in L2; the right sweep then
// starts `depth` modes later from the table, and the left sweep reads those
// modes' rho from the table instead of the stash.
//
// Each sweep runs a software pipeline over a wave's blocks: entry ids two
// blocks ahead, entry rows one block ahead, slices and stash two blocks
// ahead, with scheduling barriers so that the loads overlap the products.
//
// Layouts for a block of 16 entries (lane l, q = l / 16, c = l % 16):
//   EL (entry on lane):     lane l holds components 16t + 4q + v of entry c
//   CL (component on lane): lane l holds component 16t + c of entries 4q + v
// for comp-tile t < R/16 and v < 4.  An MFMA with a slice as A operand maps
// EL to EL (the contraction index 4q + v of chunk v is consistent between
// operands); the adjoint's outer product takes both partials in CL.
//
// Outer products are summed in registers over each run of consecutive
// blocks with the same slice.  Two ways to combine runs:
//   SLAB   (rank class 16): the wave holding a slice's first block stores its
//          run into an LDS slab, continuation runs go to per-wave edge
//          buffers, and a fixed-order flush adds them (no LDS atomics);
//   MERGE  (rank class 32): the first-block wave stores its run into an LDS
//          slab as in SLAB; a wave's first run that continues the previous
//          wave's slice stays in registers and is added to the slab after
//          the sweep, in rounds ordered by the wave's distance from the
//          slice's first wave (no edge buffers, so the slab fits beside the
//          larger rows).  The slab then goes to a per-workgroup accumulator
//          reduced in a fixed order afterwards (no atomics; measured faster
//          than adding each run, or each slab, to one gradient with float
//          atomics: 1.11 ms against 1.34 and 3.0 ms for the d=10, rank-32
//          projection of 2^20 entries);
//   DIRECT (batched kernel): runs are added to a zeroed global gradient
//          with no-return float atomics (no LDS slab).
// The per-tile work is one device function shared by the single-tensor
// kernel (tiles in grid-stride order) and the batched persistent kernel
// (work items from an atomic queue).
#include <stdlib.h>

#include <type_traits>

#include "common.h"
#include "gather_mfma.h"

namespace ttgfx {

typedef float v4f __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int a16(int x) { return (x + 15) & ~15; }

// Global-memory views of pointers.  The batched kernel reads its instances'
// pointers from memory, where the compiler cannot tell their address space
// and would use flat instructions, which also count on the LDS counter:
// every LDS wait in the sweeps would then wait for the prefetched global
// loads and the stash stores too.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gmem(const T *q) {
  return (const __attribute__((address_space(1))) T *)q;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem_w(T *q) {
  return (__attribute__((address_space(1))) T *)q;
}
// No-return float atomic add to global memory.
__device__ __forceinline__ void global_add(float *q, float v) {
  (void)__builtin_amdgcn_global_atomic_fadd_f32(gmem_w(q), v);
}

enum { ACC_SLAB = 0, ACC_DIRECT = 1, ACC_MERGE = 2 };

// Byte offsets of the LDS regions of one tile (see mf_layout).
struct MfLayout {
  int rows, slab, edges, sflag, wsum, sid, rid, perm, bslc, nblk, total, nmax;
};

namespace {

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr uint16_t kNone = 0xFFFF;

// Workgroup barrier that waits for this wave's LDS operations only.  Inside
// the sweeps no wave reads global memory written by another wave (each lane
// reads back only its own stash entries), so outstanding global stores need
// not drain at every mode boundary.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

enum { MODE_GATHER = 0, MODE_ADJOINT = 1, MODE_MSE = 2 };

// LDS layout (bytes), in this order, sized for the tensor's d and mode sizes:
//   rows   float [T + 2][R + 4]  (row T: zeros, row T+1: write sink)
//   slab   float [nmax][R][R + 4]     (SLAB, MERGE: per-slice sums)
//   edges  float [waves][R][R + 4]    (SLAB: runs continuing the previous wave's slice)
//   sflag  int   [nmax + 16]          (SLAB, MERGE: slice has a stored run; per-wave
//                                      edge slice (SLAB) or merge round (MERGE))
//   wsum   float [T + 2]              (per-entry weight g_e; [T] = 0)
//   sid    int   [T + 2]              (suffix table of sd levels: id of the
//                                      entry's last sd indices; [T] = 0)
//   rid    uint16 [sum_{k=d-1-sd}^{d-2} (T + 16 n_k)]  (table row of each
//                                      slot of perm, modes read from the table)
//   perm   uint16 [sum_k (T + 16 n_k)]
//   bslc   uint8  [sum_k ((T + 16 n_k) / 16 + 1)]
//   nblk   int   [4][MF_MAX_D]         (blocks of mode k; first slot of mode k in
//                                      perm and in rid, first block in bslc)
__host__ __device__ inline MfLayout mf_layout(int R, int T, int NTHR, int ACC, int d, const int *n, int sd) {
  const int W = NTHR / 64;
  int nmax = 1, pcap = 0, bcap = 0, rcap = 0;
  for (int k = 0; k < d; ++k) {
    nmax = n[k] > nmax ? n[k] : nmax;
    pcap += T + 16 * n[k];
    bcap += (T + 16 * n[k]) / 16 + 1;
    if (k >= d - 1 - sd && k <= d - 2) rcap += T + 16 * n[k];
  }
  MfLayout L;
  int o = 0;
  L.rows = o;
  o += a16(4 * (T + 2) * (R + 4));
  L.slab = o;
  if (ACC != ACC_DIRECT) o += 4 * nmax * R * (R + 4);
  L.edges = o;
  if (ACC == ACC_SLAB) o += 4 * W * R * (R + 4);
  L.sflag = o;
  if (ACC != ACC_DIRECT) o += a16(4 * (nmax + 16));
  L.wsum = o;
  o += a16(4 * (T + 2));
  L.sid = o;
  if (sd > 0) o += a16(4 * (T + 2));
  L.rid = o;
  o += a16(2 * rcap);
  L.perm = o;
  o += a16(2 * pcap);
  L.bslc = o;
  o += a16(bcap + 16);
  L.nblk = o;
  o += 4 * 4 * MF_MAX_D;
  L.total = o + 64;
  L.nmax = nmax;
  return L;
}

// One tile of T entries starting at entry e0 (cnt of them valid): sort,
// right sweep, residual, left sweep.  `accg` is the workgroup accumulator
// (SLAB), `loss_part` collects this thread's squared residuals (MSE).
// SUF: the suffix table may be in use (p.suf_depth levels).
template <int R, int T, int NTHR, int MODE, int ACC, bool SUF>
__device__ void run_tile(const MfInst &p, long long e0, int cnt_valid, char *smem, float *stash, int nb_max,
                         float *accg, bool first_tile, float &loss_part) {
  constexpr int NT = R / 16;      // comp tiles
  constexpr int W = NTHR / 64;    // waves
  constexpr int RS = R + 4;       // LDS row stride (padding spreads banks)
  constexpr int SS = R + 4;       // slab/edge row stride (conflict-free D stores)
  constexpr int ZROW = T;         // LDS row of zeros (padding entries read it)
  constexpr int SROW = T + 1;     // LDS row that absorbs padding writes
  const int SD = SUF ? p.suf_depth : 0;  // right partials of the last SD modes come from the suffix table
  const MfLayout L = mf_layout(R, T, NTHR, ACC, p.d, p.n, SD);
  float *rows = (float *)(smem + L.rows);
  float *slab = (float *)(smem + L.slab);
  float *edges = (float *)(smem + L.edges);
  int *sflag = (int *)(smem + L.sflag);
  int *eslice = sflag + L.nmax;
  float *wsum = (float *)(smem + L.wsum);
  int *sidv = (int *)(smem + L.sid);
  uint16_t *ridv = (uint16_t *)(smem + L.rid);
  uint16_t *perm = (uint16_t *)(smem + L.perm);
  uint8_t *bslc = (uint8_t *)(smem + L.bslc);
  int *nblk = (int *)(smem + L.nblk);
  int *pofs = nblk + MF_MAX_D;      // perm slots of mode k start at pofs[k] (multiple of 16)
  int *rofs = nblk + 2 * MF_MAX_D;  // rid slots of mode k (modes read from the table)
  int *bofs = nblk + 3 * MF_MAX_D;  // bslc entries of mode k
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c16 = lane & 15;
  const int q4 = lane >> 4;
  const int d = p.d;
  const long long M = p.M;
  const int kstart = d - 1 - SD;    // first mode the right sweep computes
  (void)slab;
  (void)edges;
  (void)sflag;
  (void)eslice;
  (void)accg;
  (void)first_tile;

  if (wave == 0) {
    // per-mode offsets of the slot arrays (lane k: sums over the modes before k)
    const int nj = (lane < d) ? p.n[lane] : 0;
    int ps = 0, bs = 0, rs = 0;
#pragma unroll
    for (int j = 0; j < MF_MAX_D; ++j) {
      const int cap = T + 16 * __builtin_amdgcn_readlane(nj, j);
      if (j < lane && j < d) {
        ps += cap;
        bs += cap / 16 + 1;
        if (j >= kstart) rs += cap;
      }
    }
    if (lane < MF_MAX_D) {
      pofs[lane] = ps;
      rofs[lane] = rs;
      bofs[lane] = bs;
    }
  }
  auto pbase = [&](int k) { return __builtin_amdgcn_readfirstlane(pofs[k]); };
  auto rbase = [&](int k) { return __builtin_amdgcn_readfirstlane(rofs[k]); };
  auto bbase = [&](int k) { return __builtin_amdgcn_readfirstlane(bofs[k]); };
  for (int c = tid; c < RS; c += NTHR) rows[ZROW * RS + c] = 0.f;
  if (tid == 0) {
    wsum[ZROW] = 0.f;
    if (SD > 0) sidv[ZROW] = 0;
  }

  // ---------------------------------------------------------------- sort
  // Stable counting sort of the tile's entries by slice index, every mode,
  // in three phases separated by barriers (scratch in the rows area, which
  // is free until the right sweep):
  //  1. wave w ranks the entries of its chunks (64 entries each) within the
  //     chunk by bit-plane ballots and records, per chunk, how many entries
  //     use each slice;
  //  2. one wave per mode turns the counts into offsets (groups padded to
  //     multiples of 16 entries; padding entries point at the zero row,
  //     so the sweeps read zeros for them without a test) and fills the
  //     block -> slice table;
  //  3. every entry is written to its place.
  // The order inside a slice group is the entry order, as before.
  {
    constexpr int CHUNKS = T / 64;
    constexpr int CPW = (CHUNKS + W - 1) / W;             // chunks per wave (wave + W i)
    constexpr int NSL = MfTraits<R>::MAX_N;               // slice values per count row
    constexpr int NBITS = NSL <= 16 ? 4 : 5;
    static_assert(sizeof(int) * MF_MAX_D * CHUNKS * NSL + 2 * MF_MAX_D * T <= sizeof(float) * T * RS,
                  "sort scratch must fit the rows area");
    int *cnt = (int *)rows;                                         // [d][CHUNKS][NSL]
    uint16_t *key = (uint16_t *)(cnt + MF_MAX_D * CHUNKS * NSL);    // [d][T]: rank << 8 | slice
    const unsigned long long below = (1ull << lane) - 1ull;
    // all index loads of the tile are issued before the first one is used
    int iv[MF_MAX_D][CPW];
#pragma unroll
    for (int k = 0; k < MF_MAX_D; ++k)
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int e = 64 * (wave + W * c) + lane;
        iv[k][c] = (k < d && wave + W * c < CHUNKS && e < cnt_valid) ? gmem(p.idx)[(long long)k * M + e0 + e] : -1;
      }
    // C-ordered id of the entry's last SD indices (suffix table; an
    // out-of-range index counts as 0, so table reads stay in bounds, and
    // such entries are dropped from that mode's blocks)
    int sfx[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) sfx[c] = 0;
#pragma unroll
    for (int k = 0; k < MF_MAX_D; ++k) {
      if (k >= d) break;
      const int nk = p.n[k];
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int ch = wave + W * c;
        if (ch >= CHUNKS) break;
        const int v = iv[k][c];
        const bool ok = v >= 0 && v < nk;  // out-of-range indices are dropped
        if (k >= d - SD) sfx[c] = sfx[c] * nk + (ok ? v : 0);
        // m: lanes of this chunk whose entry uses the same slice
        unsigned long long m = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < NBITS; ++bit) {
          const unsigned long long bb = __ballot(ok && ((v >> bit) & 1));
          m &= ((v >> bit) & 1) ? bb : ~bb;
        }
        const int rk = __popcll(m & below);
        key[k * T + 64 * ch + lane] = ok ? (uint16_t)((rk << 8) | v) : kNone;
        // the count row of a chunk belongs to one wave: zero it, then the
        // last lane of each slice value writes that value's count
        int *crow = cnt + (k * CHUNKS + ch) * NSL;
        if (lane < NSL) crow[lane] = 0;
        if (ok && (m >> lane) == 1ull) crow[v] = rk + 1;
      }
    }
    if (SD > 0) {
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int ch = wave + W * c;
        if (ch >= CHUNKS) break;
        sidv[64 * ch + lane] = sfx[c];
      }
    }
    lds_barrier();
    for (int k = wave; k < d; k += W) {
      const int nk = p.n[k];
      int c[CHUNKS];
      int run = 0;
#pragma unroll
      for (int ch = 0; ch < CHUNKS; ++ch) {
        c[ch] = (lane < nk) ? cnt[(k * CHUNKS + ch) * NSL + lane] : 0;
        run += c[ch];
      }
      const int padded = (lane < nk) ? ((run + 15) & ~15) : 0;
      // inclusive prefix sum over the NSL slice lanes: row shifts inside
      // 16-lane DPP rows (shifted-in lanes read zero), then, for 32 slices,
      // lane 15 of row 0 broadcast into row 1
      int incl = padded;
      incl += __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xF, 0xF, true);  // row_shr:1
      incl += __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xF, 0xF, true);  // row_shr:2
      incl += __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xF, 0xF, true);  // row_shr:4
      incl += __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xF, 0xF, true);  // row_shr:8
      if constexpr (NSL > 16) {
        static_assert(NSL <= 32, "slice counts must fit two DPP rows");
        incl += __builtin_amdgcn_update_dpp(0, incl, 0x142, 0xA, 0xF, false);  // row_bcast:15
      }
      const int total = __builtin_amdgcn_readlane(incl, NSL - 1);
      const int base = incl - padded;
      if (lane < nk) {
        int o = base;
#pragma unroll
        for (int ch = 0; ch < CHUNKS; ++ch) {
          cnt[(k * CHUNKS + ch) * NSL + lane] = o;
          o += c[ch];
        }
        uint16_t *pk = perm + pbase(k);
        for (int j = run; j < padded; ++j) pk[base + j] = (uint16_t)ZROW;
        if (k >= kstart && k < d - 1) {
          uint16_t *rk = ridv + rbase(k);
          for (int j = run; j < padded; ++j) rk[base + j] = 0;
        }
        uint8_t *bk = bslc + bbase(k) + base / 16;
        for (int j = 0; j < padded / 16; ++j) bk[j] = (uint8_t)lane;
      }
      if (lane == 0) nblk[k] = total / 16;
    }
    lds_barrier();
    for (int k = 0; k < d; ++k) {
      uint16_t *pk = perm + pbase(k);
      // modes whose right partial comes from the table also get, per slot,
      // the entry's row in table level d-1-k (its suffix id reduced to the
      // last d-1-k indices)
      const bool tab = k >= kstart && k < d - 1;
      uint16_t *rk = ridv + (tab ? rbase(k) : 0);
      const unsigned nrow = tab ? (unsigned)p.suf_rows[d - 2 - k] : 1u;
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int ch = wave + W * c;
        if (ch >= CHUNKS) break;
        const int kv = key[k * T + 64 * ch + lane];
        if (kv != kNone) {
          const int pos = cnt[(k * CHUNKS + ch) * NSL + (kv & 255)] + (kv >> 8);
          pk[pos] = (uint16_t)(64 * ch + lane);
          if (tab) rk[pos] = (uint16_t)((unsigned)sfx[c] % nrow);
        }
      }
    }
  }
  lds_barrier();

  if (SD > 0) {
    // rho_{kstart+1} of every entry from the deepest table level
    const float *tab = p.suf + (long long)p.suf_row0[SD - 1] * R;
    for (int x = tid; x < cnt_valid * (R / 4); x += NTHR) {
      const int e = x / (R / 4), c4 = x - e * (R / 4);
      *(v4f *)(rows + e * RS + 4 * c4) = *gmem((const v4f *)(tab + (long long)sidv[e] * R + 4 * c4));
    }
    lds_barrier();
  }

  // --------------------------------------------------------- right sweep
  // Each wave walks its blocks of mode k.  Loop bounds and slice ids are
  // wave-uniform (scalar registers): no divergent branches.  Slices load
  // U blocks ahead into U register sets used in turn (the loop is unrolled
  // by U and its first group peeled).  Every global access inside
  // the loop is unconditional (loads past the wave's last block re-read
  // it), so the compiler's memory-counter waits are exact: a block waits
  // for its own slices, not for the stash stores of the blocks before it.
  // Padding columns read the zero row.
  for (int k = kstart; k >= 0; --k) {
    const int nb = __builtin_amdgcn_readfirstlane(nblk[k]);
    const int jb = (wave * nb) / W, je = ((wave + 1) * nb) / W;
    if (jb < je) {
      const uint16_t *pk = perm + pbase(k);
      const float *gk = p.gp_right + (long long)p.sbase[k] * R * R;
      const int mysl = (lane < je - jb) ? bslc[bbase(k) + jb + lane] : 0;  // slice of block jb + lane
      // mode kinds get their own loop bodies, free of runtime branches:
      // first step (k = d-1: input e_0, nothing to stash), middle steps, and
      // the last step (k = 0: writes y)
      auto sweep = [&](auto stash_tag, auto last_tag, auto end_tag) {
        constexpr bool ST = decltype(stash_tag)::value;
        constexpr bool last = decltype(last_tag)::value;
        constexpr bool END = decltype(end_tag)::value;
        // Software pipeline over the wave's blocks, two register sets per
        // stage: the block's entry ids (LDS) are read two blocks ahead, its
        // slice (global) and entry rows (LDS; EL layout for the product, CL
        // layout for the stash) one block ahead.
        // Blocks of one mode use disjoint entries, so a later block's rows
        // may be read before this block writes its own (padding columns
        // read and write the zero row, which stays zero).  Scheduling
        // barriers keep the loads of later blocks ahead of this block's
        // products, so their latency overlaps them.
        struct Idx {
          int ent;
          int jj;
          uint2 q;  // the block's 16 entries, 4 per lane in CL order (stash)
        };
        struct Dat {
          v4f a[NT * NT];
          v4f bv[NT];
          v4f cl[NT];
          int ent;
        };
        auto ld_idx = [&](int j, Idx &x) {
          const int jj = j < je ? j : je - 1;
          x.jj = jj;
          x.ent = pk[16 * jj + c16];
          if constexpr (ST) x.q = *(const uint2 *)(pk + 16 * jj + 4 * q4);
        };
        auto ld_dat = [&](const Idx &x, Dat &o) {
          {
            const float *gs = gk + (long long)__builtin_amdgcn_readlane(mysl, x.jj - jb) * R * R;
#pragma unroll
            for (int xx = 0; xx < NT * NT; ++xx) o.a[xx] = *gmem((const v4f *)(gs + (xx * 64 + lane) * 4));
          }
          o.ent = x.ent;
          if constexpr (!last) {
#pragma unroll
            for (int t = 0; t < NT; ++t) o.bv[t] = *(const v4f *)(rows + x.ent * RS + 16 * t + 4 * q4);
          }
          if constexpr (ST) {
            const int ev[4] = {(int)(x.q.x & 0xFFFF), (int)(x.q.x >> 16), (int)(x.q.y & 0xFFFF),
                               (int)(x.q.y >> 16)};
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
              for (int v = 0; v < 4; ++v) o.cl[t][v] = rows[ev[v] * RS + 16 * t + c16];
          }
        };
        auto compute = [&](int j, const Dat &o) {
          const int ent = o.ent;
          v4f bv[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            if (last)
              bv[t] = v4f{(t == 0 && q4 == 0) ? 1.f : 0.f, 0.f, 0.f, 0.f};
            else
              bv[t] = o.bv[t];
          }
          if constexpr (ST) {
            // stash rho_{k+1} of this block in CL layout
            float *st = stash + ((long long)k * nb_max + j) * (64 * R / 4);
#pragma unroll
            for (int t = 0; t < NT; ++t) *gmem_w((v4f *)(st + (t * 64 + lane) * 4)) = o.cl[t];
          }
          v4f out[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) out[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
              for (int to = 0; to < NT; ++to) out[to] = mfma4(o.a[to * NT + ti][c], bv[ti][c], out[to]);
          if constexpr (!END) {
            // a padding column is zero (zero row in, zero out) except in the
            // first step, where the input is e_0: that one goes to the sink row
            const int w = (last && ent == ZROW) ? SROW : ent;
#pragma unroll
            for (int t = 0; t < NT; ++t) *(v4f *)(rows + w * RS + 16 * t + 4 * q4) = out[t];
          } else if (q4 == 0 && ent != ZROW) {
            wsum[ent] = out[0][0];  // component 0 of rho_1 = y
          }
        };
        Idx xi[2];
        Dat xd[2];
        ld_idx(jb, xi[0]);
        ld_idx(jb + 1, xi[1]);
        ld_dat(xi[0], xd[0]);
        // block j uses register set s = (j - jb) % 2; set s of the index
        // stage is free once block j's operands are loaded (the step before)
        auto step = [&](int j, auto slot) {
          constexpr int S = decltype(slot)::value, S1 = 1 - S;
          ld_idx(j + 2, xi[S]);
          ld_dat(xi[S1], xd[S1]);
          __builtin_amdgcn_sched_barrier(0);
          compute(j, xd[S]);
          __builtin_amdgcn_sched_barrier(0);
        };
        // whole pairs in the loop and an odd last block after it: no exit
        // between the two steps of a pair, so the memory-counter waits at
        // the loop head see the same outstanding loads on every path
        int j = jb;
        for (; j + 1 < je; j += 2) {
          step(j, std::integral_constant<int, 0>{});
          step(j + 1, std::integral_constant<int, 1>{});
        }
        if (j < je) step(j, std::integral_constant<int, 0>{});
      };
      using T1 = std::true_type;
      using F0 = std::false_type;
      constexpr bool STASH = MODE != MODE_GATHER;
      // the first computed step stashes nothing: its input is e_0 (no
      // table; d >= 2, so this step is never the last) or rho_{kstart+1}
      // from the table, which the left sweep reads there too
      if (k == d - 1)
        sweep(F0{}, T1{}, F0{});
      else if (SUF && k == kstart)
        k > 0 ? sweep(F0{}, F0{}, F0{}) : sweep(F0{}, F0{}, T1{});
      else if (k > 0)
        sweep(std::bool_constant<STASH>{}, F0{}, F0{});
      else
        sweep(std::bool_constant<STASH>{}, F0{}, T1{});
    }
    lds_barrier();
  }

  // ------------------------------------------------------------ residual
  for (int e = tid; e < cnt_valid; e += NTHR) {
    const float yv = wsum[e];
    if (p.y) gmem_w(p.y)[e0 + e] = yv;
    float w = 0.f;
    if (MODE == MODE_MSE) {
      const float rho = yv - gmem(p.t)[e0 + e];
      w = p.inv_m2 * rho;
      loss_part += rho * rho;
      if (p.gout) gmem_w(p.gout)[e0 + e] = w;
    } else if (MODE == MODE_ADJOINT) {
      w = gmem(p.gy)[e0 + e];
    }
    wsum[e] = w;
  }
  if (MODE == MODE_GATHER) {
    lds_barrier();
    return;
  }
  // lambda_1 = w_e e_0 for every entry: the left chain is linear in
  // lambda_1, so every lambda_k carries the entry's weight and the outer
  // products need no extra scaling (the zero row stays zero; the thread
  // that wrote wsum[e] above reads it here)
  for (int e = tid; e < T; e += NTHR) {
    const float w0 = (e < cnt_valid) ? wsum[e] : 0.f;
#pragma unroll
    for (int c = 0; c < R; ++c) rows[e * RS + c] = (c == 0) ? w0 : 0.f;
  }
  lds_barrier();

  // ---------------------------------------------------------- left sweep
  // Outer products are summed in registers over each run of consecutive
  // blocks with the same slice.  The wave that holds the first block of a
  // slice stores its run into slab[s]; a wave whose first run continues a
  // slice of the previous wave stores that run into its edge buffer.  The
  // flush adds slab and edges in a fixed order: no atomics, deterministic.
  // The accumulator values of the flush load at mode start.
  constexpr int FLN = (ACC == ACC_SLAB) ? (MfTraits<R>::MAX_N * R * R / 4 + NTHR - 1) / NTHR : 1;
  for (int k = 0; k < d; ++k) {
    const int nk = p.n[k];
    if constexpr (ACC != ACC_DIRECT) {
      for (int e = tid; e < nk; e += NTHR) sflag[e] = 0;
      if (lane == 0) eslice[wave] = -1;
      lds_barrier();
    }
    const int nb = __builtin_amdgcn_readfirstlane(nblk[k]);
    const int jb = (wave * nb) / W, je = ((wave + 1) * nb) / W;
    const uint16_t *pk = perm + pbase(k);
    const uint8_t *bk = bslc + bbase(k);
    const int mysl = (lane < je - jb) ? bk[jb + lane] : 0;  // slice of block jb + lane
    const int prev_sl = __builtin_amdgcn_readfirstlane(jb > 0 ? (int)bk[jb - 1] : -1);
    const bool cont_first = (jb < je) && prev_sl == __builtin_amdgcn_readfirstlane(mysl);
    float *ak = (ACC == ACC_SLAB) ? accg + (long long)p.sbase[k] * R * R : nullptr;
    v4f accp[FLN];
    if constexpr (ACC == ACC_SLAB) {
#pragma unroll
      for (int i = 0; i < FLN; ++i) {
        const int e4 = tid + i * NTHR;
        accp[i] = (!first_tile && e4 < nk * R * R / 4) ? *(const v4f *)(ak + 4 * e4) : v4f{0.f, 0.f, 0.f, 0.f};
      }
    }
    bool first_run = true;
    int rsid = -1;
    v4f racc[NT * NT];
    v4f cacc[ACC == ACC_MERGE ? NT * NT : 1];  // MERGE: the run continuing the previous wave's slice
    bool has_cont = false;
    // a finished run: SLAB stores it (owner slab or edge buffer), MERGE
    // stores owner runs and keeps a continuation in registers, DIRECT adds it
    // to the gradient target with no-return float atomics
    auto emit_run = [&](int s, bool edge) {
      if constexpr (ACC == ACC_MERGE) {
        if (edge) {
#pragma unroll
          for (int x = 0; x < NT * NT; ++x) cacc[x] = racc[x];
          has_cont = true;
        } else {
          float *dst = slab + s * R * SS;
          if (lane == 0) sflag[s] = 1;
#pragma unroll
          for (int ta = 0; ta < NT; ++ta)
#pragma unroll
            for (int tb = 0; tb < NT; ++tb)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                dst[(16 * ta + 4 * q4 + v) * SS + 16 * tb + c16] = racc[ta * NT + tb][v];
        }
      } else if constexpr (ACC == ACC_SLAB) {
        float *dst = edge ? edges + wave * R * SS : slab + s * R * SS;
        if (lane == 0) {
          if (edge) eslice[wave] = s;
          else sflag[s] = 1;
        }
#pragma unroll
        for (int ta = 0; ta < NT; ++ta)
#pragma unroll
          for (int tb = 0; tb < NT; ++tb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              dst[(16 * ta + 4 * q4 + v) * SS + 16 * tb + c16] = racc[ta * NT + tb][v];
      } else {
        float *dst = p.grad + (long long)(p.sbase[k] + s) * R * R;
#pragma unroll
        for (int ta = 0; ta < NT; ++ta)
#pragma unroll
          for (int tb = 0; tb < NT; ++tb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              global_add(dst + (16 * ta + 4 * q4 + v) * R + 16 * tb + c16, racc[ta * NT + tb][v]);
      }
    };
    // Two kinds of mode get their own loop bodies, free of runtime branches:
    // k < d-1 (chain step; rho_{k+1} from the stash or the suffix table) and
    // k = d-1 (no chain step, rho_{d+1} = e_0, no global loads).  The same
    // software pipeline as the right sweep: entry ids (and table row ids)
    // two blocks ahead; the block's lambda rows (CL layout for the outer
    // product, EL layout for the chain) and rho_{k+1} (stash or table) one
    // block ahead; slice G^k^T two blocks ahead.  (Loads consumed one step
    // after issue keep the compiler's memory-counter waits exact.)
    auto sweep = [&](auto chain_tag, auto table_tag) {
      constexpr bool CHAIN = decltype(chain_tag)::value;
      constexpr bool TAB = decltype(table_tag)::value;
      struct Idx {
        uint2 q;    // the block's 16 entries, 4 per lane in CL order
        uint2 rid;  // their rows in the table level (TAB)
        int ent;    // this lane's entry in EL order (CHAIN)
        int jj;
      };
      struct Dat {
        v4f lcl[NT];
        v4f bv[NT];
        v4f rt[NT];  // rho_{k+1} (stash or table), CL layout
        int ent;
      };
      struct Glb {
        v4f a[NT * NT];
      };
      const int lev = d - 1 - k;  // table level of rho_{k+1} (TAB)
      const uint16_t *rk = TAB ? ridv + rbase(k) : nullptr;
      const float *tab = TAB ? p.suf + (long long)p.suf_row0[lev - 1] * R : nullptr;
      auto ld_idx = [&](int j, Idx &x) {
        const int jj = j < je ? j : je - 1;
        x.jj = jj;
        x.q = *(const uint2 *)(pk + 16 * jj + 4 * q4);
        if constexpr (CHAIN) x.ent = pk[16 * jj + c16];
        if constexpr (TAB) x.rid = *(const uint2 *)(rk + 16 * jj + 4 * q4);
      };
      auto ld_dat = [&](const Idx &x, Dat &o) {
        if constexpr (CHAIN && !TAB) {
          const int jj = x.jj;
          const float *st = stash + ((long long)k * nb_max + jj) * (64 * R / 4);
#pragma unroll
          for (int t = 0; t < NT; ++t) o.rt[t] = *gmem((const v4f *)(st + (t * 64 + lane) * 4));
        }
        const int ev[4] = {(int)(x.q.x & 0xFFFF), (int)(x.q.x >> 16), (int)(x.q.y & 0xFFFF), (int)(x.q.y >> 16)};
        // lambda_k (weighted): CL (A operand of the outer product) and EL (chain)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int t = 0; t < NT; ++t) o.lcl[t][v] = rows[ev[v] * RS + 16 * t + c16];
        if constexpr (CHAIN) {
          o.ent = x.ent;
#pragma unroll
          for (int t = 0; t < NT; ++t) o.bv[t] = *(const v4f *)(rows + x.ent * RS + 16 * t + 4 * q4);
        }
        if constexpr (TAB) {
          // padding slots read row 0: their lambda is zero
          const int rv[4] = {(int)(x.rid.x & 0xFFFF), (int)(x.rid.x >> 16), (int)(x.rid.y & 0xFFFF),
                             (int)(x.rid.y >> 16)};
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int t = 0; t < NT; ++t) o.rt[t][v] = gmem(tab)[(long long)rv[v] * R + 16 * t + c16];
        }
      };
      auto ld_glob = [&](int j, Glb &g) {
        if constexpr (CHAIN) {
          const int jj = j < je ? j : je - 1;
          const float *gs = p.gp_left + ((long long)p.sbase[k] + __builtin_amdgcn_readlane(mysl, jj - jb)) * R * R;
#pragma unroll
          for (int x = 0; x < NT * NT; ++x) g.a[x] = *gmem((const v4f *)(gs + (x * 64 + lane) * 4));
        }
      };
      auto compute = [&](int j, const Dat &o, const Glb &g) {
        const int sid = __builtin_amdgcn_readlane(mysl, j - jb);
        v4f rcl[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          if constexpr (!CHAIN) {
            const float one = (t == 0 && c16 == 0) ? 1.f : 0.f;
            rcl[t] = v4f{one, one, one, one};  // rho_{d+1} = e_0
          } else {
            rcl[t] = o.rt[t];
          }
        }
        // outer products (NT * NT independent chains)
        v4f dg[NT * NT];
#pragma unroll
        for (int x = 0; x < NT * NT; ++x) dg[x] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int ta = 0; ta < NT; ++ta)
#pragma unroll
            for (int tb = 0; tb < NT; ++tb) dg[ta * NT + tb] = mfma4(o.lcl[ta][c], rcl[tb][c], dg[ta * NT + tb]);
        // chain lambda_{k+1}^T = G^T lambda_k^T
        if constexpr (CHAIN) {
          v4f out[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) out[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
              for (int to = 0; to < NT; ++to) out[to] = mfma4(g.a[to * NT + ti][c], o.bv[ti][c], out[to]);
          // a padding column reads the zero row and writes zeros back to it
#pragma unroll
          for (int t = 0; t < NT; ++t) *(v4f *)(rows + o.ent * RS + 16 * t + 4 * q4) = out[t];
        }
        // merge the block's outer products into runs
        if (sid != rsid) {
          if (rsid >= 0) {
            emit_run(rsid, first_run && cont_first);
            first_run = false;
          }
          rsid = sid;
#pragma unroll
          for (int x = 0; x < NT * NT; ++x) racc[x] = dg[x];
        } else {
#pragma unroll
          for (int x = 0; x < NT * NT; ++x) racc[x] += dg[x];
        }
      };
      Idx xi[2];
      Dat xd[2];
      Glb xg[2];
      ld_idx(jb, xi[0]);
      ld_idx(jb + 1, xi[1]);
      ld_glob(jb, xg[0]);
      ld_glob(jb + 1, xg[1]);
      ld_dat(xi[0], xd[0]);
      auto step = [&](int j, auto slot) {
        constexpr int S = decltype(slot)::value, S1 = 1 - S;
        ld_idx(j + 2, xi[S]);
        ld_dat(xi[S1], xd[S1]);
        __builtin_amdgcn_sched_barrier(0);
        compute(j, xd[S], xg[S]);
        __builtin_amdgcn_sched_barrier(0);
        ld_glob(j + 2, xg[S]);
      };
      int j = jb;  // whole pairs, then an odd last block (as in the right sweep)
      for (; j + 1 < je; j += 2) {
        step(j, std::integral_constant<int, 0>{});
        step(j + 1, std::integral_constant<int, 1>{});
      }
      if (j < je) step(j, std::integral_constant<int, 0>{});
    };
    if (jb < je) {
      if (k < d - 1) {
        if (SUF && k >= kstart)
          sweep(std::true_type{}, std::bool_constant<SUF>{});
        else
          sweep(std::true_type{}, std::false_type{});
      } else {
        sweep(std::false_type{}, std::false_type{});
      }
    }
    if (rsid >= 0) emit_run(rsid, first_run && cont_first);
    if constexpr (ACC == ACC_MERGE) {
      // merge round of this wave: 0 without a continuation run, else 1 +
      // the number of waves before it (with blocks) that lie inside the same
      // slice and continue it too; round t adds the runs of round t in
      // place, so every slice sums its runs in wave order
      int pos = 0;
      if (has_cont) {
        const int f = __builtin_amdgcn_readfirstlane(mysl);
        pos = 1;
        for (int w2 = wave - 1; w2 >= 0; --w2) {
          const int b0 = (w2 * nb) / W, b1 = ((w2 + 1) * nb) / W;
          if (b0 == b1) continue;                       // no blocks
          if (b0 > 0 && bk[b0] == f && bk[b0 - 1] == f) ++pos;  // inside f, continuing it
          else break;
        }
      }
      if (lane == 0) eslice[wave] = pos;
      lds_barrier();
      int rounds = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) rounds = max(rounds, eslice[w]);
      rounds = __builtin_amdgcn_readfirstlane(rounds);
      for (int t = 1; t <= rounds; ++t) {
        if (pos == t) {
          float *dst = slab + __builtin_amdgcn_readfirstlane(mysl) * R * SS;
#pragma unroll
          for (int ta = 0; ta < NT; ++ta)
#pragma unroll
            for (int tb = 0; tb < NT; ++tb)
#pragma unroll
              for (int v = 0; v < 4; ++v) dst[(16 * ta + 4 * q4 + v) * SS + 16 * tb + c16] += cacc[ta * NT + tb][v];
        }
        lds_barrier();
      }
      // flush into the workgroup's accumulator: a plain store on the first
      // tile, an add after (each thread owns the same elements on every
      // tile; slices without runs add zero)
      float *akm = accg + (long long)p.sbase[k] * R * R;
      for (int e4 = tid; e4 < nk * R * R / 4; e4 += NTHR) {
        const int e = 4 * e4;
        const int sl = e / (R * R), a = (e / R) % R, b = e % R;
        v4f v = sflag[sl] ? *(const v4f *)(slab + sl * R * SS + a * SS + b) : v4f{0.f, 0.f, 0.f, 0.f};
        if (!first_tile) v += *(const v4f *)(akm + e);
        *(v4f *)(akm + e) = v;
      }
      lds_barrier();
    } else {
      lds_barrier();
    }
    if constexpr (ACC == ACC_SLAB) {
      // flush this mode into the workgroup's accumulator: a plain store on
      // the first tile, an add to the values loaded at mode start after
      // (4 floats per thread and step; edge owners read once).  The same
      // thread owns the same accumulator elements on every tile, so no
      // synchronisation is needed, and no atomics sit in the in-order
      // memory counter that later loads of this wave wait on.
      int es[W];
#pragma unroll
      for (int w = 0; w < W; ++w) es[w] = eslice[w];
#pragma unroll
      for (int i = 0; i < FLN; ++i) {
        const int e4 = tid + i * NTHR;
        if (e4 >= nk * R * R / 4) break;
        const int e = 4 * e4;
        const int sl = e / (R * R), a = (e / R) % R, b = e % R;
        v4f v = accp[i];
        if (sflag[sl]) {
          v += *(const v4f *)(slab + sl * R * SS + a * SS + b);
#pragma unroll
          for (int w = 0; w < W; ++w)
            if (es[w] == sl) v += *(const v4f *)(edges + w * R * SS + a * SS + b);
        }
        *(v4f *)(ak + e) = v;
      }
      lds_barrier();
    }
  }
}

// Single tensor: tiles in grid-stride order over the entries.
struct Grid {
  int ntiles;
  int nb_max;
  float *stash;            // per workgroup: [d-1][nb_max][64 lanes][R/4]
  long long stash_stride;  // floats per workgroup
  float *acc;              // SLAB: per workgroup [total slices][R*R]
  long long acc_stride;
  float *loss_acc;         // per workgroup squared-residual sums
};

template <int R, int T, int NTHR, int MODE, int ACC>
__global__ void __launch_bounds__(NTHR) fused_kernel(MfInst p, Grid g) {
  extern __shared__ __align__(16) char smem[];
  float *stash = g.stash + (long long)blockIdx.x * g.stash_stride;
  float *accg = g.acc ? g.acc + (long long)blockIdx.x * g.acc_stride : nullptr;
  float loss_part = 0.f;
  bool first = true;
  for (int tile = blockIdx.x; tile < g.ntiles; tile += gridDim.x) {
    const long long e0 = (long long)tile * T;
    const int cnt = (int)((p.M - e0) < T ? (p.M - e0) : T);
    run_tile<R, T, NTHR, MODE, ACC, true>(p, e0, cnt, smem, stash, g.nb_max, accg, first, loss_part);
    first = false;
  }
  if (MODE == MODE_MSE) {
    // deterministic block reduction of the squared residuals
    float *red = (float *)smem;
    for (int off = 32; off > 0; off >>= 1) loss_part += __shfl_xor(loss_part, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = loss_part;
    __syncthreads();
    if (threadIdx.x == 0) {
      float v = 0.f;
      for (int w = 0; w < NTHR / 64; ++w) v += red[w];
      g.loss_acc[blockIdx.x] = v;
    }
  }
}

// Batched persistent kernel: workgroups take (tensor, first tile, tile
// count) items from an atomic counter (items are in decreasing-cost order)
// until the list is exhausted; both rank classes share the launch.  Per
// tensor: gradients accumulate into its zeroed padded buffer (DIRECT), the
// loss into loss[b] (mean over that tensor's entries).  T16 and T32 are the
// entries per tile of the two rank classes, NTHR the threads per workgroup
// (the tile shape the plan's autotuner chooses).
template <int T16, int T32, int NTHR>
__global__ void __launch_bounds__(NTHR) batched_kernel(MfBatchArgs a) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int item_sh;
  __shared__ float red[NTHR / 64];
  float *stash = a.stash + (long long)blockIdx.x * a.stash_stride;
  for (;;) {
    if (threadIdx.x == 0) item_sh = atomicAdd(a.counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(item_sh);
    __syncthreads();
    if (it >= a.nitems) break;
    const MfWorkItem w = a.items[it];
    const MfInst &p = a.table[w.inst];
    for (int t = 0; t < w.ntile; ++t) {
      float lp = 0.f;
      if (w.rclass == 16) {
        const long long e0 = (long long)(w.tile0 + t) * T16;
        const int cnt = (int)((p.M - e0) < T16 ? (p.M - e0) : T16);
        run_tile<16, T16, NTHR, MODE_MSE, ACC_DIRECT, false>(p, e0, cnt, smem, stash, a.nb16, nullptr, false, lp);
      } else {
        const long long e0 = (long long)(w.tile0 + t) * T32;
        const int cnt = (int)((p.M - e0) < T32 ? (p.M - e0) : T32);
        run_tile<32, T32, NTHR, MODE_MSE, ACC_DIRECT, false>(p, e0, cnt, smem, stash, a.nb32, nullptr, false, lp);
      }
      // this tile's share of the tensor's mean squared residual
      for (int off = 32; off > 0; off >>= 1) lp += __shfl_xor(lp, off);
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lp;
      __syncthreads();
      if (threadIdx.x == 0) {
        float s = 0.f;
        for (int wv = 0; wv < NTHR / 64; ++wv) s += red[wv];
        global_add(p.loss, s * p.inv_m);
      }
      __syncthreads();
    }
  }
}

// Suffix table build: the right partial rho_{d-l} = G^{d-l}[i_{d-l}] ..
// G^{d-1}[i_{d-1}] e_0 of every value of the last l indices, l = 1..depth.
// A group of R lanes computes one suffix of length `depth` (lane a holds
// component a), one mode at a time, and writes level l's row when the
// suffix's leading depth-l indices are zero, so every row is written once.
struct SufBuild {
  float *tab;
  int depth;
  int row0[MF_MAX_D];
  int rows[MF_MAX_D];
  int blocks;  // workgroups of the build (after the slice workgroups)
};

template <int R>
__device__ void build_suffix_rows(const TTDev &X, const SufBuild &sb, int blk) {
  const int lane = threadIdx.x & 63;
  const int grp = lane / R, a = lane - grp * R;
  constexpr int groups = 64 / R;
  const long long sfx = ((long long)blk * (blockDim.x >> 6) + (threadIdx.x >> 6)) * groups + grp;
  const int D = sb.depth;
  const bool live = sfx < sb.rows[D - 1];
  int rem = live ? (int)sfx : 0;
  float rho = 0.f;
  if constexpr (R <= 32) {
    // Up to four levels, with coalesced loads: lane b of the group holds
    // component b of rho and reads column b of the slice (rows a = 0..R-1 of
    // G[:, i, :], R consecutive floats per row across the group), forms the
    // products G[a][i][b] rho_b for every a, and a recursive-halving
    // exchange over the group sums them so that lane a ends with
    // sum_b G[a][i][b] rho_b.  Every level's loads are issued before the
    // first product.  Level 1 starts from rho = e_0 (r_d = 1).
    constexpr int DMAX = 4;
    if (D <= DMAX) {
      const int b = a;  // this lane's column
      float gv[DMAX][R];
#pragma unroll
      for (int l = 1; l <= DMAX; ++l) {
        if (l > D) break;
        const int k = X.d - l;
        const int nk = X.n[k], rk = X.r[k], rk1 = X.r[k + 1];
        const int i = rem % nk;
        rem /= nk;
        const float *G = X.data + X.off[k] + (long long)i * rk1 + b;  // G[0][i][b]
#pragma unroll
        for (int r = 0; r < R; ++r) gv[l - 1][r] = (r < rk && b < rk1) ? G[(long long)r * nk * rk1] : 0.f;
      }
      float x = (b == 0) ? 1.f : 0.f;  // rho_b
#pragma unroll
      for (int l = 1; l <= DMAX; ++l) {
        if (l > D) break;
        float pv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) pv[r] = gv[l - 1][r] * x;
#pragma unroll
        for (int h = R / 2; h >= 1; h >>= 1) {
          const bool upper = (b & h) != 0;  // keeps indices [h, 2h) of the live range
#pragma unroll
          for (int j = 0; j < h; ++j) {
            const float keep = upper ? pv[j + h] : pv[j];
            const float give = upper ? pv[j] : pv[j + h];
            pv[j] = keep + __shfl_xor(give, h);
          }
        }
        x = pv[0];  // component b of the new rho
        if (live && sfx < sb.rows[l - 1]) sb.tab[((long long)sb.row0[l - 1] + sfx) * R + b] = x;
      }
      return;
    }
  }
  for (int l = 1; l <= D; ++l) {
    const int k = X.d - l;
    const int nk = X.n[k], rk = X.r[k], rk1 = X.r[k + 1];
    const int i = rem % nk;
    rem /= nk;
    const float *G = X.data + X.off[k] + (long long)i * rk1 + (long long)a * nk * rk1;  // G[a][i][:]
    float acc = 0.f;
    if (l == 1) {
      if (a < rk) acc = G[0];  // column 0 (r_d = 1)
    } else {
      // the row of G and the partner values are read 16 at a time before
      // their sum, so the loads of a chunk are in flight together
#pragma unroll
      for (int b0 = 0; b0 < R; b0 += 16) {
        float gv[16], rv[16];
#pragma unroll
        for (int b = 0; b < 16; ++b) {
          gv[b] = (a < rk && b0 + b < rk1) ? G[b0 + b] : 0.f;
          rv[b] = __shfl(rho, grp * R + b0 + b);
        }
#pragma unroll
        for (int b = 0; b < 16; ++b) acc = fmaf(gv[b], rv[b], acc);
      }
    }
    rho = acc;
    if (live && sfx < sb.rows[l - 1]) sb.tab[((long long)sb.row0[l - 1] + sfx) * R + a] = rho;
  }
}

// Padded slice copies in MFMA A-operand order: for slice G (R x R, zero
// outside the true ranks) and comp tiles (to, ti), lane l's float4 holds
// M[16 to + l%16][16 ti + 4 (l/16) + c], c < 4, with M = G for the right
// sweep and M = G^T for the left sweep.  Workgroups past the slices build
// the suffix table of Xr.
__global__ void __launch_bounds__(256) pad_slices_kernel(TTDev Xr, TTDev Xl, int R, float *__restrict__ right,
                                                        float *__restrict__ left, int total_slices, SufBuild sb) {
  const int slice = blockIdx.x;
  if (slice >= total_slices) {
    if (sb.depth > 0 && slice - total_slices < sb.blocks) {
      if (R == 16) build_suffix_rows<16>(Xr, sb, slice - total_slices);
      else if (R == 32) build_suffix_rows<32>(Xr, sb, slice - total_slices);
      else build_suffix_rows<64>(Xr, sb, slice - total_slices);
    }
    return;
  }
  int k = 0, base = 0;
  while (k < Xr.d && slice >= base + Xr.n[k]) {
    base += Xr.n[k];
    ++k;
  }
  const int s = slice - base;
  const int NT = R / 16;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    const int c = e & 3, lane = (e >> 2) & 63, x = e >> 8;
    const int to = x / NT, ti = x % NT;
    const int row = 16 * to + (lane & 15), col = 16 * ti + 4 * (lane >> 4) + c;
    if (right) {
      float v = 0.f;  // G[row][col]
      if (row < Xr.r[k] && col < Xr.r[k + 1])
        v = Xr.data[Xr.off[k] + ((long long)row * Xr.n[k] + s) * Xr.r[k + 1] + col];
      right[(long long)slice * R * R + e] = v;
    }
    if (left) {
      float v = 0.f;  // G^T[row][col] = G[col][row]
      if (col < Xl.r[k] && row < Xl.r[k + 1])
        v = Xl.data[Xl.off[k] + ((long long)col * Xl.n[k] + s) * Xl.r[k + 1] + row];
      left[(long long)slice * R * R + e] = v;
    }
  }
}

// Stage 1 of the gradient reduction: tmp[g][e] = sum of acc[w][e] over the
// workgroups w of group g (32 per group), in increasing w.
__global__ void reduce_acc_stage1(const float *__restrict__ acc, long long acc_stride, int nwg,
                                  long long E, float *__restrict__ tmp) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int w0 = blockIdx.y * 32;
  const int w1 = (w0 + 32 < nwg) ? w0 + 32 : nwg;
  float v = 0.f;
  int w = w0;
  // eight loads in flight at a time; the additions keep workgroup order
  for (; w + 8 <= w1; w += 8) {
    float x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = acc[(long long)(w + u) * acc_stride + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += x[u];
  }
  for (; w < w1; ++w) v += acc[(long long)w * acc_stride + e];
  tmp[(long long)blockIdx.y * E + e] = v;
}

// Stage 2: out core k (a, s, b) = sum over groups (increasing) of the padded
// element (slice(k, s), a, b).  With loss set, the blocks of row d instead
// form loss = (fixed-order sum of the per-workgroup squared residuals) / M
// (one wave).
__global__ void reduce_acc_stage2(TTDev O, int R, const float *__restrict__ tmp, long long E,
                                  int ngroups, const float *__restrict__ lpart, int nwg, long long M,
                                  float *__restrict__ loss) {
  const int k = blockIdx.y;
  if (k == O.d) {
    if (!loss || blockIdx.x != 0 || threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    float v = 0.f;
    for (int w = lane; w < nwg; w += 64) v += lpart[w];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) *loss = (M > 0) ? v / (float)M : 0.f;
    return;
  }
  if (k > O.d) return;
  int sbase = 0;
  for (int j = 0; j < k; ++j) sbase += O.n[j];
  const int rk = O.r[k], nk = O.n[k], rk1 = O.r[k + 1];
  const long long total = (long long)rk * nk * rk1;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(e % rk1);
    const int s = (int)((e / rk1) % nk);
    const int a = (int)(e / ((long long)rk1 * nk));
    const long long src = ((long long)(sbase + s) * R + a) * R + b;
    float v = 0.f;
    for (int g = 0; g < ngroups; ++g) v += tmp[(long long)g * E + src];
    O.data[O.off[k] + e] = v;
  }
}

// One wave: loss = (fixed-order sum of the per-workgroup squared residuals) / M.
__global__ void reduce_loss_kernel(const float *__restrict__ part, int nwg, long long M,
                                   float *__restrict__ loss) {
  const int lane = threadIdx.x;
  float v = 0.f;
  for (int w = lane; w < nwg; w += 64) v += part[w];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (lane == 0) *loss = (M > 0) ? v / (float)M : 0.f;
}

int device_cus() {
  static int cached = -1;
  if (cached > 0) return cached;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  cached = cus;
  return cus;
}


// Tile shapes of the single-tensor kernels (entries per tile, threads per
// workgroup), two per rank class; shape 0 is the default.  At rank class 16
// the larger tile pads fewer entries (slice groups round up to 16 entries)
// while the smaller one keeps a tile's LDS under half of a CU's 160 KiB, so
// two workgroups share a CU.  Measured at d=10, n=10, r=16, 2^20 entries:
// 0.34 ms and 0.50 ms; at rank class 32 (projection, d=10, rank 32):
// 1.41 ms and 2.10 ms.
struct TileShape {
  int T, threads;
};
constexpr TileShape kShapes16[2] = {{1024, 768}, {512, 512}};
constexpr TileShape kShapes32[2] = {{512, 512}, {256, 256}};
constexpr TileShape kShape64 = {256, 512};

// Tile shapes of the batched kernel: entries per tile of rank class 16 and
// 32, threads per workgroup.  The plan's autotuner picks one.
constexpr MfBatchShape kBatchShapes[MF_BATCH_SHAPES] = {
    {1024, 512, 512}, {512, 512, 512}, {512, 256, 256}, {1024, 512, 768}};
constexpr int kLdsBytes = 160 * 1024;
constexpr int kBatchStaticLds = 1024;

// Accumulation mode of the single-tensor kernels: SLAB at rank class 16,
// MERGE at 32 when its slab fits the LDS beside the tile (else DIRECT, whose
// float atomics make the sum order vary), DIRECT for the gather-only class 64.
int acc_mode(int R, int T, int threads, int d, const int *n) {
  if (R == 16) return ACC_SLAB;
  if (R == 32 && mf_layout(R, T, threads, ACC_MERGE, d, n, 0).total <= kLdsBytes) return ACC_MERGE;
  return ACC_DIRECT;
}

bool g_deterministic = false;  // refuse float-atomic sums; plans run tensor by tensor

int g_variant[2] = {-1, -1};  // per rank class 16 / 32; -1: not chosen yet

int variant_of(int R) {
  if (R == 64) return 0;
  int &v = g_variant[R == 16 ? 0 : 1];
  if (v < 0) {
    v = 0;
    const char *e = getenv(R == 16 ? "TTGFX_TILE16" : "TTGFX_TILE32");
    if (e && (e[0] == '0' || e[0] == '1') && e[1] == 0) v = e[0] - '0';
  }
  return v;
}

TileShape shape_of(int R) {
  if (R == 16) return kShapes16[variant_of(16)];
  if (R == 32) return kShapes32[variant_of(32)];
  return kShape64;
}

int device_id() {
  int dev = 0;
  return hipGetDevice(&dev) == hipSuccess ? dev : -1;
}

// Suffix table levels of one launch (depth 0: none).
struct SuffixPlan {
  int depth;
  int row0[MF_MAX_D];
  int rows[MF_MAX_D];
  long long total_rows;
};

struct Geometry {
  int R, T, threads, acc, nb_max, total_slices, ntiles, nwg, lds;
  long long stash_stride, acc_stride;
  SuffixPlan suf;
};


// Workgroups per CU the LDS allows (the kernels' register use admits at
// least two 8-wave workgroups per CU).
int wgs_per_cu(int lds, int threads) {
  int by_lds = kLdsBytes / (lds > 0 ? lds : 1);
  int by_waves = 32 / (threads / 64);  // 8 waves per SIMD at most
  int w = by_lds < by_waves ? by_lds : by_waves;
  return w < 1 ? 1 : w;
}

// Suffix table policy.  Level l holds n_{d-l} .. n_{d-1} rows of R floats;
// a level is taken while the whole table stays within kSuffixBytes (so it
// stays in the L2 of every XCD beside the slices), while the entries
// outnumber its rows 16 to 1 (the build costs one R x R step per row and
// level, the sweep saves one per entry and level), at most d-1 levels, and
// and only as deep as the suffix ids and per-slot row ids fit the LDS
// without costing a workgroup per CU.
constexpr long long kSuffixBytes = 2ll << 20;
int g_suffix_mode = -1;  // -1 automatic, 0 off, k > 0: up to k levels, M aside

SuffixPlan suffix_plan(const tt_tensor *X, int R, int64_t M, int T, int threads, int acc) {
  SuffixPlan sf = {};
  if (g_suffix_mode == 0) return sf;
  const int l0 = mf_layout(R, T, threads, acc, X->d, X->n, 0).total;
  long long N = 1, total = 0;
  for (int l = 1; l <= X->d - 1; ++l) {
    N *= X->n[X->d - l];
    if ((total + N) * R * (long long)sizeof(float) > kSuffixBytes) break;
    if (g_suffix_mode < 0 && N * 16 > M) break;
    if (g_suffix_mode > 0 && l > g_suffix_mode) break;
    const int l1 = mf_layout(R, T, threads, acc, X->d, X->n, l).total;
    if (l1 > kLdsBytes || wgs_per_cu(l1, threads) < wgs_per_cu(l0, threads)) break;
    sf.row0[l - 1] = (int)total;
    sf.rows[l - 1] = (int)N;
    total += N;
    sf.depth = l;
  }
  sf.total_rows = total;
  return sf;
}

Geometry geometry(const tt_tensor *X, int R, int64_t M) {
  Geometry g;
  g.R = R;
  const TileShape sh = shape_of(R);
  g.T = sh.T;
  g.threads = sh.threads;
  int nmax = 1;
  g.total_slices = 0;
  for (int k = 0; k < X->d; ++k) {
    nmax = X->n[k] > nmax ? X->n[k] : nmax;
    g.total_slices += X->n[k];
  }
  g.acc = acc_mode(R, g.T, g.threads, X->d, X->n);
  g.suf = suffix_plan(X, R, M, g.T, g.threads, g.acc);
  g.lds = mf_layout(R, g.T, g.threads, g.acc, X->d, X->n, g.suf.depth).total;
  g.nb_max = g.T / 16 + nmax;
  g.ntiles = (int)((M + g.T - 1) / g.T);
  const int slots = device_cus() * wgs_per_cu(g.lds, g.threads);
  g.nwg = g.ntiles < slots ? g.ntiles : slots;
  if (g.nwg < 1) g.nwg = 1;
  // modes 0 .. d-2-depth stash rho_{k+1}; the table serves the rest
  const int stashed = X->d - 1 - g.suf.depth;
  g.stash_stride = (long long)(stashed > 1 ? stashed : 1) * g.nb_max * 64 * (R / 4);
  // per-workgroup accumulators of SLAB and MERGE
  g.acc_stride = g.acc != ACC_DIRECT ? (long long)g.total_slices * R * R : 0;
  return g;
}

template <int R, int T, int NTHR, int MODE, int ACC>
int launch_fused(const MfInst &p, const Grid &g, int nwg, int lds, hipStream_t s) {
  static int attr_dev = -2;
  const int dev = device_id();
  if (attr_dev != dev) {
    hipError_t e = hipFuncSetAttribute((const void *)fused_kernel<R, T, NTHR, MODE, ACC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (e != hipSuccess) return hip_check(e, "fused kernel LDS attribute");
    attr_dev = dev;
  }
  timer_before(s);
  hipLaunchKernelGGL((fused_kernel<R, T, NTHR, MODE, ACC>), dim3(nwg), dim3(NTHR), lds, s, p, g);
  timer_after(s);
  return launch_check("fused MFMA kernel");
}

template <int R, int T, int NTHR, int ACC>
int launch_acc(int mode, const MfInst &p, const Grid &g, int nwg, int lds, hipStream_t s) {
  if (mode == MODE_GATHER) return launch_fused<R, T, NTHR, MODE_GATHER, ACC>(p, g, nwg, lds, s);
  if constexpr (R <= 32) {
    if (mode == MODE_ADJOINT) return launch_fused<R, T, NTHR, MODE_ADJOINT, ACC>(p, g, nwg, lds, s);
    return launch_fused<R, T, NTHR, MODE_MSE, ACC>(p, g, nwg, lds, s);
  }
  return set_error(TT_ERR_UNSUPPORTED, "rank class 64 serves the gather only");
}

template <int R, int T, int NTHR>
int launch_mode(int mode, int acc, const MfInst &p, const Grid &g, int nwg, int lds, hipStream_t s) {
  if constexpr (R == 16) {
    return launch_acc<R, T, NTHR, ACC_SLAB>(mode, p, g, nwg, lds, s);
  } else {
    // the gather accumulates nothing: one instantiation serves it
    if (R == 32 && acc == ACC_MERGE && mode != MODE_GATHER)
      return launch_acc<R, T, NTHR, ACC_MERGE>(mode, p, g, nwg, lds, s);
    return launch_acc<R, T, NTHR, ACC_DIRECT>(mode, p, g, nwg, lds, s);
  }
}

int launch_geometry(int mode, const Geometry &ge, const MfInst &p, const Grid &g, hipStream_t s) {
  const TileShape sh{ge.T, ge.threads};
  if (ge.R == 16) {
    if (sh.T == kShapes16[0].T) return launch_mode<16, kShapes16[0].T, kShapes16[0].threads>(mode, ge.acc, p, g, ge.nwg, ge.lds, s);
    return launch_mode<16, kShapes16[1].T, kShapes16[1].threads>(mode, ge.acc, p, g, ge.nwg, ge.lds, s);
  }
  if (ge.R == 32) {
    if (sh.T == kShapes32[0].T) return launch_mode<32, kShapes32[0].T, kShapes32[0].threads>(mode, ge.acc, p, g, ge.nwg, ge.lds, s);
    return launch_mode<32, kShapes32[1].T, kShapes32[1].threads>(mode, ge.acc, p, g, ge.nwg, ge.lds, s);
  }
  return launch_mode<64, kShape64.T, kShape64.threads>(mode, ge.acc, p, g, ge.nwg, ge.lds, s);
}

}  // namespace

template <int R>
static bool fits_class(const tt_tensor *X) {
  if (X->d < 2 || X->d > MF_MAX_D) return false;
  for (int k = 0; k < X->d; ++k)
    if (X->n[k] > MfTraits<R>::MAX_N) return false;
  // every tile shape of the class (and the batched kernel's) fits the LDS,
  // so the choice of shape never changes which kernel serves a tensor
  TileShape shapes[2 + MF_BATCH_SHAPES];
  int ns = 0;
  if (R == 16) {
    shapes[ns++] = kShapes16[0];
    shapes[ns++] = kShapes16[1];
  } else if (R == 32) {
    shapes[ns++] = kShapes32[0];
    shapes[ns++] = kShapes32[1];
  } else {
    shapes[ns++] = kShape64;
  }
  const int nsingle = ns;
  if (R <= 32)
    for (int i = 0; i < MF_BATCH_SHAPES; ++i)
      shapes[ns++] = {R == 16 ? kBatchShapes[i].t16 : kBatchShapes[i].t32, kBatchShapes[i].threads};
  for (int i = 0; i < ns; ++i) {
    const int acc = (i < nsingle && R == 16) ? ACC_SLAB : ACC_DIRECT;
    const int cap = (i >= nsingle) ? kLdsBytes - kBatchStaticLds : kLdsBytes;
    if (mf_layout(R, shapes[i].T, shapes[i].threads, acc, X->d, X->n, 0).total > cap) return false;
  }
  return true;
}

int mfma_rank_class(const tt_tensor *L, const tt_tensor *R) {
  int mr = L ? max_rank_of(L) : 1;
  if (R && max_rank_of(R) > mr) mr = max_rank_of(R);
  return mr <= 16 ? 16 : 32;
}

bool mfma_supported(const tt_tensor *L, const tt_tensor *R) {
  const int rc = mfma_rank_class(L, R);
  const tt_tensor *ts[2] = {L, R};
  for (const tt_tensor *X : ts) {
    if (!X) continue;
    if (max_rank_of(X) > 32) return false;
    if (rc == 16 ? !fits_class<16>(X) : !fits_class<32>(X)) return false;
  }
  return true;
}

bool mfma_class_fits(const tt_tensor *X, int R) { return R == 16 ? fits_class<16>(X) : fits_class<32>(X); }

// Rank class of the gather alone (ranks up to 64), or 0 if none fits.
int mfma_gather_class(const tt_tensor *X) {
  const int mr = max_rank_of(X);
  const int rc = mr <= 16 ? 16 : (mr <= 32 ? 32 : (mr <= 64 ? 64 : 0));
  if (rc == 16) return fits_class<16>(X) ? 16 : 0;
  if (rc == 32) return fits_class<32>(X) ? 32 : 0;
  if (rc == 64) return fits_class<64>(X) ? 64 : 0;
  return 0;
}

size_t mfma_ws(const tt_tensor *X, int R, int64_t M, bool adjoint) {
  const Geometry g = geometry(X, R, M);
  size_t b = 2 * arena_bytes<float>((size_t)g.total_slices * R * R);
  if (g.suf.depth > 0) b += arena_bytes<float>((size_t)g.suf.total_rows * R);
  if (adjoint) {
    b += arena_bytes<float>((size_t)g.nwg * g.stash_stride);
    if (g.acc_stride > 0) {
      b += arena_bytes<float>((size_t)g.nwg * g.acc_stride);
      b += arena_bytes<float>((size_t)((g.nwg + 31) / 32) * g.total_slices * R * R);
    } else {
      b += arena_bytes<float>((size_t)g.total_slices * R * R);
    }
    b += arena_bytes<float>((size_t)g.nwg);
  }
  return b;
}

static int pad_and_suffix(const tt_tensor *Rt, const tt_tensor *Lt, int R, float *gpr, float *gpl,
                          const SufBuild &sb, hipStream_t s) {
  int total = 0;
  for (int k = 0; k < Rt->d; ++k) total += Rt->n[k];
  hipLaunchKernelGGL(pad_slices_kernel, dim3(total + (sb.depth > 0 ? sb.blocks : 0)), dim3(256), 0, s,
                     make_dev(Rt), make_dev(Lt ? Lt : Rt), R, gpr, gpl, total, sb);
  return launch_check("pad slices");
}

int mfma_pad(const tt_tensor *Rt, const tt_tensor *Lt, int R, float *gpr, float *gpl, hipStream_t s) {
  SufBuild none = {};
  return pad_and_suffix(Rt, Lt, R, gpr, gpl, none, s);
}

int mfma_unpad(const tt_tensor *O, int R, const float *padded, hipStream_t s) {
  long long E = 0;
  for (int k = 0; k < O->d; ++k) E += (long long)O->n[k] * R * R;
  hipLaunchKernelGGL(reduce_acc_stage2, dim3(64, O->d), dim3(256), 0, s, make_dev(O), R, padded, E, 1, nullptr, 0,
                     0LL, nullptr);
  return launch_check("unpad gradients");
}

int mfma_run(int mode, const tt_tensor *Lt, const tt_tensor *Rt, tt_tensor *O, const int32_t *idx,
             int64_t M, const float *t, const float *gy, float *y, float *gout, float *loss, void *ws,
             size_t ws_bytes, hipStream_t s) {
  const bool adjoint = mode != MODE_GATHER;
  const int R = adjoint ? mfma_rank_class(Lt, Rt) : mfma_gather_class(Rt);
  if (R == 0) return set_error(TT_ERR_UNSUPPORTED, "gather (MFMA): no rank class fits");
  const Geometry g = geometry(Rt, R, M);
  if (adjoint && g_deterministic && g.acc == ACC_DIRECT)
    return set_error(TT_ERR_UNSUPPORTED,
                     "deterministic mode: the mode sizes leave no LDS for the rank-%d slice accumulator", R);
  Arena ar(ws, ws_bytes);
  float *gpr = ar.take<float>((size_t)g.total_slices * R * R);
  float *gpl = ar.take<float>((size_t)g.total_slices * R * R);
  float *suf = g.suf.depth > 0 ? ar.take<float>((size_t)g.suf.total_rows * R) : nullptr;
  float *stash = nullptr, *acc = nullptr, *lacc = nullptr, *rtmp = nullptr, *grad = nullptr;
  if (adjoint) {
    stash = ar.take<float>((size_t)g.nwg * g.stash_stride);
    if (g.acc_stride > 0) {
      acc = ar.take<float>((size_t)g.nwg * g.acc_stride);
      rtmp = ar.take<float>((size_t)((g.nwg + 31) / 32) * g.total_slices * R * R);
    } else {
      grad = ar.take<float>((size_t)g.total_slices * R * R);
    }
    lacc = ar.take<float>((size_t)g.nwg);
  }
  if (!ar.ok()) return set_error(TT_ERR_WORKSPACE, "gather (MFMA): workspace too small");
  SufBuild sfb = {};
  if (g.suf.depth > 0 && M > 0) {
    sfb.tab = suf;
    sfb.depth = g.suf.depth;
    for (int l = 0; l < g.suf.depth; ++l) {
      sfb.row0[l] = g.suf.row0[l];
      sfb.rows[l] = g.suf.rows[l];
    }
    const int per_block = 4 * (64 / R);  // 256 threads: 4 waves of 64 / R suffixes
    sfb.blocks = (g.suf.rows[g.suf.depth - 1] + per_block - 1) / per_block;
  }
  int rc = pad_and_suffix(Rt, Lt, R, gpr, adjoint ? gpl : nullptr, sfb, s);
  if (rc) return rc;

  MfInst p = {};
  p.d = Rt->d;
  int sb = 0;
  for (int k = 0; k < Rt->d; ++k) {
    p.n[k] = Rt->n[k];
    p.sbase[k] = sb;
    sb += Rt->n[k];
  }
  p.idx = idx;
  p.M = M;
  p.gp_right = gpr;
  p.gp_left = gpl;
  p.t = t;
  p.gy = gy;
  p.y = y;
  p.gout = gout;
  p.grad = grad;
  p.inv_m2 = M > 0 ? 2.0f / (float)M : 0.f;
  p.inv_m = M > 0 ? 1.0f / (float)M : 0.f;
  p.rclass = R;
  p.suf = suf;
  p.suf_depth = sfb.depth;
  for (int l = 0; l < sfb.depth; ++l) {
    p.suf_row0[l] = sfb.row0[l];
    p.suf_rows[l] = sfb.rows[l];
  }
  Grid gr = {};
  gr.ntiles = g.ntiles;
  gr.nb_max = g.nb_max;
  gr.stash = stash;
  gr.stash_stride = g.stash_stride;
  gr.acc = acc;
  gr.acc_stride = g.acc_stride;
  gr.loss_acc = lacc;

  if (adjoint && grad) {
    if ((rc = fill_zero(grad, (long long)g.total_slices * R * R, s))) return rc;
  }
  if (M > 0) {
    rc = launch_geometry(mode, g, p, gr, s);
    if (rc) return rc;
  }
  if (!adjoint) return TT_OK;
  if (M == 0) {
    // no entries: zero gradients and loss
    for (int k = 0; k < O->d; ++k) {
      rc = fill_zero(O->data + core_off(O, k), core_elems(O, k), s);
      if (rc) return rc;
    }
    if (loss) return fill_zero(loss, 1, s);
    return TT_OK;
  }
  if (g.acc_stride > 0) {
    const TTDev od = make_dev(O);
    const long long E = (long long)g.total_slices * R * R;
    const int ngroups = (g.nwg + 31) / 32;
    hipLaunchKernelGGL(reduce_acc_stage1, dim3((unsigned)((E + 255) / 256), ngroups), dim3(256), 0, s,
                       acc, g.acc_stride, g.nwg, E, rtmp);
    if ((rc = launch_check("reduce partial gradients"))) return rc;
    // the MSE loss rides along as an extra row of blocks
    const bool with_loss = mode == MODE_MSE && loss;
    hipLaunchKernelGGL(reduce_acc_stage2, dim3(64, O->d + (with_loss ? 1 : 0)), dim3(256), 0, s, od, R, rtmp, E,
                       ngroups, lacc, g.nwg, (long long)M, with_loss ? loss : nullptr);
    if ((rc = launch_check("reduce partial gradients (2)"))) return rc;
    if (with_loss) return TT_OK;
  } else {
    if ((rc = mfma_unpad(O, R, grad, s))) return rc;
  }
  if (mode == MODE_MSE && loss) {
    hipLaunchKernelGGL(reduce_loss_kernel, dim3(1), dim3(64), 0, s, lacc, g.nwg, (long long)M, loss);
    return launch_check("reduce loss");
  }
  return TT_OK;
}

MfBatchShape mfma_batch_shape(int shape) { return kBatchShapes[shape]; }

size_t mfma_batch_lds(int shape, int d, const int *n) {
  const MfBatchShape &sh = kBatchShapes[shape];
  const int a = mf_layout(16, sh.t16, sh.threads, ACC_DIRECT, d, n, 0).total;
  const int b = mf_layout(32, sh.t32, sh.threads, ACC_DIRECT, d, n, 0).total;
  return (size_t)(a > b ? a : b);
}

int mfma_batch_wgs_per_cu(int shape, int d, const int *n) {
  return wgs_per_cu((int)mfma_batch_lds(shape, d, n) + kBatchStaticLds, kBatchShapes[shape].threads);
}

namespace {
template <int S>
const void *batch_fn() {
  constexpr MfBatchShape sh = kBatchShapes[S];
  return (const void *)batched_kernel<sh.t16, sh.t32, sh.threads>;
}
template <int S>
void batch_launch(const MfBatchArgs &a, int nwg, size_t lds, hipStream_t s) {
  constexpr MfBatchShape sh = kBatchShapes[S];
  hipLaunchKernelGGL((batched_kernel<sh.t16, sh.t32, sh.threads>), dim3(nwg), dim3(sh.threads), lds, s, a);
}
}  // namespace

int mfma_batch_prepare() {
  static int done_dev = -2;
  const int dev = device_id();
  if (done_dev == dev) return TT_OK;
  static_assert(MF_BATCH_SHAPES == 4, "one entry per shape below");
  const void *fns[MF_BATCH_SHAPES] = {batch_fn<0>(), batch_fn<1>(), batch_fn<2>(), batch_fn<3>()};
  for (const void *f : fns) {
    // the kernel also holds a few static LDS words (work item, loss partials)
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes - kBatchStaticLds);
    if (e != hipSuccess) return hip_check(e, "batched kernel LDS attribute");
  }
  done_dev = dev;
  return TT_OK;
}

int mfma_batch_launch(const MfBatchArgs &a, int shape, int nwg, size_t lds, hipStream_t s) {
  int rc = mfma_batch_prepare();
  if (rc) return rc;
  if (shape < 0 || shape >= MF_BATCH_SHAPES) return set_error(TT_ERR_ARG, "batched kernel: shape %d", shape);
  timer_before(s);
  switch (shape) {
    case 0: batch_launch<0>(a, nwg, lds, s); break;
    case 1: batch_launch<1>(a, nwg, lds, s); break;
    case 2: batch_launch<2>(a, nwg, lds, s); break;
    default: batch_launch<3>(a, nwg, lds, s); break;
  }
  timer_after(s);
  return launch_check("batched kernel");
}

int mfma_device_cus() { return device_cus(); }

void mfma_set_suffix_depth(int depth) { g_suffix_mode = depth < 0 ? -1 : depth; }

void mfma_set_deterministic(bool on) { g_deterministic = on; }

bool mfma_deterministic() { return g_deterministic; }

int mfma_suffix_depth_of(const tt_tensor *X, int R, int64_t M) { return geometry(X, R, M).suf.depth; }

bool mfma_deterministic_fits(const tt_tensor *X, int R, int64_t M) {
  return geometry(X, R, M).acc != ACC_DIRECT;
}

}  // namespace ttgfx
