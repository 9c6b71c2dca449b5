// Batched persistent plan (Batch Processing): gather + MSE + adjoint for
// many TT tensors of uneven ranks and entry counts in ONE persistent launch.
//
// tt_plan_create validates the batch, builds the work list (chunks of tiles
// of one tensor, in decreasing-cost order so that the atomic queue hands out
// the longest items first) and allocates the plan's device buffers.
// tt_plan_run issues: padded-slice copies of all tensors (one launch),
// zero-fill of gradients/losses/queue counter, the persistent kernel, and
// the unpadding of the gradients into the caller's cores.  tt_plan_capture
// records that sequence into a hipGraph (no memset nodes: fills are
// kernels) and later runs on the same stream replay it.
// tt_plan_autotune times the tile-chunk sizes of the work list and keeps the
// fastest (optionally cached in the file named by TTGFX_TUNE_CACHE).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "common.h"
#include "gather_mfma.h"
#include "kernels.h"

using namespace ttgfx;

namespace {

struct PadMeta {
  const float *data;
  long long off[TT_MAX_D];
  int r[TT_MAX_D + 1];
  int R;
  long long right;   // float offset of this tensor's padded slices (G)
  long long left;    // float offset of the transposed slices (G^T)
  long long grad;    // float offset of the padded gradient
  float *out;        // gradient output cores (caller's)
  long long out_off[TT_MAX_D];
};

struct ModeInfo {
  int d;
  int n[TT_MAX_D];
  int total;
};

// padded operand-order slices of every tensor: grid (d, b), one block per
// core, looping over its slices (one block per slice made the launch
// dispatch-bound)
__global__ void pad_batch_kernel(const PadMeta *__restrict__ meta, ModeInfo md, float *__restrict__ gp) {
  const PadMeta &m = meta[blockIdx.y];
  const int k = blockIdx.x;
  int base = 0;
  for (int j = 0; j < k; ++j) base += md.n[j];
  const int R = m.R, NT = R / 16, nk = md.n[k];
  const int r0 = m.r[k], r1 = m.r[k + 1];
  const float *G = m.data + m.off[k];
  for (int s = 0; s < nk; ++s) {
    float *right = gp + m.right + (long long)(base + s) * R * R;
    float *left = gp + m.left + (long long)(base + s) * R * R;
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
      const int c = e & 3, lane = (e >> 2) & 63, x = e >> 8;
      const int to = x / NT, ti = x % NT;
      const int row = 16 * to + (lane & 15), col = 16 * ti + 4 * (lane >> 4) + c;
      float vr = 0.f, vl = 0.f;
      if (row < r0 && col < r1) vr = G[(row * nk + s) * r1 + col];
      if (col < r0 && row < r1) vl = G[(col * nk + s) * r1 + row];
      right[e] = vr;
      left[e] = vl;
    }
  }
}

// padded gradients -> caller's cores: grid (d, b)
__global__ void unpad_batch_kernel(const PadMeta *__restrict__ meta, ModeInfo md, const float *__restrict__ gp) {
  const PadMeta &m = meta[blockIdx.y];
  const int k = blockIdx.x, R = m.R;
  int sbase = 0;
  for (int j = 0; j < k; ++j) sbase += md.n[j];
  const int rk = m.r[k], nk = md.n[k], rk1 = m.r[k + 1];
  const int total = rk * nk * rk1;  // one core: ranks and mode sizes of a plan are at most 32
  const float *g = gp + m.grad;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int b = e % rk1, t = e / rk1;
    const int s = t % nk, a = t / nk;
    m.out[m.out_off[k] + e] = g[((long long)(sbase + s) * R + a) * R + b];
  }
}

struct HostTT {
  int d;
  int32_t n[TT_MAX_D];
  int32_t r[TT_MAX_D + 1];
  int64_t off[TT_MAX_D];
  float *data;
  tt_tensor desc() const { return tt_tensor{d, n, r, off, data}; }
};

HostTT copy_tt(const tt_tensor *X) {
  HostTT h;
  memset(&h, 0, sizeof h);
  h.d = X->d;
  for (int k = 0; k < X->d; ++k) {
    h.n[k] = X->n[k];
    h.off[k] = core_off(X, k);
  }
  for (int k = 0; k <= X->d; ++k) h.r[k] = X->r[k];
  h.data = X->data;
  return h;
}

}  // namespace

struct tt_plan {
  int b = 0;
  ModeInfo md = {};
  std::vector<HostTT> X, grads;
  std::vector<int64_t> entry_off;
  std::vector<int> rclass;
  const int32_t *idx = nullptr;
  const float *t = nullptr;
  float *loss = nullptr;
  // device buffers owned by the plan
  PadMeta *dmeta = nullptr;
  MfInst *dtable = nullptr;
  MfWorkItem *ditems = nullptr;
  int *counter = nullptr;
  float *gp = nullptr;          // padded slices and padded gradients
  long long grad_begin = 0, grad_floats = 0;
  float *stash = nullptr;
  long long stash_stride = 0;
  int nmax = 1;                 // largest mode size
  int shape = 0;                // tile shape of the batched kernel (mfma_batch_shape)
  int chunk = 4;
  int nitems = 0;
  int max_items = 0;
  void *plain_ws = nullptr;
  size_t plain_ws_bytes = 0;
  hipGraphExec_t graph = nullptr;
  hipStream_t graph_stream = nullptr;
  bool graph_det = false;  // reduction policy the graph was captured under
};

namespace {

// Launch geometry of the batched kernel for one tile shape: stash blocks per
// mode of each rank class, stash floats per workgroup, workgroups.
struct ShapeGeo {
  int nb16, nb32, nwg;
  long long stash_stride;
};

ShapeGeo shape_geo(const tt_plan *P, int shape) {
  const MfBatchShape sh = mfma_batch_shape(shape);
  ShapeGeo g;
  g.nb16 = sh.t16 / 16 + P->nmax;
  g.nb32 = sh.t32 / 16 + P->nmax;
  const long long dm1 = P->md.d > 1 ? P->md.d - 1 : 1;
  g.stash_stride = std::max(dm1 * g.nb16 * 64 * 4, dm1 * g.nb32 * 64 * 8);
  g.nwg = mfma_device_cus() * mfma_batch_wgs_per_cu(shape, P->md.d, P->md.n);
  return g;
}

int build_items(tt_plan *P) {
  std::vector<MfWorkItem> items;
  std::vector<long long> cost;
  const MfBatchShape sh = mfma_batch_shape(P->shape);
  for (int j = 0; j < P->b; ++j) {
    const long long M = P->entry_off[j + 1] - P->entry_off[j];
    const int R = P->rclass[j];
    const int T = (R == 16) ? sh.t16 : sh.t32;
    const int ntiles = (int)((M + T - 1) / T);
    for (int t0 = 0; t0 < ntiles; t0 += P->chunk) {
      const int nt = std::min(P->chunk, ntiles - t0);
      items.push_back(MfWorkItem{j, t0, nt, R});
      // work per tile ~ T * R^2 (MFMA work at padded rank)
      cost.push_back((long long)nt * T * R * R);
    }
  }
  std::vector<int> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<MfWorkItem> sorted(items.size());
  for (size_t i = 0; i < order.size(); ++i) sorted[i] = items[order[i]];
  if ((int)sorted.size() > P->max_items) return set_error(TT_ERR_ARG, "plan: work list larger than allocated");
  P->nitems = (int)sorted.size();
  if (P->nitems)
    return hip_check(hipMemcpy(P->ditems, sorted.data(), sizeof(MfWorkItem) * sorted.size(), hipMemcpyHostToDevice),
                     "plan work list upload");
  return TT_OK;
}

int issue(tt_plan *P, hipStream_t s) {
  hipLaunchKernelGGL(pad_batch_kernel, dim3(P->md.d, P->b), dim3(256), 0, s, P->dmeta, P->md, P->gp);
  int rc = launch_check("plan: pad slices");
  if (rc) return rc;
  if ((rc = fill_zero(P->gp + P->grad_begin, P->grad_floats, s))) return rc;
  if ((rc = fill_zero(P->loss, P->b, s))) return rc;
  if ((rc = fill_zero((float *)P->counter, 1, s))) return rc;
  MfBatchArgs a;
  a.table = P->dtable;
  a.items = P->ditems;
  a.nitems = P->nitems;
  a.counter = P->counter;
  const ShapeGeo g = shape_geo(P, P->shape);
  a.stash = P->stash;
  a.stash_stride = g.stash_stride;
  a.nb16 = g.nb16;
  a.nb32 = g.nb32;
  if (P->nitems > 0 &&
      (rc = mfma_batch_launch(a, P->shape, g.nwg, mfma_batch_lds(P->shape, P->md.d, P->md.n), s)))
    return rc;
  hipLaunchKernelGGL(unpad_batch_kernel, dim3(P->md.d, P->b), dim3(256), 0, s, P->dmeta, P->md, P->gp);
  return launch_check("plan: unpad gradients");
}

// One fused pass per tensor (no batched kernel).
int run_plain(tt_plan *plan, hipStream_t s) {
  const int d = plan->md.d;
  for (int j = 0; j < plan->b; ++j) {
    tt_tensor x = plan->X[j].desc();
    tt_tensor g = plan->grads[j].desc();
    const int64_t M = plan->entry_off[j + 1] - plan->entry_off[j];
    const int32_t *ij = plan->idx ? plan->idx + (long long)d * plan->entry_off[j] : nullptr;
    const float *tj = plan->t ? plan->t + plan->entry_off[j] : nullptr;
    int rc = fused_mse_dispatch(&x, ij, M, tj, nullptr, nullptr, plan->loss + j, &g, plan->plain_ws,
                                plan->plain_ws_bytes, s);
    if (rc) return rc;
  }
  return TT_OK;
}

// In deterministic mode the plan runs tensor by tensor: the batched kernel
// adds finished runs with float atomics.
int issue_policy(tt_plan *P, hipStream_t s) { return mfma_deterministic() ? run_plain(P, s) : issue(P, s); }

void drop_graph(tt_plan *P) {
  if (P->graph) (void)hipGraphExecDestroy(P->graph);
  P->graph = nullptr;
  P->graph_stream = nullptr;
}

// Tuning-cache key: device architecture and CU count, d, the mode sizes'
// sum, the tensor count per rank class and the total entry count rounded
// to a power of two.
std::string signature(const tt_plan *P) {
  char buf[320];
  long long total = P->entry_off[P->b];
  int c16 = 0, c32 = 0;
  for (int j = 0; j < P->b; ++j) (P->rclass[j] == 16 ? c16 : c32)++;
  int nsum = 0;
  for (int k = 0; k < P->md.d; ++k) nsum += P->md.n[k];
  int mlog = 0;
  while ((1LL << mlog) < total) ++mlog;
  char arch[64] = "gfx";
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    for (char *c = arch; *c; ++c)
      if (*c == ':' || *c == ' ') *c = '_';
  }
  snprintf(buf, sizeof buf, "%s_cus%d_d%d_n%d_b%d_r16x%d_r32x%d_M2^%d", arch, mfma_device_cus(), P->md.d, nsum,
           P->b, c16, c32, mlog);
  return buf;
}

}  // namespace

extern "C" {

int tt_plan_create(const tt_batch *X, const int32_t *idx, const float *t, const int64_t *entry_off,
                   const tt_batch *grads, float *loss, tt_plan **plan) {
  if (!plan) return set_error(TT_ERR_ARG, "null plan pointer");
  *plan = nullptr;
  if (!X || !X->tt || X->b < 1) return set_error(TT_ERR_ARG, "X: empty or null batch");
  if (!grads || !grads->tt || grads->b != X->b) return set_error(TT_ERR_SHAPE, "grads must match X's batch size");
  if (!entry_off) return set_error(TT_ERR_ARG, "null entry_off");
  if (!loss) return set_error(TT_ERR_ARG, "null loss");
  const tt_tensor *ref = &X->tt[0];
  for (int j = 0; j < X->b; ++j) {
    char nm[32];
    snprintf(nm, sizeof nm, "X[%d]", j);
    int rc = validate_tt(&X->tt[j], nm, 32);
    if (rc) return rc;
    snprintf(nm, sizeof nm, "grads[%d]", j);
    if ((rc = validate_tt(&grads->tt[j], nm, 32))) return rc;
    if (!same_modes(&X->tt[j], ref)) return set_error(TT_ERR_SHAPE, "X[%d]: mode sizes differ from X[0]", j);
    if (!same_shape(&X->tt[j], &grads->tt[j])) return set_error(TT_ERR_SHAPE, "grads[%d] must have X[%d]'s shape", j, j);
    const int R = mfma_rank_class(&X->tt[j], nullptr);
    if (!mfma_class_fits(&X->tt[j], R))
      return set_error(TT_ERR_UNSUPPORTED, "X[%d]: d or mode sizes outside the batched kernel's limits", j);
    if (entry_off[j + 1] < entry_off[j]) return set_error(TT_ERR_ARG, "entry_off must be non-decreasing");
  }
  if (entry_off[0] != 0) return set_error(TT_ERR_ARG, "entry_off[0] must be 0");
  if (entry_off[X->b] > 0 && (!idx || !t)) return set_error(TT_ERR_ARG, "null idx or t");
  int rc = mfma_batch_prepare();
  if (rc) return rc;

  tt_plan *P = new tt_plan();
  P->b = X->b;
  P->md.d = ref->d;
  P->md.total = 0;
  for (int k = 0; k < ref->d; ++k) {
    P->md.n[k] = ref->n[k];
    P->md.total += ref->n[k];
  }
  P->idx = idx;
  P->t = t;
  P->loss = loss;
  P->entry_off.assign(entry_off, entry_off + X->b + 1);
  for (int k = 0; k < ref->d; ++k) P->nmax = std::max(P->nmax, ref->n[k]);
  // stash for the largest of the shapes' needs
  long long stash_floats = 0;
  for (int sh = 0; sh < MF_BATCH_SHAPES; ++sh) {
    const ShapeGeo g = shape_geo(P, sh);
    stash_floats = std::max(stash_floats, g.stash_stride * g.nwg);
  }

  // host tables
  std::vector<PadMeta> meta(X->b);
  std::vector<MfInst> table(X->b);
  long long off = 0;
  for (int j = 0; j < X->b; ++j) {
    P->X.push_back(copy_tt(&X->tt[j]));
    P->grads.push_back(copy_tt(&grads->tt[j]));
    const int R = mfma_rank_class(&X->tt[j], nullptr);
    P->rclass.push_back(R);
    PadMeta &m = meta[j];
    memset(&m, 0, sizeof m);
    m.data = X->tt[j].data;
    for (int k = 0; k < ref->d; ++k) {
      m.off[k] = core_off(&X->tt[j], k);
      m.out_off[k] = core_off(&grads->tt[j], k);
    }
    for (int k = 0; k <= ref->d; ++k) m.r[k] = X->tt[j].r[k];
    m.R = R;
    m.out = grads->tt[j].data;
    m.right = off;
    off += (long long)P->md.total * R * R;
    m.left = off;
    off += (long long)P->md.total * R * R;
  }
  P->grad_begin = off;
  for (int j = 0; j < X->b; ++j) {
    meta[j].grad = off;
    off += (long long)P->md.total * meta[j].R * meta[j].R;
  }
  P->grad_floats = off - P->grad_begin;
  for (int j = 0; j < X->b; ++j) {
    MfInst &p = table[j];
    memset(&p, 0, sizeof p);
    p.d = ref->d;
    int sb = 0;
    for (int k = 0; k < ref->d; ++k) {
      p.n[k] = ref->n[k];
      p.sbase[k] = sb;
      sb += ref->n[k];
    }
    const long long M = entry_off[j + 1] - entry_off[j];
    p.M = M;
    p.idx = idx ? idx + (long long)ref->d * entry_off[j] : nullptr;
    p.t = t ? t + entry_off[j] : nullptr;
    p.inv_m2 = M > 0 ? 2.0f / (float)M : 0.f;
    p.inv_m = M > 0 ? 1.0f / (float)M : 0.f;
    p.rclass = meta[j].R;
    p.loss = loss + j;
    // device pointers into gp are set after allocation
  }
  // upper bound on work items (chunk = 1)
  long long maxit = 0;
  for (int j = 0; j < X->b; ++j) {
    const int T = (meta[j].R == 16) ? MF_BATCH_MIN_T16 : MF_BATCH_MIN_T32;
    maxit += (P->entry_off[j + 1] - P->entry_off[j] + T - 1) / T;
  }
  P->max_items = (int)std::max(1LL, maxit);

  // plain path workspace (one tensor at a time)
  size_t pw = 0;
  for (int j = 0; j < X->b; ++j) {
    tt_tensor d = P->X[j].desc();
    pw = std::max(pw, fused_mse_ws(&d, entry_off[j + 1] - entry_off[j]));
  }
  P->plain_ws_bytes = pw;

  rc = hip_check(hipMalloc((void **)&P->gp, sizeof(float) * (size_t)off), "plan: slices");
  if (!rc) rc = hip_check(hipMalloc((void **)&P->dmeta, sizeof(PadMeta) * X->b), "plan: metadata");
  if (!rc) rc = hip_check(hipMalloc((void **)&P->dtable, sizeof(MfInst) * X->b), "plan: table");
  if (!rc) rc = hip_check(hipMalloc((void **)&P->ditems, sizeof(MfWorkItem) * P->max_items), "plan: items");
  if (!rc) rc = hip_check(hipMalloc((void **)&P->counter, 256), "plan: counter");
  if (!rc) rc = hip_check(hipMalloc((void **)&P->stash, sizeof(float) * (size_t)stash_floats), "plan: stash");
  if (!rc && pw) rc = hip_check(hipMalloc(&P->plain_ws, pw), "plan: plain workspace");
  if (rc) {
    tt_plan_destroy(P);
    return rc;
  }
  for (int j = 0; j < X->b; ++j) {
    table[j].gp_right = P->gp + meta[j].right;
    table[j].gp_left = P->gp + meta[j].left;
    table[j].grad = P->gp + meta[j].grad;
  }
  rc = hip_check(hipMemcpy(P->dmeta, meta.data(), sizeof(PadMeta) * X->b, hipMemcpyHostToDevice), "plan: upload");
  if (!rc) rc = hip_check(hipMemcpy(P->dtable, table.data(), sizeof(MfInst) * X->b, hipMemcpyHostToDevice), "plan: upload");
  if (!rc) rc = build_items(P);
  if (rc) {
    tt_plan_destroy(P);
    return rc;
  }
  *plan = P;
  return TT_OK;
}

int tt_plan_run(tt_plan *plan, void *stream) {
  if (!plan) return set_error(TT_ERR_ARG, "null plan");
  hipStream_t s = (hipStream_t)stream;
  if (plan->graph && plan->graph_stream == s && plan->graph_det == mfma_deterministic())
    return hip_check(hipGraphLaunch(plan->graph, s), "plan: graph launch");
  return issue_policy(plan, s);
}

int tt_plan_capture(tt_plan *plan, void *stream) {
  if (!plan) return set_error(TT_ERR_ARG, "null plan");
  hipStream_t s = (hipStream_t)stream;
  if (!s) return set_error(TT_ERR_ARG, "capture needs a non-default stream");
  drop_graph(plan);
  int rc = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "plan: begin capture");
  if (rc) return rc;
  rc = issue_policy(plan, s);
  hipGraph_t g = nullptr;
  int rc2 = hip_check(hipStreamEndCapture(s, &g), "plan: end capture");
  if (rc || rc2) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : rc2;
  }
  rc = hip_check(hipGraphInstantiate(&plan->graph, g, nullptr, nullptr, 0), "plan: instantiate");
  (void)hipGraphDestroy(g);
  if (rc) return rc;
  plan->graph_stream = s;
  plan->graph_det = mfma_deterministic();
  return TT_OK;
}

int tt_plan_run_plain(tt_plan *plan, void *stream) {
  if (!plan) return set_error(TT_ERR_ARG, "null plan");
  return run_plain(plan, (hipStream_t)stream);
}

int tt_plan_autotune(tt_plan *plan, void *stream, int32_t *chosen) {
  if (!plan) return set_error(TT_ERR_ARG, "null plan");
  hipStream_t s = (hipStream_t)stream;
  // build_items rewrites the device work list with a synchronous copy that
  // is not ordered against work already queued on s: let that work finish
  int rc0 = hip_check(hipStreamSynchronize(s), "autotune: drain the stream");
  if (rc0) return rc0;
  const char *cache = getenv("TTGFX_TUNE_CACHE");
  const std::string sig = signature(plan);
  int best = -1, best_shape = 0;
  if (cache) {
    FILE *f = fopen(cache, "r");
    if (f) {
      char key[320];
      int sh, ch;
      while (fscanf(f, "%319s %d %d", key, &sh, &ch) == 3)
        if (sig == key && sh >= 0 && sh < MF_BATCH_SHAPES && ch >= 1) {
          best_shape = sh;
          best = ch;
        }
      fclose(f);
    }
  }
  if (best < 0) {
    // every tile shape of the batched kernel with every work-item chunk
    const int cands[] = {1, 2, 4, 8, 16};
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    int rc = hip_check(hipEventCreate(&e0), "autotune event");
    if (rc) return rc;
    if ((rc = hip_check(hipEventCreate(&e1), "autotune event"))) return rc;
    for (int sh = 0; sh < MF_BATCH_SHAPES && !rc; ++sh) {
      for (int c : cands) {
        plan->shape = sh;
        plan->chunk = c;
        if ((rc = build_items(plan))) break;
        if ((rc = issue(plan, s))) break;  // warm-up
        float ms_best = 1e30f;
        for (int rep = 0; rep < 3 && !rc; ++rep) {
          rc = hip_check(hipEventRecord(e0, s), "autotune record");
          if (!rc) rc = issue(plan, s);
          if (!rc) rc = hip_check(hipEventRecord(e1, s), "autotune record");
          if (!rc) rc = hip_check(hipEventSynchronize(e1), "autotune sync");
          float ms = 0.f;
          if (!rc) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "autotune time");
          if (!rc) ms_best = std::min(ms_best, ms);
        }
        if (rc) break;
        if (ms_best < best_ms) {
          best_ms = ms_best;
          best = c;
          best_shape = sh;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (cache) {
      FILE *f = fopen(cache, "a");
      if (f) {
        fprintf(f, "%s %d %d\n", sig.c_str(), best_shape, best);
        fclose(f);
      }
    }
  }
  drop_graph(plan);
  plan->shape = best_shape;
  plan->chunk = best;
  int rc = build_items(plan);
  if (rc) return rc;
  if (chosen) *chosen = best;
  return TT_OK;
}

int tt_plan_set_config(tt_plan *plan, const int32_t *cfg) {
  if (!plan || !cfg) return set_error(TT_ERR_ARG, "plan_set_config: null argument");
  if (cfg[0] < 1) return set_error(TT_ERR_ARG, "plan_set_config: chunk %d < 1", cfg[0]);
  int shape = -1;
  for (int i = 0; i < MF_BATCH_SHAPES; ++i) {
    const MfBatchShape sh = mfma_batch_shape(i);
    if (sh.t16 == cfg[1] && sh.t32 == cfg[2] && sh.threads == cfg[3]) shape = i;
  }
  if (shape < 0)
    return set_error(TT_ERR_UNSUPPORTED, "plan_set_config: no tile shape %d/%d/%d", cfg[1], cfg[2], cfg[3]);
  drop_graph(plan);
  plan->shape = shape;
  plan->chunk = cfg[0];
  return build_items(plan);
}

int tt_plan_config(const tt_plan *plan, int32_t *cfg) {
  if (!plan || !cfg) return set_error(TT_ERR_ARG, "plan_config: null argument");
  const MfBatchShape sh = mfma_batch_shape(plan->shape);
  cfg[0] = plan->chunk;
  cfg[1] = sh.t16;
  cfg[2] = sh.t32;
  cfg[3] = sh.threads;
  return TT_OK;
}

void tt_plan_destroy(tt_plan *plan) {
  if (!plan) return;
  drop_graph(plan);
  if (plan->gp) (void)hipFree(plan->gp);
  if (plan->dmeta) (void)hipFree(plan->dmeta);
  if (plan->dtable) (void)hipFree(plan->dtable);
  if (plan->ditems) (void)hipFree(plan->ditems);
  if (plan->counter) (void)hipFree(plan->counter);
  if (plan->stash) (void)hipFree(plan->stash);
  if (plan->plain_ws) (void)hipFree(plan->plain_ws);
  delete plan;
}

}  // extern "C"
