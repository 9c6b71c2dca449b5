#!/usr/bin/env python3
"""Throughput of the TT-completion hot path on one MI355X.

One step = one fused pass over the observed entries of a d=10, n=10, r=16 TT
(2^20 uniform observed entries, planted rank-8 targets): the gather
(entry formula), the mean-squared-residual loss and the adjoint into all
core gradients, as one call of tt_gather_mse_backward.  Inputs are resident
in HBM before the timed region.

Prints one JSON line with the whole-job rate (observed entries/s), the
roofline of the dominant kernel (its duration measured with HIP events on
its launch stream) and the FP64 oracle timed on the host as a reported
baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "observed entries/s, TT gather fwd+bwd (d=10,n=10,r=16) + % roofline, batched vs plain"
# Algorithmic work of one gather forward + backward per observed entry at
# d=10, r=16 (first and last cores 1 x r and r x 1), the count of the scope
# table: forward 8 (1x16)(16x16) products plus one 16-dot = 4,128 flop;
# backward = both partial-product chains (4,128 + 4,096) and the outer
# products of all 10 modes, 2 (16 + 8*256 + 16) = 4,160: 12,352 flop.
FLOP_PER_ENTRY = 4128 + 12352
# What the fused kernel executes: the adjoint reuses the forward's right
# partials instead of recomputing them (4,128 + 4,096 + 4,160).
FLOP_EXECUTED = 4128 + 4096 + 4160
# The sparse tangent projection at d=10, canonical ranks (1,10,32,...,32,10,1):
# both interface chains and the 10 outer products per entry.
PROJ_FLOP_PER_ENTRY = 40744
# Batched workload (d=8, uniform rank r per tensor): forward + backward flop
# per entry by rank, and bytes per entry (8 indices, target, output weight,
# with the stash of one partial per mode counted once).
BATCH_FLOP = {4: 792, 8: 3120, 16: 12384, 32: 49344}
BATCH_BYTES_PER_ENTRY = 76
PEAK_MFMA_F32_TFLOPS = 157.3
PEAK_MFMA_BF16_TFLOPS = 2500.0
PEAK_VALU_F32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ["gather_mfma.hip", "gather_mfma.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fused_gather_d10_r16.json")


def batch_flop_per_entry(d, r):
    """Forward + backward flop per entry of a d-mode TT of uniform rank r
    with boundary ranks 1: forward (d-2) r x r products and one r-dot;
    backward both chains and the d outer products (the counts above)."""
    fwd = 2 * r * r * (d - 2) + 2 * r
    bwd = 2 * 2 * r * r * (d - 2) + 2 * (2 * r + (d - 2) * r * r)
    return fwd + bwd


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-peaks", action="store_true", help="skip the peak microbenchmarks")
    ap.add_argument("--no-oracle-workloads", action="store_true",
                    help="skip the oracle timings of the other workloads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20,
                    help="observed entries the oracle processes for the CPU baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (for HBM counter scaling)")
    ap.add_argument("--tables-only", action="store_true",
                    help="run only the table gather leg (for its kernel trace and HBM counters)")
    ap.add_argument("--leg", choices=["batched", "tables", "gram", "riemann", "ttm", "table1", "completion"],
                    help="run only this secondary measurement (for its kernel trace and counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary measurements (batched plan, Riemannian step, Gram, TT-matrix)")
    return ap.parse_args()


def copy_calibration():
    """A plain 512 MiB device-to-device copy, repeated: reading its
    FETCH_SIZE / WRITE_SIZE per dispatch gives the counter scale."""
    import torch
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))


def traffic_bytes():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when absent or taken on different kernel sources."""
    from paper_1801_01928_amd.profiling import source_hash
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_hash(KERNEL_SOURCES):
        return None
    return rec.get("traffic_bytes_per_launch")


def cpu_baseline(p, t, sample):
    """The FP64 oracle (gather, loss, adjoint) on the first `sample` observed
    entries, single-threaded BLAS."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import oracle
    S = min(sample, p.M)
    idx = p.idx[:, :S]
    ts = t[:S].astype(np.float64)
    cores = [c.astype(np.float64) for c in p.cores]
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        if ctx:
            ctx.__enter__()
        t0 = time.perf_counter()
        y = oracle.gather(cores, idx)
        _, g = oracle.mse_loss_and_grad(y, ts)
        oracle.gather_backward(cores, idx, g)
        dt = time.perf_counter() - t0
    finally:
        if ctx:
            ctx.__exit__(None, None, None)
    return {"value": S / dt, "unit": "entries/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of the %d observed entries (gather + MSE + adjoint, float64, %.1f s)"
                      % (S, p.M, dt)}


def _oracle_chunk(args):
    """Worker of the all-core baseline: the oracle's gather, loss and adjoint
    on one chunk of entries, single-threaded BLAS.  Returns the chunk's core
    gradients (for the parent to sum) and its time."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(limits=1)
    except ImportError:  # pragma: no cover
        ctx = None
    import oracle
    cores, idx, ts, m_total = args
    t0 = time.perf_counter()
    y = oracle.gather(cores, idx)
    _, g = oracle.mse_loss_and_grad(y, ts)
    g = g * (len(ts) / float(m_total))  # the chunk's share of the mean over all entries
    grads = oracle.gather_backward(cores, idx, g)
    dt = time.perf_counter() - t0
    del ctx  # the worker exits after the pool; its BLAS limit need not be restored
    return grads, dt


def cpu_baseline_all_cores(p, t, sample, workers):
    """The same oracle pass over `workers` processes (spawned, one BLAS thread
    each), each on its own chunk of the first workers * sample entries; the
    parent sums the chunk gradients.  Wall time from the first chunk handed
    out to the last gradient summed, after a warm-up that starts every
    worker.  Bounded waits; the pool is terminated on any failure."""
    import multiprocessing as mp
    import numpy as np
    S = min(sample * workers, p.M)
    cores = [c.astype(np.float64) for c in p.cores]
    ts = t[:S].astype(np.float64)
    bounds = np.linspace(0, S, workers + 1).astype(int)
    jobs = [(cores, p.idx[:, a:b], ts[a:b], S) for a, b in zip(bounds[:-1], bounds[1:])]
    pool = mp.get_context("spawn").Pool(workers)
    try:
        pool.map_async(_oracle_chunk, [(cores, p.idx[:, :64], ts[:64], S)] * workers, chunksize=1).get(timeout=60)
        t0 = time.perf_counter()
        res = pool.map_async(_oracle_chunk, jobs, chunksize=1).get(timeout=120)
        total = res[0][0]
        for grads, _ in res[1:]:
            total = [a + b for a, b in zip(total, grads)]
        dt = time.perf_counter() - t0
    finally:
        pool.terminate()
        pool.join()
    return {"value": S / dt, "unit": "entries/s", "cores": workers, "kind": "oracle",
            "sample": "first %d of the %d observed entries over %d processes (gather + MSE + adjoint, "
                      "float64, %.1f s)" % (S, p.M, workers, dt)}


def oracle_workloads(W):
    """The FP64 oracle timed on the other workloads, single-threaded BLAS,
    on bounded samples (each a few seconds): a full completion step of the
    small workload; the sparse projection (both sweeps, contraction, gauge,
    assembly) on the first 2^16 of the 2^20 entries of the rank-32 workload
    and its rounding; gather + MSE + adjoint of the first 8 of the 256
    batched tensors and 64 entries of their Gram matrix; the TT-matrix layer
    forward and backward on its full 4096-row batch."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle
    out = {}
    f64 = lambda cs: [np.asarray(c, np.float64) for c in cs]
    with threadpool_limits(limits=1):
        p = W.small_step()
        t = oracle.gather(p.planted, p.idx) + p.noise
        cores = f64(p.cores)
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            oracle.completion_step(cores, p.idx, t, alpha=-0.1, max_rank=4)
            ts.append(time.perf_counter() - t0)
        out["small_step"] = {"us_per_step": round(sorted(ts)[2] * 1e6, 1), "cores": 1,
                             "sample": "the whole workload (d=4 n=8 r=4, 4096 entries), median of 5"}
        q = W.riemann_d10()
        S = 1 << 16
        cq = f64(q.cores)
        t0 = time.perf_counter()
        Wt = oracle.project_sparse(cq, q.idx[:, :S], q.values[:S], alpha=-0.1, beta=1.0)[0]
        t1 = time.perf_counter()
        oracle.round_tt(Wt, 32)
        t2 = time.perf_counter()
        out["riemann_step"] = {"project_entries_per_s": round(S / (t1 - t0), 1), "round_ms": round((t2 - t1) * 1e3, 2),
                               "cores": 1, "sample": "first %d of the %d entries (projection %.1f s)" % (S, q.M, t1 - t0)}
        inst = W.batched()[:8]
        t0 = time.perf_counter()
        M = 0
        for b in inst:
            y = oracle.gather(b.cores, b.idx)
            _, g = oracle.mse_loss_and_grad(y, b.noise)
            oracle.gather_backward(b.cores, b.idx, g)
            M += b.M
        t1 = time.perf_counter()
        cs = [f64(b.cores) for b in inst]
        for a in range(8):
            for c in range(8):
                oracle.inner(cs[a], cs[c])
        t2 = time.perf_counter()
        out["batched"] = {"entries_per_s": round(M / (t1 - t0), 1), "gram_pairs_per_s": round(64 / (t2 - t1), 1),
                          "cores": 1, "sample": "tensors 0-7 of 256 (%d entries, %.1f s); 64 Gram entries" % (M, t1 - t0)}
        r = W.ttm_layer()
        t0 = time.perf_counter()
        oracle.ttm_forward(r.X, r.cores)
        t1 = time.perf_counter()
        oracle.ttm_backward(r.X, r.cores, r.dY)
        t2 = time.perf_counter()
        out["ttm_layer"] = {"fwd_ms": round((t1 - t0) * 1e3, 1), "bwd_ms": round((t2 - t1) * 1e3, 1), "cores": 1,
                            "sample": "the whole batch of 4096 rows (W materialised densely)"}
    return out


def _event_ms(fn, reps, stream=None):
    """Average milliseconds of fn() over reps calls, HIP events on the stream."""
    import torch
    stream = stream or torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
    stream.synchronize()
    return e0.elapsed_time(e1) / reps


def _percentiles(ms):
    import numpy as np
    a = np.asarray(ms, dtype=np.float64)
    return {"p10": round(float(np.percentile(a, 10)), 4), "p50": round(float(np.percentile(a, 50)), 4),
            "p90": round(float(np.percentile(a, 90)), 4), "reps": int(a.size)}


def _per_call_ms(fn, reps, stream=None):
    """Milliseconds of each of `reps` calls of fn(), each bracketed by its own
    pair of HIP events on the stream."""
    import torch
    stream = stream or torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    with torch.cuda.stream(stream):
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
    stream.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def peaks_leg(tt):
    """Measured peaks of one MI355X beside the datasheet's: a plain 1 GiB
    device copy (HBM, bytes read + written), and the library's
    microbenchmark kernels for the fp32 and bf16 matrix cores, fp32 vector
    FMA and LDS reads (median of 5 launches each)."""
    import ctypes as C
    import torch
    from paper_1801_01928_amd import _lib as L
    lib = L.load()
    out = {}
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ms = sorted(_per_call_ms(lambda: b.copy_(a), 7))[3]
    out["hbm_copy_gb_s"] = round(2 * 4 * n / (ms * 1e-3) / 1e9, 1)
    del a, b
    stream = torch.cuda.current_stream()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = 8 * cus
    sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    for kind, name, iters, unit in ((0, "mfma_f32_tflops", 1000, 1e12), (1, "mfma_bf16_tflops", 1000, 1e12),
                                    (2, "valu_f32_tflops", 4000, 1e12), (3, "lds_tb_s", 1000, 1e12)):
        launch = lambda: L.check(lib.tt_peak_launch(kind, blocks, iters, C.c_void_p(sink.data_ptr()),
                                                    C.c_void_p(stream.cuda_stream)))
        launch()
        torch.cuda.synchronize()
        ms = sorted(_per_call_ms(launch, 5))[2]
        out[name] = round(lib.tt_peak_work(kind, blocks, iters) / (ms * 1e-3) / unit, 2)
    out["datasheet"] = {"hbm_gb_s": PEAK_HBM_GBS, "mfma_f32_tflops": PEAK_MFMA_F32_TFLOPS,
                        "mfma_bf16_tflops": PEAK_MFMA_BF16_TFLOPS, "valu_f32_packed_tflops": PEAK_VALU_F32_TFLOPS,
                        "valu_f32_unpacked_tflops": PEAK_VALU_F32_TFLOPS / 2,
                        "lds_tb_s_at_128B_per_clk": round(cus * 128 * 2.4e9 / 1e12, 1)}
    return out


def batched_leg(tt, W, reps=3):
    """256 TT tensors (d=8, n=16, ranks from {4,8,16,32}, lognormal entry
    counts): one graph-captured persistent launch of gather + MSE + adjoint
    against per-tensor launches of the same kernels."""
    import numpy as np
    import torch
    inst = W.batched()
    Xs = [tt.TT.from_cores(p.cores) for p in inst]
    M = sum(p.M for p in inst)
    ts = []
    for p in inst:  # targets: planted TT gathered on the device, plus noise
        planted = tt.TT.from_cores(p.planted)
        ts.append(tt.gather(planted, p.idx) + torch.from_numpy(p.noise).cuda())
    t = torch.cat(ts)
    idx = np.concatenate([p.idx.reshape(-1) for p in inst])
    off = np.concatenate([[0], np.cumsum([p.M for p in inst])])
    plan = tt.BatchedPlan(Xs, idx, t, off)
    s = torch.cuda.Stream()
    plan.autotune(s)
    plan_cfg = plan.config()
    plan.capture(s)
    plan.run(s)
    s.synchronize()
    graph_ms = _event_ms(lambda: plan.run(s), reps, s)
    plan.run_plain(s)
    s.synchronize()
    plain_ms = _event_ms(lambda: plan.run_plain(s), reps, s)
    plan.close()
    # roofline: every tensor at the larger of its matrix-core and HBM times
    ideal_s = sum(max(q.M * BATCH_FLOP[q.meta["rank"]] / (PEAK_MFMA_F32_TFLOPS * 1e12),
                      q.M * BATCH_BYTES_PER_ENTRY / (PEAK_HBM_GBS * 1e9)) for q in inst)
    flop = sum(q.M * BATCH_FLOP[q.meta["rank"]] for q in inst)
    return {"workload": "256 TT tensors d=8 n=16, ranks U{4,8,16,32}, lognormal(ln 5e4, 0.8) entries "
                        "clipped to [1e4, 2e5], planted targets",
            "roofline": {"bound": "mfma (per tensor: max of flop/157.3 TF and 76 B/entry / 8 TB/s)",
                         "ideal_ms": round(ideal_s * 1e3, 4), "algorithmic_gflop": round(flop / 1e9, 2),
                         "frac": round(ideal_s * 1e3 / graph_ms, 4)},
            "entries": int(M), "autotuned": plan_cfg,
            "graph_ms": round(graph_ms, 3), "plain_ms": round(plain_ms, 3),
            "graph_entries_per_s": round(M / (graph_ms * 1e-3), 1),
            "plain_entries_per_s": round(M / (plain_ms * 1e-3), 1),
            "speedup": round(plain_ms / graph_ms, 3)}


def tables_leg(tt, W, reps=10):
    """The gather of the headline workload (d=10, n=10, r=16, 2^20 entries)
    from prefix/suffix tables, beside the chain gather: table build, table
    gather, and the HBM rate of the table gather over the index and output
    bytes (44 B per entry); the table rows come from the caches."""
    import torch
    p = W.gather_d10()
    X = tt.TT.from_cores(p.cores)
    idx = torch.from_numpy(p.idx).cuda()
    split, tabs = tt.halves_tables(X)
    tt.gather_halves(X, idx, tables=(split, tabs))
    tt.gather(X, idx)
    torch.cuda.synchronize()
    build_ms = _event_ms(lambda: tt.halves_tables(X, split), reps)
    gather_ms = _event_ms(lambda: tt.gather_halves(X, idx, tables=(split, tabs)), reps)
    chain_ms = _event_ms(lambda: tt.gather(X, idx), reps)
    return {"workload": "gather only, d=10 n=10 r=16, 2^20 uniform entries, tables cut at bond %d" % split,
            "table_mb": round(tabs.numel() / 1e6, 2), "build_ms": round(build_ms, 4),
            "gather_ms": round(gather_ms, 4), "chain_gather_ms": round(chain_ms, 4),
            "gather_entries_per_s": round(p.M / (gather_ms * 1e-3), 1),
            "build_plus_gather_entries_per_s": round(p.M / ((build_ms + gather_ms) * 1e-3), 1),
            "gather_gb_per_s_44b": round(44.0 * p.M / (gather_ms * 1e-3) / 1e9, 1)}


def gram_leg(tt, W, reps=3):
    """256 x 256 Gram matrix of the batched workload's tensors, ranks padded
    to 32 (12.65 MFLOP per pair, 32,896 unordered pairs)."""
    import torch
    Xs = [tt.TT.from_cores(p.cores) for p in W.batched()]
    tt.gram(Xs)
    torch.cuda.synchronize()
    with tt.KernelTimer() as kt:
        for _ in range(reps):
            tt.gram(Xs)
        torch.cuda.synchronize()
    ms = kt.ms / max(kt.launches, 1)
    flop = 416.1e9
    return {"kernel_ms": round(ms, 3), "tflops": round(flop / (ms * 1e-3) / 1e12, 2),
            "frac_of_fp32_mfma": round(flop / (ms * 1e-3) / 1e12 / PEAK_MFMA_F32_TFLOPS, 4)}


def riemann_leg(tt, W, reps=3):
    """One Riemannian step on d=10, n=10, r=32 (canonical ranks) with 2^20
    observed N(0,1) gradient values: both QR sweeps (one launch, a
    workgroup per direction), the sparse tangent projection with assembly,
    and TT rounding back to rank 32; beside the step, the projection of the
    rank-64 tangent TT onto the tangent space at X (the transport of a
    search direction), project_sum of 100 rank-10 TTs, and the Gram matrix
    of their 100 projections at a rank-10 point."""
    import torch
    p = W.riemann_d10()
    X = tt.TT.from_cores(p.cores)
    idx = torch.from_numpy(p.idx).cuda()
    z = torch.from_numpy(p.values).cuda()
    U, V = tt.orthogonalize_both(X)
    Wt = tt.project_sparse(U, V, idx, z, alpha=-0.1, add_x=1)
    tt.round_tt(Wt, 32)
    torch.cuda.synchronize()
    orth_ms = _event_ms(lambda: tt.orthogonalize_both(X), reps)
    proj_ms = _event_ms(lambda: tt.project_sparse(U, V, idx, z, alpha=-0.1, add_x=1), reps)
    with tt.KernelTimer() as kt:
        for _ in range(reps):
            tt.project_sparse(U, V, idx, z, alpha=-0.1, add_x=1)
        torch.cuda.synchronize()
    proj_kernel_ms = kt.ms / max(kt.launches, 1)
    proj_tf = PROJ_FLOP_PER_ENTRY * p.M / (proj_kernel_ms * 1e-3) / 1e12
    round_ms = _event_ms(lambda: tt.round_tt(Wt, 32), reps)
    tt.project_tt(U, V, Wt)
    torch.cuda.synchronize()
    transport_ms = _event_ms(lambda: tt.project_tt(U, V, Wt), reps)
    # project_sum of a batch of 100 random rank-10 TTs at X
    import numpy as np
    rng = np.random.default_rng(9)
    As = [tt.TT.from_cores(W.random_cores(rng, p.ns, W.uniform_ranks(len(p.ns), 10), 1 / np.sqrt(10)))
          for _ in range(100)]
    cw = rng.standard_normal(100)
    tt.project_sum(U, V, As, cw)
    torch.cuda.synchronize()
    psum_ms = _event_ms(lambda: tt.project_sum(U, V, As, cw), reps)
    # Gram matrix of 100 tangent vectors at a rank-10 point (the projections
    # of the same 100 TTs)
    X10 = tt.TT.from_cores(W.random_cores(rng, p.ns, W.canonical_ranks(p.ns, 10), 1 / np.sqrt(10)))
    U10, V10 = tt.orthogonalize_both(X10)
    Ts = [tt.project_tt(U10, V10, A) for A in As]
    tt.tangent_gram(U10, Ts)
    torch.cuda.synchronize()
    tgram_ms = _event_ms(lambda: tt.tangent_gram(U10, Ts), reps)
    return {"workload": "d=10 n=10 r=32 (canonical), 2^20 entries", "orthogonalize_both_ms": round(orth_ms, 3),
            "project_sparse_ms": round(proj_ms, 3),
            "project_entries_per_s": round(p.M / (proj_ms * 1e-3), 1),
            "project_roofline": {"bound": "mfma", "kernel": "fused_kernel<32,512,ADJOINT>",
                                 "kernel_ms": round(proj_kernel_ms, 4), "flop_per_entry": PROJ_FLOP_PER_ENTRY,
                                 "achieved": round(proj_tf, 3), "peak": PEAK_MFMA_F32_TFLOPS, "unit": "TFLOP/s",
                                 "frac": round(proj_tf / PEAK_MFMA_F32_TFLOPS, 4)},
            "round_ms": round(round_ms, 3), "step_ms": round(orth_ms + proj_ms + round_ms, 3),
            "project_tt_rank64_ms": round(transport_ms, 3),
            "project_sum_100_rank10_ms": round(psum_ms, 3),
            "tangent_gram_100_rank10_ms": round(tgram_ms, 3)}


def completion_leg(tt, W, iters=10, track=20):
    """Riemannian completion on d=10, n=10, canonical rank 16, 2^20 observed
    entries of a planted rank-8 tensor plus N(0, 0.01^2) noise, by gradient
    descent and by conjugate gradients (both with the exact line search on
    the linearised loss, every scalar on the device, no host
    synchronisation inside the loop): time per iteration over `iters`
    iterations, then `track` iterations from the same start with the
    observed loss and the held-out RMSE (2^16 held-out entries) before each
    step."""
    import torch
    p = W.completion_d10()
    X = tt.TT.from_cores(p.cores)
    planted = tt.TT.from_cores(p.planted)
    idx = torch.from_numpy(p.idx).cuda()
    idx_t = torch.from_numpy(p.meta["idx_test"]).cuda()
    t = tt.gather(planted, idx) + torch.from_numpy(p.noise).cuda()
    t_t = tt.gather(planted, idx_t)
    out = {"workload": "d=10 n=10 canonical r=16, 2^20 observed planted-rank-8 entries + N(0, 0.01^2) noise, "
                       "2^16 held-out entries"}
    for name, run in (("gd", tt.riemannian_completion), ("cg", tt.riemannian_cg)):
        run(X, idx, t, 16, 2)  # warm-up
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        run(X, idx, t, 16, iters)
        e1.record()
        torch.cuda.synchronize()
        Xn, h = run(X, idx, t, 16, track, idx_t, t_t)
        _, lt, _ = tt.gather_mse_backward(Xn, idx_t, t_t, want_y=False)
        _, lo, _ = tt.gather_mse_backward(Xn, idx, t, want_y=False)
        rec = {"iteration_ms": round(e0.elapsed_time(e1) / iters, 3),
               "loss": [round(x["loss"], 6) for x in h] + [round(float(lo.item()), 6)],
               "test_rmse": [round(x["test_rmse"], 5) for x in h] + [round(float(lt.item()) ** 0.5, 5)]}
        if name == "cg":
            rec["beta"] = [round(x["beta"], 4) for x in h]
            rec["restarts"] = sum(1 for x in h if x["restarted"])
        out[name] = rec
    return out


def table1_leg(tt, W, reps=5):
    """The operations of the paper's Table 1 at its shapes, in float32 and
    float64: TT-matrices 10^10 x 10^10 and TT vectors of size 10^10 (d=10,
    mode size 10, rank 10), batches of 100 objects; times per object of the
    batch, as the table reports them.  matvec: 100 products W x_j (outputs
    of rank 100); matmul: W W2 (one product; the batch time is 100 of them);
    norm: 100 TT vectors; gram: the 100 x 100 Gram matrix of 100 TT vectors
    (per object = per vector); project: project_sum of 100 TT vectors onto
    the tangent space at a rank-10 point (per object = per vector), and one
    projection of a rank-10 TT.  The outputs are allocated before timing.
    The HBM rate of the matvec counts its bytes read and written once."""
    import ctypes as C
    import numpy as np
    import torch
    from paper_1801_01928_amd import _lib as L
    from paper_1801_01928_amd.tt import _batch
    lib = L.load()
    d, b = 10, 100
    out = {"workload": "d=10, modes 10 (x 10 for matrices), rank 10, batch 100; ms per object"}
    stream = torch.cuda.current_stream()
    for name, dt in (("f32", torch.float32), ("f64", torch.float64)):
        rng = np.random.default_rng(11)
        mk = lambda: [rng.standard_normal((1 if k == 0 else 10, 10, 10, 1 if k == d - 1 else 10)) * 0.3
                      for k in range(d)]
        Wm = tt.TTMatrix.from_cores(mk(), dtype=dt)
        W2 = tt.TTMatrix.from_cores(mk(), dtype=dt)
        xs = [tt.TT.from_cores(W.random_cores(rng, [10] * d, W.uniform_ranks(d, 10), 0.3), dtype=dt)
              for _ in range(b)]
        ys = tt.tt_matvec(Wm, xs)
        xb, keepx = _batch(xs)
        yb, keepy = _batch(ys)
        fn = lib.tt_matvec_f64 if dt == torch.float64 else lib.tt_matvec
        call = lambda: L.check(fn(C.byref(Wm.desc()), C.byref(xb), C.byref(yb), C.c_void_p(stream.cuda_stream)))
        call()
        tt.tt_matmat(Wm, W2)
        tt.norms(xs)
        tt.gram(xs)
        torch.cuda.synchronize()
        mv = _event_ms(call, reps)
        mm = _event_ms(lambda: tt.tt_matmat(Wm, W2), reps)
        nr = _event_ms(lambda: tt.norms(xs), reps)
        gr = _event_ms(lambda: tt.gram(xs), reps)
        esize = 8 if dt == torch.float64 else 4
        nbytes = esize * (sum(y.data.numel() for y in ys) + sum(x.data.numel() for x in xs) + Wm.data.numel())
        rec = {"matvec_ms_per_object": round(mv / b, 5), "matvec_gb_per_s": round(nbytes / (mv * 1e-3) / 1e9, 1),
               "matmul_ms_per_object": round(mm, 4), "norm_ms_per_object": round(nr / b, 5),
               "gram_ms_per_object": round(gr / b, 5)}
        if dt == torch.float32:
            X10 = tt.TT.from_cores(W.random_cores(rng, [10] * d, W.canonical_ranks([10] * d, 10), 0.3))
            U, V = tt.orthogonalize_both(X10)
            cw = rng.standard_normal(b)
            tt.project_sum(U, V, xs, cw)
            tt.project_tt(U, V, xs[0])
            torch.cuda.synchronize()
            rec["project_sum_ms_per_object"] = round(_event_ms(lambda: tt.project_sum(U, V, xs, cw), reps) / b, 5)
            rec["project_one_ms"] = round(_event_ms(lambda: tt.project_tt(U, V, xs[0]), reps), 4)
        out[name] = rec
    return out


def ttm_dense_flops(ms_, ns_, rk, B):
    """Flops the dense path executes: W from the left partial products, the
    three GEMMs (Y, dX, dW_dense) and the core gradients (right partial sums
    and the contractions with the left partial products)."""
    import numpy as np
    d = len(ms_)
    U = lambda k: int(np.prod(ms_[:k])) if k else 1
    V = lambda k: int(np.prod(ns_[:k])) if k else 1
    build = sum(2 * U(k) * V(k) * rk[k] * ms_[k] * ns_[k] * rk[k + 1] for k in range(d))
    M, N = int(np.prod(ms_)), int(np.prod(ns_))
    right = sum(2 * U(k + 1) * V(k + 1) * rk[k + 1] * ms_[k + 1] * ns_[k + 1] * rk[k + 2] for k in range(d - 1))
    grads = sum(2 * rk[k] * ms_[k] * ns_[k] * rk[k + 1] * U(k) * V(k) for k in range(d))
    fwd = build + 2 * B * M * N
    bwd = build + 4 * B * M * N + right + grads
    return fwd, bwd


def ttm_leg(tt, W, reps=3):
    """TT-matrix layer 1024 x 1024 (modes 4^5, r=32) on a batch of 4096 rows:
    forward and adjoint, float32 and bf16 (float32 accumulation), on the
    path the library picks (the dense matrix) and on the core-by-core
    chain."""
    import numpy as np
    import torch
    p = W.ttm_layer()
    ms_, ns_, rk, B = p.row_modes, p.col_modes, p.ranks, p.X.shape[0]
    fwd_flop = sum(2.0 * B * np.prod(ms_[:k]) * np.prod(ns_[k + 1:]) * ns_[k] * rk[k] * ms_[k] * rk[k + 1]
                   for k in range(len(ms_)))
    dfwd, dbwd = ttm_dense_flops(ms_, ns_, rk, B)
    out = {"workload": "Y = X W^T, W 1024x1024 TT-matrix d=5 modes 4x4 r=32, batch 4096",
           "chain_fwd_gflop": round(fwd_flop / 1e9, 2),
           "dense_gflop": {"fwd": round(dfwd / 1e9, 3), "bwd": round(dbwd / 1e9, 3)}}
    for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        Wm = tt.TTMatrix.from_cores([torch.as_tensor(c).to(dt) for c in p.cores], dtype=dt)
        X = torch.as_tensor(p.X).to(dt).cuda()
        dY = torch.as_tensor(p.dY).to(dt).cuda()
        peak = PEAK_MFMA_F32_TFLOPS if name == "f32" else PEAK_MFMA_BF16_TFLOPS
        rec = {"path": tt.ttm_path(Wm, B)}
        for path in ("auto", "chain"):
            tt.ttm_set_path(path)
            tt.ttm_matmul(Wm, X)
            tt.ttm_matmul_backward(Wm, X, dY)
            torch.cuda.synchronize()
            f = _event_ms(lambda: tt.ttm_matmul(Wm, X), reps)
            b = _event_ms(lambda: tt.ttm_matmul_backward(Wm, X, dY), reps)
            if path == "auto":
                # executed flops of the dense path against the matrix-core peak
                tf = (dfwd + dbwd) / ((f + b) * 1e-3) / 1e12
                rec.update({"fwd_ms": round(f, 3), "bwd_ms": round(b, 3),
                            "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": peak,
                                         "unit": "TFLOP/s", "frac": round(tf / peak, 4),
                                         "flop_fwd_bwd": round((dfwd + dbwd) / 1e9, 2)}})
            else:
                # the backward is dX (one chain) and every dG^k (the chain of
                # T_k and V_{k+1} contractions): 3x the forward chain
                tf = 3 * fwd_flop / ((f + b) * 1e-3) / 1e12
                rec["chain"] = {"fwd_ms": round(f, 3), "bwd_ms": round(b, 3),
                                "fwd_chain_tflops": round(fwd_flop / (f * 1e-3) / 1e12, 2),
                                "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": peak,
                                             "unit": "TFLOP/s", "frac": round(tf / peak, 4),
                                             "flop_fwd_bwd": round(3 * fwd_flop / 1e9, 1)}}
        tt.ttm_set_path("auto")
        out[name] = rec
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py measures one GPU only: the library has no multi-GPU path "
                  "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    import paper_1801_01928_amd as tt

    if args.tables_only:
        import paper_1801_01928_amd as tt
        import workloads as W
        tt.load()
        print(json.dumps({"gather_tables": tables_leg(tt, W)}), flush=True)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.leg:
        torch.cuda.set_device(0)
        tt.load()
        legs = {"batched": batched_leg, "tables": tables_leg, "gram": gram_leg, "riemann": riemann_leg,
                "ttm": ttm_leg, "table1": table1_leg, "completion": completion_leg}
        print(json.dumps({args.leg: legs[args.leg](tt, W)}), flush=True)
        return

    torch.cuda.set_device(0)
    p = W.gather_d10()
    X = tt.TT.from_cores(p.cores)
    idx = torch.from_numpy(p.idx).cuda()
    planted = tt.TT.from_cores(p.planted)
    t = tt.gather(planted, idx) + torch.from_numpy(p.noise).cuda()
    torch.cuda.synchronize()

    ws = torch.empty(tt.gather_mse_workspace(X, p.M), dtype=torch.uint8, device="cuda")
    gX = X.empty_like()
    loss = torch.empty(1, dtype=torch.float32, device="cuda")

    def step():
        tt.gather_mse_backward(X, idx, t, want_y=False, ws=ws, out=gX, loss=loss)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with tt.KernelTimer() as kt:
        e0.record()
        for _ in range(args.steps):
            step()
        e1.record()
        torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    ms_per_step = total_ms / args.steps
    value = p.M * args.steps / (total_ms * 1e-3)

    kernel_ms = kt.ms / max(kt.launches, 1)
    # per-step distribution over separate event pairs (after the timed region)
    steps_ms = _per_call_ms(step, max(100, args.steps))
    achieved = FLOP_PER_ENTRY * p.M / (kernel_ms * 1e-3) / 1e12
    executed = FLOP_EXECUTED * p.M / (kernel_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_MFMA_F32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_MFMA_F32_TFLOPS, 4),
                "traffic": traffic_bytes(),
                "kernel": "fused_kernel<16,1024,768,MSE>", "kernel_ms": round(kernel_ms, 4),
                "flop_per_entry": FLOP_PER_ENTRY,
                "executed_flop_per_entry": FLOP_EXECUTED,
                "executed_frac": round(executed / PEAK_MFMA_F32_TFLOPS, 4)}

    out = {"metric": METRIC, "value": round(value, 1), "unit": "entries/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "fused TT gather + MSE + adjoint, d=10 n=10 r=16, "
                                  "2^20 uniform observed entries, planted rank-8 targets",
                      "d": 10, "n": 10, "r": 16, "M": p.M, "global_batch": p.M},
           "roofline": roofline,
           "step_ms": _percentiles(steps_ms),
           "loss": float(loss.item())}
    if not args.no_peaks:
        pk = peaks_leg(tt)
        out["peaks"] = pk
        roofline["frac_of_measured_peak"] = round(achieved / pk["mfma_f32_tflops"], 4)
    if not args.no_extras:
        # secondary measurements, each on its own workload after the timed region
        out["batched_vs_plain"] = batched_leg(tt, W)
        out["gather_tables"] = tables_leg(tt, W)
        out["gram"] = gram_leg(tt, W)
        out["riemann_step"] = riemann_leg(tt, W)
        out["ttm_layer"] = ttm_leg(tt, W)
        out["table1"] = table1_leg(tt, W)
        out["completion_loop"] = completion_leg(tt, W)
    if not args.no_cpu_baseline and not args.no_oracle_workloads:
        out["cpu_baseline_workloads"] = oracle_workloads(W)
    if not args.no_cpu_baseline:
        th = t.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(p, th, args.cpu_sample)
        workers = max(1, min(16, os.cpu_count() or 1))
        if workers > 1:
            try:
                out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(p, th, args.cpu_sample // 2, workers)
            except Exception as e:  # reported, never fatal to the JSON line
                out["cpu_baseline_all_cores"] = {"error": "%s: %s" % (type(e).__name__, e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
