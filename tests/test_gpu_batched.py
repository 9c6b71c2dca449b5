"""GPU parity of the batched persistent plan: per-tensor losses and core
gradients against the FP64 oracle (1e-5 relative), agreement with the plain
per-tensor launches, hipGraph replays, and the 256-tensor workload."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import adjoint_bound, assert_elementwise

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _small_batch():
    ns = [6, 7, 5, 6, 6]
    rng = np.random.default_rng(900)
    ranks_list = [4, 8, 16, 32, 3, 20, 12, 32, 5, 16, 28, 8]
    counts = [3000, 1, 0, 2500, 777, 1500, 4096, 5000, 1025, 64, 3333, 2048]
    insts = []
    for r, M in zip(ranks_list, counts):
        ranks = W.canonical_ranks(ns, r)
        cores = W.random_cores(rng, ns, ranks, 1.0 / np.sqrt(r))
        idx = W.random_indices(rng, ns, M)
        t = rng.standard_normal(M).astype(np.float32)
        insts.append((cores, idx, t))
    return ns, insts


def _pack(insts):
    off = [0]
    for _, idx, _ in insts:
        off.append(off[-1] + idx.shape[1])
    idx = np.concatenate([i.reshape(-1) for _, i, _ in insts]) if off[-1] else np.zeros(0, np.int32)
    t = np.concatenate([x for _, _, x in insts]) if off[-1] else np.zeros(0, np.float32)
    return idx, t, off


def _oracle(insts):
    out = []
    for cores, idx, t in insts:
        if idx.shape[1] == 0:
            out.append((0.0, [np.zeros(c.shape) for c in cores], [np.zeros(c.shape) for c in cores]))
            continue
        y = oracle.gather(cores, idx)
        loss, g = oracle.mse_loss_and_grad(y, t)
        out.append((loss, oracle.gather_backward(cores, idx, g), adjoint_bound(cores, cores, idx, g)))
    return out


def _check(plan, ref):
    """Per tensor: the loss (1e-5 relative), each core normwise (1e-5) and
    each gradient element within 1e-5 of its absolute-value bound."""
    loss = plan.loss.cpu().numpy()
    for j, item in enumerate(ref):
        lr, gr = item[0], item[1]
        assert abs(loss[j] - lr) <= TOL * max(lr, 1e-30), (j, loss[j], lr)
        got = plan.grads[j].numpy_cores()
        for k, c in enumerate(got):
            assert _rel(c, gr[k]) <= TOL, (j, k, _rel(c, gr[k]))
            if len(item) > 2:
                assert_elementwise(c, gr[k], item[2][k], TOL, "tensor %d core %d" % (j, k))


def test_batched_and_plain_match_oracle(gpu_lib):
    tt = gpu_lib
    ns, insts = _small_batch()
    idx, t, off = _pack(insts)
    Xs = [tt.TT.from_cores(c) for c, _, _ in insts]
    plan = tt.BatchedPlan(Xs, idx, t, off)
    ref = _oracle(insts)
    plan.run()
    _check(plan, ref)
    plan.run_plain()
    _check(plan, ref)
    plan.close()


def test_graph_replays_follow_eager(gpu_lib):
    import torch
    tt = gpu_lib
    ns, insts = _small_batch()
    idx, t, off = _pack(insts)
    Xs = [tt.TT.from_cores(c) for c, _, _ in insts]
    plan = tt.BatchedPlan(Xs, idx, t, off)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture(s)
    torch.cuda.synchronize()
    for rep in range(3):
        # eager work between replays: new targets in place, then an eager run
        with torch.cuda.stream(s):
            plan.t.mul_(0.5).add_(0.25 * rep)
        s.synchronize()
        plan.run_plain(s)              # eager reference (not captured)
        s.synchronize()
        ref_loss = plan.loss.clone()
        ref_grads = [g.data.clone() for g in plan.grads]
        plan.run(s)                    # graph replay
        s.synchronize()
        assert torch.allclose(plan.loss, ref_loss, rtol=1e-5, atol=1e-12)
        for g, r in zip(plan.grads, ref_grads):
            assert _rel(g.data.cpu().numpy(), r.cpu().numpy()) <= TOL
    plan.close()


def test_autotune_keeps_results(gpu_lib):
    tt = gpu_lib
    ns, insts = _small_batch()
    idx, t, off = _pack(insts)
    Xs = [tt.TT.from_cores(c) for c, _, _ in insts]
    plan = tt.BatchedPlan(Xs, idx, t, off)
    chunk = plan.autotune()
    assert chunk in (1, 2, 4, 8, 16)
    cfg = plan.config()
    assert cfg["chunk"] == chunk
    assert (cfg["tile16"], cfg["tile32"], cfg["threads"]) in ((1024, 512, 512), (512, 512, 512), (512, 256, 256),
                                                              (1024, 512, 768))
    plan.run()
    _check(plan, _oracle(insts))
    plan.close()


SHAPES = [(1024, 512, 512), (512, 512, 512), (512, 256, 256), (1024, 512, 768)]


@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_every_tile_shape_matches_oracle(gpu_lib, shape):
    """Each tile shape the autotuner can choose gives the oracle's losses and
    gradients (element by element), with chunks of 1 and 3 tiles, and
    survives a graph capture and replay."""
    import torch
    tt = gpu_lib
    ns, insts = _small_batch()
    idx, t, off = _pack(insts)
    ref = _oracle(insts)
    for chunk in (1, 3):
        print("batched tile shape", SHAPES[shape], "chunk", chunk, flush=True)
        Xs = [tt.TT.from_cores(c) for c, _, _ in insts]
        plan = tt.BatchedPlan(Xs, idx, t, off)
        plan.set_config(chunk, *SHAPES[shape])
        assert plan.config() == dict(chunk=chunk, tile16=SHAPES[shape][0], tile32=SHAPES[shape][1],
                                     threads=SHAPES[shape][2])
        plan.run()
        _check(plan, ref)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            plan.capture(s)
            plan.run(s)
        s.synchronize()
        _check(plan, ref)
        plan.close()


def test_batched_workload_256(gpu_lib):
    """The 256-tensor workload (d=8, n=16, ranks {4,8,16,32}, lognormal
    entry counts): batched equals plain for every tensor; four tensors are
    checked against the oracle.  Targets: the per-observation noise."""
    tt = gpu_lib
    inst = W.batched()
    print("batched 256 tensors, %d entries" % sum(p.M for p in inst), flush=True)
    packed = [(p.cores, p.idx, p.noise) for p in inst]
    idx, t, off = _pack(packed)
    Xs = [tt.TT.from_cores(p.cores) for p in inst]
    plan = tt.BatchedPlan(Xs, idx, t, off)
    plan.run()
    loss_b = plan.loss.cpu().numpy().copy()
    grads_b = [g.data.cpu().numpy().copy() for g in plan.grads]
    plan.run_plain()
    loss_p = plan.loss.cpu().numpy()
    for j in range(len(inst)):
        assert abs(loss_b[j] - loss_p[j]) <= TOL * loss_p[j]
        assert _rel(grads_b[j], plan.grads[j].data.cpu().numpy()) <= TOL, j
    # against the oracle: the three smallest tensors, the largest, and for
    # every rank the tensor of median entry count among that rank's tensors
    by_m = sorted(range(len(inst)), key=lambda j: inst[j].M)
    picks = by_m[:3] + by_m[-1:]
    for r in (4, 8, 16, 32):
        of_r = [j for j in by_m if inst[j].meta["rank"] == r]
        picks.append(of_r[len(of_r) // 2])
    for j in picks:
        cores, i, tj = packed[j]
        print("oracle check: tensor %d, rank %d, %d entries" % (j, inst[j].meta["rank"], inst[j].M), flush=True)
        y = oracle.gather(cores, i)
        lr, g = oracle.mse_loss_and_grad(y, tj)
        gr = oracle.gather_backward(cores, i, g)
        assert abs(loss_b[j] - lr) <= TOL * lr
        flat = np.concatenate([x.reshape(-1) for x in gr])
        assert _rel(grads_b[j], flat) <= TOL, j
        bound = np.concatenate([x.reshape(-1) for x in adjoint_bound(cores, cores, i, g)])
        assert_elementwise(grads_b[j], flat, bound, TOL, "tensor %d" % j)
    plan.close()
