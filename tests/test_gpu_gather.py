"""GPU parity of the gather, its adjoint and the fused MSE pass against the
FP64 oracle: 1e-5 relative normwise, and every element within 1e-5 of its
absolute-value bound (each entry against the product of its absolute
slices, each gradient element against the sum of |w| |L| |R| over its
entries)."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_adjoint, assert_elementwise, assert_gather, adjoint_bound, gather_bound

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _case(seed, ns, ranks, M, std=None):
    rng = np.random.default_rng(seed)
    std = std if std is not None else 1.0 / np.sqrt(max(ranks))
    cores = W.random_cores(rng, ns, ranks, std)
    idx = W.random_indices(rng, ns, M)
    g = rng.standard_normal(M).astype(np.float32)
    return cores, idx, g


CASES = [
    # (seed, ns, ranks, M)  -- several tiles plus a ragged tail, uneven ranks
    (1, [8, 8, 8, 8], [1, 4, 4, 4, 1], 4096),
    (2, [10] * 10, [1] + [16] * 9 + [1], 70001),
    (3, [10] * 10, [1, 10, 32, 32, 32, 32, 32, 32, 32, 10, 1], 20011),
    (4, [16] * 8, [1] + [8] * 7 + [1], 33333),
    (5, [5, 7, 3, 9, 4], [1, 3, 11, 6, 2, 1], 9999),
    (6, [3, 4], [1, 3, 1], 257),
    (7, [13], [1, 1], 100),                       # d = 1
    (8, [6, 6, 6], [1, 40, 40, 1], 3001),         # rank above 32
    (9, [4, 4, 4, 4], [1, 4, 16, 4, 1], 1),       # a single entry
    (12, [2] * 32, [1] + [3] * 31 + [1], 5000),   # d = TT_MAX_D (generic kernels)
    (13, [4096, 3], [1, 5, 1], 20000),            # n = TT_MAX_N
    (14, [40, 50, 30], [1, 8, 8, 1], 10000),      # modes above the MFMA classes' sizes
    # rank class 32 with slices that span several waves of a tile (the
    # slice sums of later waves are merged in rounds), one-slice modes
    (15, [2] * 6, [1] + [32] * 5 + [1], 40000),
    (16, [1, 5, 2, 1, 3], [1, 32, 32, 32, 32, 1], 30011),
]


def _ids(c):
    return "seed%d-d%d-M%d" % (c[0], len(c[1]), c[3])


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_gather_and_backward_parity(gpu_lib, case):
    import torch
    tt = gpu_lib
    seed, ns, ranks, M = case
    print("case", _ids(case), flush=True)
    cores, idx, g = _case(seed, ns, ranks, M)
    X = tt.TT.from_cores(cores)
    y = tt.gather(X, idx).cpu().numpy()
    yr = oracle.gather(cores, idx)
    assert _rel(y, yr) <= TOL
    assert_gather(y, yr, cores, idx, TOL)
    gX = tt.gather_backward(X, idx, torch.from_numpy(g))
    gr = oracle.gather_backward(cores, idx, g)
    got = gX.numpy_cores()
    for k in range(len(ns)):
        assert _rel(got[k], gr[k]) <= TOL, (k, _rel(got[k], gr[k]))
    assert_adjoint(got, gr, cores, cores, idx, g, TOL)


def test_empty_entries(gpu_lib):
    import torch
    tt = gpu_lib
    cores, _, _ = _case(11, [4, 5, 6], [1, 3, 2, 1], 1)
    X = tt.TT.from_cores(cores)
    idx = np.zeros((3, 0), np.int32)
    assert tt.gather(X, idx).numel() == 0
    gX = tt.gather_backward(X, idx, torch.zeros(0))
    assert float(gX.data.abs().max()) == 0.0
    y, loss, gX = tt.gather_mse_backward(X, idx, torch.zeros(0))
    assert float(loss.item()) == 0.0 and float(gX.data.abs().max()) == 0.0


def test_duplicates_and_repeatability(gpu_lib):
    import torch
    tt = gpu_lib
    cores, idx, g = _case(12, [3, 3, 3], [1, 2, 2, 1], 500)
    idx = np.concatenate([idx, idx[:, :200]], axis=1)
    g = np.concatenate([g, g[:200]])
    X = tt.TT.from_cores(cores)
    a = tt.gather_backward(X, idx, torch.from_numpy(g))
    b = tt.gather_backward(X, idx, torch.from_numpy(g))
    # repeated calls agree to rounding (LDS accumulation order may vary)
    assert _rel(a.data.cpu().numpy(), b.data.cpu().numpy()) <= 1e-6
    gr = oracle.gather_backward(cores, idx, g)
    for k, c in enumerate(a.numpy_cores()):
        assert _rel(c, gr[k]) <= TOL
    assert_adjoint(a.numpy_cores(), gr, cores, cores, idx, g, TOL)


@pytest.mark.parametrize("M", [4096, 100003])
def test_fused_mse_parity(gpu_lib, M):
    tt = gpu_lib
    p = W.gather_d10(M=M)
    X = tt.TT.from_cores(p.cores)
    t = (oracle.gather(p.planted, p.idx) + p.noise).astype(np.float32)
    y, loss, gX = tt.gather_mse_backward(X, p.idx, t)
    yr = oracle.gather(p.cores, p.idx)
    lr, gr = oracle.mse_loss_and_grad(yr, t)
    assert _rel(y.cpu().numpy(), yr) <= TOL
    assert_gather(y.cpu().numpy(), yr, p.cores, p.idx, TOL)
    assert abs(float(loss.item()) - lr) <= TOL * lr
    grr = oracle.gather_backward(p.cores, p.idx, gr)
    for k, c in enumerate(gX.numpy_cores()):
        assert _rel(c, grr[k]) <= TOL, k
    assert_adjoint(gX.numpy_cores(), grr, p.cores, p.cores, p.idx, gr, TOL, "fused MSE")


def test_autograd_function(gpu_lib):
    import torch
    tt = gpu_lib
    cores, idx, g = _case(13, [6, 5, 7, 4], [1, 5, 6, 3, 1], 5000)
    X = tt.TT.from_cores(cores)
    X.data.requires_grad_(True)
    y = tt.tt_gather(X, idx)
    y.backward(torch.from_numpy(g).cuda())
    gr = oracle.gather_backward(cores, idx, g)
    flat = np.concatenate([x.reshape(-1) for x in gr])
    assert _rel(X.data.grad.cpu().numpy(), flat) <= TOL
    bound = np.concatenate([x.reshape(-1) for x in adjoint_bound(cores, cores, idx, g)])
    assert_elementwise(X.data.grad.cpu().numpy(), flat, bound, TOL, "autograd")


@pytest.fixture(scope="module")
def full_d10():
    """The d=10, n=10, r=16 workload at 2^20 entries with its oracle results."""
    p = W.gather_d10()
    t = (oracle.gather(p.planted, p.idx) + p.noise).astype(np.float32)
    yr = oracle.gather(p.cores, p.idx)
    lr, gr = oracle.mse_loss_and_grad(yr, t)
    grads = oracle.gather_backward(p.cores, p.idx, gr)
    ybound = gather_bound(p.cores, p.idx)
    gbound = adjoint_bound(p.cores, p.cores, p.idx, gr)
    return p, t, yr, lr, grads, ybound, gbound


def test_full_size_d10_r16(gpu_lib, full_d10):
    """Full size (2^20 entries) in the launch configuration the benchmark
    times: every output compared with the oracle."""
    tt = gpu_lib
    p, t, yr, lr, grads, ybound, gbound = full_d10
    print("full d10 r16 M=2^20", flush=True)
    X = tt.TT.from_cores(p.cores)
    y, loss, gX = tt.gather_mse_backward(X, p.idx, t)
    assert _rel(y.cpu().numpy(), yr) <= TOL
    assert_elementwise(y.cpu().numpy(), yr, ybound, TOL, "y")
    assert abs(float(loss.item()) - lr) <= TOL * lr
    for k, c in enumerate(gX.numpy_cores()):
        assert _rel(c, grads[k]) <= TOL, (k, _rel(c, grads[k]))
        assert_elementwise(c, grads[k], gbound[k], TOL, "core %d" % k)


def test_full_size_finite_differences(gpu_lib, full_d10):
    """64 random core entries: exact central differences of the FP64 loss
    agree with the GPU gradient."""
    tt = gpu_lib
    p, t, yr, lr, grads, ybound, gbound = full_d10
    X = tt.TT.from_cores(p.cores)
    _, _, gX = tt.gather_mse_backward(X, p.idx, t)
    got = np.concatenate([c.reshape(-1) for c in gX.numpy_cores()])
    flat = np.concatenate([c.reshape(-1).astype(np.float64) for c in p.cores])
    sizes = [c.size for c in p.cores]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    rng = np.random.default_rng(16)
    pick = rng.choice(flat.size, size=64, replace=False)
    sub = np.arange(0, p.M, 16)   # every 16th entry keeps the FP64 loss cheap
    idx = p.idx[:, sub]
    ts = t[sub].astype(np.float64)
    base = [c.astype(np.float64) for c in p.cores]
    yb = oracle.gather(base, idx)
    _, gs = oracle.mse_loss_and_grad(yb, ts)
    gsub = np.concatenate([c.reshape(-1) for c in oracle.gather_backward(base, idx, gs)])
    fd, an = [], []
    for j in pick:
        k = int(np.searchsorted(offs, j, side="right") - 1)
        pos = np.unravel_index(j - offs[k], p.cores[k].shape)
        mask = idx[k] == pos[1]          # only entries through this slice change
        h = 0.1 * max(1.0, abs(flat[j]))
        vals = []
        for s in (1, -1):
            cs = list(base)
            cs[k] = base[k].copy()
            cs[k][pos] += s * h
            yp = yb.copy()
            yp[mask] = oracle.gather(cs, idx[:, mask])
            vals.append(oracle.mse_loss_and_grad(yp, ts)[0])
        fd.append((vals[0] - vals[1]) / (2 * h))
        an.append(gsub[j])
    assert _rel(an, fd) <= 1e-8          # the oracle gradient is exact
    ref = np.concatenate([c.reshape(-1) for c in grads])
    bnd = np.concatenate([c.reshape(-1) for c in gbound])
    assert _rel(got[pick], ref[pick]) <= TOL
    # each picked entry on its own, against the full-set oracle gradient
    for j in pick:
        assert abs(got[j] - ref[j]) <= TOL * bnd[j], (int(j), got[j], ref[j], bnd[j])


def test_fused_pass_graph_replays(gpu_lib):
    """The fused pass captured into a hipGraph (through torch.cuda.graph) and
    replayed three times, with new targets written and an eager call made
    between replays: every replay equals the eager result bit for bit (the
    rank-16 path sums in a fixed order)."""
    import torch
    tt = gpu_lib
    p = W.small_step(M=5000)
    ns, ranks = p.ns, [1] + [16] * (len(p.ns) - 1) + [1]
    rng = np.random.default_rng(77)
    cores = [(rng.standard_normal((ranks[k], ns[k], ranks[k + 1])) / 4).astype(np.float32) for k in range(len(ns))]
    X = tt.TT.from_cores(cores)
    idx = torch.as_tensor(p.idx).cuda()
    t = torch.zeros(p.M, device="cuda")
    nbytes = tt.gather_mse_workspace(X, p.M)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ws_ref = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    gX, loss = X.empty_like(), torch.empty(1, device="cuda")
    gX_ref, loss_ref = X.empty_like(), torch.empty(1, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tt.gather_mse_backward(X, idx, t, want_y=False, ws=ws, out=gX, loss=loss)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        tt.gather_mse_backward(X, idx, t, want_y=False, ws=ws, out=gX, loss=loss)
    for rep in range(3):
        t.copy_(torch.as_tensor(rng.standard_normal(p.M).astype(np.float32)).cuda())
        tt.gather_mse_backward(X, idx, t, want_y=False, ws=ws_ref, out=gX_ref, loss=loss_ref)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(gX.data, gX_ref.data), rep
        assert torch.equal(loss, loss_ref), rep
        # and against the oracle
        y = oracle.gather(cores, p.idx)
        tr = t.cpu().numpy().astype(np.float64)
        g = 2.0 * (y - tr) / p.M
        ref = oracle.gather_backward(cores, p.idx, g)
        got = tt.TT(ns, ranks, gX.data).numpy_cores()
        for a, b in zip(got, ref):
            assert _rel(a, b) <= TOL
        assert_adjoint(got, ref, cores, cores, p.idx, g, TOL, "replay %d" % rep)


RANK64_CASES = [
    (51, [10] * 10, W.canonical_ranks([10] * 10, 64), 70001),   # tangent rank of a rank-32 point
    (52, [16, 16, 16, 16], [1, 16, 64, 16, 1], 30001),
    (53, [6, 6, 6], [1, 6, 36, 1], 1000),
    (54, [5, 9, 7, 3], [1, 5, 45, 21, 1], 257),
]


@pytest.mark.parametrize("case", range(len(RANK64_CASES)))
def test_gather_rank64_class(gpu_lib, case):
    """Ranks 33..64 take the rank-64 MFMA gather (tiles of 256 entries):
    parity with the oracle gather, several tiles and a ragged tail."""
    import torch
    tt = gpu_lib
    seed, ns, ranks, M = RANK64_CASES[case]
    print("rank-64 gather", ns, max(ranks), M, flush=True)
    rng = np.random.default_rng(seed)
    cores = W.random_cores(rng, ns, ranks, 1 / np.sqrt(max(ranks)))
    idx = W.random_indices(rng, ns, M)
    X = tt.TT.from_cores(cores)
    y = tt.gather(X, torch.as_tensor(idx).cuda()).cpu().numpy()
    yr = oracle.gather(cores, idx)
    assert _rel(y, yr) <= TOL
    assert_gather(y, yr, cores, idx, TOL)
