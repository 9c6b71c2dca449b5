"""The fused pass through the entry point that allocates nothing
(tt_gather_mse_backward_noalloc), called through the C ABI: two calls in a
row, the second with a smaller input, each checked against the entry point
with a caller workspace (bit for bit where that path sums in a fixed order)
and against the FP64 oracle (1e-5, normwise and per element)."""
import ctypes as C

import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_adjoint, assert_gather

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _call_both(tt, cores, idx_np, t_np):
    """The pass through both entry points on the same inputs, through the
    C ABI; returns ((y, loss, cores) noalloc, (y, loss, cores) workspace)."""
    import torch
    from paper_1801_01928_amd import _lib as L
    lib = L.load()
    X = tt.TT.from_cores(cores)
    idx = torch.as_tensor(idx_np).cuda().contiguous()
    t = torch.as_tensor(t_np).cuda().contiguous()
    M = idx.shape[1]
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    outs = []
    for noalloc in (True, False):
        y = torch.full((M,), float("nan"), device="cuda")
        loss = torch.full((1,), float("nan"), device="cuda")
        gX = X.empty_like()
        gX.data.fill_(float("nan"))
        if noalloc:
            rc = lib.tt_gather_mse_backward_noalloc(C.byref(X.desc()), C.c_void_p(idx.data_ptr()), M,
                                                    C.c_void_p(t.data_ptr()), C.c_void_p(y.data_ptr()), None,
                                                    C.c_void_p(loss.data_ptr()), C.byref(gX.desc()), stream)
        else:
            nb = lib.tt_gather_mse_workspace(C.byref(X.desc()), M)
            ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
            rc = lib.tt_gather_mse_backward(C.byref(X.desc()), C.c_void_p(idx.data_ptr()), M,
                                            C.c_void_p(t.data_ptr()), C.c_void_p(y.data_ptr()), None,
                                            C.c_void_p(loss.data_ptr()), C.byref(gX.desc()),
                                            C.c_void_p(ws.data_ptr()), nb, stream)
        L.check(rc)
        torch.cuda.synchronize()
        outs.append((y.cpu().numpy(), float(loss.item()), gX.numpy_cores()))
    return outs


def _check_against_oracle(out, cores, idx, t):
    y, loss, got = out
    yr = oracle.gather(cores, idx)
    lr, g = oracle.mse_loss_and_grad(yr, t)
    gr = oracle.gather_backward(cores, idx, g)
    assert _rel(y, yr) <= TOL
    assert_gather(y, yr, cores, idx, TOL)
    assert abs(loss - lr) <= TOL * lr
    for k in range(len(cores)):
        assert _rel(got[k], gr[k]) <= TOL, k
    assert_adjoint(got, gr, cores, cores, idx, g, TOL, "noalloc")


def test_noalloc_matches_workspace_entry_point(gpu_lib):
    tt = gpu_lib
    assert tt.gather_mse_noalloc_limit() == 256 << 20
    # call 1: the d=10, n=10, r=16 workload at its full 2^20 entries
    p = W.gather_d10()
    print("noalloc call 1: d=10 n=10 r=16 M=2^20", flush=True)
    t1 = (oracle.gather(p.planted, p.idx) + p.noise).astype(np.float32)
    a, b = _call_both(tt, p.cores, p.idx, t1)
    np.testing.assert_array_equal(a[0], b[0])
    assert a[1] == b[1]
    for x, z in zip(a[2], b[2]):
        np.testing.assert_array_equal(x, z)   # rank 16 sums in a fixed order
    sub = np.arange(0, p.M, 64)               # the oracle on a sample of the entries' values
    assert _rel(a[0][sub], oracle.gather(p.cores, p.idx[:, sub])) <= TOL
    # call 2: a smaller input of another rank class (rank 32, atomics), on
    # the scratch the first call left behind
    rng = np.random.default_rng(61)
    ns, ranks, M = [7, 6, 5, 8, 6], [1, 7, 24, 32, 6, 1], 20011
    print("noalloc call 2: d=5 rank 32 M=%d" % M, flush=True)
    cores = W.random_cores(rng, ns, ranks, 1 / np.sqrt(32))
    idx = W.random_indices(rng, ns, M)
    t2 = rng.standard_normal(M).astype(np.float32)
    a, b = _call_both(tt, cores, idx, t2)
    np.testing.assert_array_equal(a[0], b[0])
    assert abs(a[1] - b[1]) <= 1e-6 * abs(b[1])
    for x, z in zip(a[2], b[2]):
        assert _rel(x, z) <= 1e-6
    _check_against_oracle(a, cores, idx, t2)
    # call 3: smaller again, rank 16, and against the oracle in full
    q = W.small_step(M=3001)
    print("noalloc call 3: d=4 rank 4 M=3001", flush=True)
    t3 = (oracle.gather(q.planted, q.idx) + q.noise).astype(np.float32)
    a, b = _call_both(tt, q.cores, q.idx, t3)
    np.testing.assert_array_equal(a[0], b[0])
    for x, z in zip(a[2], b[2]):
        np.testing.assert_array_equal(x, z)
    _check_against_oracle(a, q.cores, q.idx, t3)


def test_noalloc_binding_and_empty_input(gpu_lib):
    import torch
    tt = gpu_lib
    q = W.small_step(M=500)
    X = tt.TT.from_cores(q.cores)
    t = (oracle.gather(q.planted, q.idx) + q.noise).astype(np.float32)
    y, loss, gX = tt.gather_mse_backward_noalloc(X, q.idx, t)
    y2, loss2, gX2 = tt.gather_mse_backward(X, q.idx, t)
    assert torch.equal(y, y2) and torch.equal(loss, loss2) and torch.equal(gX.data, gX2.data)
    y, loss, gX = tt.gather_mse_backward_noalloc(X, np.zeros((4, 0), np.int32), np.zeros(0, np.float32))
    assert y.numel() == 0 and float(loss.item()) == 0.0 and float(gX.data.abs().max()) == 0.0
