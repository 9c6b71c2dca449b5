"""GPU parity of the TT-matrix layer (Y = X W^T, dX = dY W, dG^k) against the
FP64 oracle, which materialises W.

float32: normwise relative error <= 1e-5 for Y and dX and per core for dG
(fp32 sums of at most a few thousand products per MFMA accumulator, then a
fixed-order sum of partials).  bf16 (inputs, cores and intermediates in
bfloat16, float32 accumulation): the oracle is fed the same bf16-rounded
inputs; each of the d-1 intermediates is rounded to bf16 once (relative
error <= 2^-9 per element), so the bound is (d-1) * 2^-8 normwise."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from parity import assert_elementwise

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _case(seed, ms, ns, ranks, B):
    rng = np.random.default_rng(seed)
    r = max(ranks)
    cores = [(rng.standard_normal((ranks[k], ms[k], ns[k], ranks[k + 1])) / np.sqrt(r)).astype(np.float32)
             for k in range(len(ms))]
    X = rng.standard_normal((B, int(np.prod(ns)))).astype(np.float32)
    dY = rng.standard_normal((B, int(np.prod(ms)))).astype(np.float32)
    return cores, X, dY


def _bf16(a):
    return torch.as_tensor(a).to(torch.bfloat16)


@pytest.fixture(params=["chain", "dense"])
def ttm_path(gpu_lib, request):
    """Each layer test runs on both evaluation paths (one core per step;
    W built once and multiplied on the matrix cores)."""
    tt = gpu_lib
    tt.ttm_set_path(request.param)
    yield tt
    tt.ttm_set_path("auto")


CASES = [
    ([4, 4, 4], [4, 4, 4], [1, 8, 8, 1], 64),
    ([2, 3, 5], [4, 2, 3], [1, 3, 7, 1], 37),          # ragged batch, odd sizes
    ([7], [5], [1, 1], 19),                            # d = 1: a dense matrix
    ([4, 4, 4, 4, 4], [4, 4, 4, 4, 4], [1, 32, 32, 32, 32, 1], 70),
    ([8, 2, 4], [2, 4, 4], [1, 16, 32, 1], 129),       # m r = 128 (largest fused step)
    ([3, 3, 3, 3], [2, 2, 2, 2], [1, 1, 1, 1, 1], 33),  # rank 1
    ([16, 8], [8, 16], [1, 8, 1], 200),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fp32_forward_backward(ttm_path, case):
    tt = ttm_path
    ms, ns, ranks, B = CASES[case]
    print("ttm fp32", ms, ns, ranks, B, flush=True)
    cores, X, dY = _case(500 + case, ms, ns, ranks, B)
    Wm = tt.TTMatrix.from_cores(cores)
    Xg = torch.as_tensor(X).cuda()
    dYg = torch.as_tensor(dY).cuda()
    Y = tt.ttm_matmul(Wm, Xg).cpu().numpy()
    assert rel(Y, oracle.ttm_forward(X, cores)) <= 1e-5
    dX, dG = tt.ttm_matmul_backward(Wm, Xg, dYg)
    rdX, rdG = oracle.ttm_backward(X, cores, dY)
    assert rel(dX.cpu().numpy(), rdX) <= 1e-5
    got = tt.TTMatrix(ms, ns, ranks, dG).numpy_cores()
    for g, r in zip(got, rdG):
        assert rel(g, r) <= 1e-5
    # outputs requested one at a time agree with the joint call bit for bit
    dX2, none = tt.ttm_matmul_backward(Wm, Xg, dYg, want_dw=False)
    assert none is None and torch.equal(dX2, dX)
    none, dG2 = tt.ttm_matmul_backward(Wm, Xg, dYg, want_dx=False)
    assert none is None and torch.equal(dG2, dG)


@pytest.mark.parametrize("case", [0, 1, 3, 4])
def test_bf16_forward_backward(ttm_path, case):
    tt = ttm_path
    ms, ns, ranks, B = CASES[case]
    print("ttm bf16", ms, ns, ranks, B, flush=True)
    cores, X, dY = _case(600 + case, ms, ns, ranks, B)
    cb = [_bf16(c) for c in cores]
    Xb, dYb = _bf16(X), _bf16(dY)
    # the oracle sees exactly the bf16 values
    c64 = [c.double().numpy() for c in cb]
    X64, dY64 = Xb.double().numpy(), dYb.double().numpy()
    Wm = tt.TTMatrix.from_cores(cb, dtype=torch.bfloat16)
    tol = max(len(ms) - 1, 1) * 2.0 ** -8
    Y = tt.ttm_matmul(Wm, Xb.cuda()).cpu().numpy()
    assert rel(Y, oracle.ttm_forward(X64, c64)) <= tol
    dX, dG = tt.ttm_matmul_backward(Wm, Xb.cuda(), dYb.cuda())
    rdX, rdG = oracle.ttm_backward(X64, c64, dY64)
    assert rel(dX.cpu().numpy(), rdX) <= tol
    got = tt.TTMatrix(ms, ns, ranks, dG).numpy_cores()
    for g, r in zip(got, rdG):
        assert rel(g, r) <= tol


def test_empty_batch(ttm_path):
    tt = ttm_path
    cores, X, dY = _case(700, [4, 4], [4, 4], [1, 4, 1], 0)
    Wm = tt.TTMatrix.from_cores(cores)
    Y = tt.ttm_matmul(Wm, torch.zeros((0, 16), device="cuda"))
    assert Y.shape == (0, 16)
    dX, dG = tt.ttm_matmul_backward(Wm, torch.zeros((0, 16), device="cuda"), torch.zeros((0, 16), device="cuda"))
    assert dX.shape == (0, 16)
    assert float(dG.abs().max()) == 0.0


def test_autograd_and_finite_differences(ttm_path):
    """tt_linear through torch.autograd; L = <dY, Y> is linear in every core
    entry, so a central difference with a large step is exact up to fp32
    rounding of the forward."""
    tt = ttm_path
    ms, ns, ranks, B = [4, 4, 4], [4, 4, 4], [1, 8, 8, 1], 96
    cores, X, dY = _case(800, ms, ns, ranks, B)
    Wm = tt.TTMatrix.from_cores(cores)
    flat = Wm.data.clone().requires_grad_(True)
    Wv = tt.TTMatrix(ms, ns, ranks, flat)
    x = torch.as_tensor(X).cuda().requires_grad_(True)
    Y = tt.tt_linear(x, Wv)
    dYg = torch.as_tensor(dY).cuda()
    (Y * dYg).sum().backward()
    rdX, rdG = oracle.ttm_backward(X, cores, dY)
    assert rel(x.grad.cpu().numpy(), rdX) <= 1e-5
    assert rel(flat.grad.cpu().numpy(), np.concatenate([g.reshape(-1) for g in rdG])) <= 1e-5
    rng = np.random.default_rng(801)
    scale = float(np.linalg.norm(dY) * np.linalg.norm(oracle.ttm_forward(X, cores)))
    for _ in range(16):
        e = int(rng.integers(0, Wm.data.numel()))
        h = 0.5
        vals = []
        for s in (1.0, -1.0):
            d2 = Wm.data.clone()
            d2[e] += s * h
            Yp = tt.ttm_matmul(tt.TTMatrix(ms, ns, ranks, d2), x.detach())
            vals.append(float((Yp.double() * dYg.double()).sum()))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - float(flat.grad[e])) <= 1e-5 * scale


def test_ttm_layer_full_size(ttm_path):
    """The 1024 x 1024 layer (modes 4^5, r = 32) on a batch of 4096 rows,
    float32, against the full oracle; the Euler identity <dG^k, G^k> = <dY, Y>
    holds for every core."""
    tt = ttm_path
    p = W.ttm_layer()
    print("ttm layer 4096 x 1024, r = 32", flush=True)
    Wm = tt.TTMatrix.from_cores(p.cores)
    Xg = torch.as_tensor(p.X).cuda()
    dYg = torch.as_tensor(p.dY).cuda()
    Y = tt.ttm_matmul(Wm, Xg).cpu().numpy()
    dX, dG = tt.ttm_matmul_backward(Wm, Xg, dYg)
    rY = oracle.ttm_forward(p.X, p.cores)
    assert rel(Y, rY) <= 1e-5
    rdX, rdG = oracle.ttm_backward(p.X, p.cores, p.dY)
    assert rel(dX.cpu().numpy(), rdX) <= 1e-5
    # absolute-value sums of the same products bound every element
    aX, aC, adY = np.abs(p.X), [np.abs(c) for c in p.cores], np.abs(p.dY)
    bY = oracle.ttm_forward(aX, aC)
    bdX, bdG = oracle.ttm_backward(aX, aC, adY)
    assert_elementwise(Y, rY, bY, 1e-5, "Y")
    assert_elementwise(dX.cpu().numpy(), rdX, bdX, 1e-5, "dX")
    got = tt.TTMatrix(p.row_modes, p.col_modes, p.ranks, dG).numpy_cores()
    L0 = float(np.sum(p.dY.astype(np.float64) * rY))
    for k, (g, r) in enumerate(zip(got, rdG)):
        assert rel(g, r) <= 1e-5, (k, rel(g, r))
        assert_elementwise(g, r, bdG[k], 1e-5, "dG core %d" % k)
        euler = float(np.sum(g.astype(np.float64) * p.cores[k]))
        assert abs(euler - L0) <= 1e-5 * np.linalg.norm(g) * np.linalg.norm(p.cores[k])


def test_ttm_layer_full_size_bf16(ttm_path):
    tt = ttm_path
    p = W.ttm_layer()
    print("ttm layer bf16", flush=True)
    cb = [_bf16(c) for c in p.cores]
    Xb, dYb = _bf16(p.X), _bf16(p.dY)
    Wm = tt.TTMatrix.from_cores(cb, dtype=torch.bfloat16)
    Y = tt.ttm_matmul(Wm, Xb.cuda()).cpu().numpy()
    c64 = [c.double().numpy() for c in cb]
    X64, dY64 = Xb.double().numpy(), dYb.double().numpy()
    tol = 4 * 2.0 ** -8
    assert rel(Y, oracle.ttm_forward(X64, c64)) <= tol
    dX, dG = tt.ttm_matmul_backward(Wm, Xb.cuda(), dYb.cuda())
    rdX, rdG = oracle.ttm_backward(X64, c64, dY64)
    assert rel(dX.cpu().numpy(), rdX) <= tol
    got = tt.TTMatrix(p.row_modes, p.col_modes, p.ranks, dG).numpy_cores()
    for g, r in zip(got, rdG):
        assert rel(g, r) <= tol


MATVEC_CASES = [
    # (seed, row modes, column modes, W ranks, x ranks, vectors)
    (40, [2, 3, 5], [3, 4, 2], [1, 3, 4, 1], [1, 2, 5, 1], 3),     # ragged modes and ranks
    (41, [7], [5], [1, 1], [1, 1], 2),                              # d = 1: a dense matvec
    (42, [3, 2, 2], [2, 2, 3], [1, 2, 2, 1], [1, 2, 3, 1], 65),     # two launches of 64 + 1
    (43, [10] * 10, [10] * 10, [1] + [10] * 9 + [1], [1] + [10] * 9 + [1], 21),  # d=10, rank 10 x 10: row-block path
    (46, [3, 3, 3], [8, 8, 8], [1, 2, 2, 1], [1, 64, 64, 1], 2),   # x core 64x8x64: beyond LDS, grid-stride path
    (47, [4, 3], [3, 4], [1, 20, 1], [1, 16, 1], 2),            # output rows of 320: the per-(a, i) LDS path
]


@pytest.mark.parametrize("case", range(len(MATVEC_CASES)))
def test_tt_matvec_matches_oracle(gpu_lib, case):
    """tt_matvec against the oracle's TT-format product, core by core: every
    element within 1e-5 of the same sum taken over absolute values."""
    tt = gpu_lib
    seed, ms, ns, rw, rx, b = MATVEC_CASES[case]
    print("matvec", ms, ns, rw, rx, b, flush=True)
    rng = np.random.default_rng(seed)
    Wc = [rng.standard_normal((rw[k], ms[k], ns[k], rw[k + 1])).astype(np.float32) for k in range(len(ms))]
    xs = [[rng.standard_normal((rx[k], ns[k], rx[k + 1])).astype(np.float32) for k in range(len(ms))]
          for _ in range(b)]
    W = tt.TTMatrix.from_cores(Wc)
    ys = tt.tt_matvec(W, [tt.TT.from_cores(x) for x in xs])
    absW = [np.abs(c) for c in Wc]
    for x, y in zip(xs, ys):
        want = oracle.tt_matvec(Wc, x)
        bound = oracle.tt_matvec(absW, [np.abs(c) for c in x])
        got = y.numpy_cores()
        assert [g.shape for g in got] == [w.shape for w in want]
        for g, w, bd in zip(got, want, bound):
            assert np.all(np.abs(g.astype(np.float64) - w) <= 1e-5 * bd + 1e-30)


MATMAT_CASES = [
    # (seed, row modes, inner modes, column modes, A ranks, B ranks)
    (44, [2, 3, 5], [3, 4, 2], [2, 1, 3], [1, 3, 4, 1], [1, 2, 5, 1]),
    (45, [10] * 4, [10] * 4, [10] * 4, [1, 10, 10, 10, 1], [1, 10, 10, 10, 1]),
    # Table 1's shape (d=10, modes 10, ranks 10): row chunks of 4, 4 and 2
    (48, [10] * 10, [10] * 10, [10] * 10, [1] + [10] * 9 + [1], [1] + [10] * 9 + [1]),
]


@pytest.mark.parametrize("case", range(len(MATMAT_CASES)))
def test_tt_matmat_matches_oracle(gpu_lib, case):
    """tt_matmat against the oracle's TT-format product, core by core, each
    element within 1e-5 of its absolute-value sum."""
    tt = gpu_lib
    seed, ms, ns, ls, ra, rb = MATMAT_CASES[case]
    print("matmat", ms, ns, ls, ra, rb, flush=True)
    rng = np.random.default_rng(seed)
    d = len(ms)
    A = [rng.standard_normal((ra[k], ms[k], ns[k], ra[k + 1])).astype(np.float32) for k in range(d)]
    B = [rng.standard_normal((rb[k], ns[k], ls[k], rb[k + 1])).astype(np.float32) for k in range(d)]
    Cm = tt.tt_matmat(tt.TTMatrix.from_cores(A), tt.TTMatrix.from_cores(B))
    flat = Cm.data.cpu().numpy().astype(np.float64)
    want = oracle.tt_matmat(A, B)
    bound = oracle.tt_matmat([np.abs(c) for c in A], [np.abs(c) for c in B])
    for k in range(d):
        got = flat[Cm.offs[k]:Cm.offs[k + 1]].reshape(want[k].shape)
        assert np.all(np.abs(got - want[k]) <= 1e-5 * bound[k] + 1e-30)
