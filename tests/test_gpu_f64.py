"""GPU parity of the float64 variants of Table 1's operations (the paper
times matvec, matmul, norm and gram in double precision) against the FP64
oracle: every element within 1e-12 of the same sum over absolute values
(products), the squared norm within 1e-12 relative, the Gram entries within
1e-12 sqrt(G_aa G_bb).  The float32 Gram is checked at Table 1's shape too
(100 TT vectors, d=10, n=10, rank 10)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
F64 = torch.float64


MATVEC_CASES = [
    (40, [2, 3, 5], [3, 4, 2], [1, 3, 4, 1], [1, 2, 5, 1], 3),     # ragged modes and ranks
    (41, [7], [5], [1, 1], [1, 1], 2),                              # d = 1
    (42, [3, 2, 2], [2, 2, 3], [1, 2, 2, 1], [1, 2, 3, 1], 65),     # two launches of 64 + 1
    (43, [10] * 10, [10] * 10, [1] + [10] * 9 + [1], [1] + [10] * 9 + [1], 21),  # Table 1's shape: row-block path
    (46, [3, 3, 3], [8, 8, 8], [1, 2, 2, 1], [1, 48, 48, 1], 2),   # float64 slices beyond the LDS path
    (47, [4, 3], [3, 4], [1, 20, 1], [1, 16, 1], 2),            # output rows of 320: the per-(a, i) LDS path
]


@pytest.mark.parametrize("case", range(len(MATVEC_CASES)))
def test_tt_matvec_f64(gpu_lib, case):
    tt = gpu_lib
    seed, ms, ns, rw, rx, b = MATVEC_CASES[case]
    print("matvec f64", ms, ns, rw, rx, b, flush=True)
    rng = np.random.default_rng(seed)
    Wc = [rng.standard_normal((rw[k], ms[k], ns[k], rw[k + 1])) for k in range(len(ms))]
    xs = [[rng.standard_normal((rx[k], ns[k], rx[k + 1])) for k in range(len(ms))] for _ in range(b)]
    Wm = tt.TTMatrix.from_cores(Wc, dtype=F64)
    ys = tt.tt_matvec(Wm, [tt.TT.from_cores(x, dtype=F64) for x in xs])
    absW = [np.abs(c) for c in Wc]
    for x, y in zip(xs, ys):
        assert y.data.dtype == F64
        want = oracle.tt_matvec(Wc, x)
        bound = oracle.tt_matvec(absW, [np.abs(c) for c in x])
        for g, w, bd in zip(y.numpy_cores(), want, bound):
            assert g.shape == w.shape
            assert np.all(np.abs(g - w) <= TOL * bd + 1e-300)


@pytest.mark.parametrize("case", [0, 1, 2])
def test_tt_matmat_f64(gpu_lib, case):
    tt = gpu_lib
    seed, ms, ns, ls, ra, rb = [(44, [2, 3, 5], [3, 4, 2], [2, 1, 3], [1, 3, 4, 1], [1, 2, 5, 1]),
                                (45, [10] * 4, [10] * 4, [10] * 4, [1, 10, 10, 10, 1], [1, 10, 10, 10, 1]),
                                (48, [10] * 10, [10] * 10, [10] * 10, [1] + [10] * 9 + [1],
                                 [1] + [10] * 9 + [1])][case]
    rng = np.random.default_rng(seed)
    d = len(ms)
    A = [rng.standard_normal((ra[k], ms[k], ns[k], ra[k + 1])) for k in range(d)]
    B = [rng.standard_normal((rb[k], ns[k], ls[k], rb[k + 1])) for k in range(d)]
    Cm = tt.tt_matmat(tt.TTMatrix.from_cores(A, dtype=F64), tt.TTMatrix.from_cores(B, dtype=F64))
    want = oracle.tt_matmat(A, B)
    bound = oracle.tt_matmat([np.abs(c) for c in A], [np.abs(c) for c in B])
    for g, w, bd in zip(Cm.numpy_cores(), want, bound):
        assert np.all(np.abs(g - w) <= TOL * bd + 1e-300)


NORM_CASES = [
    (50, [7], [1, 1], 3),
    (51, [5, 7, 3, 9, 4], [1, 3, 11, 6, 2, 1], 70),
    (52, [4, 4, 4], [1, 4, 64, 1], 2),
    (53, [10] * 10, [1] + [10] * 9 + [1], 100),          # Table 1's shape
    (55, [8] * 5, [1, 8, 64, 64, 8, 1], 3),              # one slice per group in float64
]


@pytest.mark.parametrize("case", range(len(NORM_CASES)))
def test_norms_f64(gpu_lib, case):
    tt = gpu_lib
    seed, ns, ranks, b = NORM_CASES[case]
    rng = np.random.default_rng(seed)
    As = [[rng.standard_normal((ranks[k], ns[k], ranks[k + 1])) / np.sqrt(max(ranks)) for k in range(len(ns))]
          for _ in range(b)]
    got = tt.norms([tt.TT.from_cores(a, dtype=F64) for a in As]).cpu().numpy()
    want2 = np.array([oracle.inner(a, a) for a in As])
    assert np.all(np.abs(got ** 2 - want2) <= TOL * want2)


def _batch(rng, count, ns, rmax, fixed=None):
    out = []
    for _ in range(count):
        r = fixed or int(rng.integers(1, rmax + 1))
        ranks = W.canonical_ranks(ns, r)
        out.append([rng.standard_normal((ranks[k], ns[k], ranks[k + 1])) / np.sqrt(r) for k in range(len(ns))])
    return out


@pytest.mark.parametrize("ns,count,rmax", [([4, 5, 3, 4], 7, 6), ([8] * 5, 13, 16), ([16] * 6, 5, 32),
                                            ([6], 3, 1)])
def test_gram_f64_symmetric(gpu_lib, ns, count, rmax):
    tt = gpu_lib
    rng = np.random.default_rng(len(ns) * 10 + count)
    As = _batch(rng, count, ns, rmax)
    G = tt.gram([tt.TT.from_cores(a, dtype=F64) for a in As]).cpu().numpy()
    ref = oracle.gram(As)
    scale = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
    assert G.dtype == np.float64
    assert np.all(np.abs(G - ref) <= TOL * scale + 1e-300)
    assert np.array_equal(G, G.T)


def test_gram_f64_two_batches(gpu_lib):
    tt = gpu_lib
    rng = np.random.default_rng(7)
    ns = [10] * 6
    As, Bs = _batch(rng, 5, ns, 32), _batch(rng, 9, ns, 20)
    G = tt.gram([tt.TT.from_cores(a, dtype=F64) for a in As], [tt.TT.from_cores(b, dtype=F64) for b in Bs])
    ref = oracle.gram(As, Bs)
    da = np.array([oracle.inner(a, a) for a in As])
    db = np.array([oracle.inner(b, b) for b in Bs])
    assert np.all(np.abs(G.cpu().numpy() - ref) <= TOL * np.sqrt(np.outer(da, db)) + 1e-300)


@pytest.mark.parametrize("dtype", [torch.float32, F64])
def test_gram_table1_shape(gpu_lib, dtype):
    """100 TT vectors with d=10, n=10, rank 10: the full Gram matrix against
    the oracle (1e-5 sqrt(G_aa G_bb) in float32, 1e-12 in float64)."""
    tt = gpu_lib
    rng = np.random.default_rng(13)
    ns = [10] * 10
    As = _batch(rng, 100, ns, 10, fixed=10)
    if dtype == torch.float32:
        As = [[c.astype(np.float32) for c in a] for a in As]
    G = tt.gram([tt.TT.from_cores(a, dtype=dtype) for a in As]).cpu().numpy().astype(np.float64)
    ref = oracle.gram(As)
    tol = 1e-5 if dtype == torch.float32 else TOL
    scale = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
    assert np.all(np.abs(G - ref) <= tol * scale)


def test_f64_descriptor_refused_by_float32_entry_points(gpu_lib):
    """A float64 TT cannot reach a float32-only entry point: the argument
    types refuse its descriptor before any call."""
    import ctypes
    tt = gpu_lib
    X = tt.TT.from_cores([np.ones((1, 3, 2)), np.ones((2, 3, 1))], dtype=F64)
    with pytest.raises(ctypes.ArgumentError):
        tt.gather(X, np.zeros((2, 4), np.int32))
