"""GPU parity of the Gram matrix of TT batches against the FP64 oracle:
|G_ab - G_ab^ref| <= 1e-5 sqrt(G_aa G_bb) (Cauchy-Schwarz scale)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _batch(seed, count, ns, rmax, rng_ranks=True):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        r = int(rng.integers(1, rmax + 1)) if rng_ranks else rmax
        ranks = W.canonical_ranks(ns, r)
        out.append(W.random_cores(rng, ns, ranks, 1.0 / np.sqrt(r)))
    return out


def _check(G, ref, diagA, diagB):
    scale = np.sqrt(np.outer(diagA, diagB))
    assert np.all(np.abs(G - ref) <= 1e-5 * scale + 1e-30), np.max(np.abs(G - ref) / scale)


@pytest.mark.parametrize("ns,count,rmax", [([4, 5, 3, 4], 7, 6), ([8] * 5, 13, 16),
                                            ([16] * 8, 9, 32), ([3, 3], 5, 3), ([6], 6, 1)])
def test_gram_symmetric(gpu_lib, ns, count, rmax):
    tt = gpu_lib
    As = _batch(len(ns) * 100 + count, count, ns, rmax)
    G = tt.gram([tt.TT.from_cores(a) for a in As]).cpu().numpy()
    ref = oracle.gram(As)
    _check(G, ref, np.diag(ref), np.diag(ref))
    assert np.array_equal(G, G.T)


def test_gram_two_batches(gpu_lib):
    tt = gpu_lib
    ns = [10] * 6
    As = _batch(1, 6, ns, 32)
    Bs = _batch(2, 11, ns, 20)
    G = tt.gram([tt.TT.from_cores(a) for a in As], [tt.TT.from_cores(b) for b in Bs]).cpu().numpy()
    ref = oracle.gram(As, Bs)
    _check(G, ref, [oracle.inner(a, a) for a in As], [oracle.inner(b, b) for b in Bs])


def test_gram_batched_workload_sampled(gpu_lib):
    """The 256-instance batched workload (d=8, n=16, ranks in {4,8,16,32}):
    the full Gram on the GPU, the diagonal and 300 sampled pairs in FP64."""
    tt = gpu_lib
    inst = W.batched()
    print("gram 256 x 256", flush=True)
    G = tt.gram([tt.TT.from_cores(p.cores) for p in inst]).cpu().numpy()
    cores = [[c.astype(np.float64) for c in p.cores] for p in inst]
    diag = np.array([oracle.inner(c, c) for c in cores])
    assert np.all(np.abs(np.diag(G) - diag) <= 1e-5 * diag)
    rng = np.random.default_rng(44)
    for _ in range(300):
        a, b = rng.integers(0, len(inst), size=2)
        ref = oracle.inner(cores[a], cores[b])
        assert abs(G[a, b] - ref) <= 1e-5 * np.sqrt(diag[a] * diag[b])
    assert np.array_equal(G, G.T)


NORM_CASES = [
    # (seed, ns, ranks, members)
    (50, [7], [1, 1], 3),                                   # d = 1
    (51, [5, 7, 3, 9, 4], [1, 3, 11, 6, 2, 1], 70),         # ragged; two launches of 64 + 6
    (52, [4, 4, 4], [1, 4, 64, 1], 2),                      # rank 64 (the limit)
    (53, [10] * 10, [1] + [10] * 9 + [1], 100),             # d=10, rank 10, batch 100
    (54, [10] * 4, [1, 10, 32, 32, 1], 5),                  # r r' = 1024: groups of 8 slices, then 2
    (55, [8] * 5, [1, 8, 64, 64, 8, 1], 3),                 # r r' = 4096: four groups of 2 slices
]


@pytest.mark.parametrize("case", range(len(NORM_CASES)))
def test_norms_match_oracle(gpu_lib, case):
    """tt_norms against the oracle (exact inner product in FP64): the
    squared norm within 1e-5 relative, the inner-product tolerance.  The
    cases include cores processed in several slice groups with a ragged
    last group."""
    tt = gpu_lib
    seed, ns, ranks, b = NORM_CASES[case]
    print("norms", ns, ranks, b, flush=True)
    rng = np.random.default_rng(seed)
    As = [W.random_cores(rng, ns, ranks, 1.0 / np.sqrt(max(ranks))) for _ in range(b)]
    got = tt.norms([tt.TT.from_cores(a) for a in As]).cpu().numpy().astype(np.float64)
    want2 = np.array([oracle.inner(a, a) for a in As])
    assert np.all(np.abs(got ** 2 - want2) <= 1e-5 * want2), np.max(np.abs(got ** 2 - want2) / want2)
