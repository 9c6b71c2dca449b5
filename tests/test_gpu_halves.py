"""GPU parity of the gather by prefix/suffix tables (tt_halves_*) against the
FP64 oracle's gather (the entry formula), 1e-5 relative, normwise: every
lane-group width of the row dot (r_split = 4, 8, 16, 32, 64), the scalar
path (other r_split), forced and automatic splits, d = 2 and d > 16, ragged
sizes, table reuse, and the 2^20-entry workload against the chain gather."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _case(seed, ns, ranks, M):
    rng = np.random.default_rng(seed)
    cores = W.random_cores(rng, ns, ranks, 1.0 / np.sqrt(max(ranks)))
    idx = W.random_indices(rng, ns, M)
    return cores, idx


CASES = [
    # (seed, ns, ranks, M, split or None = automatic)
    (21, [10] * 10, [1] + [16] * 9 + [1], 70001, None),                      # r_s = 16, split 5
    (22, [10] * 10, [1] + [16] * 9 + [1], 30011, 2),                         # lopsided split
    (23, [10] * 10, [1] + [16] * 9 + [1], 30011, 8),
    (24, [10] * 10, [1, 10, 32, 32, 32, 32, 32, 32, 32, 10, 1], 20011, None),  # r_s = 32
    (25, [8, 8, 8, 8, 8], [1, 8, 64, 64, 8, 1], 9001, 2),                    # r_s = 64
    (26, [8, 8, 8, 8], [1, 4, 4, 4, 1], 4096, None),                         # r_s = 4
    (27, [16] * 8, [1] + [8] * 7 + [1], 33333, None),                        # r_s = 8
    (28, [5, 7, 3, 9, 4], [1, 3, 11, 6, 2, 1], 9999, None),                  # scalar path
    (29, [5, 7, 3, 9, 4], [1, 3, 11, 6, 2, 1], 9999, 2),                     # scalar, r_s = 11
    (30, [3, 4], [1, 3, 1], 257, None),                                      # d = 2
    (31, [2] * 17, [1] + [4] * 16 + [1], 5000, None),                        # d > 16
    (32, [8, 8, 8, 8, 8], [1, 8, 64, 64, 8, 1], 1, 2),                       # one entry, 16 lanes
]


def _ids(c):
    return "seed%d-d%d-M%d-s%s" % (c[0], len(c[1]), c[3], c[4])


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_halves_gather_parity(gpu_lib, case):
    tt = gpu_lib
    seed, ns, ranks, M, split = case
    print("case", _ids(case), flush=True)
    cores, idx = _case(seed, ns, ranks, M)
    X = tt.TT.from_cores(cores)
    y = tt.gather_halves(X, idx, split=split).cpu().numpy()
    assert y.shape == (M,)
    assert _rel(y, oracle.gather(cores, idx)) <= TOL


def test_halves_tables_reused_and_empty(gpu_lib):
    """One build serves several gathers; M = 0 gives an empty result."""
    tt = gpu_lib
    cores, idx = _case(33, [10] * 6, [1, 10, 16, 16, 16, 10, 1], 12345)
    X = tt.TT.from_cores(cores)
    tabs = tt.halves_tables(X)
    assert tabs[0] == tt.halves_split(X) == 3
    y1 = tt.gather_halves(X, idx, tables=tabs).cpu().numpy()
    idx2 = W.random_indices(np.random.default_rng(34), [10] * 6, 777)
    y2 = tt.gather_halves(X, idx2, tables=tabs).cpu().numpy()
    assert _rel(y1, oracle.gather(cores, idx)) <= TOL
    assert _rel(y2, oracle.gather(cores, idx2)) <= TOL
    y0 = tt.gather_halves(X, np.zeros((6, 0), np.int32), tables=tabs)
    assert tuple(y0.shape) == (0,)


def test_halves_full_size(gpu_lib):
    """The d=10, n=10, r=16 workload at 2^20 entries: sampled entries against
    the oracle, all entries against the chain gather."""
    import torch
    tt = gpu_lib
    p = W.gather_d10()
    X = tt.TT.from_cores(p.cores)
    idx = torch.from_numpy(p.idx).cuda()
    y = tt.gather_halves(X, idx).cpu().numpy()
    yc = tt.gather(X, idx).cpu().numpy()
    assert _rel(y, yc) <= TOL
    sel = np.random.default_rng(35).choice(p.M, 4096, replace=False)
    assert _rel(y[sel], oracle.gather(p.cores, p.idx[:, sel])) <= TOL
