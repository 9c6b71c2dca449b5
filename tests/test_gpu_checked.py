"""GPU tests of the index check (tt_check_indices) and of the binding's
checked mode (TTGFX_CHECKED=1 turns out-of-range indices into TT_ERR_INDEX).
Integer work: the count and the first bad entry must equal numpy's exactly."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _expected(idx, ns):
    bad = np.zeros(idx.shape[1], dtype=bool)
    for k, n in enumerate(ns):
        bad |= (idx[k] < 0) | (idx[k] >= n)
    where = np.flatnonzero(bad)
    return int(bad.sum()), int(where[0]) if where.size else idx.shape[1]


def _planted(seed, ns, M, nbad):
    rng = np.random.default_rng(seed)
    idx = np.stack([rng.integers(0, n, M) for n in ns]).astype(np.int32)
    if nbad:
        ent = rng.choice(M, size=nbad, replace=False)
        modes = rng.integers(0, len(ns), nbad)
        kinds = rng.integers(0, 4, nbad)
        for e, k, kind in zip(ent, modes, kinds):
            idx[k, e] = [-1, ns[k], np.iinfo(np.int32).min, np.iinfo(np.int32).max][kind]
    return idx


CASES = [
    ([3, 4, 5], 1, 0),
    ([3, 4, 5], 1, 1),
    ([10] * 10, 1000, 0),
    ([10] * 10, 1000, 7),            # ragged last workgroup
    ([7, 2], 65536 * 9 + 5, 300),    # several grid-stride passes
    ([10] * 10, 1 << 20, 1),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_check_indices_counts(gpu_lib, case):
    tt = gpu_lib
    ns, M, nbad = CASES[case]
    print("check_indices", ns, M, nbad, flush=True)
    idx = _planted(900 + case, ns, M, nbad)
    X = tt.TT(ns, [1] * (len(ns) + 1))
    got = tt.check_indices(X, torch.as_tensor(idx).cuda())
    assert got == _expected(idx, ns)


def test_check_indices_boundary_values(gpu_lib):
    tt = gpu_lib
    ns = [4, 6]
    idx = np.array([[0, 3, 4, 0, 0], [5, 0, 0, 6, -1]], dtype=np.int32)
    X = tt.TT(ns, [1, 2, 1])
    assert tt.check_indices(X, torch.as_tensor(idx).cuda()) == (3, 2)
    assert tt.check_indices(X, torch.zeros((2, 0), dtype=torch.int32, device="cuda")) == (0, 0)


def test_checked_mode_raises(gpu_lib, monkeypatch):
    tt = gpu_lib
    from paper_1801_01928_amd import _lib as L
    p = W.small_step()
    X = tt.TT.from_cores(p.cores)
    good = torch.as_tensor(p.idx).cuda()
    bad = good.clone()
    bad[1, 17] = p.ns[1]
    t = torch.zeros(good.shape[1], device="cuda")
    y0 = tt.gather(X, good)
    # (unchecked calls with such indices are undefined behaviour: never made)
    monkeypatch.setenv("TTGFX_CHECKED", "1")
    assert torch.equal(tt.gather(X, good), y0)
    for call in (lambda: tt.gather(X, bad),
                 lambda: tt.gather_backward(X, bad, t),
                 lambda: tt.gather_mse_backward(X, bad, t)):
        with pytest.raises(L.TTError) as ei:
            call()
        assert ei.value.code == L.TT_ERR_INDEX
        assert "entry 17" in str(ei.value)
    U = tt.orthogonalize(X, L.TT_LR)
    V = tt.orthogonalize(X, L.TT_RL)
    with pytest.raises(L.TTError) as ei:
        tt.project_sparse(U, V, bad, t)
    assert ei.value.code == L.TT_ERR_INDEX
    flat = bad.reshape(-1)
    M = good.shape[1]
    with pytest.raises(L.TTError) as ei:
        tt.BatchedPlan([X, X], torch.cat([good.reshape(-1), flat]), torch.cat([t, t]), [0, M, 2 * M])
    assert ei.value.code == L.TT_ERR_INDEX
