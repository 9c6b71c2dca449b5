"""GPU parity of the suffix-table path of the slice-grouped kernels against
the FP64 oracle.  Entries that share their last l indices share the right
partial G^{d-l}[i_{d-l}] .. G^{d-1}[i_{d-1}] e_0 (the entry formula of the
Introduction, regrouped); the kernels read those partials from a table
built once per call.  Every case runs with the table off, at one level, and
at the deepest level the size cap allows (down to d-1 levels, where the
right sweep computes mode 0 alone), and each result is checked element by
element against the oracle (1e-5 of the absolute-value bound)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from parity import assert_adjoint, assert_gather

pytestmark = pytest.mark.gpu

TOL = 1e-5

CASES = [
    # (seed, ns, ranks, M)
    (21, [10] * 10, [1] + [16] * 9 + [1], 30011),
    (22, [5, 7, 3, 9, 4], [1, 3, 11, 6, 2, 1], 9999),     # ragged modes and ranks
    (23, [4, 5, 3], [1, 3, 2, 1], 3001),                   # d = 3: two levels = d-1
    (24, [6, 9], [1, 5, 1], 777),                          # d = 2: one level = d-1
    (25, [10] * 6, [1, 10, 32, 32, 32, 10, 1], 20011),     # rank class 32
    (26, [6, 6, 6], [1, 40, 40, 1], 3001),                 # gather rank class 64
]
DEPTHS = [0, 1, 15]


@pytest.fixture
def depth_policy(gpu_lib):
    yield gpu_lib.set_suffix_depth
    gpu_lib.set_suffix_depth(-1)


def _case(seed, ns, ranks, M):
    rng = np.random.default_rng(seed)
    cores = W.random_cores(rng, ns, ranks, 1.0 / np.sqrt(max(ranks)))
    idx = W.random_indices(rng, ns, M)
    g = rng.standard_normal(M).astype(np.float32)
    return cores, idx, g


@pytest.mark.parametrize("depth", DEPTHS)
@pytest.mark.parametrize("case", range(len(CASES)))
def test_suffix_table_gather_adjoint_fused(gpu_lib, depth_policy, case, depth):
    tt = gpu_lib
    seed, ns, ranks, M = CASES[case]
    depth_policy(depth)
    cores, idx, g = _case(seed, ns, ranks, M)
    X = tt.TT.from_cores(cores)
    print("suffix case", seed, ns, ranks, M, "depth", depth, "->", tt.suffix_depth(X, M), flush=True)
    if depth == 0:
        assert tt.suffix_depth(X, M) == 0
    y = tt.gather(X, idx).cpu().numpy()
    yr = oracle.gather(cores, idx)
    assert_gather(y, yr, cores, idx, TOL)
    if max(ranks) > 32:
        return  # rank class 64 serves the gather alone
    assert tt.suffix_depth(X, M) == (0 if depth == 0 else min(depth, len(ns) - 1, 4))
    gX = tt.gather_backward(X, idx, torch.from_numpy(g))
    gr = oracle.gather_backward(cores, idx, g)
    assert_adjoint(gX.numpy_cores(), gr, cores, cores, idx, g, TOL, "adjoint depth %d" % depth)
    t = (yr + 0.1 * g).astype(np.float32)
    y2, loss, gF = tt.gather_mse_backward(X, idx, t)
    lr, gl = oracle.mse_loss_and_grad(yr, t)
    assert_gather(y2.cpu().numpy(), yr, cores, idx, TOL)
    assert abs(float(loss.item()) - lr) <= TOL * lr
    grr = oracle.gather_backward(cores, idx, gl)
    assert_adjoint(gF.numpy_cores(), grr, cores, cores, idx, gl, TOL, "fused depth %d" % depth)


DEEP = [
    # (seed, ns, ranks, M): small modes, so the table reaches past four levels
    (27, [2] * 12, [1, 2, 4, 8, 16, 16, 16, 16, 16, 8, 4, 2, 1], 40000),
    (28, [2] * 10, [1, 2, 4, 8, 16, 32, 16, 8, 4, 2, 1], 30000),   # rank class 32
]


@pytest.mark.parametrize("case", DEEP, ids=lambda c: "seed%d" % c[0])
def test_suffix_table_deep(gpu_lib, depth_policy, case):
    """Tables deeper than four levels (built one level at a time) against
    the oracle: gather, adjoint and fused pass."""
    tt = gpu_lib
    seed, ns, ranks, M = case
    depth_policy(15)
    cores, idx, g = _case(seed, ns, ranks, M)
    X = tt.TT.from_cores(cores)
    depth = tt.suffix_depth(X, M)
    print("deep suffix case", seed, "depth", depth, flush=True)
    assert depth > 4
    yr = oracle.gather(cores, idx)
    assert_gather(tt.gather(X, idx).cpu().numpy(), yr, cores, idx, TOL)
    gX = tt.gather_backward(X, idx, torch.from_numpy(g))
    assert_adjoint(gX.numpy_cores(), oracle.gather_backward(cores, idx, g), cores, cores, idx, g, TOL, "adjoint")
    t = (yr + 0.1 * g).astype(np.float32)
    y2, loss, gF = tt.gather_mse_backward(X, idx, t)
    lr, gl = oracle.mse_loss_and_grad(yr, t)
    assert abs(float(loss.item()) - lr) <= TOL * lr
    assert_adjoint(gF.numpy_cores(), oracle.gather_backward(cores, idx, gl), cores, cores, idx, gl, TOL, "fused")


def test_suffix_table_projection(gpu_lib, depth_policy):
    """The sparse tangent projection (left sweep over U, right sweep and
    table over V) at the deepest table: element-wise against the oracle."""
    from test_gpu_riemann import assert_tangent_elementwise, rel_tt
    tt = gpu_lib
    depth_policy(15)
    rng = np.random.default_rng(31)
    ns = [10] * 8
    ranks = W.canonical_ranks(ns, 16)
    cores = W.random_cores(rng, ns, ranks, 0.25)
    idx = W.random_indices(rng, ns, 20011)
    z = rng.standard_normal(idx.shape[1]).astype(np.float32)
    X = tt.TT.from_cores(cores)
    U = tt.orthogonalize(X, tt.TT_LR)
    V = tt.orthogonalize(X, tt.TT_RL)
    Wg = tt.project_sparse(U, V, idx, z, alpha=-0.5, add_x=1)
    ref = oracle.project_sparse(cores, idx, z, alpha=-0.5, beta=1.0)
    assert rel_tt(Wg.numpy_cores(), ref[0]) <= 1e-4
    assert_tangent_elementwise(Wg.numpy_cores(), ref, idx, z, -0.5, 1.0)


def test_suffix_table_headline_depth(gpu_lib):
    """The fused pass at d=10, n=10, rank 16 over 2^20 entries takes four
    levels (10^4 rows of the deepest) under the automatic policy."""
    tt = gpu_lib
    p = W.gather_d10()
    X = tt.TT.from_cores(p.cores)
    assert tt.suffix_depth(X, p.M) == 4
