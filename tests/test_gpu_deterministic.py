"""Fixed-order sums: the slice-grouped adjoint, fused pass and projection
repeat bitwise, with and without the deterministic policy
(tt_set_deterministic); results stay within the oracle parity bar (1e-5 for
the adjoint and the fused pass, 1e-4 for the projection, every element
against its absolute-value bound); under the policy the batched plan equals
its tensor-by-tensor path bitwise, and shapes only the atomic kernels serve
are refused."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_adjoint, assert_gather

pytestmark = pytest.mark.gpu


@pytest.fixture(params=[True, False], ids=["policy", "default"])
def det(gpu_lib, request):
    tt = gpu_lib
    tt.set_deterministic(request.param)
    assert tt.deterministic() == request.param
    yield tt
    tt.set_deterministic(False)


@pytest.fixture
def det_on(gpu_lib):
    tt = gpu_lib
    tt.set_deterministic(True)
    yield tt
    tt.set_deterministic(False)


def _cores(seed, ns, ranks, M):
    rng = np.random.default_rng(seed)
    cores = W.random_cores(rng, ns, ranks, 1.0 / np.sqrt(max(ranks)))
    idx = W.random_indices(rng, ns, M)
    g = rng.standard_normal(M).astype(np.float32)
    return cores, idx, g


ADJ = [
    (21, [10] * 10, [1, 10, 32, 32, 32, 32, 32, 32, 32, 10, 1], 50021),
    (22, [2] * 6, [1] + [32] * 5 + [1], 40000),          # slices across many waves
    (23, [10] * 10, [1] + [16] * 9 + [1], 30001),        # rank class 16
]


@pytest.mark.parametrize("case", ADJ, ids=lambda c: "seed%d" % c[0])
def test_adjoint_bitwise_and_oracle(det, case):
    import torch
    tt = det
    seed, ns, ranks, M = case
    print("deterministic adjoint", seed, flush=True)
    cores, idx, g = _cores(seed, ns, ranks, M)
    X = tt.TT.from_cores(cores)
    gt = torch.from_numpy(g)
    a = [c.copy() for c in tt.gather_backward(X, idx, gt).numpy_cores()]
    b = tt.gather_backward(X, idx, gt).numpy_cores()
    for k in range(len(ns)):
        assert np.array_equal(a[k], b[k]), k
    assert_adjoint(a, oracle.gather_backward(cores, idx, g), cores, cores, idx, g, 1e-5)


def test_fused_pass_bitwise_and_oracle(det):
    tt = det
    ns, ranks, M = [10] * 10, [1, 10, 32, 32, 32, 32, 32, 32, 32, 10, 1], 65536
    cores, idx, _ = _cores(24, ns, ranks, M)
    t = np.random.default_rng(25).standard_normal(M).astype(np.float32)
    X = tt.TT.from_cores(cores)
    runs = []
    for _ in range(2):
        y, loss, gX = tt.gather_mse_backward(X, idx, t)
        runs.append((y.cpu().numpy(), float(loss.item()), [c.copy() for c in gX.numpy_cores()]))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert runs[0][1] == runs[1][1]
    for k in range(len(ns)):
        assert np.array_equal(runs[0][2][k], runs[1][2][k]), k
    yr = oracle.gather(cores, idx)
    lr, gr = oracle.mse_loss_and_grad(yr, t)
    assert_gather(runs[0][0], yr, cores, idx, 1e-5)
    assert abs(runs[0][1] - lr) <= 1e-5 * lr
    assert_adjoint(runs[0][2], oracle.gather_backward(cores, idx, gr), cores, cores, idx, gr, 1e-5)


def test_projection_bitwise_and_oracle(det):
    """The sparse projection at d=10, canonical rank 32, 2^17 entries."""
    tt = det
    from test_gpu_riemann import assert_tangent_elementwise, rel_tt
    ns = [10] * 10
    ranks = W.canonical_ranks(ns, 32)
    cores, idx, z = _cores(26, ns, ranks, 1 << 17)
    X = tt.TT.from_cores(cores)
    U, V = tt.orthogonalize_both(X)
    a = [c.copy() for c in tt.project_sparse(U, V, idx, z, alpha=-0.1, add_x=1).numpy_cores()]
    b = tt.project_sparse(U, V, idx, z, alpha=-0.1, add_x=1).numpy_cores()
    for k in range(len(ns)):
        assert np.array_equal(a[k], b[k]), k
    ref = oracle.project_sparse(cores, idx, z, alpha=-0.1, beta=1.0)
    assert rel_tt(a, ref[0]) <= 1e-4
    assert_tangent_elementwise(a, ref, idx, z, -0.1, 1.0)


def test_plan_runs_tensor_by_tensor(det_on):
    """Under the policy tt_plan_run is the per-tensor path: bitwise equal to
    tt_plan_run_plain and to itself, and on the oracle (1e-5)."""
    import torch
    tt = det_on
    from test_gpu_batched import _check, _oracle, _pack, _small_batch
    ns, insts = _small_batch()
    idx, t, off = _pack(insts)
    Xs = [tt.TT.from_cores(c) for c, _, _ in insts]
    plan = tt.BatchedPlan(Xs, idx, t, off)
    out = []
    for run in (plan.run, plan.run, plan.run_plain):
        run()
        torch.cuda.synchronize()
        out.append((plan.loss.cpu().numpy().copy(), [g.data.cpu().numpy().copy() for g in plan.grads]))
    for o in out[1:]:
        assert np.array_equal(o[0], out[0][0])
        for a, b in zip(o[1], out[0][1]):
            assert np.array_equal(a, b)
    _check(plan, _oracle(insts))
    plan.close()


def test_refuses_generic_shapes(det_on):
    """Ranks above 32 have no fixed-order accumulator: the call fails before
    any device work, and the default policy then runs it."""
    import torch
    tt = det_on
    cores, idx, g = _cores(27, [6, 6, 6], [1, 40, 40, 1], 3001)
    X = tt.TT.from_cores(cores)
    with pytest.raises(RuntimeError, match="deterministic"):
        tt.gather_backward(X, idx, torch.from_numpy(g))
    tt.set_deterministic(False)
    got = tt.gather_backward(X, idx, torch.from_numpy(g)).numpy_cores()
    assert_adjoint(got, oracle.gather_backward(cores, idx, g), cores, cores, idx, g, 1e-5)
