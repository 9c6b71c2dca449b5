"""GPU parity of the Riemannian gradients (Riemannian Geometry Operations:
the projection of the Euclidean gradient onto the tangent space) against
the FP64 oracle:
  - tt_observed_loss (squared, Huber, logistic): loss and per-entry
    gradient element by element;
  - the Riemannian gradient of an observed-entry loss (gather, loss,
    sparse projection) against the oracle's dense projector on a tiny shape
    and its sparse projection at d=10;
  - tt_riemannian_grad from per-core Euclidean gradients that automatic
    differentiation of f(X + xi(dG)) at dG = 0 returns, for an observed
    loss (through the library's differentiable gather) and for a dense
    f = |X - A|^2 / 2 (through torch on the host), against the dense
    projector."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from parity import assert_elementwise

pytestmark = pytest.mark.gpu

KINDS = ["squared", "huber", "logistic"]


def _targets(rng, kind, M):
    t = rng.standard_normal(M)
    return (np.sign(t) if kind == "logistic" else t).astype(np.float32)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("M", [0, 1, 1000, 100003])
def test_observed_loss_matches_oracle(gpu_lib, kind, M):
    tt = gpu_lib
    rng = np.random.default_rng(81 + M)
    y = (1.7 * rng.standard_normal(M)).astype(np.float32)
    t = _targets(rng, kind, M)
    loss, g = tt.observed_loss(torch.as_tensor(y).cuda(), torch.as_tensor(t).cuda(), kind, 0.6)
    lr, gr = oracle.observed_loss(y, t, kind, 0.6)
    if M == 0:
        assert float(loss.item()) == 0.0 and g.numel() == 0
        return
    assert abs(float(loss.item()) - lr) <= 1e-5 * abs(lr)
    # each gradient element within 1e-5 of its own magnitude, plus the
    # rounding of y - t (|y| + |t|) for the residual-based losses
    bound = np.abs(gr) + (0 if kind == "logistic" else (np.abs(y) + np.abs(t)) / max(M, 1))
    assert_elementwise(g.cpu().numpy(), gr, bound, 1e-5, "observed loss gradient (%s)" % kind)


def _tiny(seed):
    rng = np.random.default_rng(seed)
    ns, ranks = [3, 4, 3, 2], [1, 2, 3, 2, 1]
    X = W.random_cores(rng, ns, ranks, 0.8)
    return rng, ns, ranks, X


def _dense_rel(Wc, ref):
    got = oracle.full([c.astype(np.float64) for c in Wc])
    return np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)


@pytest.mark.parametrize("kind", KINDS)
def test_riemannian_grad_observed_equals_dense_projector(gpu_lib, kind):
    tt = gpu_lib
    rng, ns, ranks, X = _tiny(90 + KINDS.index(kind))
    M = 40
    idx = W.random_indices(rng, ns, M)
    t = _targets(rng, kind, M)
    Xg = tt.TT.from_cores(X)
    loss, Wt = tt.riemannian_grad_observed(Xg, idx, t, kind, 0.5)
    y = oracle.gather(X, idx)
    lr, g = oracle.observed_loss(y, t, kind, 0.5)
    G = np.zeros(ns)
    np.add.at(G, tuple(idx), g)
    ref = oracle.riemannian_grad_dense([c.astype(np.float64) for c in X], G)
    assert abs(float(loss.item()) - lr) <= 1e-5 * abs(lr)
    assert _dense_rel(Wt.numpy_cores(), ref) <= 1e-5


@pytest.mark.parametrize("kind", ["huber", "logistic"])
def test_riemannian_grad_observed_d10(gpu_lib, kind):
    """d=10, n=10, canonical rank 16, 50,000 entries: the tangent TT against
    the oracle's sparse projection of the oracle's gradient, by exact TT
    difference norm (1e-4) and values at the observed entries."""
    tt = gpu_lib
    rng = np.random.default_rng(95)
    ns = [10] * 10
    ranks = W.canonical_ranks(ns, 16)
    X = W.random_cores(rng, ns, ranks, 0.25)
    M = 50000
    idx = W.random_indices(rng, ns, M)
    t = _targets(rng, kind, M)
    Xg = tt.TT.from_cores(X)
    _, Wt = tt.riemannian_grad_observed(Xg, idx, t, kind, 0.05)
    X64 = [c.astype(np.float64) for c in X]
    _, g = oracle.observed_loss(oracle.gather(X64, idx), t, kind, 0.05)
    ref = oracle.project_sparse(X64, idx, g)[0]
    Wc = Wt.numpy_cores()
    diff = oracle.add(Wc, oracle.scale(ref, -1.0))
    assert np.sqrt(max(oracle.inner(diff, diff), 0.0)) <= 1e-4 * oracle.norm(ref)
    sub = idx[:, :4096]
    vg, vr = oracle.gather(Wc, sub), oracle.gather(ref, sub)
    assert np.linalg.norm(vg - vr) <= 1e-4 * np.linalg.norm(vr)


def _tangent_param(U, V, ns, ranks, dG):
    """Cores of X + xi(dG) = [[V_k, 0], [dG_k, U_k]] ... as torch tensors
    (differentiable in the dG_k); U, V are lists of torch cores."""
    d = len(ns)
    cores = []
    for k in range(d):
        if k == 0:
            cores.append(torch.cat([dG[0], U[0]], dim=2))
        elif k == d - 1:
            cores.append(torch.cat([V[k], U[k] + dG[k]], dim=0))
        else:
            top = torch.cat([V[k], torch.zeros(ranks[k], ns[k], ranks[k + 1], dtype=V[k].dtype,
                                                device=V[k].device)], dim=2)
            bot = torch.cat([dG[k], U[k]], dim=2)
            cores.append(torch.cat([top, bot], dim=0))
    return cores


@pytest.mark.parametrize("kind", KINDS)
def test_riemannian_grad_from_autodiff_of_observed_loss(gpu_lib, kind):
    """Zhat_k = d f(X + xi(dG)) / d dG_k at dG = 0 by torch autograd through
    the library's differentiable gather (whose backward is the adjoint
    kernel), then tt_riemannian_grad: equals the dense projector applied to
    the Euclidean gradient."""
    tt = gpu_lib
    rng, ns, ranks, X = _tiny(100 + KINDS.index(kind))
    M = 40
    idx = W.random_indices(rng, ns, M)
    t = _targets(rng, kind, M)
    Xg = tt.TT.from_cores(X)
    U, V = tt.orthogonalize_both(Xg)
    Uc = [c.detach() for c in U.cores()]
    Vc = [c.detach() for c in V.cores()]
    dG = [torch.zeros(ranks[k], ns[k], ranks[k + 1], device="cuda", requires_grad=True) for k in range(len(ns))]
    cores = _tangent_param(Uc, Vc, ns, ranks, dG)
    Wr = [1] + [2 * r for r in ranks[1:-1]] + [1]
    flat = torch.cat([c.reshape(-1) for c in cores])
    y = tt.tt_gather(tt.TT(ns, Wr, flat), idx)
    tg = torch.as_tensor(t).cuda()
    if kind == "squared":
        f = ((y - tg) ** 2).mean()
    elif kind == "huber":
        r = y - tg
        f = torch.where(r.abs() <= 0.5, 0.5 * r * r, 0.5 * (r.abs() - 0.25)).mean()
    else:
        f = torch.nn.functional.softplus(-tg * y).mean()
    f.backward()
    Wt = tt.riemannian_grad(U, V, [g.grad.detach() for g in dG])
    lr, g = oracle.observed_loss(oracle.gather(X, idx), t, kind, 0.5)
    assert abs(float(f.item()) - lr) <= 1e-5 * abs(lr)
    G = np.zeros(ns)
    np.add.at(G, tuple(idx), g)
    ref = oracle.riemannian_grad_dense([c.astype(np.float64) for c in X], G)
    assert _dense_rel(Wt.numpy_cores(), ref) <= 1e-5


def test_riemannian_grad_from_autodiff_of_dense_function(gpu_lib):
    """f(X) = |X - A|^2 / 2 for a TT A, written with dense torch operations
    on the host (float64): its Zhat from autograd of f(X + xi(dG)) at
    dG = 0, then tt_riemannian_grad on the GPU, against the dense projector
    applied to X - A; with alpha = -0.3 and add_x = 1, the retraction input
    X - 0.3 grad f."""
    tt = gpu_lib
    rng, ns, ranks, X = _tiny(110)
    A = W.random_cores(rng, ns, [1, 2, 2, 2, 1], 0.8)
    Xg = tt.TT.from_cores(X)
    U, V = tt.orthogonalize_both(Xg)
    Uc = [torch.as_tensor(c, dtype=torch.float64) for c in U.numpy_cores()]
    Vc = [torch.as_tensor(c, dtype=torch.float64) for c in V.numpy_cores()]
    dG = [torch.zeros(ranks[k], ns[k], ranks[k + 1], dtype=torch.float64, requires_grad=True)
          for k in range(len(ns))]
    cores = _tangent_param(Uc, Vc, ns, ranks, dG)

    def full(cs):
        t = cs[0]
        for c in cs[1:]:
            t = torch.tensordot(t, c, dims=([t.dim() - 1], [0]))
        return t.reshape(ns)

    Ad = torch.as_tensor(oracle.full(A))
    f = 0.5 * ((full(cores) - Ad) ** 2).sum()
    f.backward()
    zhat = [g.grad.detach().to(torch.float32).cuda() for g in dG]
    Xd = oracle.full([c.astype(np.float64) for c in X])
    ref = oracle.riemannian_grad_dense([c.astype(np.float64) for c in X], Xd - oracle.full(A))
    Wt = tt.riemannian_grad(U, V, zhat)
    assert _dense_rel(Wt.numpy_cores(), ref) <= 1e-5
    Wr = tt.riemannian_grad(U, V, zhat, alpha=-0.3, add_x=1)
    assert _dense_rel(Wr.numpy_cores(), Xd - 0.3 * ref) <= 1e-5
