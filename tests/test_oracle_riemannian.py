"""Pins of the FP64 oracle's Riemannian step: QR sweeps, sparse tangent
projection, tangent assembly and TT rounding.

The tangent-space projector is pinned against the range of the Jacobian of
the TT parametrisation (an independent construction of the tangent space),
rounding against a dense TT-SVD of the full tensor and against Eckart-Young,
and the sweeps against orthonormality and tensor invariance.
"""
import numpy as np
import pytest

import oracle
from oracle import riemannian as R
from workloads import random_tt, random_indices, canonical_ranks, small_step


def _rng(s):
    return np.random.default_rng(2000 + s)


def _X(seed, ns, r):
    return [c.astype(np.float64) for c in random_tt(seed, ns, canonical_ranks(ns, r))]


# ----------------------------------------------------------------------- QR

def test_qr_pos():
    A = _rng(0).standard_normal((12, 5))
    Q, R = oracle.qr_pos(A)
    np.testing.assert_allclose(Q.T @ Q, np.eye(5), atol=1e-14)
    assert np.all(np.diag(R) >= 0)
    np.testing.assert_allclose(np.tril(R, -1), 0, atol=0)
    np.testing.assert_allclose(Q @ R, A, atol=1e-13)


@pytest.mark.parametrize("ns,r", [([3, 4, 3, 5], 3), ([4, 4, 4, 4, 4], 6), ([5, 2, 6], 4)])
def test_orthogonalize_sweeps(ns, r):
    X = _X(1, ns, r)
    F = oracle.full(X)
    U = oracle.orthogonalize_lr(X)
    V = oracle.orthogonalize_rl(X)
    np.testing.assert_allclose(oracle.full(U), F, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(oracle.full(V), F, rtol=1e-12, atol=1e-13)
    for k in range(len(ns) - 1):
        UL = U[k].reshape(-1, U[k].shape[2])
        np.testing.assert_allclose(UL.T @ UL, np.eye(UL.shape[1]), atol=1e-13)
        VR = V[k + 1].reshape(V[k + 1].shape[0], -1)
        np.testing.assert_allclose(VR @ VR.T, np.eye(VR.shape[0]), atol=1e-13)
    nrm = np.linalg.norm(F)
    assert np.linalg.norm(U[-1]) == pytest.approx(nrm, rel=1e-12)
    assert np.linalg.norm(V[0]) == pytest.approx(nrm, rel=1e-12)
    # the first QR of the sweep is LAPACK's after the sign fix (uniqueness)
    Q, _ = np.linalg.qr(X[0].reshape(-1, X[0].shape[2]))
    Q = Q * np.sign(np.diag(np.linalg.qr(X[0].reshape(-1, X[0].shape[2]))[1]))[None, :]
    np.testing.assert_allclose(U[0].reshape(Q.shape), Q, atol=1e-13)


def test_orthogonalize_reduces_infeasible_ranks():
    """Ranks above min(r_{k-1} n_k, r_k) shrink to it."""
    ns = [2, 3, 2]
    X = [c.astype(np.float64) for c in random_tt(3, ns, [1, 5, 5, 1])]
    U = oracle.orthogonalize_lr(X)
    assert [c.shape[2] for c in U] == [2, 5, 1]
    V = oracle.orthogonalize_rl(X)
    assert [c.shape[0] for c in V] == [1, 5, 2]
    np.testing.assert_allclose(oracle.full(U), oracle.full(X), atol=1e-13)
    np.testing.assert_allclose(oracle.full(V), oracle.full(X), atol=1e-13)


# --------------------------------------------------------------- projection

def _jacobian_projector(X):
    """Orthogonal projector onto the range of d vec(full(X)) / d(cores): the
    tangent space of the fixed-rank manifold, built without any of the
    projection formulas.  full() is multilinear, so each Jacobian column is
    full() with one core replaced by a unit tensor."""
    cols = []
    for k in range(len(X)):
        for j in range(X[k].size):
            E = np.zeros(X[k].size); E[j] = 1
            Xk = list(X); Xk[k] = E.reshape(X[k].shape)
            cols.append(oracle.full(Xk).reshape(-1))
    J = np.stack(cols, axis=1)
    Uj, s, _ = np.linalg.svd(J, full_matrices=False)
    rank = int(np.sum(s > 1e-10 * s[0]))
    B = Uj[:, :rank]
    return B @ B.T, rank


def _manifold_dim(ns, rk):
    return sum(rk[k] * ns[k] * rk[k + 1] for k in range(len(ns))) - sum(r * r for r in rk[1:-1])


@pytest.mark.parametrize("ns,r", [([3, 3, 3], 2), ([2, 3, 2, 3], 2), ([3, 4, 3], 3)])
def test_dense_projector_is_jacobian_range(ns, r):
    X = _X(4, ns, r)
    U = oracle.orthogonalize_lr(X)
    V = oracle.orthogonalize_rl(X)
    P = oracle.dense_projector(U, V)
    PJ, rank = _jacobian_projector(X)
    rk = canonical_ranks(ns, r)
    assert rank == _manifold_dim(ns, rk)
    np.testing.assert_allclose(P, PJ, atol=1e-10)
    np.testing.assert_allclose(P @ P, P, atol=1e-12)
    np.testing.assert_allclose(P, P.T, atol=1e-12)
    assert np.trace(P) == pytest.approx(rank, abs=1e-9)


def _dense_sparse(ns, idx, z):
    Z = np.zeros(ns)
    np.add.at(Z, tuple(idx), z)
    return Z


@pytest.mark.parametrize("ns,r", [([3, 3, 3], 2), ([3, 4, 3, 2], 3), ([4, 4, 4, 4], 4)])
def test_project_sparse_equals_dense_projector(ns, r):
    rng = _rng(5)
    X = _X(5, ns, r)
    idx = random_indices(rng, ns, 60)
    z = rng.standard_normal(60)
    W, U, V, dG = oracle.project_sparse(X, idx, z, alpha=1.0, beta=0.0)
    P = oracle.dense_projector(U, V)
    Z = _dense_sparse(ns, idx, z)
    np.testing.assert_allclose(oracle.full(W).reshape(-1), P @ Z.reshape(-1), atol=1e-12)
    # gauge condition on the tangent cores
    for k in range(len(ns) - 1):
        UL = U[k].reshape(-1, U[k].shape[2])
        np.testing.assert_allclose(UL.T @ dG[k].reshape(UL.shape[0], -1), 0, atol=1e-12)
    # rank of the tangent TT is 2r in the interior
    assert [c.shape[2] for c in W][:-1] == [2 * c.shape[2] for c in U][:-1]


def _all_entries(ns):
    return np.indices(ns).reshape(len(ns), -1)


def test_projection_idempotent_identity_and_symmetric():
    rng = _rng(6)
    ns, r = [3, 4, 3, 3], 3
    X = _X(6, ns, r)
    grid = _all_entries(ns)
    idx = random_indices(rng, ns, 80)
    z = rng.standard_normal(80)
    W1 = oracle.project_sparse(X, idx, z)[0]
    F1 = oracle.full(W1)
    # idempotence: project the (dense) projection again
    W2 = oracle.project_sparse(X, grid, F1.reshape(-1))[0]
    np.testing.assert_allclose(oracle.full(W2), F1, atol=1e-12)
    # identity on X itself: P_X(X) = X
    FX = oracle.full(X)
    WX = oracle.project_sparse(X, grid, FX.reshape(-1))[0]
    np.testing.assert_allclose(oracle.full(WX), FX, atol=1e-12)
    # symmetry <P Z1, Z2> = <Z1, P Z2>
    idx2 = random_indices(rng, ns, 70)
    z2 = rng.standard_normal(70)
    Z1 = _dense_sparse(ns, idx, z)
    Z2 = _dense_sparse(ns, idx2, z2)
    F2 = oracle.full(oracle.project_sparse(X, idx2, z2)[0])
    assert np.sum(F1 * Z2) == pytest.approx(np.sum(Z1 * F2), rel=1e-11)
    # beta=1 adds X; alpha scales
    W3 = oracle.project_sparse(X, idx, z, alpha=-0.1, beta=1.0)[0]
    np.testing.assert_allclose(oracle.full(W3), FX - 0.1 * F1, atol=1e-12)


def test_projection_identity_on_random_tangent_vector():
    """xi built from random gauge-satisfying tangent cores is fixed by P."""
    rng = _rng(7)
    ns, r = [3, 3, 4, 3], 3
    X = _X(7, ns, r)
    U = oracle.orthogonalize_lr(X)
    V = oracle.orthogonalize_rl(X)
    dG = []
    for k in range(len(ns)):
        H = rng.standard_normal(U[k].shape)
        if k < len(ns) - 1:
            UL = U[k].reshape(-1, U[k].shape[2])
            HL = H.reshape(UL.shape[0], -1)
            H = (HL - UL @ (UL.T @ HL)).reshape(H.shape)
        dG.append(H)
    xi = oracle.full(oracle.tangent_tt(U, V, dG))
    W = oracle.project_sparse(X, _all_entries(ns), xi.reshape(-1))[0]
    np.testing.assert_allclose(oracle.full(W), xi, atol=1e-12)


def test_projection_linearity_project_sum():
    """P(sum c_i A_i) = sum c_i P(A_i) (the identity project_sum relies on)."""
    rng = _rng(8)
    ns, r = [3, 4, 3], 3
    X = _X(8, ns, r)
    parts = [(random_indices(rng, ns, 30), rng.standard_normal(30)) for _ in range(3)]
    c = [0.5, -2.0, 1.25]
    idx = np.concatenate([p[0] for p in parts], axis=1)
    z = np.concatenate([ci * p[1] for ci, p in zip(c, parts)])
    lhs = oracle.full(oracle.project_sparse(X, idx, z)[0])
    rhs = sum(ci * oracle.full(oracle.project_sparse(X, p[0], p[1])[0]) for ci, p in zip(c, parts))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_projection_inner_identity_without_dense():
    """<P_X Z, xi> = sum_m z_m xi(i^m) for a tangent xi (P is symmetric and
    fixes xi); only TT inner products and gathers, so it scales."""
    rng = _rng(9)
    ns, r = [6] * 6, 5
    X = _X(9, ns, r)
    idx = random_indices(rng, ns, 3000)
    z = rng.standard_normal(3000)
    W, U, V, _ = oracle.project_sparse(X, idx, z)
    dG = []
    for k in range(len(ns)):
        H = rng.standard_normal(U[k].shape)
        if k < len(ns) - 1:
            UL = U[k].reshape(-1, U[k].shape[2])
            HL = H.reshape(UL.shape[0], -1)
            H = (HL - UL @ (UL.T @ HL)).reshape(H.shape)
        dG.append(H)
    xi = oracle.tangent_tt(U, V, dG)
    lhs = oracle.inner(W, xi)
    rhs = np.dot(z, oracle.gather(xi, idx))
    assert lhs == pytest.approx(rhs, rel=1e-10)


# ------------------------------------------------------------------ rounding

def _tt_svd_dense(F, max_rank):
    """TT-SVD of a dense tensor: truncated SVDs of successive unfoldings."""
    ns = F.shape
    cores = []
    C = F.reshape(1, -1)
    r0 = 1
    for k in range(len(ns) - 1):
        C = C.reshape(r0 * ns[k], -1)
        Uf, s, Vt = np.linalg.svd(C, full_matrices=False)
        rk = min(max_rank, s.shape[0])
        cores.append(Uf[:, :rk].reshape(r0, ns[k], rk))
        C = s[:rk, None] * Vt[:rk]
        r0 = rk
    cores.append(C.reshape(r0, ns[-1], 1))
    return cores


@pytest.mark.parametrize("ns,r,rmax", [([3, 4, 3, 4], 4, 2), ([4, 4, 4], 4, 3), ([2, 3, 4, 3, 2], 5, 2)])
def test_round_matches_dense_tt_svd_and_error_identity(ns, r, rmax):
    X = _X(10, ns, r)
    Y, disc = oracle.round_tt(X, rmax)
    F = oracle.full(X)
    ref = oracle.full(_tt_svd_dense(F, rmax))
    np.testing.assert_allclose(oracle.full(Y), ref, atol=1e-12)
    err2 = np.sum((F - oracle.full(Y)) ** 2)
    assert err2 == pytest.approx(np.sum(disc), rel=1e-9, abs=1e-20)
    assert max(c.shape[2] for c in Y) <= rmax
    # quasi-optimality: error^2 <= (d-1) * max_k (best rank-rmax error of unfolding k)^2
    tails = []
    for k in range(1, len(ns)):
        s = np.linalg.svd(F.reshape(int(np.prod(ns[:k])), -1), compute_uv=False)
        tails.append(np.sum(s[rmax:] ** 2))
    assert err2 <= (len(ns) - 1) * max(tails) * (1 + 1e-9) + 1e-24
    assert err2 >= max(tails) * (1 - 1e-9) - 1e-24


def test_round_d2_is_eckart_young():
    A = [c.astype(np.float64) for c in random_tt(11, [7, 9], [1, 6, 1])]
    M = A[0][0] @ A[1][:, :, 0]
    Y, disc = oracle.round_tt(A, 3)
    Uf, s, Vt = np.linalg.svd(M)
    best = (Uf[:, :3] * s[:3]) @ Vt[:3]
    np.testing.assert_allclose(oracle.full(Y), best, atol=1e-12)
    assert disc[0] == pytest.approx(np.sum(s[3:] ** 2), rel=1e-12)


def test_round_exact_when_ranks_suffice():
    """round(X + X, r) = 2X (the sum has rank 2r but represents a rank-r tensor)."""
    ns, r = [3, 4, 4, 3], 3
    X = _X(12, ns, r)
    Y, disc = oracle.round_tt(oracle.add(X, X), r)
    np.testing.assert_allclose(oracle.full(Y), 2 * oracle.full(X), atol=1e-12)
    assert np.all(disc < 1e-20 * np.sum(oracle.full(X) ** 2) + 1e-24)
    assert [c.shape[2] for c in Y] == canonical_ranks(ns, r)[1:]


def test_small_step_pipeline_consistent():
    """One completion step on the small workload: the retraction input is
    X - 0.1 P_X(grad) and the rounded point keeps rank <= 4."""
    p = small_step()
    X = [c.astype(np.float64) for c in p.cores]
    t = oracle.gather(p.planted, p.idx) + p.noise
    out = oracle.completion_step(X, p.idx, t, alpha=-0.1, max_rank=4)
    P = oracle.dense_projector(out["U"], out["V"])
    Z = _dense_sparse(p.ns, p.idx, out["g"])
    expect = oracle.full(X).reshape(-1) - 0.1 * (P @ Z.reshape(-1))
    np.testing.assert_allclose(oracle.full(out["W"]).reshape(-1), expect, atol=1e-12)
    assert max(c.shape[2] for c in out["Y"]) <= 4
    err2 = np.sum((oracle.full(out["W"]) - oracle.full(out["Y"])) ** 2)
    assert err2 == pytest.approx(np.sum(out["disc_sq"]), rel=1e-8, abs=1e-18)


# ------------------------------------------------ completion loop (line search)
def test_line_search_is_the_minimiser():
    """The step minimises the observed loss of the first-order model along
    -P: the quadratic's central-difference derivative vanishes there (exact
    for a quadratic), and no grid point does better; P = 0 gives step 0."""
    from oracle import riemannian as R
    rng = np.random.default_rng(31)
    M = 500
    y, t, p = rng.standard_normal(M), rng.standard_normal(M), rng.standard_normal(M)
    a = R.line_search_step(y, t, p)

    def q(s):
        e = y - s * p - t
        return float(np.mean(e * e))

    h = 1e-3 * (1.0 + abs(a))
    assert abs(q(a + h) - q(a - h)) / (2 * h) <= 1e-9
    for s in np.linspace(a - 2.0, a + 2.0, 401):
        assert q(a) <= q(s) + 1e-14
    assert q(a) <= q(0.0)
    assert R.line_search_step(y, t, np.zeros(M)) == 0.0


def test_completion_recovers_planted_tensor():
    """Noiseless planted rank-2 tensor, d=4, n=8, 2000 of 4096 entries
    observed (with repetition), from a random rank-2 start: Riemannian
    gradient descent with the exact line search recovers it (held-out RMSE
    below 1e-8) and the observed loss never increases."""
    from oracle import riemannian as R
    from workloads import random_cores
    ns = [8] * 4
    rng = np.random.default_rng(21)
    planted = random_cores(rng, ns, [1, 2, 2, 2, 1], 1 / np.sqrt(2))
    X0 = random_cores(rng, ns, [1, 2, 2, 2, 1], 0.5)
    idx = random_indices(rng, ns, 2000)
    t = oracle.gather(planted, idx)
    idx_t = random_indices(rng, ns, 1000)
    t_t = oracle.gather(planted, idx_t)
    X, h = R.riemannian_completion(X0, idx, t, 2, 50, idx_t, t_t)
    e = oracle.gather(X, idx_t) - t_t
    assert float(np.sqrt(np.mean(e * e))) < 1e-8
    assert h[0]["test_rmse"] > 0.1
    losses = [x["loss"] for x in h]
    for a, b in zip(losses, losses[1:]):
        assert b <= a * (1 + 1e-9) + 1e-30


def test_completion_with_noise_reaches_noise_level():
    """The small planted problem with N(0, 0.01^2) noise: after 20 steps the
    observed loss is within 1.5x of the noise variance and the held-out RMSE
    fell at least tenfold."""
    from oracle import riemannian as R
    p = small_step()
    rng = np.random.default_rng(11)
    idx_t = random_indices(rng, p.ns, 2000)
    t_t = oracle.gather(p.planted, idx_t)
    t = oracle.gather(p.planted, p.idx) + p.noise
    X, h = R.riemannian_completion(p.cores, p.idx, t, 4, 20, idx_t, t_t)
    y = oracle.gather(X, p.idx)
    loss = float(np.mean((y - t) ** 2))
    assert loss < 1.5 * 1e-4
    e = oracle.gather(X, idx_t) - t_t
    assert float(np.sqrt(np.mean(e * e))) < 0.1 * h[0]["test_rmse"]


# ------------------------------------------------ projection of a TT tensor
@pytest.mark.parametrize("ns,r,sr", [([3, 4, 3, 2], 3, [1, 2, 5, 3, 1]), ([2, 3, 2], 2, [1, 4, 3, 1]),
                                     ([3, 3, 3, 3], 2, [1, 3, 3, 3, 1])])
def test_project_tt_equals_dense_projector(ns, r, sr):
    from oracle import riemannian as R
    X = random_tt(1, ns, canonical_ranks(ns, r))
    Y = random_tt(2, ns, sr)
    W, U, V, dG = R.project_tt(X, Y)
    P = R.dense_projector(U, V)
    want = P @ oracle.full(Y).reshape(-1)
    got = oracle.full(W).reshape(-1)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_project_tt_of_one_hot_is_the_sparse_projection():
    """A one-hot tensor e_i as a rank-1 TT projects exactly as the sparse
    projection of the single entry i with weight 1."""
    from oracle import riemannian as R
    ns = [3, 4, 3, 2]
    X = random_tt(3, ns, canonical_ranks(ns, 3))
    i = np.array([[1], [3], [0], [1]], dtype=np.int32)
    onehot = [np.zeros((1, n, 1)) for n in ns]
    for k in range(len(ns)):
        onehot[k][0, i[k, 0], 0] = 1.0
    a = oracle.full(R.project_tt(X, onehot)[0])
    b = oracle.full(R.project_sparse(X, i, np.array([1.0]))[0])
    assert np.abs(a - b).max() <= 1e-14


def test_project_tt_identity_idempotence_linearity():
    from oracle import riemannian as R
    ns = [3, 3, 4, 3]
    X = random_tt(4, ns, canonical_ranks(ns, 3))
    Y1 = random_tt(5, ns, [1, 3, 4, 2, 1])
    Y2 = random_tt(6, ns, [1, 2, 2, 2, 1])
    fx = oracle.full(X)
    # P_X(X) = X
    assert np.abs(oracle.full(R.project_tt(X, X)[0]) - fx).max() <= 1e-12 * np.abs(fx).max()
    # P(P(Y)) = P(Y)
    P1 = R.project_tt(X, Y1)[0]
    assert np.abs(oracle.full(R.project_tt(X, P1)[0]) - oracle.full(P1)).max() <= 1e-12 * np.abs(oracle.full(P1)).max()
    # P(2 Y1 - 3 Y2) = 2 P(Y1) - 3 P(Y2)
    Ysum = oracle.add(oracle.scale(Y1, 2.0), oracle.scale(Y2, -3.0))
    lhs = oracle.full(R.project_tt(X, Ysum)[0])
    rhs = 2 * oracle.full(P1) - 3 * oracle.full(R.project_tt(X, Y2)[0])
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


# ------------------------------------------------------ conjugate gradients

def _cg_problem():
    from workloads import random_cores
    ns = [8] * 4
    rng = np.random.default_rng(21)
    planted = random_cores(rng, ns, [1, 2, 2, 2, 1], 1 / np.sqrt(2))
    X0 = [c.astype(np.float64) for c in random_cores(rng, ns, [1, 2, 2, 2, 1], 0.5)]
    idx = random_indices(rng, ns, 2000)
    t = oracle.gather(planted, idx)
    idx_t = random_indices(rng, ns, 1000)
    return X0, idx, t, idx_t, oracle.gather(planted, idx_t)


def _tt_dist(A, B):
    D = oracle.add(A, oracle.scale(B, -1.0))
    return np.sqrt(max(oracle.inner(D, D), 0.0)) / np.sqrt(oracle.inner(B, B))


def test_cg_first_step_is_gradient_descent():
    """With no previous direction, eta = -P_X(grad): the CG step is the
    gradient step (same step length along the opposite sign convention)."""
    from oracle import riemannian as R
    X0, idx, t, _, _ = _cg_problem()
    cg = R.cg_iteration(X0, idx, t, 2)
    gd = R.completion_iteration(X0, idx, t, 2)
    assert cg["beta"] == 0.0
    assert cg["step"] == pytest.approx(gd["step"], rel=1e-12)
    assert _tt_dist(cg["Y"], gd["Y"]) < 1e-12


def test_cg_direction_beta_and_line_search():
    """Second step, checked with dense tensors: beta equals the
    Polak-Ribiere+ quotient formed with the dense projector at the new point
    (transport of the previous gradient), eta = -xi + beta P_X(eta') is a
    tangent vector (P_X eta = eta) and a descent direction, and the step
    zeroes the derivative of the linearised observed loss along eta."""
    from oracle import riemannian as R
    X0, idx, t, _, _ = _cg_problem()
    s1 = R.cg_iteration(X0, idx, t, 2)
    X1 = s1["Y"]
    s2 = R.cg_iteration(X1, idx, t, 2, s1)
    Pd = R.dense_projector(oracle.orthogonalize_lr(X1), oracle.orthogonalize_rl(X1))
    xi = oracle.full(s2["xi"]).reshape(-1)
    xi_prev = oracle.full(s1["xi"]).reshape(-1)
    eta_prev = oracle.full(s1["eta"]).reshape(-1)
    beta = max(0.0, float(xi @ (xi - Pd @ xi_prev)) / float(xi_prev @ xi_prev))
    assert beta > 0.0
    assert s2["beta"] == pytest.approx(beta, rel=1e-9)
    eta = oracle.full(s2["eta"]).reshape(-1)
    np.testing.assert_allclose(eta, -xi + beta * (Pd @ eta_prev), atol=1e-12 * np.abs(eta).max())
    np.testing.assert_allclose(Pd @ eta, eta, atol=1e-12 * np.abs(eta).max())
    assert float(xi @ eta) < 0.0
    y = oracle.gather(X1, idx)
    ev = oracle.gather(s2["eta"], idx)
    assert abs(float(np.dot(y + s2["step"] * ev - t, ev))) <= 1e-10 * float(np.dot(ev, ev)) * abs(s2["step"])


def test_cg_recovers_planted_tensor_faster_than_gd():
    """The noiseless planted rank-2 problem: after 30 steps CG's held-out
    RMSE is below 1e-8 and a hundred times below gradient descent's."""
    from oracle import riemannian as R
    X0, idx, t, idx_t, t_t = _cg_problem()
    Xc, hc = R.riemannian_cg(X0, idx, t, 2, 30, idx_t, t_t)
    Xg, _ = R.riemannian_completion(X0, idx, t, 2, 30, idx_t, t_t)
    ec = oracle.gather(Xc, idx_t) - t_t
    eg = oracle.gather(Xg, idx_t) - t_t
    rc, rg = float(np.sqrt(np.mean(ec * ec))), float(np.sqrt(np.mean(eg * eg)))
    assert rc < 1e-8 and rc < rg / 100
    assert all(h["beta"] >= 0.0 for h in hc)


def test_project_sum_linearity_and_dense_projector():
    """project_sum of a batch equals the weighted sum of the single
    projections, and the dense projector applied to the dense weighted sum,
    with X added for beta = 1."""
    from oracle import riemannian as R
    ns = [3, 4, 3, 2]
    X = _X(31, ns, 3)
    As = [_X(40 + i, ns, 2) for i in range(3)]
    c = [0.7, -1.3, 0.4]
    W = R.project_sum(X, As, c, alpha=0.5, beta=1.0)[0]
    single = [R.project_tt(X, A)[0] for A in As]
    dense = oracle.full(X) + 0.5 * sum(ci * oracle.full(S) for ci, S in zip(c, single))
    np.testing.assert_allclose(oracle.full(W), dense, atol=1e-12)
    P = R.dense_projector(oracle.orthogonalize_lr(X), oracle.orthogonalize_rl(X))
    z = sum(ci * oracle.full(A).reshape(-1) for ci, A in zip(c, As))
    np.testing.assert_allclose(oracle.full(W).reshape(-1), oracle.full(X).reshape(-1) + 0.5 * (P @ z), atol=1e-12)


def test_tangent_gram_dense_and_block_identity():
    """The tangent Gram matrix equals the Gram matrix of the dense tensors,
    and the sum of the dG block inner products (the gauge condition makes
    the tangent terms orthogonal); it is symmetric positive semidefinite."""
    from oracle import riemannian as R
    ns = [3, 4, 3, 2]
    X = _X(61, ns, 3)
    outs = [R.project_tt(X, _X(70 + i, ns, 2)) for i in range(4)]
    Ws = [o[0] for o in outs]
    G = R.tangent_gram(Ws)
    F = np.stack([oracle.full(W).reshape(-1) for W in Ws])
    np.testing.assert_allclose(G, F @ F.T, atol=1e-12)
    blocks = np.array([[sum(np.vdot(a, b) for a, b in zip(oi[3], oj[3])) for oj in outs] for oi in outs])
    np.testing.assert_allclose(G, blocks, atol=1e-12)
    assert np.array_equal(G, G.T) or np.allclose(G, G.T, atol=1e-14)
    assert np.linalg.eigvalsh(G).min() > -1e-12


@pytest.mark.parametrize("kind", ["squared", "huber", "logistic"])
def test_observed_loss_gradient_is_the_derivative(kind):
    """Central differences of the observed loss in each y_m match g_m (the
    losses are smooth away from Huber's two kinks, which the draw avoids)."""
    rng = np.random.default_rng(71)
    M = 40
    y = rng.standard_normal(M) * 1.5
    t = np.sign(rng.standard_normal(M)) if kind == "logistic" else rng.standard_normal(M)
    delta = 0.7
    if kind == "huber":
        r = y - t
        keep = np.abs(np.abs(r) - delta) > 1e-2
        y, t = y[keep], t[keep]
    L, g = R.observed_loss(y, t, kind, delta)
    h = 1e-6
    for m in range(len(y)):
        yp, ym = y.copy(), y.copy()
        yp[m] += h
        ym[m] -= h
        fd = (R.observed_loss(yp, t, kind, delta)[0] - R.observed_loss(ym, t, kind, delta)[0]) / (2 * h)
        assert abs(fd - g[m]) <= 1e-6 * max(1.0, abs(g[m])) / len(y)


def test_observed_loss_closed_forms():
    """Huber with delta above every residual is half the squared loss; Huber
    with a tiny delta is delta times the mean absolute residual (to first
    order); the logistic loss is log 2 at y = 0 for either label and
    symmetric under (y, t) -> (-y, -t)."""
    rng = np.random.default_rng(72)
    y, t = rng.standard_normal(50), rng.standard_normal(50)
    Ls, gs = R.observed_loss(y, t, "squared")
    Lh, gh = R.observed_loss(y, t, "huber", delta=100.0)
    assert abs(Lh - 0.5 * Ls) <= 1e-15 and np.allclose(gh, 0.5 * gs, rtol=0, atol=1e-15)
    d = 1e-6
    Lt, _ = R.observed_loss(y, t, "huber", delta=d)
    assert abs(Lt - d * np.mean(np.abs(y - t))) <= d * d
    lab = np.sign(rng.standard_normal(50))
    L0, _ = R.observed_loss(np.zeros(50), lab, "logistic")
    assert abs(L0 - np.log(2.0)) <= 1e-15
    La, ga = R.observed_loss(y, lab, "logistic")
    Lb, gb = R.observed_loss(-y, -lab, "logistic")
    assert abs(La - Lb) <= 1e-15 and np.allclose(ga, -gb, rtol=0, atol=1e-15)


def test_riemannian_gradient_gives_the_directional_derivative():
    """For tangent vectors xi at X, <P_X G, xi> equals the derivative of the
    observed loss along xi (central differences of f(X + h xi), exact for
    the squared loss since f is quadratic along a line): the defining
    property of the Riemannian gradient; and P_X G of a sparse G is the
    sparse projection."""
    from oracle import core as K
    rng = np.random.default_rng(73)
    ns, ranks = [3, 4, 3, 2], [1, 2, 3, 2, 1]
    X = [rng.standard_normal((ranks[k], ns[k], ranks[k + 1])) for k in range(4)]
    M = 30
    idx = np.stack([rng.integers(0, n, M) for n in ns]).astype(np.int32)
    t = rng.standard_normal(M)
    for kind in ("squared", "huber", "logistic"):
        tk = np.sign(t) if kind == "logistic" else t
        f = lambda cores: R.observed_loss(K.gather(cores, idx), tk, kind, 0.5)[0]
        _, g = R.observed_loss(K.gather(X, idx), tk, kind, 0.5)
        G = np.zeros(ns)
        np.add.at(G, tuple(idx), g)
        PG = R.riemannian_grad_dense(X, G)
        Wsp = R.project_sparse(X, idx, g)[0]
        assert np.abs(K.full(Wsp) - PG).max() <= 1e-12 * max(1.0, np.abs(PG).max())
        U = R.orthogonalize_lr(X)
        V = R.orthogonalize_rl(X)
        for j in range(3):
            H = [rng.standard_normal(c.shape) for c in X]
            xi_cores = R.tangent_tt(U, V, R.tangent_cores(U, H), 1.0, 0.0)
            xi = K.full(xi_cores)
            h = 1e-5
            Xp = K.add(X, K.scale(xi_cores, h))
            Xm = K.add(X, K.scale(xi_cores, -h))
            fd = (f(Xp) - f(Xm)) / (2 * h)
            assert abs(fd - float(np.sum(PG * xi))) <= 1e-6 * max(1.0, abs(fd))
