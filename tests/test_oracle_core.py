"""Pins of the FP64 oracle's TT-format core: gather, adjoint, inner products.

Each test checks the oracle against something other than itself: closed
forms, textbook routines (matrix products, Kronecker products), invariants of
the mathematics, exact finite differences, or CPU autograd.
"""
import json
import os

import numpy as np
import pytest

import oracle
from workloads import random_tt, random_indices, uniform_ranks, small_step

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(s):
    return np.random.default_rng(1000 + s)


# --------------------------------------------------------------------- format

def test_storage_count_golden():
    """Introduction: storage r*n*(r*(d-2)+2) for a uniform TT; the cores the
    generator draws have exactly that many scalars."""
    cases = json.load(open(os.path.join(GOLDEN, "storage_count.json")))["cases"]
    for c in cases:
        d, n, r = c["d"], c["n"], c["r"]
        assert oracle.storage_count(d, n, r) == c["count"]
        cores = random_tt(0, [n] * d, uniform_ranks(d, r))
        assert sum(x.size for x in cores) == c["count"]


def test_full_d2_is_matrix_product():
    """d=2: the entry formula is the matrix product G^1 G^2 (textbook)."""
    A = random_tt(1, [5, 7], [1, 3, 1])
    M = A[0][0].astype(np.float64) @ A[1][:, :, 0].astype(np.float64)
    np.testing.assert_allclose(oracle.full(A), M, rtol=1e-14, atol=1e-14)


def test_full_rank1_is_outer_product():
    """r=1: A = a_1 (x) a_2 (x) ... (x) a_d (C-ordered outer product)."""
    A = random_tt(2, [3, 4, 2, 5], [1, 1, 1, 1, 1])
    vs = [c[0, :, 0].astype(np.float64) for c in A]
    T = vs[0]
    for v in vs[1:]:
        T = np.multiply.outer(T, v)
    np.testing.assert_allclose(oracle.full(A), T, rtol=1e-14)


def _sum_tt(xs):
    """Exact rank-2 TT of f(i_1..i_d) = sum_k x_k[i_k]: G^1[i] = [x_1[i], 1],
    G^k[i] = [[1, 0], [x_k[i], 1]], G^d[i] = [1; x_d[i]]."""
    d = len(xs)
    cores = []
    for k, x in enumerate(xs):
        n = len(x)
        if k == 0:
            c = np.zeros((1, n, 2)); c[0, :, 0] = x; c[0, :, 1] = 1
        elif k == d - 1:
            c = np.zeros((2, n, 1)); c[0, :, 0] = 1; c[1, :, 0] = x
        else:
            c = np.zeros((2, n, 2)); c[0, :, 0] = 1; c[1, :, 0] = x; c[1, :, 1] = 1
        cores.append(c)
    return cores


def test_gather_closed_form_sum_function():
    """A rank-2 TT with a closed-form entry: catches transposed or
    mis-ordered slices (the lower-triangular middle cores are not symmetric)."""
    rng = _rng(3)
    ns = [4, 3, 5, 2, 6]
    xs = [rng.standard_normal(n) for n in ns]
    X = _sum_tt(xs)
    idx = random_indices(rng, ns, 500)
    expect = sum(xs[k][idx[k]] for k in range(len(ns)))
    np.testing.assert_allclose(oracle.gather(X, idx), expect, rtol=1e-13, atol=1e-13)
    F = oracle.full(X)
    grid = np.indices(ns)
    np.testing.assert_allclose(F, sum(xs[k][grid[k]] for k in range(len(ns))), rtol=1e-13, atol=1e-13)


def test_gather_matches_full_small_step():
    """Brute force: every one of the 8^4 cells of the small-step TT."""
    p = small_step()
    X = [c.astype(np.float64) for c in p.cores]
    F = oracle.full(X)
    grid = np.indices(p.ns).reshape(len(p.ns), -1)
    np.testing.assert_allclose(oracle.gather(X, grid), F.reshape(-1), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(oracle.gather(X, p.idx), F[tuple(p.idx)], rtol=1e-12, atol=1e-14)


def test_gather_d2_and_r1():
    rng = _rng(4)
    A = random_tt(5, [6, 9], [1, 4, 1])
    idx = random_indices(rng, [6, 9], 300)
    M = A[0][0].astype(np.float64) @ A[1][:, :, 0].astype(np.float64)
    np.testing.assert_allclose(oracle.gather(A, idx), M[idx[0], idx[1]], rtol=1e-13)
    B = random_tt(6, [3, 4, 5], [1, 1, 1, 1])
    idx = random_indices(rng, [3, 4, 5], 100)
    prod = np.prod([B[k][0, idx[k], 0].astype(np.float64) for k in range(3)], axis=0)
    np.testing.assert_allclose(oracle.gather(B, idx), prod, rtol=1e-13)


def test_gather_multilinear():
    """The entry formula is linear in each core."""
    rng = _rng(5)
    ns, rk = [4, 5, 3, 6], [1, 3, 2, 4, 1]
    X = [c.astype(np.float64) for c in random_tt(7, ns, rk)]
    idx = random_indices(rng, ns, 200)
    for k in range(4):
        A = rng.standard_normal(X[k].shape)
        B = rng.standard_normal(X[k].shape)
        a, b = 1.7, -0.3
        XA = list(X); XA[k] = A
        XB = list(X); XB[k] = B
        XC = list(X); XC[k] = a * A + b * B
        np.testing.assert_allclose(oracle.gather(XC, idx),
                                   a * oracle.gather(XA, idx) + b * oracle.gather(XB, idx),
                                   rtol=1e-12, atol=1e-12)


def test_gather_empty():
    X = random_tt(8, [3, 3], [1, 2, 1])
    assert oracle.gather(X, np.zeros((2, 0), np.int32)).shape == (0,)
    g = oracle.gather_backward(X, np.zeros((2, 0), np.int32), np.zeros(0))
    assert all(np.all(x == 0) for x in g)


# -------------------------------------------------------------------- adjoint

def _problem(seed, ns, rk, M):
    rng = _rng(seed)
    X = [c.astype(np.float64) for c in random_tt(seed, ns, rk)]
    idx = random_indices(rng, ns, M)
    g = rng.standard_normal(M)
    return rng, X, idx, g


def test_adjoint_dot_product():
    """<gather(X with G^k := H), g> = <H, grad_k(g)> (y is linear in G^k)."""
    rng, X, idx, g = _problem(10, [4, 5, 3, 6, 2], [1, 3, 4, 2, 3, 1], 400)
    grads = oracle.gather_backward(X, idx, g)
    for k in range(len(X)):
        H = rng.standard_normal(X[k].shape)
        XH = list(X); XH[k] = H
        lhs = np.dot(oracle.gather(XH, idx), g)
        rhs = np.sum(H * grads[k])
        assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs))


def test_adjoint_euler_identity():
    """<grad_k, G^k> = sum_m g_m y_m for every k (degree-1 homogeneity)."""
    rng, X, idx, g = _problem(11, [5, 4, 6, 3], [1, 4, 3, 5, 1], 600)
    y = oracle.gather(X, idx)
    grads = oracle.gather_backward(X, idx, g)
    s = np.dot(g, y)
    for k in range(len(X)):
        assert abs(np.sum(grads[k] * X[k]) - s) <= 1e-11 * max(1.0, abs(s))


def test_adjoint_exact_central_differences():
    """The MSE is quadratic in any single core entry, so the central
    difference quotient is exact up to roundoff."""
    rng, X, idx, _ = _problem(12, [4, 4, 4, 4], [1, 3, 3, 3, 1], 300)
    t = rng.standard_normal(300)
    y = oracle.gather(X, idx)
    loss, g = oracle.mse_loss_and_grad(y, t)
    grads = oracle.gather_backward(X, idx, g)
    for _ in range(24):
        k = rng.integers(0, 4)
        pos = tuple(rng.integers(0, s) for s in X[k].shape)
        h = 0.1 * max(1.0, abs(X[k][pos]))
        vals = []
        for sgn in (1, -1):
            Xp = [c.copy() for c in X]
            Xp[k][pos] += sgn * h
            vals.append(oracle.mse_loss_and_grad(oracle.gather(Xp, idx), t)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - grads[k][pos]) <= 1e-10 * max(1.0, abs(fd))


def test_adjoint_matches_torch_autograd():
    """CPU autograd of a float64 chain agrees with the hand-written adjoint."""
    torch = pytest.importorskip("torch")
    rng, X, idx, g = _problem(13, [3, 5, 4], [1, 2, 3, 1], 250)
    Ct = [torch.tensor(c, requires_grad=True) for c in X]
    it = torch.tensor(idx.astype(np.int64))
    v = Ct[0][0][it[0]]                                   # (M, r1)
    for k in range(1, 3):
        S = Ct[k].permute(1, 0, 2)[it[k]]                 # (M, r_k, r_{k+1})
        v = torch.bmm(v[:, None, :], S)[:, 0, :]
    (v[:, 0] * torch.tensor(g)).sum().backward()
    grads = oracle.gather_backward(X, idx, g)
    for k in range(3):
        np.testing.assert_allclose(grads[k], Ct[k].grad.numpy(), rtol=1e-12, atol=1e-13)


def test_adjoint_duplicates_sum():
    """A repeated multi-index contributes once per occurrence."""
    rng, X, idx, g = _problem(14, [3, 3, 3], [1, 2, 2, 1], 50)
    idx2 = np.concatenate([idx, idx[:, :10]], axis=1)
    g2 = np.concatenate([g, g[:10]])
    g1 = g.copy(); g1[:10] *= 2
    a = oracle.gather_backward(X, idx2, g2)
    b = oracle.gather_backward(X, idx, g1)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=1e-13, atol=1e-14)


def test_mse_loss_closed_form():
    y = np.array([1.0, 2.0, 4.0]); t = np.array([0.0, 2.0, 1.0])
    loss, g = oracle.mse_loss_and_grad(y, t)
    assert loss == pytest.approx((1 + 0 + 9) / 3)
    np.testing.assert_allclose(g, [2 / 3, 0, 2.0])


# ---------------------------------------------------------- inner, gram, add

def test_inner_matches_full():
    A = random_tt(20, [3, 4, 2, 3], [1, 2, 3, 2, 1])
    B = random_tt(21, [3, 4, 2, 3], [1, 3, 1, 4, 1])
    ref = np.sum(oracle.full(A) * oracle.full(B))
    assert oracle.inner(A, B) == pytest.approx(ref, rel=1e-12)
    assert oracle.norm(A) == pytest.approx(np.linalg.norm(oracle.full(A)), rel=1e-12)


def test_gram_symmetric_psd_and_padding():
    ns = [3, 4, 3]
    As = [random_tt(30 + i, ns, [1, 1 + i % 3, 2, 1]) for i in range(6)]
    G = oracle.gram(As)
    np.testing.assert_allclose(G, G.T)
    assert np.linalg.eigvalsh(G).min() > -1e-10 * np.abs(G).max()
    F = np.stack([oracle.full(a).reshape(-1) for a in As])
    np.testing.assert_allclose(G, F @ F.T, rtol=1e-12, atol=1e-12)
    Ap = [oracle.pad_ranks(a, [1, 4, 4, 1]) for a in As]
    np.testing.assert_allclose(oracle.gram(Ap), G, rtol=1e-13, atol=1e-13)
    Bs = [random_tt(50 + i, ns, [1, 2, 2, 1]) for i in range(3)]
    FB = np.stack([oracle.full(b).reshape(-1) for b in Bs])
    np.testing.assert_allclose(oracle.gram(As, Bs), F @ FB.T, rtol=1e-12, atol=1e-12)


def test_add_and_scale():
    A = random_tt(40, [3, 2, 4], [1, 2, 3, 1])
    B = random_tt(41, [3, 2, 4], [1, 3, 2, 1])
    np.testing.assert_allclose(oracle.full(oracle.add(A, B)), oracle.full(A) + oracle.full(B), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(oracle.full(oracle.scale(A, -2.5)), -2.5 * oracle.full(A), rtol=1e-13)
