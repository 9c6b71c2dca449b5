"""Pins of the FP64 oracle's TT-matrix layer (Y = X W^T and its adjoint).

W is pinned against Kronecker products (a rank-1 TT-matrix is the C-ordered
Kronecker product of its core slices; a rank-2 one can represent a Kronecker
sum), the adjoint against exact central differences, the Euler identity and
the generic sparse adjoint of the TT view.
"""
import numpy as np
import pytest

import oracle


def _rng(s):
    return np.random.default_rng(3000 + s)


def _cores(rng, ms, ns, ranks):
    return [rng.standard_normal((ranks[k], ms[k], ns[k], ranks[k + 1])) for k in range(len(ms))]


def test_rank1_is_kronecker_product():
    rng = _rng(0)
    ms, ns = [2, 3, 2], [3, 2, 4]
    A = [rng.standard_normal((m, n)) for m, n in zip(ms, ns)]
    cores = [a[None, :, :, None] for a in A]
    W = oracle.ttm_full(cores)
    np.testing.assert_allclose(W, np.kron(np.kron(A[0], A[1]), A[2]), rtol=1e-13)


def test_rank2_kronecker_sum():
    """cores [[A, I]] , [[I], [B]] give A (x) I + I (x) B."""
    rng = _rng(1)
    A = rng.standard_normal((3, 3))
    B = rng.standard_normal((4, 4))
    c1 = np.zeros((1, 3, 3, 2)); c1[0, :, :, 0] = A; c1[0, :, :, 1] = np.eye(3)
    c2 = np.zeros((2, 4, 4, 1)); c2[0, :, :, 0] = np.eye(4); c2[1, :, :, 0] = B
    W = oracle.ttm_full([c1, c2])
    np.testing.assert_allclose(W, np.kron(A, np.eye(4)) + np.kron(np.eye(3), B), rtol=1e-13, atol=1e-14)


def test_forward_is_row_batch_product():
    rng = _rng(2)
    ms, ns, rk = [2, 3, 2], [2, 2, 3], [1, 3, 2, 1]
    cores = _cores(rng, ms, ns, rk)
    X = rng.standard_normal((5, 12))
    W = oracle.ttm_full(cores)
    np.testing.assert_allclose(oracle.ttm_forward(X, cores), X @ W.T, rtol=1e-13)
    # entry formula for one element of W
    i, j = (1, 2, 0), (0, 1, 2)
    v = np.ones((1, 1))
    for k in range(3):
        v = v @ cores[k][:, i[k], j[k], :]
    row = (i[0] * ms[1] + i[1]) * ms[2] + i[2]
    col = (j[0] * ns[1] + j[1]) * ns[2] + j[2]
    assert W[row, col] == pytest.approx(v[0, 0], rel=1e-13)


def test_backward_exact_fd_euler_and_sparse_adjoint():
    rng = _rng(3)
    ms, ns, rk = [2, 3, 2], [3, 2, 2], [1, 3, 4, 1]
    cores = _cores(rng, ms, ns, rk)
    X = rng.standard_normal((6, 12))
    dY = rng.standard_normal((6, 12))
    dX, dG = oracle.ttm_backward(X, cores, dY)
    Y = oracle.ttm_forward(X, cores)
    L0 = np.sum(dY * Y)
    # Euler identity: L is linear in each core
    for k in range(3):
        assert np.sum(dG[k] * cores[k]) == pytest.approx(L0, rel=1e-11)
    # exact central differences (L linear in every parameter)
    for _ in range(20):
        k = rng.integers(0, 3)
        pos = tuple(rng.integers(0, s) for s in cores[k].shape)
        h = 0.5
        vals = []
        for s in (1, -1):
            c2 = [c.copy() for c in cores]
            c2[k][pos] += s * h
            vals.append(np.sum(dY * oracle.ttm_forward(X, c2)))
        assert (vals[0] - vals[1]) / (2 * h) == pytest.approx(dG[k][pos], rel=1e-10, abs=1e-11)
    for _ in range(10):
        pos = (rng.integers(0, 6), rng.integers(0, 12))
        X2 = X.copy(); X2[pos] += 1.0
        assert np.sum(dY * oracle.ttm_forward(X2, cores)) - L0 == pytest.approx(dX[pos], rel=1e-10, abs=1e-11)
    # the generic adjoint on the TT view (modes m_k n_k, every entry observed)
    view = [c.reshape(c.shape[0], c.shape[1] * c.shape[2], c.shape[3]) for c in cores]
    W = oracle.ttm_full(cores)
    dW = dY.T @ X
    T = dW.reshape(ms + ns).transpose(0, 3, 1, 4, 2, 5).reshape(-1)
    grid = np.indices([m * n for m, n in zip(ms, ns)]).reshape(3, -1)
    ga = oracle.gather_backward(view, grid, T)
    for k in range(3):
        np.testing.assert_allclose(ga[k].reshape(cores[k].shape), dG[k], rtol=1e-11, atol=1e-12)
    assert W.shape == (12, 12)


def test_tt_matvec_dense_product_and_identity():
    """The TT-format product equals the dense matrix-vector product, its
    ranks multiply, and an identity TT-matrix (rank-1 eye cores) returns the
    vector's own cores."""
    import oracle
    rng = np.random.default_rng(5)
    ms, ns, rw, rx = [2, 3, 2], [3, 2, 4], [1, 2, 3, 1], [1, 3, 2, 1]
    Wc = [rng.standard_normal((rw[k], ms[k], ns[k], rw[k + 1])) for k in range(3)]
    xc = [rng.standard_normal((rx[k], ns[k], rx[k + 1])) for k in range(3)]
    y = oracle.tt_matvec(Wc, xc)
    assert [c.shape for c in y] == [(1, 2, 6), (6, 3, 6), (6, 2, 1)]
    np.testing.assert_allclose(oracle.full(y).reshape(-1), oracle.ttm_full(Wc) @ oracle.full(xc).reshape(-1),
                               rtol=1e-12, atol=1e-12)
    eye = [np.eye(n).reshape(1, n, n, 1) for n in ns]
    for a, b in zip(oracle.tt_matvec(eye, xc), xc):
        assert np.array_equal(a, b)


def test_tt_matmat_dense_product_and_matvec():
    """The TT-format matrix product equals the dense product of the dense
    matrices; with a one-column right factor it is the matvec."""
    import oracle
    rng = np.random.default_rng(6)
    ms, ns, ls, ra, rb = [2, 3, 2], [3, 2, 2], [2, 1, 3], [1, 2, 3, 1], [1, 3, 2, 1]
    A = [rng.standard_normal((ra[k], ms[k], ns[k], ra[k + 1])) for k in range(3)]
    B = [rng.standard_normal((rb[k], ns[k], ls[k], rb[k + 1])) for k in range(3)]
    Cc = oracle.tt_matmat(A, B)
    assert [c.shape for c in Cc] == [(1, 2, 2, 6), (6, 3, 1, 6), (6, 2, 3, 1)]
    np.testing.assert_allclose(oracle.ttm_full(Cc), oracle.ttm_full(A) @ oracle.ttm_full(B), rtol=1e-12, atol=1e-12)
    x = [rng.standard_normal((rb[k], ns[k], rb[k + 1])) for k in range(3)]
    as_mat = oracle.tt_matmat(A, [c.reshape(c.shape[0], c.shape[1], 1, c.shape[2]) for c in x])
    for a, b in zip(as_mat, oracle.tt_matvec(A, x)):
        np.testing.assert_array_equal(a[:, :, 0, :], b)
