"""FP64 oracle: the TT-matrix layer Y = X W^T and its adjoint.

Test infrastructure only (see the package docstring).

Paper, Implementation Details: a TT-matrix used as a neural-network layer
through ``t3f.matmul(tt_matrix, x)``.  A TT-matrix core G^k has shape
(r_k, m_k, n_k, r_{k+1}) with m_k the row (output) mode and n_k the column
(input) mode, and W[(i_1..i_d), (j_1..j_d)] = G^1[i_1, j_1] ... G^d[i_d, j_d]
(the entry formula applied to the paired indices (i_k, j_k)).  The product
is taken with x as a column; a batch of rows X therefore gives Y = X W^T.
Row and column multi-indices are C-ordered.
"""
import numpy as np

from .core import full


def _tt_view(cores):
    """The TT-matrix as a TT tensor with mode sizes m_k * n_k (index i_k*n_k + j_k)."""
    return [np.asarray(c, dtype=np.float64).reshape(c.shape[0], c.shape[1] * c.shape[2], c.shape[3])
            for c in cores]


def ttm_full(cores):
    """Dense W (prod m_k x prod n_k) of a TT-matrix."""
    d = len(cores)
    ms = [c.shape[1] for c in cores]
    ns = [c.shape[2] for c in cores]
    t = full(_tt_view(cores))  # shape (m1 n1, ..., md nd)
    t = t.reshape([x for pair in zip(ms, ns) for x in pair])  # (m1, n1, ..., md, nd)
    t = t.transpose(list(range(0, 2 * d, 2)) + list(range(1, 2 * d, 2)))
    return t.reshape(int(np.prod(ms)), int(np.prod(ns)))


def ttm_forward(X, cores):
    """Y = X W^T for a batch of input rows X (B x prod n_k)."""
    return np.asarray(X, dtype=np.float64) @ ttm_full(cores).T


def ttm_backward(X, cores, dY):
    """Adjoint of ``ttm_forward``: returns (dX, [dG^k]).

    dX = dY W.  With dW = dY^T X (the gradient of <dY, X W^T> with respect to
    W), the gradient with respect to core k is the sum over all entries of W of
    dW times the derivative of the entry, i.e. dW contracted with the left
    interface (product of cores 1..k-1) and the right interface (product of
    cores k+1..d) of the TT view; the entry formula is linear in each core.
    """
    X = np.asarray(X, dtype=np.float64)
    dY = np.asarray(dY, dtype=np.float64)
    W = ttm_full(cores)
    dX = dY @ W
    dW = dY.T @ X
    d = len(cores)
    ms = [c.shape[1] for c in cores]
    ns = [c.shape[2] for c in cores]
    # dW in TT-view order (m1 n1, ..., md nd)
    T = dW.reshape(ms + ns).transpose([a for k in range(d) for a in (k, d + k)])
    T = T.reshape([m * n for m, n in zip(ms, ns)])
    V = _tt_view(cores)
    grads = []
    for k in range(d):
        # left interface (P x r_k) and right interface (r_{k+1} x S)
        if k == 0:
            Lk = np.ones((1, 1))
        else:
            t = V[0]
            for c in V[1:k]:
                t = np.tensordot(t, c, axes=([t.ndim - 1], [0]))
            Lk = t.reshape(-1, t.shape[-1])
        if k == d - 1:
            Rk = np.ones((1, 1))
        else:
            t = V[k + 1]
            for c in V[k + 2:]:
                t = np.tensordot(t, c, axes=([t.ndim - 1], [0]))
            Rk = t.reshape(t.shape[0], -1)
        mk = V[k].shape[1]
        Tk = T.reshape(Lk.shape[0], mk, Rk.shape[1])
        g = np.tensordot(Lk.T, Tk, axes=([1], [0]))          # (r_k, mk, S)
        g = np.tensordot(g, Rk.T, axes=([2], [0]))           # (r_k, mk, r_{k+1})
        grads.append(g.reshape(cores[k].shape))
    return dX, grads


def tt_matvec(W, x):
    """The TT-matrix by TT-vector product in the TT format (Implementation
    Details: products of TT objects; Table 1 times it as matvec): for W
    cores (r_k, m_k, n_k, r_{k+1}) and x cores (s_k, n_k, s_{k+1}), the cores
    y_k[(a, b), i, (a', b')] = sum_j W_k[a, i, j, a'] x_k[b, j, b'], bond
    index a s_k + b.  Exact; the ranks multiply."""
    out = []
    for Wk, xk in zip(W, x):
        Wk = np.asarray(Wk, dtype=np.float64)
        xk = np.asarray(xk, dtype=np.float64)
        r0, m, n, r1 = Wk.shape
        s0, _, s1 = xk.shape
        out.append(np.einsum("aijc,bjd->abicd", Wk, xk).reshape(r0 * s0, m, r1 * s1))
    return out


def tt_matmat(A, B):
    """The TT-matrix by TT-matrix product in the TT format (Table 1 times it
    as matmul): for A cores (r_k, m_k, n_k, r_{k+1}) and B cores
    (s_k, n_k, l_k, s_{k+1}), C_k[(a, b), i, l, (a', b')] =
    sum_j A_k[a, i, j, a'] B_k[b, j, l, b'], bond index a s_k + b."""
    out = []
    for Ak, Bk in zip(A, B):
        Ak = np.asarray(Ak, dtype=np.float64)
        Bk = np.asarray(Bk, dtype=np.float64)
        r0, m, n, r1 = Ak.shape
        s0, _, lk, s1 = Bk.shape
        out.append(np.einsum("aijc,bjld->abilcd", Ak, Bk).reshape(r0 * s0, m, lk, r1 * s1))
    return out
