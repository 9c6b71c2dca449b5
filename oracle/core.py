"""FP64 oracle: TT format, gather, its adjoint, inner products and Gram.

Test infrastructure only (see the package docstring).  Parity of every
function here is pinned in ``tests/test_oracle_core.py`` against brute force,
closed forms and invariants that do not reuse the function under test.
"""
import numpy as np
import scipy.sparse as sp

_CHUNK = 65536  # entries per vectorised chunk (bounds the size of temporaries)


def storage_count(d, n, r):
    """Number of scalars of a uniform TT tensor: r*n*(r*(d-2)+2).

    Paper, Introduction: the storage formula stated after the TT-core
    definition (cores G^1 n x r, G^2..G^{d-1} r x n x r, G^d r x n).
    """
    return r * n * (r * (d - 2) + 2)


def ranks_of(cores):
    """Bond ranks (r_0, ..., r_d) of a TT given as cores (r_k, n_k, r_{k+1})."""
    return [cores[0].shape[0]] + [c.shape[2] for c in cores]


def full(cores):
    """Dense tensor of a TT by chained tensordot (tiny sizes only).

    Paper, Introduction, entry formula: A[i_1..i_d] is the sum over all
    auxiliary indices alpha_k of the products of core elements.  Contracting
    the cores one bond at a time evaluates exactly that sum for every
    multi-index at once; the result is C-ordered (i_1 slowest).
    """
    cores = [np.asarray(c, dtype=np.float64) for c in cores]
    t = cores[0]
    for c in cores[1:]:
        t = np.tensordot(t, c, axes=([t.ndim - 1], [0]))
    # t has shape (1, n_1, ..., n_d, 1)
    return t.reshape(t.shape[1:-1])


def _slices(core, ik):
    """Core slices G^k[i] for a vector of mode indices: shape (m, r_k, r_{k+1})."""
    return core.transpose(1, 0, 2)[ik]


def gather(cores, idx):
    """Entries of a TT at observed multi-indices.

    Paper, Introduction, entry formula: y_m = G^1[i_1] G^2[i_2] ... G^d[i_d],
    the product of the core slices selected by the multi-index.  Evaluated left
    to right as a row vector times one slice per mode.
    """
    cores = [np.asarray(c, dtype=np.float64) for c in cores]
    idx = np.asarray(idx)
    d, M = idx.shape
    assert d == len(cores)
    y = np.empty(M, dtype=np.float64)
    for s in range(0, M, _CHUNK):
        e = min(M, s + _CHUNK)
        v = _slices(cores[0], idx[0, s:e])[:, 0, :]  # (m, r_1)
        for k in range(1, d):
            S = _slices(cores[k], idx[k, s:e])  # (m, r_k, r_{k+1})
            v = np.matmul(v[:, None, :], S)[:, 0, :]
        y[s:e] = v[:, 0]
    return y


def sparse_adjoint(left_cores, right_cores, idx, w):
    """Weighted sum of the per-entry core derivatives (the gather's adjoint).

    For every mode k and slice i it returns
        Z_k[:, i, :] = sum over m with i_k^m = i of  w_m * L_m^{(k)T} R_m^{(k)T}
    with the left partial L_m^{(k)} = left[0][i_1] ... left[k-1][i_{k-1}]
    (a row of size r_k) and the right partial
    R_m^{(k)} = right[k+1][i_{k+1}] ... right[d-1][i_d] (a column of size
    r_{k+1}).  Repeated multi-indices contribute once per occurrence.

    With ``left = right = X`` this is the gradient of sum_m w_m y_m with
    respect to every core (the entry formula is linear in each core: the
    automatic-differentiation feature of the abstract).  With the left- and
    right-orthonormal cores of X it is the core contraction of the tangent
    projection of a sparse tensor: Riemannian Geometry Operations section,
    project_sum of M one-hot rank-1 tensors weighted by w.

    The sum over entries for each slice is a one-hot (M x n_k) matrix product,
    i.e. the definition written as a sparse matrix times the per-entry outer
    products.
    """
    left_cores = [np.asarray(c, dtype=np.float64) for c in left_cores]
    right_cores = [np.asarray(c, dtype=np.float64) for c in right_cores]
    idx = np.asarray(idx)
    w = np.asarray(w, dtype=np.float64)
    d, M = idx.shape
    shapes = []
    for k in range(d):
        rl = left_cores[k].shape[0] if k > 0 else 1
        rr = right_cores[k].shape[2] if k < d - 1 else 1
        n = right_cores[k].shape[1]
        shapes.append((rl, n, rr))
    out = [np.zeros(s) for s in shapes]
    for s0 in range(0, M, _CHUNK):
        e0 = min(M, s0 + _CHUNK)
        m = e0 - s0
        ik = idx[:, s0:e0]
        # right partials R^{(k)} for k = d-1 .. 0 (column vectors, shape (m, r_{k+1}))
        R = [None] * d
        R[d - 1] = np.ones((m, 1))
        for k in range(d - 1, 0, -1):
            S = _slices(right_cores[k], ik[k])
            R[k - 1] = np.matmul(S, R[k][:, :, None])[:, :, 0]
        L = np.ones((m, 1))
        for k in range(d):
            contrib = w[s0:e0, None, None] * L[:, :, None] * R[k][:, None, :]
            onehot = sp.csr_matrix(
                (np.ones(m), (ik[k], np.arange(m))), shape=(shapes[k][1], m))
            acc = onehot @ contrib.reshape(m, -1)  # (n_k, r_k * r_{k+1})
            out[k] += acc.reshape(shapes[k][1], shapes[k][0], shapes[k][2]).transpose(1, 0, 2)
            if k < d - 1:
                S = _slices(left_cores[k], ik[k])
                L = np.matmul(L[:, None, :], S)[:, 0, :]
    return out


def gather_backward(cores, idx, gy):
    """Gradient of sum_m gy_m * y_m with respect to every core.

    Adjoint of ``gather`` (automatic differentiation, abstract and
    Introduction): the entry formula is linear in each core, so the
    derivative of y_m with respect to G^k[:, i_k^m, :] is the outer product of
    the left and right partial products.  See ``sparse_adjoint``.
    """
    return sparse_adjoint(cores, cores, idx, gy)


def mse_loss_and_grad(y, t):
    """Completion loss L = mean((y - t)^2) and its gradient g = 2 (y - t) / M.

    Paper, Introduction: tensor completion minimises the residual between the
    low-rank tensor and the known elements.  The squared residual averaged over
    the observed entries is the reading used here.
    """
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    M = y.shape[0]
    rho = y - t
    loss = float(np.dot(rho, rho) / M) if M else 0.0
    return loss, (2.0 / M) * rho if M else rho


def inner(A, B):
    """Frobenius inner product <A, B> of two TT tensors of the same mode sizes.

    Computed by the bond-by-bond contraction Phi_0 = 1,
    Phi_k = sum_i A^k[i]^T Phi_{k-1} B^k[i], <A, B> = Phi_d: the sum over all
    multi-indices of products of entries (Introduction, entry formula), with
    the sums over indices moved inside.  Used by the Gram matrix of the
    Riemannian Geometry Operations section and by the Table 1 'gram' and
    'norm' operations.
    """
    phi = np.ones((1, 1))
    for a, b in zip(A, B):
        a = np.asarray(a, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        phi = sum(a[:, i, :].T @ phi @ b[:, i, :] for i in range(a.shape[1]))
    return float(phi[0, 0])


def gram(As, Bs=None):
    """Gram matrix G[a, b] = <As[a], Bs[b]> of two lists of TT tensors."""
    sym = Bs is None
    Bs = As if sym else Bs
    G = np.empty((len(As), len(Bs)))
    for a in range(len(As)):
        for b in range(len(Bs)):
            if sym and b < a:
                G[a, b] = G[b, a]
            else:
                G[a, b] = inner(As[a], Bs[b])
    return G


def norm(A):
    """Frobenius norm of a TT tensor (Table 1, 'norm')."""
    return float(np.sqrt(max(inner(A, A), 0.0)))


def add(A, B):
    """TT of A + B by block concatenation of the cores.

    First core [A^1 B^1] (side by side), last core [A^d; B^d] (stacked),
    middle cores block diagonal diag(A^k, B^k); each entry of the result is
    then A[i] + B[i] by the entry formula.
    """
    A = [np.asarray(x, dtype=np.float64) for x in A]
    B = [np.asarray(x, dtype=np.float64) for x in B]
    d = len(A)
    if d == 1:
        return [A[0] + B[0]]
    out = []
    for k, (a, b) in enumerate(zip(A, B)):
        ra0, n, ra1 = a.shape
        rb0, _, rb1 = b.shape
        if k == 0:
            c = np.concatenate([a, b], axis=2)
        elif k == d - 1:
            c = np.concatenate([a, b], axis=0)
        else:
            c = np.zeros((ra0 + rb0, n, ra1 + rb1))
            c[:ra0, :, :ra1] = a
            c[ra0:, :, ra1:] = b
        out.append(c)
    return out


def scale(A, c):
    """TT of c * A (multiplication by a number, Implementation Details):
    the first core is scaled."""
    return [np.asarray(A[0], dtype=np.float64) * c] + [np.asarray(x, dtype=np.float64) for x in A[1:]]


def pad_ranks(A, ranks):
    """Zero-pad the bond ranks of a TT to ``ranks`` (the tensor is unchanged)."""
    out = []
    for k, a in enumerate(A):
        r0, n, r1 = a.shape
        c = np.zeros((ranks[k], n, ranks[k + 1]), dtype=np.float64)
        c[:r0, :, :r1] = a
        out.append(c)
    return out
