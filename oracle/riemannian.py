"""FP64 oracle: orthogonalization sweeps, sparse tangent projection, TT rounding.

Test infrastructure only (see the package docstring).

The paper names these operations (Implementation Details: ``t3f.round`` with
``max_tt_rank``; Riemannian Geometry Operations: the projection P_B A onto the
tangent space of the fixed-rank manifold, ``project_sum``, Riemannian
gradients P_X df/dX) but gives no algorithm for them.  They follow the
standard TT algorithms of the literature the paper cites: QR sweeps and
TT-SVD rounding from the TT-format paper (Oseledets 2011), the tangent-space
parametrisation with left/right orthonormal cores and the gauge condition
from the Riemannian TT paper (Steinlechner 2016).  Readings that the paper
leaves open (sign conventions, rank feasibility, rounding direction) are fixed
as documented in each function.
"""
import numpy as np

from .core import sparse_adjoint


def qr_pos(A):
    """Reduced Householder QR (LAPACK) with the sign fixed so diag(R) >= 0.

    The sign reading (diag(R) >= 0, sign(0) taken as +1) makes Q and R unique
    for a matrix of full column rank.
    """
    Q, R = np.linalg.qr(np.asarray(A, dtype=np.float64), mode="reduced")
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * s[None, :], R * s[:, None]


def orthogonalize_lr(cores):
    """Left-to-right orthogonalization sweep.

    For k = 1..d-1: QR of the left unfolding reshape(G^k, r_{k-1} n_k x r_k),
    G^k <- Q (left-orthonormal, rank min(r_{k-1} n_k, r_k)), and the R factor
    is multiplied into G^{k+1}.  The tensor is unchanged; the last core
    carries it (its norm is the tensor's Frobenius norm).
    """
    G = [np.array(c, dtype=np.float64) for c in cores]
    d = len(G)
    for k in range(d - 1):
        r0, n, r1 = G[k].shape
        Q, R = qr_pos(G[k].reshape(r0 * n, r1))
        G[k] = Q.reshape(r0, n, Q.shape[1])
        G[k + 1] = np.tensordot(R, G[k + 1], axes=([1], [0]))
    return G


def orthogonalize_rl(cores):
    """Right-to-left orthogonalization sweep (mirror of ``orthogonalize_lr``).

    For k = d..2: LQ of the right unfolding reshape(G^k, r_{k-1} x n_k r_k),
    computed as the QR of its transpose, A = L Q with diag(L) >= 0;
    G^k <- Q (right-orthonormal rows) and G^{k-1} <- G^{k-1} L.
    """
    G = [np.array(c, dtype=np.float64) for c in cores]
    d = len(G)
    for k in range(d - 1, 0, -1):
        r0, n, r1 = G[k].shape
        Q, R = qr_pos(G[k].reshape(r0, n * r1).T)  # A^T = Q R  =>  A = R^T Q^T
        G[k] = Q.T.reshape(Q.shape[1], n, r1)
        G[k - 1] = np.tensordot(G[k - 1], R.T, axes=([2], [0]))
    return G


def project_sparse_cores(U, V, idx, z):
    """Core contractions Zhat_k of a sparse tensor with the tangent-space
    interfaces of X.

    Zhat_k[a, i, b] = sum over m with i_k^m = i of
        z_m (U^1[i_1]..U^{k-1}[i_{k-1}])[a] (V^{k+1}[i_{k+1}]..V^d[i_d])[b],
    i.e. the adjoint of the gather taken with the left-orthonormal cores U on
    the left and the right-orthonormal cores V on the right.  By the linearity
    used by ``project_sum`` (Riemannian Geometry Operations section) this is
    the projection of sum_m z_m e_{i^m}, a weighted sum of M one-hot rank-1 TT
    tensors, computed one observed entry at a time.
    """
    return sparse_adjoint(U, V, idx, z)


def project_tt_cores(U, V, Y):
    """Core contractions Zhat_k of a TT tensor Y with the tangent-space
    interfaces of X (projection of a TT onto the tangent space, Riemannian
    Geometry Operations section: P_B A for TT tensors A and B).

    Left interfaces Psi_0 = 1, Psi_k = sum_i U^k[i]^T Psi_{k-1} Y^k[i]
    (r_k x s_k); right interfaces Phi_{d+1} = 1,
    Phi_k = sum_i V^k[i] Phi_{k+1} Y^k[i]^T (r_{k-1} x s_{k-1}); then
    Zhat_k[i] = Psi_{k-1} Y^k[i] Phi_{k+1}^T.  Each entry is the inner
    product of Y with the tensor U_<k (x) e_i (x) V_>k, the same quantity the
    sparse projection accumulates one observed entry at a time.
    """
    d = len(U)
    Y = [np.asarray(c, dtype=np.float64) for c in Y]
    psi = [np.ones((1, 1))]
    for k in range(d - 1):
        psi.append(np.einsum("aib,ac,cid->bd", U[k], psi[k], Y[k]))
    phi = [None] * (d + 1)
    phi[d] = np.ones((1, 1))
    for k in range(d - 1, 0, -1):
        phi[k] = np.einsum("aib,bc,dic->ad", V[k], phi[k + 1], Y[k])
    return [np.einsum("ac,cid,bd->aib", psi[k], Y[k], phi[k + 1]) for k in range(d)]


def project_tt(X, Y, alpha=1.0, beta=0.0):
    """Projection of the TT tensor Y onto the tangent space of X, returned as
    the rank-2r TT  beta*X + alpha*P_X(Y)  (Riemannian Geometry Operations:
    P_B A).  Orthogonalize X both ways, contract Y with the interfaces
    (``project_tt_cores``), fix the gauge, assemble.  Returns (W, U, V, dG).
    """
    U = orthogonalize_lr(X)
    V = orthogonalize_rl(X)
    _check_interfaces(U, V)
    dG = tangent_cores(U, project_tt_cores(U, V, Y))
    return tangent_tt(U, V, dG, alpha, beta), U, V, dG


def tangent_cores(U, Zhat):
    """Gauge-fixed tangent cores dG from the core contractions Zhat.

    dG_k = Zhat_k - U_k (U_k^L^T Zhat_k^L) for k < d (left unfoldings), which
    imposes the gauge U_k^L^T dG_k^L = 0; dG_d = Zhat_d.  These are the
    parameters of the orthogonal projection onto the tangent space of the
    fixed-rank manifold at X.
    """
    d = len(U)
    out = []
    for k in range(d):
        Z = np.asarray(Zhat[k], dtype=np.float64)
        if k < d - 1:
            r0, n, r1 = U[k].shape
            UL = U[k].reshape(r0 * n, r1)
            ZL = Z.reshape(r0 * n, r1)
            out.append((ZL - UL @ (UL.T @ ZL)).reshape(r0, n, r1))
        else:
            out.append(Z.copy())
    return out


def tangent_tt(U, V, dG, alpha=1.0, beta=0.0):
    """The tangent vector beta*X + alpha*sum_k U_<k dG_k V_>k as a TT of rank 2r.

    Cores: W_1 = [alpha dG_1, U_1]; W_k = [[V_k, 0], [alpha dG_k, U_k]];
    W_d = [[V_d], [beta S_d + alpha dG_d]], where S_d is the last core of the
    left-orthogonalized X (U[-1]).  Elements of one tangent space add by this
    block structure, the fact ``project_sum`` relies on (Riemannian Geometry
    Operations section).  beta = 1 gives the retraction input X + alpha P_X(Z).
    """
    d = len(U)
    assert d >= 2
    W = []
    for k in range(d):
        if k == 0:
            W.append(np.concatenate([alpha * dG[0], U[0]], axis=2))
        elif k == d - 1:
            W.append(np.concatenate([V[k], beta * U[k] + alpha * dG[k]], axis=0))
        else:
            r0, n, r1 = U[k].shape
            c = np.zeros((2 * r0, n, 2 * r1))
            c[:r0, :, :r1] = V[k]
            c[r0:, :, :r1] = alpha * dG[k]
            c[r0:, :, r1:] = U[k]
            W.append(c)
    return W


def _check_interfaces(U, V):
    for k in range(len(U) - 1):
        if U[k].shape[2] != V[k + 1].shape[0]:
            raise ValueError(
                "left- and right-orthogonalized ranks differ at bond %d (%d vs %d):"
                " X is not at feasible ranks" % (k + 1, U[k].shape[2], V[k + 1].shape[0]))


def project_sparse(X, idx, z, alpha=1.0, beta=0.0):
    """Projection of the sparse tensor Z = sum_m z_m e_{i^m} onto the tangent
    space of X, returned as the rank-2r TT  beta*X + alpha*P_X(Z).

    Riemannian Geometry Operations section: P_X Z, computed as project_sum of
    one-hot rank-1 tensors.  Steps: orthogonalize X both ways, contract Z with
    the interfaces (``project_sparse_cores``), fix the gauge
    (``tangent_cores``), assemble (``tangent_tt``).  Returns (W, U, V, dG).
    """
    U = orthogonalize_lr(X)
    V = orthogonalize_rl(X)
    _check_interfaces(U, V)
    Zhat = project_sparse_cores(U, V, idx, z)
    dG = tangent_cores(U, Zhat)
    return tangent_tt(U, V, dG, alpha, beta), U, V, dG


def round_tt(cores, max_rank):
    """TT rounding to ranks <= max_rank (``t3f.round``, Implementation Details).

    TT-SVD rounding of the cited TT-format paper: a right-to-left
    orthogonalization sweep, then for k = 1..d-1 the SVD of the left unfolding
    reshape(G^k, r_{k-1} n_k x r_k); the leading min(max_rank, r_{k-1} n_k, r_k)
    singular triplets are kept (singular values in descending order), G^k <- U,
    and Sigma V^T is multiplied into G^{k+1}.  Each kept left singular vector
    is sign-fixed so that its largest-magnitude component is positive.
    Returns (cores, disc_sq) with disc_sq[k] the sum of the discarded squared
    singular values at bond k+1; their total equals ||Y - round(Y)||_F^2.
    """
    G = orthogonalize_rl(cores)
    d = len(G)
    disc = []
    for k in range(d - 1):
        r0, n, r1 = G[k].shape
        Uf, s, Vt = np.linalg.svd(G[k].reshape(r0 * n, r1), full_matrices=False)
        rk = min(max_rank, s.shape[0])
        disc.append(float(np.sum(s[rk:] ** 2)))
        Uk = Uf[:, :rk]
        SVt = s[:rk, None] * Vt[:rk]
        j = np.argmax(np.abs(Uk), axis=0)
        sgn = np.where(Uk[j, np.arange(rk)] < 0, -1.0, 1.0)
        Uk = Uk * sgn[None, :]
        SVt = SVt * sgn[:, None]
        G[k] = Uk.reshape(r0, n, rk)
        G[k + 1] = np.tensordot(SVt, G[k + 1], axes=([1], [0]))
    return G, np.array(disc)


def completion_step(X, idx, t, alpha=-0.1, max_rank=None):
    """One Riemannian tensor-completion step on the observed set.

    Introduction (the completion example: fit a low-TT-rank tensor to known
    entries by Riemannian optimization) with the Riemannian gradient
    P_X(df/dX) of the Riemannian Geometry Operations section:
      y = gather(X), L = mean((y - t)^2), g = 2 (y - t) / M,
      core gradients = gather_backward(g),
      W = X + alpha * P_X(sum_m g_m e_{i^m}),  Y = round(W, max_rank).
    """
    from .core import gather, gather_backward, mse_loss_and_grad

    if max_rank is None:
        max_rank = max(c.shape[2] for c in X)
    y = gather(X, idx)
    loss, g = mse_loss_and_grad(y, t)
    grads = gather_backward(X, idx, g)
    W, U, V, dG = project_sparse(X, idx, g, alpha=alpha, beta=1.0)
    Y, disc = round_tt(W, max_rank)
    return dict(y=y, loss=loss, g=g, grads=grads, U=U, V=V, dG=dG, W=W, Y=Y, disc_sq=disc)


def left_interface(U, k):
    """Left interface matrix U_{<=k} (prod n_1..n_k x r_k) of the first k cores."""
    if k == 0:
        return np.ones((1, 1))
    t = U[0]
    for c in U[1:k]:
        t = np.tensordot(t, c, axes=([t.ndim - 1], [0]))
    return t.reshape(-1, t.shape[-1])


def right_interface(V, k):
    """Right interface matrix V_{>=k} (r_{k-1} x prod n_k..n_d), 1-based k."""
    d = len(V)
    if k > d:
        return np.ones((1, 1))
    t = V[k - 1]
    for c in V[k:]:
        t = np.tensordot(t, c, axes=([t.ndim - 1], [0]))
    return t.reshape(t.shape[0], -1)


def dense_projector(U, V):
    """Dense matrix of the tangent-space projector at X (tiny sizes only).

    P = sum_{k=1}^{d} P_<=k-1 (x) I_{n_k} (x) P_>=k+1
        - sum_{k=1}^{d-1} P_<=k (x) P_>=k+1,
    with P_<=k = U_<=k U_<=k^T from the left-orthonormal cores and
    P_>=k = V_>=k^T V_>=k from the right-orthonormal cores (P_<=0 = P_>=d+1 = 1);
    C-ordered Kronecker products match the C-ordered multi-index.
    """
    d = len(U)
    ns = [c.shape[1] for c in U]
    N = int(np.prod(ns))

    def PL(k):
        Ul = left_interface(U, k)
        return Ul @ Ul.T

    def PR(k):
        Vr = right_interface(V, k)
        return Vr.T @ Vr

    P = np.zeros((N, N))
    for k in range(1, d + 1):
        P += np.kron(np.kron(PL(k - 1), np.eye(ns[k - 1])), PR(k + 1))
    for k in range(1, d):
        P -= np.kron(PL(k), PR(k + 1))
    return P


def line_search_step(y, t, p):
    """Exact line search on the linearised completion loss.

    Along the descent direction xi = -P, with P = P_X(grad) and p_m = P(i^m)
    its values at the observed entries, the first-order model X + a xi has
    the observed loss (1/M) sum_m (y_m - a p_m - t_m)^2, a quadratic in a
    minimised at a* = sum_m (y_m - t_m) p_m / sum_m p_m^2 (0 when P vanishes
    on the observed set).  This is the step rule of Riemannian completion in
    the TT format (Steinlechner 2016, cited with the Riemannian Geometry
    Operations section), applied to the completion loss of the Introduction.
    """
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    pp = float(np.dot(p, p))
    if pp == 0.0:
        return 0.0
    return float(np.dot(y - t, p)) / pp


def completion_iteration(X, idx, t, max_rank):
    """One Riemannian gradient-descent step of tensor completion with the
    exact linearised line search:
      y = gather(X), L = mean((y - t)^2), g = 2 (y - t) / M,
      P = P_X(sum_m g_m e_{i^m})  (rank-2r tangent TT),
      a* = line_search_step(y, t, gather(P)),
      Y = round(X - a* P, max_rank).
    Returns dict(loss, step, Y, P_values).
    """
    from .core import gather, mse_loss_and_grad

    y = gather(X, idx)
    loss, g = mse_loss_and_grad(y, t)
    P, U, V, dG = project_sparse(X, idx, g, alpha=1.0, beta=0.0)
    pv = gather(P, idx)
    a = line_search_step(y, t, pv)
    W = tangent_tt(U, V, dG, -a, 1.0)
    Y, disc = round_tt(W, max_rank)
    return dict(loss=loss, step=a, Y=Y, P_values=pv, disc_sq=disc)


def riemannian_completion(X0, idx, t, max_rank, iters, idx_test=None, t_test=None):
    """Riemannian gradient descent for tensor completion: ``iters`` steps of
    ``completion_iteration`` from X0.  Returns (X, history) with history a
    list of dict(loss, step, test_rmse) per step (test_rmse of the iterate
    before the step, on the held-out entries, when given)."""
    from .core import gather

    X = [np.asarray(c, dtype=np.float64) for c in X0]
    hist = []
    for _ in range(iters):
        rmse = None
        if idx_test is not None:
            e = gather(X, idx_test) - np.asarray(t_test, dtype=np.float64)
            rmse = float(np.sqrt(np.mean(e * e)))
        out = completion_iteration(X, idx, t, max_rank)
        hist.append(dict(loss=out["loss"], step=out["step"], test_rmse=rmse))
        X = out["Y"]
    return X, hist


def cg_iteration(X, idx, t, max_rank, prev=None):
    """One step of Riemannian conjugate gradients for tensor completion
    (the nonlinear CG of Riemannian TT completion in the literature cited
    with the Riemannian Geometry Operations section, Steinlechner 2016):
      y = gather(X), L = mean((y - t)^2), g = 2 (y - t) / M,
      xi = P_X(sum_m g_m e_{i^m})              (Riemannian gradient),
      with the previous step's gradient xi' and direction eta' (tangent
      TTs at the previous point) carried over by projection,
        T xi' = P_X(xi'),  T eta' = P_X(eta'),
      beta = max(0, <xi, xi - T xi'> / <xi', xi'>)      (Polak-Ribiere+),
      eta = -xi + beta T eta', reset to -xi on the first step and whenever
        <xi, eta> >= 0 (not a descent direction; beta is then 0),
      a = -sum_m (y_m - t_m) eta(i^m) / sum_m eta(i^m)^2   (exact line
        search of the linearised observed loss along eta),
      Y = round(X + a eta, max_rank).
    Inner products are exact TT inner products.  ``prev`` is the dict this
    function returned for the previous step (None on the first).
    Returns dict(loss, step, beta, Y, xi, eta, xi_sq): xi and eta as TTs at
    X (rank-2r tangent TTs), xi_sq = <xi, xi>.
    """
    from .core import gather, inner, mse_loss_and_grad

    y = gather(X, idx)
    loss, g = mse_loss_and_grad(y, t)
    xi, U, V, dG = project_sparse(X, idx, g, alpha=1.0, beta=0.0)
    xi_sq = inner(xi, xi)
    beta = 0.0
    dE = [-c for c in dG]
    if prev is not None and prev["xi_sq"] > 0.0:
        Txi = project_tt(X, prev["xi"])[3]
        Teta = project_tt(X, prev["eta"])[3]
        Txi_tt = tangent_tt(U, V, Txi, 1.0, 0.0)
        beta = max(0.0, (xi_sq - inner(xi, Txi_tt)) / prev["xi_sq"])
        cand = [-a + beta * b for a, b in zip(dG, Teta)]
        if inner(xi, tangent_tt(U, V, cand, 1.0, 0.0)) < 0.0:
            dE = cand
        else:
            beta = 0.0
    eta = tangent_tt(U, V, dE, 1.0, 0.0)
    ev = gather(eta, idx)
    a = -line_search_step(y, t, ev)
    Y, _ = round_tt(tangent_tt(U, V, dE, a, 1.0), max_rank)
    return dict(loss=loss, step=a, beta=beta, Y=Y, xi=xi, eta=eta, xi_sq=xi_sq)


def riemannian_cg(X0, idx, t, max_rank, iters, idx_test=None, t_test=None):
    """Riemannian conjugate gradients for tensor completion: ``iters`` steps
    of ``cg_iteration`` from X0.  Returns (X, history) with history a list of
    dict(loss, step, beta, test_rmse) per step (test_rmse of the iterate
    before the step, when held-out entries are given)."""
    from .core import gather

    X = [np.asarray(c, dtype=np.float64) for c in X0]
    hist = []
    prev = None
    for _ in range(iters):
        rmse = None
        if idx_test is not None:
            e = gather(X, idx_test) - np.asarray(t_test, dtype=np.float64)
            rmse = float(np.sqrt(np.mean(e * e)))
        prev = cg_iteration(X, idx, t, max_rank, prev)
        hist.append(dict(loss=prev["loss"], step=prev["step"], beta=prev["beta"], test_rmse=rmse))
        X = prev["Y"]
    return X, hist


def project_sum(X, As, c, alpha=1.0, beta=0.0):
    """``project_sum`` (Riemannian Geometry Operations): the tangent vector
    beta*X + alpha * sum_i c_i P_X(A_i), for a batch of TT tensors A_i.  The
    projection is linear, so this is P_X of the weighted TT sum
    sum_i c_i A_i (formed by TT addition, ranks adding up).  Returns
    (W, U, V, dG) as ``project_tt``."""
    from .core import add, scale
    Y = scale([np.asarray(g, dtype=np.float64) for g in As[0]], float(c[0]))
    for A, ci in zip(As[1:], c[1:]):
        Y = add(Y, scale([np.asarray(g, dtype=np.float64) for g in A], float(ci)))
    return project_tt(X, Y, alpha, beta)


def tangent_gram(Ws):
    """Gram matrix of tangent vectors given as TTs (Riemannian Geometry
    Operations: the tangent space carries the ambient inner product; Table 1
    times the Gram matrix): G[i][j] = <W_i, W_j> by exact TT inner products."""
    from .core import inner
    b = len(Ws)
    W64 = [[np.asarray(g, dtype=np.float64) for g in W] for W in Ws]
    G = np.empty((b, b))
    for i in range(b):
        for j in range(b):
            G[i, j] = inner(W64[i], W64[j])
    return G


def observed_loss(y, t, kind, delta=1.0):
    """A loss over the observed entries, L = (1/M) sum_m phi(y_m, t_m), and
    its gradient g_m = dL/dy_m = phi'(y_m, t_m) / M, for the completion use
    case of the Introduction with other per-entry losses than the squared
    residual (the Riemannian gradient of the Riemannian Geometry Operations
    section is then P_X(sum_m g_m e_{i^m})).  kind:
      'squared'   phi = (y - t)^2,                  phi' = 2 (y - t);
      'huber'     r = y - t; phi = r^2 / 2 for |r| <= delta, else
                  delta (|r| - delta / 2);         phi' = r, else delta sign(r);
      'logistic'  labels t in {-1, +1}; phi = log(1 + exp(-t y)),
                  phi' = -t / (1 + exp(t y)).
    The definitions written out, in float64."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    M = y.shape[0]
    if M == 0:
        return 0.0, np.zeros(0)
    if kind == "squared":
        r = y - t
        phi, dphi = r * r, 2.0 * r
    elif kind == "huber":
        r = y - t
        small = np.abs(r) <= delta
        phi = np.where(small, 0.5 * r * r, delta * (np.abs(r) - 0.5 * delta))
        dphi = np.where(small, r, delta * np.sign(r))
    elif kind == "logistic":
        z = t * y
        phi = np.log1p(np.exp(-z))
        dphi = -t / (1.0 + np.exp(z))
    else:
        raise ValueError("unknown loss kind %r" % (kind,))
    return float(np.sum(phi) / M), dphi / M


def riemannian_grad_dense(X, G):
    """P_X G for a dense tensor G (tiny sizes only): the Riemannian gradient
    of a function whose Euclidean gradient at X is G (Riemannian Geometry
    Operations: the Riemannian gradient is the projection of the Euclidean
    one onto the tangent space).  The dense projector of ``dense_projector``
    applied to vec(G); returns a dense tensor of G's shape."""
    U = orthogonalize_lr(X)
    V = orthogonalize_rl(X)
    G = np.asarray(G, dtype=np.float64)
    return (dense_projector(U, V) @ G.reshape(-1)).reshape(G.shape)
