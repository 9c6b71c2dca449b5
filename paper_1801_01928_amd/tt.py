"""TT tensors on the device and thin wrappers over the C ABI.

PyTorch supplies device memory and the current stream; every computation is
a call into libttgfx.  A ``TT`` stores its cores in one flat float32 buffer
(core k, shape (r_k, n_k, r_{k+1}), row-major, at a packed offset), which is
exactly the descriptor layout of include/ttgfx.h with ``off = NULL``.
"""
import ctypes as C
import os

import numpy as np
import torch

from . import _lib as L


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _workspace(nbytes, device):
    nbytes = int(nbytes)
    if nbytes <= 0:
        return None, 0
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


class TT:
    """A TT tensor (Introduction: the TT format) with packed float32 cores
    (float64 for the double-precision Table 1 operations: tt_matvec,
    tt_matmat, norms and gram take either; every other entry point takes
    float32, and a float64 descriptor is refused by its argument types)."""

    def __init__(self, ns, ranks, data=None, device="cuda", dtype=torch.float32):
        self.ns = [int(x) for x in ns]
        self.ranks = [int(x) for x in ranks]
        if len(self.ranks) != len(self.ns) + 1:
            raise ValueError("ranks must have d+1 entries")
        self.sizes = [self.ranks[k] * self.ns[k] * self.ranks[k + 1] for k in range(self.d)]
        self.offs = [0]
        for s in self.sizes:
            self.offs.append(self.offs[-1] + s)
        if data is None:
            data = torch.empty(self.offs[-1], dtype=dtype, device=device)
        if data.dtype not in (torch.float32, torch.float64) or data.dim() != 1 or data.numel() != self.offs[-1] \
                or not data.is_contiguous():
            raise ValueError("data must be a contiguous float32 or float64 vector of %d elements" % self.offs[-1])
        self.data = data
        self._desc = None

    @property
    def d(self):
        return len(self.ns)

    @property
    def device(self):
        return self.data.device

    @classmethod
    def from_cores(cls, cores, device="cuda", dtype=torch.float32):
        npdt = np.float64 if dtype == torch.float64 else np.float32
        cores = [np.asarray(c, dtype=npdt) if not torch.is_tensor(c) else c for c in cores]
        ns = [int(c.shape[1]) for c in cores]
        ranks = [int(cores[0].shape[0])] + [int(c.shape[2]) for c in cores]
        flat = torch.cat([torch.as_tensor(c, dtype=dtype).reshape(-1) for c in cores])
        return cls(ns, ranks, flat.to(device).contiguous(), device=device)

    @property
    def is_f64(self):
        return self.data.dtype == torch.float64

    def core(self, k):
        return self.data[self.offs[k]:self.offs[k + 1]].view(self.ranks[k], self.ns[k], self.ranks[k + 1])

    def cores(self):
        return [self.core(k) for k in range(self.d)]

    def numpy_cores(self):
        return [c.detach().cpu().numpy() for c in self.cores()]

    def empty_like(self):
        return TT(self.ns, self.ranks, device=self.device, dtype=self.data.dtype)

    def desc(self):
        """The ``tt_tensor`` descriptor (``tt_tensor_f64`` for float64 cores;
        host arrays kept alive by this object)."""
        if self._desc is None or self._desc.data != self.data.data_ptr():
            d = self.d
            self._n = (C.c_int32 * d)(*self.ns)
            self._r = (C.c_int32 * (d + 1))(*self.ranks)
            kind = L.tt_tensor_f64 if self.is_f64 else L.tt_tensor
            self._desc = kind(d, self._n, self._r, None, self.data.data_ptr())
        return self._desc


def _idx(idx, d, device):
    if not torch.is_tensor(idx):
        idx = torch.as_tensor(np.asarray(idx, dtype=np.int32))
    idx = idx.to(device=device, dtype=torch.int32).contiguous()
    if idx.dim() != 2 or idx.shape[0] != d:
        raise ValueError("idx must have shape (d, M)")
    return idx


def _vec(v, M, device):
    v = torch.as_tensor(v).to(device=device, dtype=torch.float32).contiguous()
    if v.numel() != M:
        raise ValueError("expected %d values" % M)
    return v


def check_indices(X, idx):
    """Index check (tt_check_indices): returns (bad, first), the number of
    entries of idx (d, M) with some index outside [0, n_k) of X's modes and
    the smallest such entry (M when there is none)."""
    lib = L.load()
    idx = _idx(idx, X.d, X.device)
    M = idx.shape[1]
    out = torch.empty(2, dtype=torch.int64, device=X.device)
    L.check(lib.tt_check_indices(C.byref(X.desc()), _ptr(idx), M, _ptr(out), _stream(X.device)))
    bad, first = (int(v) for v in out.cpu())
    return bad, first


def _checked(X, idx):
    """Checked mode, on when TTGFX_CHECKED=1: raise TT_ERR_INDEX before a
    call whose indices leave [0, n_k) (the library's entry points treat such
    indices as undefined behaviour).  Synchronizes with the device."""
    if os.environ.get("TTGFX_CHECKED", "0") != "1":
        return
    bad, first = check_indices(X, idx)
    if bad:
        raise L.TTError(L.TT_ERR_INDEX, "%d of %d entries have an index outside [0, n_k); the first is "
                        "entry %d with indices %s" % (bad, idx.shape[1], first, idx[:, first].tolist()))


def gather(X, idx):
    """y[m] = G^1[i_1^m] ... G^d[i_d^m] (the entry formula) for idx (d, M)."""
    lib = L.load()
    idx = _idx(idx, X.d, X.device)
    _checked(X, idx)
    M = idx.shape[1]
    y = torch.empty(M, dtype=torch.float32, device=X.device)
    ws, nb = _workspace(L.check(lib.tt_gather_workspace(C.byref(X.desc()), M)), X.device)
    L.check(lib.tt_gather(C.byref(X.desc()), _ptr(idx), M, _ptr(y), _ptr(ws), nb, _stream(X.device)))
    return y


def halves_split(X):
    """Bond at which the prefix/suffix tables of X are smallest."""
    return int(L.check(L.load().tt_halves_split(C.byref(X.desc()))))


def halves_tables(X, split=None):
    """Prefix and suffix tables of X cut at bond ``split`` (the smallest
    when None): returns (split, tables), tables a uint8 device tensor."""
    lib = L.load()
    split = halves_split(X) if split is None else int(split)
    nb = int(L.check(lib.tt_halves_bytes(C.byref(X.desc()), split)))
    tables = torch.empty(max(nb, 1), dtype=torch.uint8, device=X.device)
    L.check(lib.tt_halves_build(C.byref(X.desc()), split, _ptr(tables), nb, _stream(X.device)))
    return split, tables


def gather_halves(X, idx, split=None, tables=None):
    """The gather computed from prefix/suffix tables (built here unless
    ``tables`` = (split, buffer) from ``halves_tables`` is given)."""
    lib = L.load()
    idx = _idx(idx, X.d, X.device)
    _checked(X, idx)
    M = idx.shape[1]
    if tables is None:
        split, buf = halves_tables(X, split)
    else:
        split, buf = tables
    y = torch.empty(M, dtype=torch.float32, device=X.device)
    L.check(lib.tt_halves_gather(C.byref(X.desc()), int(split), _ptr(buf), buf.numel(), _ptr(idx), M, _ptr(y),
                                 _stream(X.device)))
    return y


def gather_backward(X, idx, gy):
    """Core gradients of sum_m gy[m] y[m] (the gather's adjoint)."""
    lib = L.load()
    idx = _idx(idx, X.d, X.device)
    _checked(X, idx)
    M = idx.shape[1]
    gy = _vec(gy, M, X.device)
    gX = X.empty_like()
    ws, nb = _workspace(L.check(lib.tt_gather_backward_workspace(C.byref(X.desc()), M)), X.device)
    L.check(lib.tt_gather_backward(C.byref(X.desc()), _ptr(idx), M, _ptr(gy), C.byref(gX.desc()),
                                   _ptr(ws), nb, _stream(X.device)))
    return gX


def set_suffix_depth(depth):
    """Suffix-table policy of the gather / adjoint / fused kernels for later
    calls: -1 automatic (default), 0 never, k > 0 up to k levels."""
    L.check(L.load().tt_set_suffix_depth(int(depth)))


def set_deterministic(on):
    """Reduction policy for later adjoint, fused-pass, projection and plan
    calls: True sums every gradient in a fixed order (bitwise repeatable),
    False (default) lets rank class 32 and the batched plan add with float
    atomics."""
    L.check(L.load().tt_set_deterministic(1 if on else 0))


def deterministic():
    """The current reduction policy."""
    return bool(L.load().tt_deterministic())


def suffix_depth(X, M):
    """Suffix-table levels a fused pass over X with M entries takes now."""
    return int(L.check(L.load().tt_suffix_depth(C.byref(X.desc()), int(M))))


def gather_mse_workspace(X, M):
    """Workspace bytes of ``gather_mse_backward`` for M entries."""
    return int(L.check(L.load().tt_gather_mse_workspace(C.byref(X.desc()), int(M))))


def gather_mse_backward(X, idx, t, want_y=True, ws=None, out=None, loss=None, want_g=False):
    """Fused completion-loss pass: returns (y, loss, core gradients) for
    loss = mean((y - t)^2), or (y, g, loss, core gradients) with
    g = dloss/dy when want_g.  ``ws`` (uint8 device tensor), ``out`` (a TT
    of X's shape) and ``loss`` (1-element float32 tensor) may be given to
    reuse buffers across calls."""
    lib = L.load()
    idx = _idx(idx, X.d, X.device)
    _checked(X, idx)
    M = idx.shape[1]
    t = _vec(t, M, X.device)
    y = torch.empty(M, dtype=torch.float32, device=X.device) if want_y else None
    g = torch.empty(M, dtype=torch.float32, device=X.device) if want_g else None
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    gX = out if out is not None else X.empty_like()
    need = gather_mse_workspace(X, M)
    if ws is None or ws.numel() < need:
        ws, nb = _workspace(need, X.device)
    else:
        nb = ws.numel()
    L.check(lib.tt_gather_mse_backward(C.byref(X.desc()), _ptr(idx), M, _ptr(t), _ptr(y), _ptr(g),
                                       _ptr(loss), C.byref(gX.desc()), _ptr(ws), nb, _stream(X.device)))
    if want_g:
        return y, g, loss, gX
    return y, loss, gX


def gather_mse_backward_noalloc(X, idx, t, want_y=True, out=None, loss=None, want_g=False):
    """``gather_mse_backward`` through the entry point that allocates nothing
    on the device (its workspace is the library's fixed scratch array).
    ``out`` and ``loss`` may be given, as may ``idx`` and ``t`` as device
    tensors, so that a caller allocates nothing per call either."""
    lib = L.load()
    idx = _idx(idx, X.d, X.device)
    _checked(X, idx)
    M = idx.shape[1]
    t = _vec(t, M, X.device)
    y = torch.empty(M, dtype=torch.float32, device=X.device) if want_y else None
    g = torch.empty(M, dtype=torch.float32, device=X.device) if want_g else None
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    gX = out if out is not None else X.empty_like()
    L.check(lib.tt_gather_mse_backward_noalloc(C.byref(X.desc()), _ptr(idx), M, _ptr(t), _ptr(y), _ptr(g),
                                               _ptr(loss), C.byref(gX.desc()), _stream(X.device)))
    if want_g:
        return y, g, loss, gX
    return y, loss, gX


def gather_mse_noalloc_limit():
    """Bytes of the fixed scratch array behind ``gather_mse_backward_noalloc``."""
    return int(L.load().tt_gather_mse_noalloc_limit())


class KernelTimer:
    """Times the library's dominant kernels with HIP events recorded on the
    launch stream (tt_timer_start / tt_timer_stop)."""

    def __enter__(self):
        L.check(L.load().tt_timer_start())
        self.ms = 0.0
        self.launches = 0
        return self

    def __exit__(self, *exc):
        ms = C.c_float(0)
        n = C.c_int32(0)
        L.check(L.load().tt_timer_stop(C.byref(ms), C.byref(n)))
        self.ms = float(ms.value)
        self.launches = int(n.value)
        return False


class _GatherFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, flat, idx, ns, ranks):
        X = TT(ns, ranks, flat.detach())
        ctx.save_for_backward(flat.detach(), idx)
        ctx.meta = (ns, ranks)
        return gather(X, idx)

    @staticmethod
    def backward(ctx, gy):
        flat, idx = ctx.saved_tensors
        ns, ranks = ctx.meta
        g = gather_backward(TT(ns, ranks, flat), idx, gy.contiguous())
        return g.data, None, None, None


def tt_gather(X, idx):
    """Differentiable gather: gradients flow to ``X.data`` through the
    hand-written adjoint kernel."""
    idx = _idx(idx, X.d, X.device)
    return _GatherFn.apply(X.data, idx, tuple(X.ns), tuple(X.ranks))


def _ranks_call(fn, X, *args):
    out = (C.c_int32 * (X.d + 1))()
    L.check(fn(C.byref(X.desc()), *args, out))
    return list(out)


def orthogonalize(X, direction):
    """QR sweep (direction L.TT_LR or L.TT_RL); returns a new TT with the
    reduced ranks.  LR: cores 1..d-1 left-orthonormal; RL: cores 2..d
    right-orthonormal."""
    lib = L.load()
    ranks = _ranks_call(lib.tt_orthogonalize_ranks, X, int(direction))
    out = TT(X.ns, ranks, device=X.device)
    ws, nb = _workspace(L.check(lib.tt_orthogonalize_workspace(C.byref(X.desc()), int(direction))), X.device)
    L.check(lib.tt_orthogonalize(C.byref(X.desc()), int(direction), C.byref(out.desc()), _ptr(ws), nb,
                                 _stream(X.device)))
    return out


def orthogonalize_both(X):
    """(U, V) = (orthogonalize(X, LR), orthogonalize(X, RL)) in one launch
    (tt_orthogonalize_both)."""
    lib = L.load()
    U = TT(X.ns, _ranks_call(lib.tt_orthogonalize_ranks, X, L.TT_LR), device=X.device)
    V = TT(X.ns, _ranks_call(lib.tt_orthogonalize_ranks, X, L.TT_RL), device=X.device)
    ws, nb = _workspace(L.check(lib.tt_orthogonalize_both_workspace(C.byref(X.desc()))), X.device)
    L.check(lib.tt_orthogonalize_both(C.byref(X.desc()), C.byref(U.desc()), C.byref(V.desc()), _ptr(ws), nb,
                                      _stream(X.device)))
    return U, V


def project_sparse(U, V, idx, z, alpha=1.0, add_x=0):
    """Tangent projection of the sparse tensor sum_m z[m] e_{i^m} at X, with
    U = orthogonalize(X, LR) and V = orthogonalize(X, RL); returns the rank-2r
    TT  add_x * X + alpha * P_X(Z)."""
    lib = L.load()
    idx = _idx(idx, U.d, U.device)
    _checked(U, idx)
    M = idx.shape[1]
    z = _vec(z, M, U.device)
    W = TT(U.ns, [1] + [2 * r for r in U.ranks[1:-1]] + [1], device=U.device)
    ws, nb = _workspace(L.check(lib.tt_project_sparse_workspace(C.byref(U.desc()), M)), U.device)
    L.check(lib.tt_project_sparse(C.byref(U.desc()), C.byref(V.desc()), _ptr(idx), M, _ptr(z),
                                  C.c_float(alpha), int(add_x), C.byref(W.desc()), _ptr(ws), nb,
                                  _stream(U.device)))
    return W


def round_tt(Y, max_rank, with_status=False):
    """TT rounding to ranks <= max_rank (t3f.round); returns (TT, disc_sq)
    with disc_sq[k] the discarded squared singular values at bond k+1, and
    with ``with_status`` also a device int32 holding the number of bonds
    whose Jacobi SVD did not converge (tt_round_status)."""
    lib = L.load()
    ranks = _ranks_call(lib.tt_round_ranks, Y, int(max_rank))
    out = TT(Y.ns, ranks, device=Y.device)
    disc = torch.zeros(max(Y.d - 1, 1), dtype=torch.float32, device=Y.device)
    status = torch.full((1,), -1, dtype=torch.int32, device=Y.device) if with_status else None
    ws, nb = _workspace(L.check(lib.tt_round_workspace(C.byref(Y.desc()), int(max_rank))), Y.device)
    L.check(lib.tt_round_status(C.byref(Y.desc()), int(max_rank), C.byref(out.desc()), _ptr(disc), _ptr(status),
                                _ptr(ws), nb, _stream(Y.device)))
    if with_status:
        return out, disc[:max(Y.d - 1, 0)], status
    return out, disc[:max(Y.d - 1, 0)]


def riemannian_step(X, idx, t, alpha=-0.1, max_rank=None):
    """One Riemannian completion step: loss and Euclidean core gradients of
    mean((y - t)^2), then Y = round(X + alpha * P_X(grad), max_rank).
    Returns dict(loss, grads, W, Y, disc_sq)."""
    if max_rank is None:
        max_rank = max(X.ranks)
    idx = _idx(idx, X.d, X.device)
    M = idx.shape[1]
    y, g, loss, grads = gather_mse_backward(X, idx, t, want_g=True)
    U, V = orthogonalize_both(X)
    W = project_sparse(U, V, idx, g, alpha=alpha, add_x=1)
    Y, disc = round_tt(W, max_rank)
    return dict(y=y, loss=loss, grads=grads, U=U, V=V, W=W, Y=Y, disc_sq=disc)


def project_tt(U, V, Y, alpha=1.0, add_x=0):
    """Projection of the TT tensor Y onto the tangent space at X, with
    U = orthogonalize(X, LR) and V = orthogonalize(X, RL); returns the
    rank-2r TT  add_x * X + alpha * P_X(Y)  (tt_project_tt)."""
    lib = L.load()
    W = TT(U.ns, [1] + [2 * r for r in U.ranks[1:-1]] + [1], device=U.device)
    ws, nb = _workspace(L.check(lib.tt_project_tt_workspace(C.byref(U.desc()), C.byref(Y.desc()))), U.device)
    L.check(lib.tt_project_tt(C.byref(U.desc()), C.byref(V.desc()), C.byref(Y.desc()), C.c_float(alpha),
                              int(add_x), C.byref(W.desc()), _ptr(ws), nb, _stream(U.device)))
    return W


def tangent_combine_dev(U, P, alpha, scale, add_x, out=None):
    """``tangent_combine`` with the coefficient scale * alpha[0] read on the
    device (alpha: a one-element device tensor), so no host round trip."""
    W = out if out is not None else TT(P.ns, P.ranks, device=P.device)
    L.check(L.load().tt_tangent_combine_dev(C.byref(U.desc()), C.byref(P.desc()), _ptr(alpha), C.c_float(scale),
                                            int(add_x), C.byref(W.desc()), _stream(P.device)))
    return W


def cg_direction(U, xi, Txi, Teta, prev_xi_sq, eta, scalars):
    """Direction update of Riemannian CG on the device (tt_cg_direction):
    eta = -xi + beta Teta with the Polak-Ribiere+ beta, reset to -xi when it
    is not a descent direction; Txi = Teta = None on the first step.
    scalars (5 device floats) receives <xi, xi>, beta, the reset flag,
    <xi, eta> and <xi, Txi>."""
    first = Txi is None
    L.check(L.load().tt_cg_direction(C.byref(U.desc()), C.byref(xi.desc()),
                                     None if first else C.byref(Txi.desc()),
                                     None if first else C.byref(Teta.desc()),
                                     C.c_void_p(0) if first else _ptr(prev_xi_sq), C.byref(eta.desc()),
                                     _ptr(scalars), _stream(U.device)))
    return eta


def tangent_combine(U, P, alpha, add_x, out=None):
    """add_x X + alpha P_X(Z) from P = project_sparse(U, V, idx, z, 1, 0)
    (tt_tangent_combine); ``out`` may be P itself."""
    W = out if out is not None else TT(P.ns, P.ranks, device=P.device)
    L.check(L.load().tt_tangent_combine(C.byref(U.desc()), C.byref(P.desc()), C.c_float(alpha), int(add_x),
                                        C.byref(W.desc()), _stream(P.device)))
    return W


def project_sum(U, V, As, c, alpha=1.0, add_x=0):
    """project_sum (tt_project_sum): the rank-2r TT  add_x * X +
    alpha * sum_i c[i] P_X(As[i])  for TTs As of one shape, with U, V the
    two sweeps of X."""
    lib = L.load()
    c = (C.c_float * len(As))(*[float(x) for x in c])
    A, keep = _batch(As)
    W = TT(U.ns, [1] + [2 * r for r in U.ranks[1:-1]] + [1], device=U.device)
    ws, nb = _workspace(L.check(lib.tt_project_sum_workspace(C.byref(U.desc()), C.byref(A))), U.device)
    L.check(lib.tt_project_sum(C.byref(U.desc()), C.byref(V.desc()), C.byref(A), c, C.c_float(alpha), int(add_x),
                               C.byref(W.desc()), _ptr(ws), nb, _stream(U.device)))
    return W


def tangent_inner(U, A, B):
    """<A, B> of two tangent TTs at the point with left sweep U, as a device
    tensor of one float (tt_tangent_inner)."""
    out = torch.empty(1, dtype=torch.float32, device=A.device)
    L.check(L.load().tt_tangent_inner(C.byref(U.desc()), C.byref(A.desc()), C.byref(B.desc()), _ptr(out),
                                      _stream(A.device)))
    return out


def norms(As):
    """Frobenius norms of TT tensors of one shape (tt_norms; tt_norms_f64
    for float64 TTs), as a device tensor of len(As) values."""
    A, keep = _batch(As)
    f64 = As[0].is_f64
    out = torch.empty(len(As), dtype=torch.float64 if f64 else torch.float32, device=As[0].device)
    fn = L.load().tt_norms_f64 if f64 else L.load().tt_norms
    L.check(fn(C.byref(A), _ptr(out), _stream(As[0].device)))
    return out


def tangent_gram(U, As):
    """Gram matrix G[i][j] = <As[i], As[j]> of tangent TTs at the point with
    left sweep U (tt_tangent_gram), as a (b, b) device tensor."""
    lib = L.load()
    A, keep = _batch(As)
    G = torch.empty((len(As), len(As)), dtype=torch.float32, device=U.device)
    ws, nb = _workspace(L.check(lib.tt_tangent_gram_workspace(C.byref(U.desc()), C.byref(A))), U.device)
    L.check(lib.tt_tangent_gram(C.byref(U.desc()), C.byref(A), _ptr(G), _ptr(ws), nb, _stream(U.device)))
    return G


def tangent_axpby(U, a, A, b, B, out=None):
    """a A + b B for two tangent TTs at the point with left sweep U
    (tt_tangent_axpby); ``out`` may be A or B."""
    W = out if out is not None else TT(A.ns, A.ranks, device=A.device)
    L.check(L.load().tt_tangent_axpby(C.byref(U.desc()), C.c_float(a), C.byref(A.desc()), C.c_float(b),
                                      C.byref(B.desc()), C.byref(W.desc()), _stream(A.device)))
    return W


def observed_loss(y, t, kind="squared", delta=1.0):
    """Per-entry loss over the observed entries (tt_observed_loss): returns
    (loss, g), L = mean(phi(y, t)) and g = phi'(y, t) / M as device tensors,
    for kind 'squared', 'huber' (parameter delta) or 'logistic' (labels
    t in {-1, +1})."""
    lib = L.load()
    y = torch.as_tensor(y).to(dtype=torch.float32).contiguous()
    dev = y.device
    M = y.numel()
    t = _vec(t, M, dev)
    g = torch.empty(M, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ws, nb = _workspace(L.check(lib.tt_observed_loss_workspace(M)), dev)
    L.check(lib.tt_observed_loss(_ptr(y), _ptr(t), M, L.TT_LOSS[kind], C.c_float(delta), _ptr(g), _ptr(loss),
                                 _ptr(ws), nb, _stream(dev)))
    return loss, g


def riemannian_grad_observed(X, idx, t, kind="squared", delta=1.0, UV=None):
    """Riemannian gradient of an observed-entry loss at X: y = gather(X),
    (L, g) = observed_loss(y, t), then P_X(sum_m g_m e_{i^m}) by the sparse
    projection.  Returns (loss, W) with W the rank-2r tangent TT; UV may
    pass the two sweeps of X."""
    idx = _idx(idx, X.d, X.device)
    y = gather(X, idx)
    loss, g = observed_loss(y, t, kind, delta)
    U, V = UV if UV is not None else orthogonalize_both(X)
    return loss, project_sparse(U, V, idx, g, alpha=1.0, add_x=0)


def riemannian_grad(U, V, zhat, alpha=1.0, add_x=0):
    """Gauge-fixed tangent TT add_x X + alpha P_X(grad f) from the per-core
    Euclidean gradients zhat (a TT of X's shape, or a list of cores) of f in
    the tangent parametrisation at dG = 0 (tt_riemannian_grad)."""
    lib = L.load()
    Z = zhat if isinstance(zhat, TT) else TT.from_cores(zhat, device=U.device)
    W = TT(U.ns, [1] + [2 * r for r in U.ranks[1:-1]] + [1], device=U.device)
    ws, nb = _workspace(L.check(lib.tt_riemannian_grad_workspace(C.byref(U.desc()))), U.device)
    L.check(lib.tt_riemannian_grad(C.byref(U.desc()), C.byref(V.desc()), C.byref(Z.desc()), C.c_float(alpha),
                                   int(add_x), C.byref(W.desc()), _ptr(ws), nb, _stream(U.device)))
    return W


def line_search_terms(P, idx, y, t):
    """Line-search terms (tt_line_search) as a device tensor of 3 floats:
    sum_m P(i^m)^2, sum_m (y_m - t_m) P(i^m) and their quotient (the step
    a of X - a P; 0 when the first is 0)."""
    lib = L.load()
    idx = _idx(idx, P.d, P.device)
    _checked(P, idx)
    M = idx.shape[1]
    y = _vec(y, M, P.device)
    t = _vec(t, M, P.device)
    out = torch.empty(3, dtype=torch.float32, device=P.device)
    ws, nb = _workspace(L.check(lib.tt_line_search_workspace(C.byref(P.desc()), M)), P.device)
    L.check(lib.tt_line_search(C.byref(P.desc()), _ptr(idx), M, _ptr(y), _ptr(t), _ptr(out), _ptr(ws), nb,
                               _stream(P.device)))
    return out


def completion_iteration(X, idx, t, max_rank=None):
    """One step of Riemannian gradient descent for tensor completion with the
    exact line search on the linearised observed loss: g = dL/dy of the
    fused pass, P = P_X(sum_m g_m e_{i^m}), step a = sum (y - t) P(i) /
    sum P(i)^2 (tt_line_search, on the device), Y = round(X - a P,
    max_rank) with X - a P re-weighted from P by tt_tangent_combine_dev,
    which reads a on the device.  No host synchronisation.
    Returns dict(loss, ls, Y): loss (one device float) and ls (three device
    floats: the two line-search sums and a)."""
    if max_rank is None:
        max_rank = max(X.ranks)
    idx = _idx(idx, X.d, X.device)
    y, g, loss, _ = gather_mse_backward(X, idx, t, want_g=True)
    U, V = orthogonalize_both(X)
    P = project_sparse(U, V, idx, g, alpha=1.0, add_x=0)
    ls = line_search_terms(P, idx, y, t)
    W = tangent_combine_dev(U, P, ls[2:3], -1.0, 1, out=P)  # X - a P, without a second projection
    Y, _ = round_tt(W, max_rank)
    return dict(loss=loss, ls=ls, Y=Y)


def _history(rows, keys):
    """Device scalars of a run's steps to floats, in one transfer."""
    if not rows:
        return []
    flat = torch.cat([torch.cat([r[k].reshape(-1)[:1] for k in keys]) for r in rows]).cpu().tolist()
    n = len(keys)
    return [dict(zip(keys, flat[i * n:(i + 1) * n])) for i in range(len(rows))]


def riemannian_completion(X0, idx, t, max_rank, iters, idx_test=None, t_test=None):
    """Riemannian gradient descent for tensor completion: ``iters`` steps of
    ``completion_iteration`` from X0, with no host synchronisation inside
    the loop.  Returns (X, history), one dict(loss, step, test_rmse) per
    step; test_rmse is the held-out RMSE of the iterate before the step
    (from the fused pass on the test entries), None without test entries."""
    X = X0
    idx = _idx(idx, X.d, X.device)
    t = _vec(t, idx.shape[1], X.device)
    if idx_test is not None:
        idx_test = _idx(idx_test, X.d, X.device)
        t_test = _vec(t_test, idx_test.shape[1], X.device)
    rows = []
    for _ in range(iters):
        row = {}
        if idx_test is not None:
            _, row["test_mse"], _ = gather_mse_backward(X, idx_test, t_test, want_y=False)
        out = completion_iteration(X, idx, t, max_rank)
        row["loss"], row["step"] = out["loss"], out["ls"][2:3]
        rows.append(row)
        X = out["Y"]
    keys = ["loss", "step"] + (["test_mse"] if idx_test is not None else [])
    hist = _history(rows, keys)
    for h in hist:
        h["test_rmse"] = max(h.pop("test_mse"), 0.0) ** 0.5 if "test_mse" in h else None
    return X, hist


def cg_iteration(X, idx, t, max_rank=None, prev=None):
    """One step of Riemannian conjugate gradients for tensor completion:
    xi = P_X(grad) from the fused pass and the sparse projection; with the
    previous step's xi', eta' (``prev``), their transports P_X(xi'),
    P_X(eta') by tt_project_tt; the direction eta = -xi + beta P_X(eta')
    with the Polak-Ribiere+ beta, reset to -xi when it is not a descent
    direction (tt_cg_direction); the exact linearised line search along eta
    (tt_line_search), Y = round(X + a eta) with a = -ls[2] read on the
    device.  No host synchronisation.  Returns dict(loss, ls, scalars, Y,
    xi, eta): loss, ls (as for completion_iteration, along eta) and the five
    CG scalars of tt_cg_direction are device tensors; xi, eta are tangent
    TTs at X for the next step.  ``cg_values`` turns them into floats."""
    if max_rank is None:
        max_rank = max(X.ranks)
    idx = _idx(idx, X.d, X.device)
    y, g, loss, _ = gather_mse_backward(X, idx, t, want_g=True)
    U, V = orthogonalize_both(X)
    xi = project_sparse(U, V, idx, g, alpha=1.0, add_x=0)
    sc = torch.empty(5, dtype=torch.float32, device=X.device)
    if prev is not None:
        Txi = project_tt(U, V, prev["xi"])
        Teta = project_tt(U, V, prev["eta"])
        eta = cg_direction(U, xi, Txi, Teta, prev["scalars"][0:1], Teta, sc)
    else:
        eta = cg_direction(U, xi, None, None, None, TT(xi.ns, xi.ranks, device=xi.device), sc)
    ls = line_search_terms(eta, idx, y, t)
    W = tangent_combine_dev(U, eta, ls[2:3], -1.0, 1)  # X + a eta, a = -ls[2]
    Y, _ = round_tt(W, max_rank)
    return dict(loss=loss, ls=ls, scalars=sc, Y=Y, xi=xi, eta=eta)


def cg_values(out):
    """Floats of one CG step for reporting: loss, step a (Y = round(X + a
    eta)), beta, whether the direction was reset, and <xi, xi>."""
    v = torch.cat([out["loss"].reshape(1), out["ls"], out["scalars"]]).cpu().tolist()
    return dict(loss=v[0], step=-v[3], beta=v[5], restarted=bool(v[6] > 0.5), xi_sq=v[4])


def riemannian_cg(X0, idx, t, max_rank, iters, idx_test=None, t_test=None):
    """Riemannian conjugate gradients for tensor completion: ``iters`` steps
    of ``cg_iteration`` from X0, with no host synchronisation inside the
    loop.  Returns (X, history), one dict(loss, step, beta, restarted,
    test_rmse) per step (test_rmse of the iterate before the step)."""
    X = X0
    idx = _idx(idx, X.d, X.device)
    t = _vec(t, idx.shape[1], X.device)
    if idx_test is not None:
        idx_test = _idx(idx_test, X.d, X.device)
        t_test = _vec(t_test, idx_test.shape[1], X.device)
    rows = []
    prev = None
    for _ in range(iters):
        row = {}
        if idx_test is not None:
            _, row["test_mse"], _ = gather_mse_backward(X, idx_test, t_test, want_y=False)
        prev = cg_iteration(X, idx, t, max_rank, prev)
        row.update(loss=prev["loss"], step=prev["ls"][2:3], beta=prev["scalars"][1:2],
                   restarted=prev["scalars"][2:3])
        rows.append(row)
        X = prev["Y"]
    keys = ["loss", "step", "beta", "restarted"] + (["test_mse"] if idx_test is not None else [])
    hist = _history(rows, keys)
    for h in hist:
        h["step"] = -h["step"]
        h["restarted"] = bool(h["restarted"] > 0.5)
        h["test_rmse"] = max(h.pop("test_mse"), 0.0) ** 0.5 if "test_mse" in h else None
    return X, hist


def _batch(tts):
    """A tt_batch (tt_batch_f64 for float64) descriptor over TT objects of
    one precision (kept alive by the returned tuple)."""
    f64 = tts[0].is_f64
    if any(t.is_f64 != f64 for t in tts):
        raise ValueError("a batch holds TTs of one precision")
    kind, bkind = (L.tt_tensor_f64, L.tt_batch_f64) if f64 else (L.tt_tensor, L.tt_batch)
    arr = (kind * len(tts))(*[t.desc() for t in tts])
    return bkind(len(tts), arr), arr


def gram(As, Bs=None):
    """Gram matrix G[a][b] = <As[a], Bs[b]> (Bs = None: As with itself,
    computed once per unordered pair; tt_gram_f64 for float64 TTs).  Ranks
    up to 32; ranks may differ between tensors."""
    lib = L.load()
    dev = As[0].device
    A, keepA = _batch(As)
    B, keepB = _batch(Bs) if Bs is not None else (None, None)
    pB = C.byref(B) if B is not None else None
    nb = len(Bs) if Bs is not None else len(As)
    f64 = As[0].is_f64
    if Bs is not None and Bs[0].is_f64 != f64:
        raise ValueError("gram takes two batches of one precision")
    G = torch.empty((len(As), nb), dtype=torch.float64 if f64 else torch.float32, device=dev)
    wsq, run = (lib.tt_gram_f64_workspace, lib.tt_gram_f64) if f64 else (lib.tt_gram_workspace, lib.tt_gram)
    ws, n = _workspace(L.check(wsq(C.byref(A), pB)), dev)
    L.check(run(C.byref(A), pB, _ptr(G), _ptr(ws), n, _stream(dev)))
    return G


class BatchedPlan:
    """Batched persistent gather + MSE + adjoint over TT tensors of uneven
    ranks and entry counts (tt_plan_*).  ``idx`` holds, for tensor j, the
    (d, M_j) index block flattened at element d * entry_off[j]; ``t`` the
    targets at entry_off[j].  Gradients land in ``self.grads`` (a list of TT)
    and per-tensor losses in ``self.loss``."""

    def __init__(self, Xs, idx, t, entry_off):
        lib = L.load()
        self.Xs = list(Xs)
        dev = self.Xs[0].device
        self.idx = torch.as_tensor(idx).to(device=dev, dtype=torch.int32).contiguous().reshape(-1)
        self.t = torch.as_tensor(t).to(device=dev, dtype=torch.float32).contiguous()
        self.entry_off = (C.c_int64 * len(entry_off))(*[int(x) for x in entry_off])
        for j, X in enumerate(self.Xs):
            e0, e1 = int(entry_off[j]), int(entry_off[j + 1])
            _checked(X, self.idx[X.d * e0:X.d * e1].view(X.d, e1 - e0))
        self.grads = [X.empty_like() for X in self.Xs]
        self.loss = torch.empty(len(self.Xs), dtype=torch.float32, device=dev)
        self._bx, self._kx = _batch(self.Xs)
        self._bg, self._kg = _batch(self.grads)
        self._plan = C.c_void_p()
        L.check(lib.tt_plan_create(C.byref(self._bx), _ptr(self.idx), _ptr(self.t), self.entry_off,
                                   C.byref(self._bg), _ptr(self.loss), C.byref(self._plan)))
        self.device = dev

    def run(self, stream=None):
        s = C.c_void_p(stream.cuda_stream) if stream is not None else _stream(self.device)
        L.check(L.load().tt_plan_run(self._plan, s))

    def run_plain(self, stream=None):
        s = C.c_void_p(stream.cuda_stream) if stream is not None else _stream(self.device)
        L.check(L.load().tt_plan_run_plain(self._plan, s))

    def capture(self, stream):
        L.check(L.load().tt_plan_capture(self._plan, C.c_void_p(stream.cuda_stream)))

    def autotune(self, stream=None):
        s = C.c_void_p(stream.cuda_stream) if stream is not None else _stream(self.device)
        chosen = C.c_int32(0)
        L.check(L.load().tt_plan_autotune(self._plan, s, C.byref(chosen)))
        return int(chosen.value)

    def config(self):
        """The plan's launch: dict(chunk, tile16, tile32, threads) (entries
        per tile of the two rank classes, threads per workgroup)."""
        cfg = (C.c_int32 * 4)()
        L.check(L.load().tt_plan_config(self._plan, cfg))
        return dict(chunk=cfg[0], tile16=cfg[1], tile32=cfg[2], threads=cfg[3])

    def set_config(self, chunk, tile16, tile32, threads):
        """Set the launch (one of the autotuner's tile shapes); synchronizes
        the device first, since the work list is rewritten."""
        torch.cuda.synchronize(self.device)
        cfg = (C.c_int32 * 4)(int(chunk), int(tile16), int(tile32), int(threads))
        L.check(L.load().tt_plan_set_config(self._plan, cfg))

    def close(self):
        if self._plan:
            L.load().tt_plan_destroy(self._plan)
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TTMatrix:
    """A TT-matrix (Implementation Details: the ``t3f.matmul`` layer) with
    cores G^k of shape (r_k, m_k, n_k, r_{k+1}) packed in one flat buffer of
    dtype float32 or bfloat16; W[(i_1..i_d), (j_1..j_d)] =
    G^1[i_1, j_1] ... G^d[i_d, j_d] with C-ordered multi-indices."""

    def __init__(self, row_modes, col_modes, ranks, data):
        self.ms = [int(x) for x in row_modes]
        self.ns = [int(x) for x in col_modes]
        self.ranks = [int(x) for x in ranks]
        d = len(self.ms)
        if len(self.ns) != d or len(self.ranks) != d + 1:
            raise ValueError("row modes, column modes and ranks disagree in length")
        self.sizes = [self.ranks[k] * self.ms[k] * self.ns[k] * self.ranks[k + 1] for k in range(d)]
        self.offs = [0]
        for s in self.sizes:
            self.offs.append(self.offs[-1] + s)
        if data.dtype not in (torch.float32, torch.bfloat16, torch.float64) or data.dim() != 1 \
                or data.numel() != self.offs[-1] or not data.is_contiguous():
            raise ValueError("data must be a contiguous float32, bfloat16 or float64 vector of %d elements"
                             % self.offs[-1])
        self.data = data
        self._desc = None

    @property
    def d(self):
        return len(self.ms)

    @property
    def dtype_code(self):
        return {torch.float32: 0, torch.bfloat16: 1, torch.float64: 2}[self.data.dtype]

    @classmethod
    def from_cores(cls, cores, dtype=torch.float32, device="cuda"):
        npdt = np.float64 if dtype == torch.float64 else np.float32
        cores = [torch.as_tensor(np.asarray(c, dtype=npdt)) if not torch.is_tensor(c) else c for c in cores]
        ranks = [int(cores[0].shape[0])] + [int(c.shape[3]) for c in cores]
        mid = torch.float64 if dtype == torch.float64 else torch.float32
        flat = torch.cat([c.to(mid).reshape(-1) for c in cores]).to(dtype)
        return cls([c.shape[1] for c in cores], [c.shape[2] for c in cores], ranks,
                   flat.to(device).contiguous())

    def core(self, k):
        return self.data[self.offs[k]:self.offs[k + 1]].view(self.ranks[k], self.ms[k], self.ns[k],
                                                             self.ranks[k + 1])

    def numpy_cores(self):
        return [(self.core(k) if self.dtype_code == 2 else self.core(k).float()).cpu().numpy() for k in range(self.d)]

    def desc(self):
        if self._desc is None or self._desc.data != self.data.data_ptr():
            d = self.d
            self._m = (C.c_int32 * d)(*self.ms)
            self._n = (C.c_int32 * d)(*self.ns)
            self._r = (C.c_int32 * (d + 1))(*self.ranks)
            self._desc = L.tt_matrix(d, self._m, self._n, self._r, None, self.data.data_ptr())
        return self._desc


def _ttm_input(W, X, cols):
    want = torch.bfloat16 if W.dtype_code else torch.float32
    if X.dtype != want or X.dim() != 2 or X.shape[1] != cols or not X.is_contiguous():
        raise ValueError("expected a contiguous %s matrix with %d columns" % (want, cols))
    return X


def tt_matvec(W, xs):
    """y_j = W x_j in the TT format (tt_matvec, tt_matvec_f64) for a float32
    or float64 TTMatrix W and TT vectors xs of one shape and W's precision:
    exact products of ranks r_k s_k."""
    f64 = W.dtype_code == 2
    if W.dtype_code == 1 or any(x.is_f64 != f64 for x in xs):
        raise ValueError("tt_matvec takes float32 or float64 operands of one precision")
    lib = L.load()
    ranks = [a * b for a, b in zip(W.ranks, xs[0].ranks)]
    ys = [TT(W.ms, ranks, device=xs[0].device, dtype=xs[0].data.dtype) for _ in xs]
    X, keepx = _batch(xs)
    Y, keepy = _batch(ys)
    fn = lib.tt_matvec_f64 if f64 else lib.tt_matvec
    L.check(fn(C.byref(W.desc()), C.byref(X), C.byref(Y), _stream(xs[0].device)))
    return ys


def tt_matmat(A, B):
    """C = A B in the TT format (tt_matmat, tt_matmat_f64) for float32 or
    float64 TTMatrix objects of one precision: exact, modes A.ms x B.ns,
    ranks the products of A's and B's."""
    if A.dtype_code == 1 or A.dtype_code != B.dtype_code:
        raise ValueError("tt_matmat takes float32 or float64 TT-matrices of one precision")
    ranks = [a * b for a, b in zip(A.ranks, B.ranks)]
    n = sum(ranks[k] * A.ms[k] * B.ns[k] * ranks[k + 1] for k in range(A.d))
    Cm = TTMatrix(A.ms, B.ns, ranks, torch.empty(n, dtype=A.data.dtype, device=A.data.device))
    fn = L.load().tt_matmat_f64 if A.dtype_code == 2 else L.load().tt_matmat
    L.check(fn(C.byref(A.desc()), C.byref(B.desc()), C.byref(Cm.desc()), _stream(A.data.device)))
    return Cm


def ttm_set_path(path):
    """Evaluation path of the TT-matrix layer for later calls: "auto"
    (default), "chain" (one core per step) or "dense" (W built once, GEMMs
    on the matrix cores)."""
    codes = {"auto": 0, "chain": 1, "dense": 2}
    L.check(L.load().tt_matmul_set_path(codes[path]))


def ttm_path(W, B):
    """The path ("chain" or "dense") a layer call on B rows takes now."""
    code = L.check(L.load().tt_matmul_path(C.byref(W.desc()), int(B), W.dtype_code))
    return {1: "chain", 2: "dense"}[code]


def ttm_matmul(W, X):
    """Y = X W^T (float32) for a batch of rows X (B x prod n), X in W's dtype."""
    lib = L.load()
    Nt, Mt = int(np.prod(W.ns)), int(np.prod(W.ms))
    X = _ttm_input(W, X, Nt)
    B = X.shape[0]
    Y = torch.empty((B, Mt), dtype=torch.float32, device=X.device)
    # the forward needs a subset of the backward's workspace
    ws, n = _workspace(L.check(lib.tt_matmul_workspace(C.byref(W.desc()), B, W.dtype_code)), X.device)
    L.check(lib.tt_matmul(C.byref(W.desc()), _ptr(X), B, _ptr(Y), W.dtype_code, _ptr(ws), n,
                          _stream(X.device)))
    return Y


def ttm_matmul_backward(W, X, dY, want_dx=True, want_dw=True):
    """Adjoint of ``ttm_matmul``: dX = dY W (float32) and the core gradients
    of <dY, X W^T> as a flat float32 vector in W's packed layout."""
    lib = L.load()
    Nt, Mt = int(np.prod(W.ns)), int(np.prod(W.ms))
    dY = _ttm_input(W, dY, Mt)
    B = dY.shape[0]
    if want_dw:
        X = _ttm_input(W, X, Nt)
    dX = torch.empty((B, Nt), dtype=torch.float32, device=dY.device) if want_dx else None
    dW = torch.empty(W.offs[-1], dtype=torch.float32, device=dY.device) if want_dw else None
    ws, n = _workspace(L.check(lib.tt_matmul_workspace(C.byref(W.desc()), B, W.dtype_code)), dY.device)
    L.check(lib.tt_matmul_backward(C.byref(W.desc()), _ptr(X if want_dw else None), B, _ptr(dY), _ptr(dX),
                                   _ptr(dW), W.dtype_code, _ptr(ws), n, _stream(dY.device)))
    return dX, dW


class _TTLinearFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, flat, ms, ns, ranks):
        W = TTMatrix(ms, ns, ranks, flat.detach())
        ctx.save_for_backward(x.detach(), flat.detach())
        ctx.meta = (ms, ns, ranks)
        return ttm_matmul(W, x.detach().contiguous())

    @staticmethod
    def backward(ctx, gy):
        x, flat = ctx.saved_tensors
        ms, ns, ranks = ctx.meta
        W = TTMatrix(ms, ns, ranks, flat)
        gy = gy.to(flat.dtype).contiguous()
        dX, dW = ttm_matmul_backward(W, x, gy, ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        return (dX.to(x.dtype) if dX is not None else None,
                dW.to(flat.dtype) if dW is not None else None, None, None, None)


def tt_linear(x, W):
    """Differentiable y = x W^T through the hand-written TT-matrix kernels;
    gradients flow to ``x`` and ``W.data``."""
    return _TTLinearFn.apply(x, W.data, tuple(W.ms), tuple(W.ns), tuple(W.ranks))
