"""GPU parity of the Riemannian step: QR sweeps, sparse tangent projection
with assembly, TT rounding and one full completion step, against the FP64
oracle.  Cores are gauge-dependent, so tensors are compared (normwise, by
exact FP64 TT inner products); tolerances 1e-5 for sweeps that leave the
tensor unchanged, 1e-4 for projection and rounding."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import absolute, assert_elementwise, gather_bound

pytestmark = pytest.mark.gpu


def tangent_blocks(Wc, ranks):
    """Blocks of an assembled tangent TT (ranks 2r): per core the alpha*dG
    block, and the U and V blocks where the core has them.  Layout: W_1 =
    [alpha dG_1, U_1]; W_k = [[V_k, 0], [alpha dG_k, U_k]];
    W_d = [[V_d], [beta S_d + alpha dG_d]]."""
    d = len(Wc)
    out = []
    for k, c in enumerate(Wc):
        c = np.asarray(c, np.float64)
        r0, r1 = ranks[k], ranks[k + 1]
        if k == 0:
            out.append({"dG": c[:, :, :r1], "U": c[:, :, r1:]})
        elif k == d - 1:
            out.append({"V": c[:r0], "dG": c[r0:]})
        else:
            out.append({"V": c[:r0, :, :r1], "dG": c[r0:, :, :r1], "U": c[r0:, :, r1:], "zero": c[:r0, :, r1:]})
    return out


def tangent_core_bounds(U, V, idx, z, alpha):
    """Per element of alpha*dG_k: |alpha| (|Zhat|_abs + |U_k| (|U_k|^T |Zhat|_abs)),
    where |Zhat|_abs is the sparse contraction over |U|, |V| and |z| (the sum
    of the absolute terms of Zhat, then of the gauge fix dG = Zhat - U U^T Zhat)."""
    Za = oracle.sparse_adjoint(absolute(U), absolute(V), idx, np.abs(np.asarray(z, np.float64)))
    out = []
    d = len(U)
    for k in range(d):
        if k < d - 1:
            r0, n, r1 = U[k].shape
            UL = np.abs(np.asarray(U[k], np.float64)).reshape(r0 * n, r1)
            ZL = Za[k].reshape(r0 * n, r1)
            out.append(abs(alpha) * (ZL + UL @ (UL.T @ ZL)).reshape(r0, n, r1))
        else:
            out.append(abs(alpha) * Za[k])
    return out


def assert_tangent_elementwise(Wg, ref, idx, z, alpha, beta, tol=1e-4):
    """Element-by-element comparison of an assembled tangent TT with the
    oracle's: the alpha*dG blocks within ``tol`` of their absolute-value
    bounds (plus, in the last core with beta != 0, tol times the largest
    element of S_d), the orthonormal U and V blocks within ``tol``
    absolutely (their columns have unit norm), the zero blocks exactly zero."""
    Wr, Uo, Vo, dGo = ref
    ranks = oracle.ranks_of(Uo)
    bounds = tangent_core_bounds(Uo, Vo, idx, z, alpha)
    gb = tangent_blocks(Wg, ranks)
    rb = tangent_blocks(Wr, ranks)
    d = len(Wg)
    for k in range(d):
        g, r = gb[k], rb[k]
        bd = bounds[k]
        if k == d - 1 and beta != 0.0:
            # beta S_d + alpha dG_d: the part of S_d (the last core of the
            # left-to-right sweep) is held to tol times its largest element
            bd = bd + abs(beta) * float(np.abs(np.asarray(Uo[k], np.float64)).max())
        assert_elementwise(g["dG"], r["dG"], bd, tol, "dG block of core %d" % k)
        for key in ("U", "V"):
            if key in g:
                err = float(np.abs(g[key] - r[key]).max())
                assert err <= tol, (k, key, err)
        if "zero" in g:
            assert not np.any(g["zero"]), k


def rel_tt(A, B):
    """||A - B||_F / ||B||_F for TTs given as lists of cores (FP64)."""
    A = [np.asarray(c, np.float64) for c in A]
    B = [np.asarray(c, np.float64) for c in B]
    nb = oracle.norm(B)
    return oracle.norm(oracle.add(A, oracle.scale(B, -1.0))) / (nb if nb > 0 else 1.0)


def _orth_err(cores, left):
    err = 0.0
    for c in cores:
        c = np.asarray(c, np.float64)
        M = c.reshape(-1, c.shape[2]) if left else c.reshape(c.shape[0], -1)
        G = M.T @ M if left else M @ M.T
        err = max(err, np.abs(G - np.eye(G.shape[0])).max())
    return err


SHAPES = [
    ([8, 8, 8, 8], W.canonical_ranks([8] * 4, 4)),
    ([10] * 10, W.canonical_ranks([10] * 10, 32)),
    ([16] * 8, W.uniform_ranks(8, 8)),
    ([3, 4, 5, 3], [1, 3, 5, 4, 1]),        # ranks above feasibility shrink
    ([6, 5, 7], [1, 6, 7, 1]),
    ([4, 4, 4, 4, 4], [1, 4, 16, 16, 4, 1]),
    ([16, 16, 16, 16], [1, 16, 48, 16, 1]),  # 768-row unfolding: QR in global memory
]


@pytest.mark.parametrize("case", range(len(SHAPES)))
def test_orthogonalize(gpu_lib, case):
    tt = gpu_lib
    ns, ranks = SHAPES[case]
    print("orthogonalize", ns, ranks, flush=True)
    cores = W.random_tt(100 + case, ns, ranks, std=1.0 / np.sqrt(max(ranks)))
    X = tt.TT.from_cores(cores)
    for direction, ref_fn, left in ((tt.TT_LR, oracle.orthogonalize_lr, True),
                                    (tt.TT_RL, oracle.orthogonalize_rl, False)):
        O = tt.orthogonalize(X, direction)
        ref = ref_fn(cores)
        got = O.numpy_cores()
        assert [c.shape for c in got] == [c.shape for c in ref]
        assert rel_tt(got, cores) <= 1e-5
        inner = got[:-1] if left else got[1:]
        assert _orth_err(inner, left) <= 1e-5
        # with full-rank unfoldings and diag(R) >= 0 the cores are unique
        for g, r in zip(got, ref):
            assert np.linalg.norm(g - r) <= 1e-4 * max(np.linalg.norm(r), 1e-30)


@pytest.mark.parametrize("case", range(len(SHAPES)))
def test_orthogonalize_both_equals_two_sweeps(gpu_lib, case):
    """One launch with both sweeps writes exactly what two single-direction
    calls write (the same arithmetic on separate buffers), on every shape
    above, including the global-memory QR."""
    tt = gpu_lib
    ns, ranks = SHAPES[case]
    print("orthogonalize_both", ns, ranks, flush=True)
    X = tt.TT.from_cores(W.random_tt(150 + case, ns, ranks, std=1.0 / np.sqrt(max(ranks))))
    U, V = tt.orthogonalize_both(X)
    U1 = tt.orthogonalize(X, tt.TT_LR)
    V1 = tt.orthogonalize(X, tt.TT_RL)
    assert U.ranks == U1.ranks and V.ranks == V1.ranks
    for a, b in zip(U.numpy_cores() + V.numpy_cores(), U1.numpy_cores() + V1.numpy_cores()):
        np.testing.assert_array_equal(a, b)


ROUND = [
    ([8, 8, 8, 8], [1, 8, 8, 8, 1], 4),
    ([10] * 6, [1, 10, 40, 40, 40, 10, 1], 16),
    ([5, 7], [1, 5, 1], 3),                  # d = 2: Eckart-Young
    ([4, 5, 3, 6], [1, 4, 12, 6, 1], 64),    # nothing to truncate
    ([10] * 10, [1, 20, 64, 64, 64, 64, 64, 64, 64, 20, 1], 32),
    ([12, 12, 12, 12], [1, 12, 64, 12, 1], 20),  # 768-row unfoldings: QR in global memory
]


@pytest.mark.parametrize("case", range(len(ROUND)))
def test_round(gpu_lib, case):
    tt = gpu_lib
    ns, ranks, rmax = ROUND[case]
    print("round", ns, ranks, rmax, flush=True)
    cores = W.random_tt(200 + case, ns, ranks, std=1.0 / np.sqrt(max(ranks)))
    Y = tt.TT.from_cores(cores)
    O, disc = tt.round_tt(Y, rmax)
    ref, dref = oracle.round_tt(cores, rmax)
    got = O.numpy_cores()
    assert [c.shape for c in got] == [c.shape for c in ref]
    assert rel_tt(got, ref) <= 1e-4
    ny2 = oracle.inner(cores, cores)
    assert np.abs(disc.cpu().numpy() - dref).max() <= 1e-4 * ny2
    # float32 Householder / Jacobi: loss of orthogonality O(m u), m <= 640 rows
    assert _orth_err(got[:-1], True) <= 1e-4


def test_round_ill_conditioned_converges(gpu_lib):
    """Rounding of a TT whose bond singular values fall over six decades
    (each core's right bond scaled by 10^(-6 j / r)): the Jacobi SVD of every
    bond converges (status 0) and the result matches the oracle's rounding."""
    tt = gpu_lib
    ns, r, rmax = [6] * 6, 24, 12
    ranks = W.canonical_ranks(ns, r)
    cores = W.random_tt(310, ns, ranks, std=1.0 / np.sqrt(r))
    graded = []
    for k, c in enumerate(cores):
        c = c.astype(np.float64)
        if k < len(cores) - 1:
            rr = c.shape[2]
            c = c * (10.0 ** (-6.0 * np.arange(rr) / rr))[None, None, :]
        graded.append(c.astype(np.float32))
    O, disc, status = tt.round_tt(tt.TT.from_cores(graded), rmax, with_status=True)
    assert int(status.item()) == 0
    ref, dref = oracle.round_tt(graded, rmax)
    assert rel_tt(O.numpy_cores(), ref) <= 1e-4
    ny2 = oracle.inner(graded, graded)
    assert np.abs(disc.cpu().numpy() - dref).max() <= 1e-4 * ny2


def test_round_exact_sum(gpu_lib):
    """round(X + X, r) represents 2X exactly (ranks suffice)."""
    tt = gpu_lib
    ns = [6] * 5
    ranks = W.canonical_ranks(ns, 5)
    cores = W.random_tt(300, ns, ranks, std=0.4)
    S = [c.astype(np.float32) for c in oracle.add(cores, cores)]
    O, disc = tt.round_tt(tt.TT.from_cores(S), 5)
    assert rel_tt(O.numpy_cores(), oracle.scale(cores, 2.0)) <= 1e-5
    assert float(disc.abs().max()) <= 1e-6 * oracle.inner(S, S)


PROJ = [
    ([8, 8, 8, 8], 4, 4096),
    ([6] * 6, 5, 20001),
    ([10] * 10, 16, 50000),
    ([10] * 10, 32, 30001),
    ([16] * 8, 8, 40000),
]


@pytest.mark.parametrize("case", range(len(PROJ)))
@pytest.mark.parametrize("alpha,add_x", [(1.0, 0), (-0.1, 1)])
def test_project_sparse(gpu_lib, case, alpha, add_x):
    tt = gpu_lib
    ns, r, M = PROJ[case]
    print("project", ns, r, M, alpha, add_x, flush=True)
    rng = np.random.default_rng(400 + case)
    ranks = W.canonical_ranks(ns, r)
    cores = W.random_cores(rng, ns, ranks, 1.0 / np.sqrt(r))
    idx = W.random_indices(rng, ns, M)
    z = rng.standard_normal(M).astype(np.float32)
    X = tt.TT.from_cores(cores)
    U = tt.orthogonalize(X, tt.TT_LR)
    V = tt.orthogonalize(X, tt.TT_RL)
    Wg = tt.project_sparse(U, V, idx, z, alpha=alpha, add_x=add_x)
    ref = oracle.project_sparse(cores, idx, z, alpha=alpha, beta=float(add_x))
    assert rel_tt(Wg.numpy_cores(), ref[0]) <= 1e-4
    assert_tangent_elementwise(Wg.numpy_cores(), ref, idx, z, alpha, float(add_x))


def test_completion_step_small(gpu_lib):
    """The small workload: loss, core gradients, projection and rounding."""
    tt = gpu_lib
    p = W.small_step()
    t = (oracle.gather(p.planted, p.idx) + p.noise).astype(np.float32)
    X = tt.TT.from_cores(p.cores)
    out = tt.riemannian_step(X, p.idx, t, alpha=-0.1, max_rank=4)
    ref = oracle.completion_step([c.astype(np.float64) for c in p.cores], p.idx, t, alpha=-0.1, max_rank=4)
    assert abs(float(out["loss"].item()) - ref["loss"]) <= 1e-5 * ref["loss"]
    for g, r in zip(out["grads"].numpy_cores(), ref["grads"]):
        assert np.linalg.norm(g - r) <= 1e-5 * np.linalg.norm(r)
    assert rel_tt(out["W"].numpy_cores(), ref["W"]) <= 1e-4
    assert rel_tt(out["Y"].numpy_cores(), ref["Y"]) <= 1e-4
    assert np.abs(out["disc_sq"].cpu().numpy() - ref["disc_sq"]).max() <= 1e-4 * oracle.inner(ref["W"], ref["W"])


def test_riemann_d10_full_size_properties(gpu_lib):
    """Full size (d=10, n=10, r=32, 2^20 entries): properties that hold at
    any size, checked with FP64 oracle arithmetic on the GPU outputs:
    <P_X Z, xi> = sum_m z_m xi(i^m) for xi = X and for a tangent vector
    with one non-zero tangent core; rounding's error identity; ranks."""
    tt = gpu_lib
    p = W.riemann_d10()
    print("riemann d10 r32 M=2^20", flush=True)
    X = tt.TT.from_cores(p.cores)
    U = tt.orthogonalize(X, tt.TT_LR)
    V = tt.orthogonalize(X, tt.TT_RL)
    Pz = tt.project_sparse(U, V, p.idx, p.values, alpha=1.0, add_x=0).numpy_cores()
    cores = [c.astype(np.float64) for c in p.cores]
    z = p.values.astype(np.float64)
    lhs = oracle.inner(Pz, cores)
    rhs = float(np.dot(z, oracle.gather(cores, p.idx)))
    assert abs(lhs - rhs) <= 1e-4 * np.sqrt(oracle.inner(Pz, Pz) * oracle.inner(cores, cores))
    # a tangent vector U_<k dH V_>k (gauge-fixed dH at k = 4)
    Uo = oracle.orthogonalize_lr(cores)
    Vo = oracle.orthogonalize_rl(cores)
    k = 4
    rng = np.random.default_rng(7)
    H = rng.standard_normal(Uo[k].shape)
    UL = Uo[k].reshape(-1, Uo[k].shape[2])
    H = (H.reshape(UL.shape[0], -1) - UL @ (UL.T @ H.reshape(UL.shape[0], -1))).reshape(H.shape)
    xi = Uo[:k] + [H] + Vo[k + 1:]
    lhs = oracle.inner(Pz, xi)
    rhs = float(np.dot(z, oracle.gather(xi, p.idx)))
    assert abs(lhs - rhs) <= 1e-4 * np.sqrt(oracle.inner(Pz, Pz) * oracle.inner(xi, xi))
    # retraction input X - 0.1 P_X(Z) and its rounding to r = 32
    Wt = tt.project_sparse(U, V, p.idx, p.values, alpha=-0.1, add_x=1)
    Wc = Wt.numpy_cores()
    assert rel_tt(Wc, oracle.add(cores, oracle.scale(Pz, -0.1))) <= 1e-5
    Y, disc = tt.round_tt(Wt, 32)
    Yc = Y.numpy_cores()
    assert Y.ranks == W.canonical_ranks(p.ns, 32)
    err2 = oracle.inner(oracle.add(Wc, oracle.scale(Yc, -1.0)), oracle.add(Wc, oracle.scale(Yc, -1.0)))
    assert abs(err2 - float(disc.double().sum())) <= 1e-3 * err2 + 1e-5 * oracle.inner(Wc, Wc)
    assert _orth_err(Yc[:-1], True) <= 1e-4


@pytest.fixture(scope="module")
def riemann_full():
    """The d=10, n=10, canonical rank-32 workload at 2^20 entries and the
    oracle's retraction input X - 0.1 P_X(Z) (with U, V and dG)."""
    p = W.riemann_d10()
    ref = oracle.project_sparse([c.astype(np.float64) for c in p.cores], p.idx, p.values, alpha=-0.1, beta=1.0)
    return p, ref


@pytest.mark.timeout(900)
def test_riemann_d10_full_size_oracle(gpu_lib, riemann_full):
    """Full size against the oracle's projection, in the launch
    configuration the benchmark times: the exact TT-difference norm of the
    retraction input X - 0.1 P_X(Z) (1e-4), every tangent core element
    within 1e-4 of its absolute-value bound, and the values at a seeded
    sample of 2^17 observed entries plus 4096 uniform probes (1e-4 normwise
    and per entry against the product of the absolute slices)."""
    tt = gpu_lib
    p, ref = riemann_full
    print("riemann d10 r32 M=2^20 against the oracle", flush=True)
    X = tt.TT.from_cores(p.cores)
    U, V = tt.orthogonalize_both(X)
    Wg = tt.project_sparse(U, V, p.idx, p.values, alpha=-0.1, add_x=1).numpy_cores()
    Wr = ref[0]
    assert [c.shape for c in Wg] == [c.shape for c in Wr]
    assert rel_tt(Wg, Wr) <= 1e-4
    assert_tangent_elementwise(Wg, ref, p.idx, p.values, -0.1, 1.0)
    rng = np.random.default_rng(33)
    sample = np.sort(rng.choice(p.M, size=1 << 17, replace=False))
    probes = np.concatenate([p.idx[:, sample], W.random_indices(rng, p.ns, 4096)], axis=1)
    vg = oracle.gather(Wg, probes)
    vr = oracle.gather(Wr, probes)
    assert np.linalg.norm(vg - vr) <= 1e-4 * np.linalg.norm(vr)
    assert_elementwise(vg, vr, gather_bound(Wr, probes), 1e-4, "tangent values")
