"""GPU parity of the Riemannian completion loop: the line-search terms
(tt_line_search) against FP64 sums over the oracle's gather of the same
tangent TT, single iterations against the oracle's iteration, and recovery
of a planted tensor.  Tolerances: 1e-5 relative for the fp32 sums (fixed-
order partial sums of at most 2^20 terms); 1e-4 for iterates (the
projection and rounding tolerance)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle import riemannian as R

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _tt_rel(A, B):
    """||A - B|| / ||B|| for TTs given as core lists, by exact inner products."""
    nb2 = oracle.inner(B, B)
    d2 = oracle.inner(A, A) - 2 * oracle.inner(A, B) + nb2
    return float(np.sqrt(max(d2, 0.0) / nb2))


LS_CASES = [
    ([8] * 4, [1, 4, 4, 4, 1], 4096),
    ([10] * 10, W.canonical_ranks([10] * 10, 16), 70001),   # tangent rank 32, ragged tail
    # P's prefix/suffix tables have fewer rows than M: the table gather
    ([10] * 6, W.canonical_ranks([10] * 6, 16), 20011),      # split rank 32
    ([10] * 8, W.canonical_ranks([10] * 8, 32), 30011),      # split rank 64
]


@pytest.mark.parametrize("case", range(len(LS_CASES)))
def test_line_search_terms_match_oracle(gpu_lib, case):
    tt = gpu_lib
    ns, ranks, M = LS_CASES[case]
    print("line search", ns[0], len(ns), max(ranks), M, flush=True)
    rng = np.random.default_rng(40 + case)
    cores = W.random_cores(rng, ns, ranks, 1 / np.sqrt(max(ranks)))
    idx = W.random_indices(rng, ns, M)
    t = rng.standard_normal(M).astype(np.float32)
    X = tt.TT.from_cores(cores)
    idxg = torch.as_tensor(idx).cuda()
    y, g, loss, _ = tt.gather_mse_backward(X, idxg, torch.as_tensor(t).cuda(), want_g=True)
    U = tt.orthogonalize(X, tt.TT_LR)
    V = tt.orthogonalize(X, tt.TT_RL)
    P = tt.project_sparse(U, V, idxg, g, alpha=1.0, add_x=0)
    got = tt.line_search_terms(P, idxg, y, torch.as_tensor(t).cuda()).cpu().numpy()
    pv = oracle.gather([c.astype(np.float64) for c in P.numpy_cores()], idx)
    yv = y.cpu().numpy().astype(np.float64)
    want = [float(np.dot(pv, pv)), float(np.dot(yv - t, pv))]
    assert abs(got[0] - want[0]) <= 1e-5 * abs(want[0])
    assert abs(got[1] - want[1]) <= 1e-5 * np.sqrt(np.dot(yv - t, yv - t) * want[0])
    # the step quotient, computed on the device
    assert abs(got[2] - want[1] / want[0]) <= 2e-5 * np.sqrt(np.dot(yv - t, yv - t) / want[0])


def test_line_search_empty(gpu_lib):
    tt = gpu_lib
    X = tt.TT([4, 4], [1, 2, 1])
    e = torch.zeros((2, 0), dtype=torch.int32, device="cuda")
    z = torch.zeros(0, device="cuda")
    assert tt.line_search_terms(X, e, z, z).cpu().tolist() == [0.0, 0.0, 0.0]


def test_completion_iterations_match_oracle(gpu_lib):
    """Three steps from the same start on the small planted problem: loss and
    step size per step, and the iterate after each step, against the oracle
    run on the GPU's own previous iterate (so errors do not compound)."""
    tt = gpu_lib
    p = W.small_step()
    t = oracle.gather(p.planted, p.idx) + p.noise
    X = tt.TT.from_cores(p.cores)
    idxg = torch.as_tensor(p.idx).cuda()
    tg = torch.as_tensor(t.astype(np.float32)).cuda()
    for it in range(3):
        print("completion iteration", it, flush=True)
        Xc = [c.astype(np.float64) for c in X.numpy_cores()]
        ref = R.completion_iteration(Xc, p.idx, t.astype(np.float32), 4)
        out = tt.completion_iteration(X, idxg, tg, 4)
        loss, step = float(out["loss"]), float(out["ls"][2])
        assert abs(loss - ref["loss"]) <= 1e-5 * ref["loss"]
        assert abs(step - ref["step"]) <= 1e-4 * abs(ref["step"])
        assert _tt_rel(out["Y"].numpy_cores(), ref["Y"]) <= 1e-4
        X = out["Y"]


def test_completion_recovers_planted_tensor(gpu_lib):
    """The noiseless planted rank-2 problem of the oracle pin, run on the
    GPU: held-out RMSE falls below 1e-4 (fp32 floor) within 40 steps."""
    tt = gpu_lib
    ns = [8] * 4
    rng = np.random.default_rng(21)
    planted = W.random_cores(rng, ns, [1, 2, 2, 2, 1], 1 / np.sqrt(2))
    X0 = W.random_cores(rng, ns, [1, 2, 2, 2, 1], 0.5)
    idx = W.random_indices(rng, ns, 2000)
    t = oracle.gather(planted, idx).astype(np.float32)
    idx_t = W.random_indices(rng, ns, 1000)
    t_t = oracle.gather(planted, idx_t).astype(np.float32)
    X, h = tt.riemannian_completion(tt.TT.from_cores(X0), idx, t, 2, 40, idx_t, t_t)
    e = oracle.gather([c.astype(np.float64) for c in X.numpy_cores()], idx_t) - t_t
    assert h[0]["test_rmse"] > 0.1
    assert float(np.sqrt(np.mean(e * e))) < 1e-4


@pytest.mark.parametrize("add_x", [0, 1])
def test_tangent_combine_equals_projection(gpu_lib, add_x):
    """Re-weighting P = P_X(Z) (alpha 1, no X) gives what the projection
    returns for (alpha, add_x) directly, in a new TT and in place."""
    tt = gpu_lib
    rng = np.random.default_rng(60 + add_x)
    ns = [8] * 5
    ranks = W.canonical_ranks(ns, 6)
    X = tt.TT.from_cores(W.random_cores(rng, ns, ranks, 0.4))
    idx = torch.as_tensor(W.random_indices(rng, ns, 3000)).cuda()
    z = torch.as_tensor(rng.standard_normal(3000).astype(np.float32)).cuda()
    U = tt.orthogonalize(X, tt.TT_LR)
    V = tt.orthogonalize(X, tt.TT_RL)
    alpha = -0.37
    want = tt.project_sparse(U, V, idx, z, alpha=alpha, add_x=add_x).data
    P = tt.project_sparse(U, V, idx, z, alpha=1.0, add_x=0)
    got = tt.tangent_combine(U, P, alpha, add_x).data
    scale = float(want.abs().max())
    assert float((got - want).abs().max()) <= 1e-6 * scale
    tt.tangent_combine(U, P, alpha, add_x, out=P)
    assert torch.equal(P.data, got)


PROJ_CASES = [
    (70, [3, 4, 3, 2], 3, [1, 2, 5, 3, 1]),
    (71, [8] * 5, 6, [1, 7, 12, 12, 5, 1]),
    (72, [10] * 10, 16, [1] + [32] * 9 + [1]),
]


@pytest.mark.parametrize("case", range(len(PROJ_CASES)))
def test_project_tt_matches_oracle(gpu_lib, case):
    """P_X(Y) for a TT Y (tt_project_tt) against the FP64 oracle, compared as
    tensors through exact inner products; add_x = 1 as well."""
    tt = gpu_lib
    seed, ns, r, sr = PROJ_CASES[case]
    print("project_tt", ns, r, max(sr), flush=True)
    rng = np.random.default_rng(seed)
    Xc = W.random_cores(rng, ns, W.canonical_ranks(ns, r), 1 / np.sqrt(r))
    Yc = W.random_cores(rng, ns, sr, 1 / np.sqrt(max(sr)))
    X = tt.TT.from_cores(Xc)
    U = tt.orthogonalize(X, tt.TT_LR)
    V = tt.orthogonalize(X, tt.TT_RL)
    Y = tt.TT.from_cores(Yc)
    for alpha, add_x in ((1.0, 0), (-0.3, 1)):
        got = tt.project_tt(U, V, Y, alpha=alpha, add_x=add_x).numpy_cores()
        want = R.project_tt(Xc, Yc, alpha=alpha, beta=float(add_x))[0]
        assert _tt_rel(got, want) <= 1e-4


def test_project_tt_one_hot_equals_sparse_projection(gpu_lib):
    tt = gpu_lib
    ns = [8] * 5
    rng = np.random.default_rng(73)
    X = tt.TT.from_cores(W.random_cores(rng, ns, W.canonical_ranks(ns, 6), 0.4))
    U = tt.orthogonalize(X, tt.TT_LR)
    V = tt.orthogonalize(X, tt.TT_RL)
    i = [3, 1, 7, 0, 5]
    onehot = [np.zeros((1, n, 1), np.float32) for n in ns]
    for k in range(len(ns)):
        onehot[k][0, i[k], 0] = 1.0
    a = tt.project_tt(U, V, tt.TT.from_cores(onehot)).numpy_cores()
    idx = torch.as_tensor(np.array(i, np.int32).reshape(-1, 1)).cuda()
    b = tt.project_sparse(U, V, idx, torch.ones(1, device="cuda")).numpy_cores()
    assert _tt_rel(a, b) <= 1e-5


@pytest.mark.parametrize("case", [([8] * 5, 6, 3000), ([10] * 6, 16, 20000), ([6, 6], 4, 200)])
def test_tangent_inner_and_axpby(gpu_lib, case):
    """Tangent algebra at one point: <A, B> from the dG blocks against the
    exact TT inner product of the two tangent TTs, and a A + b B (out of
    place and in place) against the TT sum, on projections of two sparse
    tensors."""
    tt = gpu_lib
    ns, r, M = case
    print("tangent algebra", ns, r, M, flush=True)
    rng = np.random.default_rng(70 + len(ns))
    X = tt.TT.from_cores(W.random_cores(rng, ns, W.canonical_ranks(ns, r), 1 / np.sqrt(r)))
    U = tt.orthogonalize(X, tt.TT_LR)
    V = tt.orthogonalize(X, tt.TT_RL)
    idx = torch.as_tensor(W.random_indices(rng, ns, M)).cuda()
    A = tt.project_sparse(U, V, idx, torch.as_tensor(rng.standard_normal(M).astype(np.float32)).cuda())
    B = tt.project_sparse(U, V, idx, torch.as_tensor(rng.standard_normal(M).astype(np.float32)).cuda())
    Ac = [c.astype(np.float64) for c in A.numpy_cores()]
    Bc = [c.astype(np.float64) for c in B.numpy_cores()]
    for P, Q, Pc, Qc in ((A, B, Ac, Bc), (A, A, Ac, Ac)):
        got = float(tt.tangent_inner(U, P, Q).item())
        want = oracle.inner(Pc, Qc)
        assert abs(got - want) <= 1e-5 * np.sqrt(oracle.inner(Pc, Pc) * oracle.inner(Qc, Qc))
    want = oracle.add(oracle.scale(Ac, -0.7), oracle.scale(Bc, 1.9))
    Wn = tt.tangent_axpby(U, -0.7, A, 1.9, B)
    assert _tt_rel([c.astype(np.float64) for c in Wn.numpy_cores()], want) <= 1e-5
    tt.tangent_axpby(U, -0.7, A, 1.9, B, out=B)
    assert _tt_rel([c.astype(np.float64) for c in B.numpy_cores()], want) <= 1e-5


def test_cg_iterations_match_oracle(gpu_lib):
    """Four CG steps on the small planted problem: loss, beta, step and the
    iterate after each step against the oracle's step run on the GPU's own
    iterate and previous gradient and direction (so errors do not
    compound)."""
    tt = gpu_lib
    p = W.small_step()
    t = oracle.gather(p.planted, p.idx) + p.noise
    X = tt.TT.from_cores(p.cores)
    idxg = torch.as_tensor(p.idx).cuda()
    tg = torch.as_tensor(t.astype(np.float32)).cuda()
    prev_gpu = prev_ref = None
    saw_beta = False
    for it in range(4):
        print("cg iteration", it, flush=True)
        Xc = [c.astype(np.float64) for c in X.numpy_cores()]
        if prev_gpu is not None:
            prev_ref = dict(xi=[c.astype(np.float64) for c in prev_gpu["xi"].numpy_cores()],
                            eta=[c.astype(np.float64) for c in prev_gpu["eta"].numpy_cores()],
                            xi_sq=oracle.inner([c.astype(np.float64) for c in prev_gpu["xi"].numpy_cores()],
                                               [c.astype(np.float64) for c in prev_gpu["xi"].numpy_cores()]))
        ref = R.cg_iteration(Xc, p.idx, t.astype(np.float32), 4, prev_ref)
        out = tt.cg_iteration(X, idxg, tg, 4, prev_gpu)
        v = tt.cg_values(out)
        assert abs(v["loss"] - ref["loss"]) <= 1e-5 * ref["loss"]
        assert abs(v["beta"] - ref["beta"]) <= 1e-3 * max(ref["beta"], 1e-3)
        saw_beta = saw_beta or ref["beta"] > 0.0
        assert abs(v["step"] - ref["step"]) <= 1e-4 * abs(ref["step"])
        assert _tt_rel(out["Y"].numpy_cores(), ref["Y"]) <= 1e-4
        X, prev_gpu = out["Y"], out
    assert saw_beta


def test_cg_iterations_match_oracle_d10(gpu_lib):
    """Three CG steps at the completion workload's shape (d=10, n=10,
    canonical rank 16, planted rank 8) on 2^16 of its observed entries:
    loss, beta, restart decision and step against the oracle's step run on
    the GPU's own iterate, previous gradient and direction."""
    tt = gpu_lib
    p = W.completion_d10(M=1 << 16)
    t = (oracle.gather(p.planted, p.idx) + p.noise).astype(np.float32)
    X = tt.TT.from_cores(p.cores)
    idxg = torch.as_tensor(p.idx).cuda()
    tg = torch.as_tensor(t).cuda()
    prev_gpu = prev_ref = None
    for it in range(3):
        print("cg d10 iteration", it, flush=True)
        Xc = [c.astype(np.float64) for c in X.numpy_cores()]
        if prev_gpu is not None:
            xi = [c.astype(np.float64) for c in prev_gpu["xi"].numpy_cores()]
            prev_ref = dict(xi=xi, eta=[c.astype(np.float64) for c in prev_gpu["eta"].numpy_cores()],
                            xi_sq=oracle.inner(xi, xi))
        ref = R.cg_iteration(Xc, p.idx, t, 16, prev_ref)
        out = tt.cg_iteration(X, idxg, tg, 16, prev_gpu)
        v = tt.cg_values(out)
        print("  loss %.6g/%.6g beta %.6g/%.6g step %.6g/%.6g" % (v["loss"], ref["loss"], v["beta"], ref["beta"],
                                                                 v["step"], ref["step"]), flush=True)
        assert abs(v["loss"] - ref["loss"]) <= 1e-5 * ref["loss"]
        assert abs(v["beta"] - ref["beta"]) <= 1e-3 * max(ref["beta"], 1e-3)
        assert abs(v["step"] - ref["step"]) <= 1e-4 * abs(ref["step"])
        assert _tt_rel(out["Y"].numpy_cores(), ref["Y"]) <= 1e-4
        X, prev_gpu = out["Y"], out


def test_cg_recovers_planted_tensor(gpu_lib):
    """The noiseless planted rank-2 problem of the gradient-descent test: CG
    on the GPU reaches a held-out RMSE below 1e-4 in 20 steps (gradient
    descent needs about 40)."""
    tt = gpu_lib
    ns = [8] * 4
    rng = np.random.default_rng(21)
    planted = W.random_cores(rng, ns, [1, 2, 2, 2, 1], 1 / np.sqrt(2))
    X0 = W.random_cores(rng, ns, [1, 2, 2, 2, 1], 0.5)
    idx = W.random_indices(rng, ns, 2000)
    t = oracle.gather(planted, idx).astype(np.float32)
    idx_t = W.random_indices(rng, ns, 1000)
    t_t = oracle.gather(planted, idx_t).astype(np.float32)
    X, h = tt.riemannian_cg(tt.TT.from_cores(X0), idx, t, 2, 20, idx_t, t_t)
    e = oracle.gather([c.astype(np.float64) for c in X.numpy_cores()], idx_t) - t_t
    assert h[0]["test_rmse"] > 0.1
    assert float(np.sqrt(np.mean(e * e))) < 1e-4
    assert any(x["beta"] > 0.0 for x in h)


SUM_CASES = [
    # (seed, ns, X rank, batch rank, batch size): one launch chunk, and 70
    # members across two chunks of 64
    (80, [3, 4, 3, 2], 3, 2, 3),
    (81, [8] * 5, 6, 4, 9),
    (82, [10] * 8, 12, 4, 70),
    (84, [5, 7], 3, 5, 65),               # d = 2; a last chunk of one member
    (85, [5, 7, 3, 9, 4], 4, 64, 3),      # ragged modes; members of rank 64 at X rank 4
    (86, [4] * 4, 3, 2, 64),              # exactly one full chunk
]


@pytest.mark.parametrize("case", range(len(SUM_CASES)))
def test_project_sum_matches_oracle(gpu_lib, case):
    """project_sum of a batch (tt_project_sum) against the FP64 oracle, as
    tensors through exact inner products, with and without X added."""
    tt = gpu_lib
    seed, ns, r, ra, b = SUM_CASES[case]
    print("project_sum", ns, r, ra, b, flush=True)
    rng = np.random.default_rng(seed)
    Xc = W.random_cores(rng, ns, W.canonical_ranks(ns, r), 1 / np.sqrt(r))
    As = [W.random_cores(rng, ns, W.uniform_ranks(len(ns), ra), 1 / np.sqrt(ra)) for _ in range(b)]
    c = rng.standard_normal(b)
    X = tt.TT.from_cores(Xc)
    U, V = tt.orthogonalize_both(X)
    At = [tt.TT.from_cores(a) for a in As]
    for alpha, add_x in ((1.0, 0), (-0.3, 1)):
        got = tt.project_sum(U, V, At, c, alpha=alpha, add_x=add_x).numpy_cores()
        want = R.project_sum(Xc, As, c.astype(np.float32), alpha=alpha, beta=float(add_x))[0]
        assert _tt_rel(got, want) <= 1e-4


def test_project_sum_cancelling_weights(gpu_lib):
    """Weights that cancel (A with 0.5 and -0.5, B with 0) leave only X:
    the result is X itself as a tangent TT."""
    tt = gpu_lib
    rng = np.random.default_rng(87)
    ns = [6, 5, 7, 4]
    Xc = W.random_cores(rng, ns, W.canonical_ranks(ns, 5), 0.4)
    A = W.random_cores(rng, ns, W.uniform_ranks(4, 7), 0.3)
    B = W.random_cores(rng, ns, W.uniform_ranks(4, 7), 0.3)
    X = tt.TT.from_cores(Xc)
    U, V = tt.orthogonalize_both(X)
    At = [tt.TT.from_cores(a) for a in (A, A, B)]
    got = tt.project_sum(U, V, At, [0.5, -0.5, 0.0], alpha=2.0, add_x=1).numpy_cores()
    assert _tt_rel(got, Xc) <= 1e-5


GRAM_CASES = [
    # (seed, ns, X rank, Y rank, members)
    (90, [6, 5, 7, 4], 5, 3, 70),     # two pack chunks, a ragged 8 x 8 tile
    (91, [5, 7], 3, 2, 1),            # d = 2, one member
    (92, [10] * 10, 10, 10, 9),       # d = 10, n = 10, rank 10
]


@pytest.mark.parametrize("case", range(len(GRAM_CASES)))
def test_tangent_gram_matches_oracle(gpu_lib, case):
    """tt_tangent_gram on tangent TTs that the oracle projected (cast to
    float32) against the oracle's Gram matrix of the same TTs, entrywise
    relative to sqrt(G_ii G_jj); the result is exactly symmetric."""
    import torch
    tt = gpu_lib
    seed, ns, r, ry, b = GRAM_CASES[case]
    print("tangent_gram", ns, r, ry, b, flush=True)
    rng = np.random.default_rng(seed)
    Xc = W.random_cores(rng, ns, W.canonical_ranks(ns, r), 1 / np.sqrt(r))
    outs = [R.project_tt(Xc, W.random_cores(rng, ns, W.uniform_ranks(len(ns), ry), 1 / np.sqrt(ry)))
            for _ in range(b)]
    U = tt.TT.from_cores([u.astype(np.float32) for u in outs[0][1]])
    Ws = [[g.astype(np.float32) for g in o[0]] for o in outs]
    G = tt.tangent_gram(U, [tt.TT.from_cores(w) for w in Ws])
    assert torch.equal(G, G.t())
    got = G.cpu().numpy().astype(np.float64)
    want = R.tangent_gram(Ws)
    scale = np.sqrt(np.outer(np.diag(want), np.diag(want)))
    assert np.all(np.abs(got - want) <= 1e-5 * scale)


def test_project_sum_of_one_is_project_tt(gpu_lib):
    """A batch of one with weight 1 gives exactly the single projection."""
    import torch
    tt = gpu_lib
    rng = np.random.default_rng(83)
    ns = [8] * 5
    X = tt.TT.from_cores(W.random_cores(rng, ns, W.canonical_ranks(ns, 6), 0.4))
    Y = tt.TT.from_cores(W.random_cores(rng, ns, [1, 7, 12, 12, 5, 1], 0.3))
    U, V = tt.orthogonalize_both(X)
    a = tt.project_sum(U, V, [Y], [1.0], alpha=-0.7, add_x=1)
    b = tt.project_tt(U, V, Y, alpha=-0.7, add_x=1)
    assert torch.equal(a.data, b.data)
