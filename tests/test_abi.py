"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ttgfx.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(tt_[a-z_]+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def lib():
    import paper_1801_01928_amd as tt
    return tt.load()


def test_exports_every_declared_symbol(lib):
    from paper_1801_01928_amd._lib import SIGNATURES
    names = _declared()
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(lib, n), n
        assert n in SIGNATURES, n
    assert lib.tt_version() == 1


def _desc(ns, ranks, data=0x1000):
    from paper_1801_01928_amd._lib import tt_tensor
    d = len(ns)
    n = (C.c_int32 * d)(*ns)
    r = (C.c_int32 * (d + 1))(*ranks)
    t = tt_tensor(d, n, r, None, data)
    t._keep = (n, r)
    return t


def test_validation_errors_before_device(lib):
    from paper_1801_01928_amd import _lib as L
    X = _desc([3, 4], [1, 2, 1])
    # negative M
    assert lib.tt_gather(C.byref(X), C.c_void_p(0x10), -1, C.c_void_p(0x10), None, 0, None) == L.TT_ERR_ARG
    assert "negative" in L.last_error()
    # null idx with M > 0
    assert lib.tt_gather(C.byref(X), None, 5, C.c_void_p(0x10), None, 0, None) == L.TT_ERR_ARG
    # bad boundary rank
    B = _desc([3, 4], [2, 2, 1])
    assert lib.tt_gather(C.byref(B), C.c_void_p(0x10), 5, C.c_void_p(0x10), None, 0, None) == L.TT_ERR_SHAPE
    # rank above the maximum
    H = _desc([3, 4], [1, 65, 1])
    assert lib.tt_gather(C.byref(H), C.c_void_p(0x10), 5, C.c_void_p(0x10), None, 0, None) == L.TT_ERR_UNSUPPORTED
    # d out of range
    Z = _desc([3], [1, 1])
    Z.d = 0
    assert lib.tt_gather(C.byref(Z), C.c_void_p(0x10), 5, C.c_void_p(0x10), None, 0, None) == L.TT_ERR_ARG
    # null data
    N = _desc([3, 4], [1, 2, 1], data=0)
    assert lib.tt_gather(C.byref(N), C.c_void_p(0x10), 5, C.c_void_p(0x10), None, 0, None) == L.TT_ERR_ARG
    # M = 0 is a no-op success (no device work)
    assert lib.tt_gather(C.byref(X), None, 0, None, None, 0, None) == L.TT_OK
    # shape mismatch of the gradient descriptor
    G = _desc([3, 4], [1, 3, 1])
    assert lib.tt_gather_backward(C.byref(X), C.c_void_p(0x10), 5, C.c_void_p(0x10), C.byref(G),
                                  None, 0, None) == L.TT_ERR_SHAPE
    # workspace too small
    ws = lib.tt_gather_backward_workspace(C.byref(X), 5)
    assert ws > 0
    assert lib.tt_gather_backward(C.byref(X), C.c_void_p(0x10), 5, C.c_void_p(0x10), C.byref(X),
                                  C.c_void_p(0x10), ws - 1, None) == L.TT_ERR_WORKSPACE
    assert "workspace" in L.last_error()


def _mdesc(ms, ns, ranks, data=0x1000):
    from paper_1801_01928_amd._lib import tt_matrix
    d = len(ms)
    m = (C.c_int32 * d)(*ms)
    n = (C.c_int32 * d)(*ns)
    r = (C.c_int32 * (d + 1))(*ranks)
    t = tt_matrix(d, m, n, r, None, data)
    t._keep = (m, n, r)
    return t


def test_matmul_validation_before_device(lib):
    from paper_1801_01928_amd import _lib as L
    W = _mdesc([4, 4], [4, 4], [1, 8, 1])
    assert lib.tt_matmul_workspace(C.byref(W), 16, 0) > 0
    # on the chain, bf16 intermediates need half the bytes of float32 ones
    # (plus fixed parts)
    try:
        assert lib.tt_matmul_set_path(1) == 0
        assert lib.tt_matmul_workspace(C.byref(W), 4096, 1) < lib.tt_matmul_workspace(C.byref(W), 4096, 0)
    finally:
        lib.tt_matmul_set_path(0)
    assert lib.tt_matmul_workspace(C.byref(W), 16, 2) == L.TT_ERR_ARG
    assert lib.tt_matmul_workspace(C.byref(W), -1, 0) == L.TT_ERR_ARG
    # a mode size times a rank above the fused step limit of 128
    big = _mdesc([8, 4], [4, 4], [1, 32, 1])
    assert lib.tt_matmul_workspace(C.byref(big), 16, 0) == L.TT_ERR_UNSUPPORTED
    assert "128" in L.last_error()
    bad = _mdesc([4, 4], [4, 4], [2, 8, 1])
    assert lib.tt_matmul(C.byref(bad), C.c_void_p(0x10), 4, C.c_void_p(0x10), 0, None, 0, None) == L.TT_ERR_SHAPE
    nul = _mdesc([4, 4], [4, 4], [1, 8, 1], data=0)
    assert lib.tt_matmul(C.byref(nul), C.c_void_p(0x10), 4, C.c_void_p(0x10), 0, None, 0, None) == L.TT_ERR_ARG
    # null X with a non-empty batch, and an empty batch (no device work)
    assert lib.tt_matmul(C.byref(W), None, 4, C.c_void_p(0x10), 0, None, 0, None) == L.TT_ERR_ARG
    assert lib.tt_matmul(C.byref(W), None, 0, None, 0, None, 0, None) == L.TT_OK
    # workspace too small
    assert lib.tt_matmul(C.byref(W), C.c_void_p(0x10), 4, C.c_void_p(0x10), 0, C.c_void_p(0x10), 8,
                         None) == L.TT_ERR_WORKSPACE
    assert lib.tt_matmul_backward(C.byref(W), C.c_void_p(0x10), 4, None, C.c_void_p(0x10), None, 0,
                                  C.c_void_p(0x10), 1 << 30, None) == L.TT_ERR_ARG
    # nothing requested: success without device work
    assert lib.tt_matmul_backward(C.byref(W), None, 4, None, None, None, 0, None, 0, None) == L.TT_OK


def test_check_indices_validation_before_device(lib):
    from paper_1801_01928_amd import _lib as L
    X = _desc([3, 4], [1, 2, 1])
    assert lib.tt_check_indices(C.byref(X), C.c_void_p(0x10), 5, None, None) == L.TT_ERR_ARG
    assert "null out" in L.last_error()
    assert lib.tt_check_indices(C.byref(X), C.c_void_p(0x10), -1, C.c_void_p(0x10), None) == L.TT_ERR_ARG
    assert lib.tt_check_indices(C.byref(X), None, 5, C.c_void_p(0x10), None) == L.TT_ERR_ARG
    Z = _desc([3], [1, 1])
    Z.d = 0
    assert lib.tt_check_indices(C.byref(Z), C.c_void_p(0x10), 5, C.c_void_p(0x10), None) == L.TT_ERR_ARG


def test_tangent_combine_validation_before_device(lib):
    from paper_1801_01928_amd import _lib as L
    U = _desc([3, 4, 5], [1, 2, 2, 1])
    P = _desc([3, 4, 5], [1, 4, 4, 1])
    bad = _desc([3, 4, 5], [1, 4, 3, 1])
    assert lib.tt_tangent_combine(C.byref(U), C.byref(bad), 1.0, 1, C.byref(bad), None) == L.TT_ERR_SHAPE
    assert lib.tt_tangent_combine(C.byref(U), C.byref(P), 1.0, 1, C.byref(bad), None) == L.TT_ERR_SHAPE
    assert lib.tt_tangent_combine(C.byref(U), C.byref(P), 1.0, 2, C.byref(P), None) == L.TT_ERR_ARG
    one = _desc([3], [1, 1])
    assert lib.tt_tangent_combine(C.byref(one), C.byref(one), 1.0, 1, C.byref(one), None) == L.TT_ERR_ARG


def test_halves_host_logic(lib):
    """Split choice, table bytes and argument checks of the prefix/suffix
    gather: host-only code, no device call."""
    from paper_1801_01928_amd import _lib as L

    def al(b):
        return (b + 255) // 256 * 256

    X = _desc([10] * 10, [1] + [16] * 9 + [1])
    assert lib.tt_halves_split(C.byref(X)) == 5
    # left levels j = 1..5: 10^j rows of r_j floats; right levels j = 9..5:
    # 10^(10-j) rows of r_j floats (r_j = 16 except nothing at the ends here)
    want = sum(al(4 * 10 ** j * 16) for j in range(1, 6)) + sum(al(4 * 10 ** (10 - j) * 16) for j in range(5, 10))
    assert lib.tt_halves_bytes(C.byref(X), 5) == want
    # uneven modes: the smaller tables sit where the products balance
    U = _desc([2, 2, 2, 2, 64, 64], [1, 2, 4, 4, 4, 4, 1])
    s = lib.tt_halves_split(C.byref(U))
    sizes = []
    for c in range(1, 6):
        pl = 1
        for k in range(c):
            pl *= [2, 2, 2, 2, 64, 64][k]
        pr = 2 * 2 * 2 * 2 * 64 * 64 // pl
        sizes.append((pl + pr) * [1, 2, 4, 4, 4, 4, 1][c])
    assert s == 1 + sizes.index(min(sizes))
    # d = 1 has no bond to cut; split outside [1, d-1]
    D1 = _desc([7], [1, 1])
    assert lib.tt_halves_split(C.byref(D1)) == L.TT_ERR_UNSUPPORTED
    assert lib.tt_halves_bytes(C.byref(X), 0) == L.TT_ERR_ARG
    assert lib.tt_halves_bytes(C.byref(X), 10) == L.TT_ERR_ARG
    # a level over 2^30 rows
    Big = _desc([4096] * 6, [1, 2, 2, 2, 2, 2, 1])
    assert lib.tt_halves_bytes(C.byref(Big), 3) == L.TT_ERR_UNSUPPORTED
    # missing or short table buffer, null idx, negative M
    nb = lib.tt_halves_bytes(C.byref(X), 5)
    assert lib.tt_halves_build(C.byref(X), 5, None, 0, None) == L.TT_ERR_WORKSPACE
    assert lib.tt_halves_build(C.byref(X), 5, C.c_void_p(0x1000), nb - 1, None) == L.TT_ERR_WORKSPACE
    assert lib.tt_halves_gather(C.byref(X), 5, C.c_void_p(0x1000), nb - 1, C.c_void_p(0x10), 4,
                                C.c_void_p(0x10), None) == L.TT_ERR_WORKSPACE
    assert lib.tt_halves_gather(C.byref(X), 5, C.c_void_p(0x1000), nb, None, 4, C.c_void_p(0x10),
                                None) == L.TT_ERR_ARG
    assert lib.tt_halves_gather(C.byref(X), 5, C.c_void_p(0x1000), nb, C.c_void_p(0x10), -1,
                                C.c_void_p(0x10), None) == L.TT_ERR_ARG
    # M = 0 is a no-op success
    assert lib.tt_halves_gather(C.byref(X), 5, C.c_void_p(0x1000), nb, None, 0, None, None) == 0


def test_tangent_algebra_and_orthogonalize_both_validation(lib):
    """Shape and argument checks of tt_tangent_inner, tt_tangent_axpby and
    tt_orthogonalize_both, all on the host before any device work."""
    from paper_1801_01928_amd import _lib as L
    U = _desc([3, 4, 5], [1, 2, 2, 1])
    P = _desc([3, 4, 5], [1, 4, 4, 1])
    bad = _desc([3, 4, 5], [1, 4, 3, 1])
    other = _desc([3, 4, 6], [1, 4, 4, 1])
    out = C.c_void_p(0x10)
    assert lib.tt_tangent_inner(C.byref(U), C.byref(P), C.byref(bad), out, None) == L.TT_ERR_SHAPE
    assert lib.tt_tangent_inner(C.byref(U), C.byref(other), C.byref(P), out, None) == L.TT_ERR_SHAPE
    assert lib.tt_tangent_inner(C.byref(U), C.byref(P), C.byref(P), None, None) == L.TT_ERR_ARG
    one = _desc([3], [1, 1])
    assert lib.tt_tangent_inner(C.byref(one), C.byref(one), C.byref(one), out, None) == L.TT_ERR_ARG
    assert lib.tt_tangent_axpby(C.byref(U), 1.0, C.byref(P), 2.0, C.byref(P), C.byref(bad), None) == L.TT_ERR_SHAPE
    assert lib.tt_tangent_axpby(C.byref(U), 1.0, C.byref(bad), 2.0, C.byref(P), C.byref(P), None) == L.TT_ERR_SHAPE
    # orthogonalize_both: output ranks must be the reduced ones of each direction
    X = _desc([3, 4, 5], [1, 3, 5, 1])       # LR ranks (1, 3, 5, 1); RL ranks (1, 3, 5, 1)
    Xs = _desc([3, 4, 5], [1, 3, 4, 1])
    assert lib.tt_orthogonalize_both_workspace(C.byref(X)) > 0
    assert lib.tt_orthogonalize_both(C.byref(X), C.byref(Xs), C.byref(X), C.c_void_p(0x1000), 1 << 30,
                                     None) == L.TT_ERR_SHAPE
    assert lib.tt_orthogonalize_both(C.byref(X), C.byref(X), C.byref(Xs), C.c_void_p(0x1000), 1 << 30,
                                     None) == L.TT_ERR_SHAPE
    assert lib.tt_orthogonalize_both(C.byref(X), C.byref(X), C.byref(X), None, 0, None) == L.TT_ERR_WORKSPACE
    assert lib.tt_orthogonalize_both(C.byref(X), C.byref(X), C.byref(other), C.c_void_p(0x1000), 1 << 30,
                                     None) == L.TT_ERR_SHAPE


def test_project_sum_validation_before_device(lib):
    """tt_project_sum rejects empty batches, mixed shapes, wrong output
    ranks and a missing weight array before any device work."""
    from paper_1801_01928_amd import _lib as L
    U = _desc([3, 4, 5], [1, 2, 2, 1])
    W = _desc([3, 4, 5], [1, 4, 4, 1])
    a1 = _desc([3, 4, 5], [1, 3, 3, 1])
    a2 = _desc([3, 4, 5], [1, 3, 2, 1])
    arr = (L.tt_tensor * 2)(a1, a2)
    mixed = L.tt_batch(2, arr)
    same = L.tt_batch(1, arr)
    empty = L.tt_batch(0, arr)
    c = (C.c_float * 2)(1.0, 2.0)
    ws = C.c_void_p(0x1000)
    assert lib.tt_project_sum(C.byref(U), C.byref(U), C.byref(empty), c, 1.0, 0, C.byref(W), ws, 1 << 30,
                              None) == L.TT_ERR_ARG
    assert lib.tt_project_sum(C.byref(U), C.byref(U), C.byref(mixed), c, 1.0, 0, C.byref(W), ws, 1 << 30,
                              None) == L.TT_ERR_SHAPE
    assert lib.tt_project_sum(C.byref(U), C.byref(U), C.byref(same), None, 1.0, 0, C.byref(W), ws, 1 << 30,
                              None) == L.TT_ERR_ARG
    assert lib.tt_project_sum(C.byref(U), C.byref(U), C.byref(same), c, 1.0, 0, C.byref(a1), ws, 1 << 30,
                              None) == L.TT_ERR_SHAPE
    assert lib.tt_project_sum(C.byref(U), C.byref(U), C.byref(same), c, 1.0, 0, C.byref(W), None, 0,
                              None) == L.TT_ERR_WORKSPACE
    assert lib.tt_project_sum_workspace(C.byref(U), C.byref(same)) > 0


def test_tangent_gram_validation_before_device(lib):
    """tt_tangent_gram rejects empty batches, members that are not tangent
    TTs of U's shape, a missing output and a short workspace before any
    device work; the workspace is the b x S matrix of dG blocks."""
    from paper_1801_01928_amd import _lib as L
    U = _desc([3, 4, 5], [1, 2, 2, 1])
    t1 = _desc([3, 4, 5], [1, 4, 4, 1])
    bad = _desc([3, 4, 5], [1, 3, 3, 1])
    arr = (L.tt_tensor * 3)(t1, t1, bad)
    two = L.tt_batch(2, arr)
    mixed = L.tt_batch(3, arr)
    empty = L.tt_batch(0, arr)
    G = C.c_void_p(0x2000)
    ws = C.c_void_p(0x1000)
    assert lib.tt_tangent_gram(C.byref(U), C.byref(empty), G, ws, 1 << 30, None) == L.TT_ERR_ARG
    assert lib.tt_tangent_gram(C.byref(U), C.byref(mixed), G, ws, 1 << 30, None) == L.TT_ERR_SHAPE
    assert lib.tt_tangent_gram(C.byref(U), C.byref(two), None, ws, 1 << 30, None) == L.TT_ERR_ARG
    assert lib.tt_tangent_gram(C.byref(U), C.byref(two), G, None, 0, None) == L.TT_ERR_WORKSPACE
    S = 3 * 2 + 2 * 4 * 2 + 2 * 5
    need = lib.tt_tangent_gram_workspace(C.byref(U), C.byref(two))
    assert need >= 2 * S * 4
    assert lib.tt_tangent_gram_workspace(C.byref(U), C.byref(mixed)) == L.TT_ERR_SHAPE


def test_matvec_validation_before_device(lib):
    """tt_matvec rejects an empty batch, mismatched batch sizes, a vector
    whose modes are not W's column modes, and outputs whose ranks are not
    the products, before any device work."""
    from paper_1801_01928_amd import _lib as L
    m = (C.c_int32 * 2)(2, 3)
    n = (C.c_int32 * 2)(3, 4)
    r = (C.c_int32 * 3)(1, 2, 1)
    W = L.tt_matrix(2, m, n, r, None, C.c_void_p(0x3000))
    x = _desc([3, 4], [1, 3, 1])
    xbad = _desc([3, 5], [1, 3, 1])
    y = _desc([2, 3], [1, 6, 1])
    ybad = _desc([2, 3], [1, 5, 1])
    xs = (L.tt_tensor * 2)(x, xbad)
    ys = (L.tt_tensor * 2)(y, ybad)
    one_x, one_y = L.tt_batch(1, xs), L.tt_batch(1, ys)
    assert lib.tt_matvec(C.byref(W), C.byref(L.tt_batch(0, xs)), C.byref(one_y), None) == L.TT_ERR_ARG
    assert lib.tt_matvec(C.byref(W), C.byref(one_x), C.byref(L.tt_batch(2, ys)), None) == L.TT_ERR_ARG
    assert lib.tt_matvec(C.byref(W), C.byref(L.tt_batch(2, xs)), C.byref(L.tt_batch(2, ys)), None) == L.TT_ERR_SHAPE
    ys2 = (L.tt_tensor * 1)(ybad)
    assert lib.tt_matvec(C.byref(W), C.byref(one_x), C.byref(L.tt_batch(1, ys2)), None) == L.TT_ERR_SHAPE


def test_matmat_validation_before_device(lib):
    """tt_matmat rejects mismatched inner modes and output ranks that are
    not the products before any device work."""
    from paper_1801_01928_amd import _lib as L
    def mat(m, n, r, ptr):
        arrs = ((C.c_int32 * len(m))(*m), (C.c_int32 * len(n))(*n), (C.c_int32 * len(r))(*r))
        return L.tt_matrix(len(m), arrs[0], arrs[1], arrs[2], None, C.c_void_p(ptr)), arrs
    A, ka = mat([2, 3], [3, 4], [1, 2, 1], 0x1000)
    B, kb = mat([3, 4], [2, 2], [1, 3, 1], 0x2000)
    Bbad, kbb = mat([3, 5], [2, 2], [1, 3, 1], 0x2000)
    Cg, kc = mat([2, 3], [2, 2], [1, 6, 1], 0x3000)
    Cbad, kcb = mat([2, 3], [2, 2], [1, 5, 1], 0x3000)
    assert lib.tt_matmat(C.byref(A), C.byref(Bbad), C.byref(Cg), None) == L.TT_ERR_SHAPE
    assert lib.tt_matmat(C.byref(A), C.byref(B), C.byref(Cbad), None) == L.TT_ERR_SHAPE
    assert lib.tt_matmat(C.byref(A), C.byref(B), None, None) == L.TT_ERR_ARG


def test_noalloc_rejects_shapes_beyond_its_scratch(lib):
    """The no-allocation fused pass refuses, on the host and before any
    device work, a shape whose workspace exceeds its fixed scratch array."""
    from paper_1801_01928_amd import _lib as L
    limit = lib.tt_gather_mse_noalloc_limit()
    assert limit == 256 << 20
    X = _desc([32] * 16, [1] + [32] * 15 + [1])
    M = 1 << 20
    assert lib.tt_gather_mse_workspace(C.byref(X), M) > limit
    rc = lib.tt_gather_mse_backward_noalloc(C.byref(X), C.c_void_p(0x10), M, C.c_void_p(0x10), None, None,
                                            None, C.byref(X), None)
    assert rc == L.TT_ERR_WORKSPACE
    assert "scratch" in L.last_error()
    # invalid descriptors are still reported as such
    B = _desc([3, 4], [2, 2, 1])
    assert lib.tt_gather_mse_backward_noalloc(C.byref(B), C.c_void_p(0x10), 5, C.c_void_p(0x10), None, None,
                                              None, C.byref(B), None) == L.TT_ERR_SHAPE


def test_suffix_table_policy(lib):
    """Suffix-table depth of the fused pass (host logic, no device work):
    levels are taken while the entries outnumber the deepest level's rows 16
    to 1 and the table stays within 2 MiB, at most d-1; the policy knob
    forces a depth or turns the table off, and workspace sizes follow it."""
    X = _desc([10] * 10, [1] + [16] * 9 + [1])
    try:
        assert lib.tt_suffix_depth(C.byref(X), 1 << 20) == 4      # 10^4 * 16 <= 2^20 < 10^5 * 16
        assert lib.tt_suffix_depth(C.byref(X), 1000) == 1
        assert lib.tt_suffix_depth(C.byref(X), 100) == 0
        ws_auto = lib.tt_gather_mse_workspace(C.byref(X), 1 << 20)
        lib.tt_set_suffix_depth(0)
        assert lib.tt_suffix_depth(C.byref(X), 1 << 20) == 0
        ws_off = lib.tt_gather_mse_workspace(C.byref(X), 1 << 20)
        assert ws_off > ws_auto  # the table replaces 4 of 9 stashed modes
        lib.tt_set_suffix_depth(9)
        # 2 MiB cap at rank class 16: 11,110 rows (64 B each) fit, 111,110 do not
        assert lib.tt_suffix_depth(C.byref(X), 100) == 4
        Y = _desc([4, 5, 3], [1, 3, 2, 1])
        assert lib.tt_suffix_depth(C.byref(Y), 7) == 2            # d-1 levels
        Z = _desc([10] * 6, [1] + [32] * 5 + [1])
        assert lib.tt_suffix_depth(C.byref(Z), 7) == 4            # 11,110 rows of 128 B
    finally:
        lib.tt_set_suffix_depth(-1)
    assert lib.tt_suffix_depth(C.byref(X), 1 << 20) == 4


def test_deterministic_policy(lib):
    """Reduction policy (host logic, no device work): workspaces do not
    depend on it, and shapes without a fixed-order accumulator (ranks above
    32) are refused before any device work while it is on."""
    from paper_1801_01928_amd import _lib as L
    X16 = _desc([10] * 10, [1] + [16] * 9 + [1])
    X32 = _desc([10] * 10, [1, 10] + [32] * 7 + [10, 1])
    X64 = _desc([6, 6, 6], [1, 40, 40, 1])
    M = 1 << 16
    assert lib.tt_deterministic() == 0
    w16, w32 = lib.tt_gather_backward_workspace(C.byref(X16), M), lib.tt_gather_backward_workspace(C.byref(X32), M)
    try:
        assert lib.tt_set_deterministic(1) == 0 and lib.tt_deterministic() == 1
        assert lib.tt_gather_backward_workspace(C.byref(X16), M) == w16
        assert lib.tt_gather_backward_workspace(C.byref(X32), M) == w32
        ws = lib.tt_gather_backward_workspace(C.byref(X64), 3001)
        rc = lib.tt_gather_backward(C.byref(X64), C.c_void_p(0x10), 3001, C.c_void_p(0x10), C.byref(X64),
                                    C.c_void_p(0x1000), ws, None)
        assert rc == L.TT_ERR_UNSUPPORTED
        assert "deterministic" in L.last_error()
    finally:
        lib.tt_set_deterministic(0)
    assert lib.tt_deterministic() == 0


def test_matmul_path_policy(lib):
    """Path choice of the TT-matrix layer (host logic, no device work): the
    automatic policy takes the dense matrix when its GEMM flops, 2 B prod m
    prod n, are below the core-by-core chain's; the knob forces either path;
    W above 2^28 elements always takes the chain; workspaces follow the
    path, including an empty batch."""
    from paper_1801_01928_amd import _lib as L
    layer = _mdesc([4] * 5, [4] * 5, [1, 32, 32, 32, 32, 1])   # chain 105 GFLOP, dense 8.6 at B = 4096
    thin = _mdesc([4, 4], [4, 4], [1, 1, 1])                    # rank 1: the chain is cheaper
    huge = _mdesc([128] * 3, [128] * 3, [1, 1, 1, 1])           # W of 2^42 elements
    try:
        assert lib.tt_matmul_path(C.byref(layer), 4096, 0) == 2
        assert lib.tt_matmul_path(C.byref(thin), 4096, 0) == 1
        assert lib.tt_matmul_path(C.byref(huge), 4, 0) == 1
        w_dense = lib.tt_matmul_workspace(C.byref(layer), 4096, 0)
        assert lib.tt_matmul_set_path(1) == 0
        assert lib.tt_matmul_path(C.byref(layer), 4096, 0) == 1
        w_chain = lib.tt_matmul_workspace(C.byref(layer), 4096, 0)
        assert w_chain > w_dense  # the chain keeps B-sized intermediates
        assert lib.tt_matmul_set_path(2) == 0
        assert lib.tt_matmul_path(C.byref(thin), 4096, 0) == 2
        assert lib.tt_matmul_path(C.byref(huge), 4, 0) == 1
        for B in (0, 1, 255, 256, 4096):
            assert lib.tt_matmul_workspace(C.byref(layer), B, 0) > 0
            assert lib.tt_matmul_workspace(C.byref(layer), B, 1) > 0
        assert lib.tt_matmul_set_path(3) == L.TT_ERR_ARG
    finally:
        lib.tt_matmul_set_path(0)
