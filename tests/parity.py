"""Element-by-element parity bounds shared by the GPU tests.

A float32 sum of products is accurate to a small multiple of the unit
roundoff times the same sum taken over absolute values.  Feeding the oracle
absolute-valued inputs therefore gives, for every output element, that
absolute sum (every term becomes non-negative), and each GPU element is held
to ``tol`` times it.  The normwise checks stay beside these in the tests.
"""
import numpy as np

import oracle


def absolute(cores):
    return [np.abs(np.asarray(c, dtype=np.float64)) for c in cores]


def gather_bound(cores, idx):
    """|G^1[i_1]| |G^2[i_2]| ... |G^d[i_d]| per entry (products of the
    absolute-valued slices; the entry formula of the Introduction over |G|)."""
    return oracle.gather(absolute(cores), idx)


def adjoint_bound(left, right, idx, w):
    """Per core element, the sum over its entries of |w_m| |L_m| |R_m|: the
    oracle's sparse adjoint over absolute cores and weights."""
    return oracle.sparse_adjoint(absolute(left), absolute(right), idx, np.abs(np.asarray(w, np.float64)))


def worst(got, want, bound):
    """Largest |got - want| / bound over the elements (0 where both are 0)."""
    got = np.asarray(got, np.float64).ravel()
    want = np.asarray(want, np.float64).ravel()
    bound = np.asarray(bound, np.float64).ravel()
    err = np.abs(got - want)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(err == 0, 0.0, err / bound)
    return float(q.max()) if q.size else 0.0


def assert_elementwise(got, want, bound, tol, what=""):
    """Every element within ``tol`` times its absolute-value bound."""
    q = worst(got, want, bound)
    assert q <= tol, "%s: worst element error %.3e of its bound (tol %.1e)" % (what, q, tol)


def assert_gather(y, yr, cores, idx, tol=1e-5, what="gather"):
    assert_elementwise(y, yr, gather_bound(cores, idx), tol, what)


def assert_adjoint(got_cores, want_cores, left, right, idx, w, tol=1e-5, what="adjoint"):
    bounds = adjoint_bound(left, right, idx, w)
    for k, (g, r, b) in enumerate(zip(got_cores, want_cores, bounds)):
        assert_elementwise(g, r, b, tol, "%s core %d" % (what, k))
