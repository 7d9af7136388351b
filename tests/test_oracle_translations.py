"""Pins for the oracle's multipole and local translations (Secs. 4.2, 4.3).

Each check is fixed by the mathematics, not by the oracle's own formulas:
  - the uncompressed M2M of eq. mpole_translated_full_coeffs is the binomial theorem, so
    translating the moments of a point set equals forming them at the new centre;
  - the uncompressed L2L of eq. l2l-expr re-centres a polynomial, so it evaluates to the
    same values everywhere;
  - for PDEs whose terms all have one order (Laplace, biharmonic) the compressed M2M is
    exact (Sec. 4.3, Theorem truncation_equal), and so is the compressed L2L of a local
    expansion (its polynomial satisfies the PDE exactly);
  - for PDEs with terms of several orders (Helmholtz, Yukawa) the compressed M2M differs
    from the exact potential at the level of the truncation error (Sec. 4.3); the same
    bound is taken for the compressed L2L (a reading: the paper states it for M2M), and the
    difference decays with the order.
"""
import numpy as np
import pytest

from oracle import compressed as Z
from oracle import kernels as K
from oracle import taylor as T

KERNELS = [("laplace", 0.0), ("biharmonic", 0.0), ("helmholtz", 1.0), ("yukawa", 2.0)]
EQUAL_ORDER = [("laplace", 0.0), ("biharmonic", 0.0)]
VARYING_ORDER = [("helmholtz", 1.0), ("yukawa", 2.0)]


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


@pytest.fixture(scope="module")
def cluster():
    g = np.random.Generator(np.random.PCG64(5))
    c_child = np.array([0.25, -0.25, 0.25])
    src = c_child + g.uniform(-0.25, 0.25, (30, 3))
    w = g.standard_normal(30)
    return c_child, np.zeros(3), src, w


def multipole_eval(kernel, param, p, c, beta, x):
    """sum_{q in j} beta_q G^(q)(x - c): the compressed multipole expansion at x."""
    J = Z.kept(kernel, param, p)
    return np.array([np.dot(beta, K.deriv_table_rec(kernel, param, xx - c, J)) for xx in x])


def test_full_m2m_is_the_binomial_theorem(cluster):
    c1, c2, src, w = cluster
    p = 6
    moved = T.m2m_full(p, c2 - c1, T.p2m_full(p, c1, src, w))
    assert rel(moved, T.p2m_full(p, c2, src, w)) < 1e-13


def test_full_m2m_composes(cluster):
    c1, _, src, w = cluster
    p = 5
    a = T.p2m_full(p, c1, src, w)
    h1, h2 = np.array([0.1, -0.2, 0.3]), np.array([-0.4, 0.05, 0.2])
    assert rel(T.m2m_full(p, h2, T.m2m_full(p, h1, a)), T.m2m_full(p, h1 + h2, a)) < 1e-13


def test_full_l2l_recentres_the_polynomial():
    g = np.random.Generator(np.random.PCG64(6))
    p = 6
    L = g.standard_normal(len(T.graded_order(p)))
    c, h = np.array([0.1, 0.2, -0.3]), np.array([0.3, -0.1, 0.2])
    x = c + g.uniform(-0.5, 0.5, (7, 3))
    assert rel(T.l2p_full(p, c + h, T.l2l_full(p, h, L), x), T.l2p_full(p, c, L, x)) < 1e-12


@pytest.mark.parametrize("kernel,param", KERNELS)
def test_translation_by_zero_is_the_identity(kernel, param):
    g = np.random.Generator(np.random.PCG64(7))
    p = 6
    n = len(Z.kept(kernel, param, p))
    beta, theta = g.standard_normal(n), g.standard_normal(n)
    assert np.allclose(Z.m2m(kernel, param, p, np.zeros(3), beta), beta, rtol=0, atol=1e-14)
    assert np.allclose(Z.l2l(kernel, param, p, np.zeros(3), theta), theta, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("kernel,param", EQUAL_ORDER)
def test_compressed_m2m_is_exact_for_equal_order_pdes(cluster, kernel, param):
    c1, c2, src, w = cluster
    for p in (2, 5, 8):
        moved = Z.m2m(kernel, param, p, c2 - c1, Z.p2m(kernel, param, p, c1, src, w))
        assert rel(moved, Z.p2m(kernel, param, p, c2, src, w)) < 1e-13


@pytest.mark.parametrize("kernel,param", VARYING_ORDER)
def test_compressed_m2m_error_is_at_truncation_level(cluster, kernel, param):
    c1, c2, src, w = cluster
    x = np.array([[3.0, 0.5, -0.4], [0.3, 2.8, 1.0], [-2.5, -1.5, 2.0]])
    exact = K.direct_sum(kernel, param, src, w, x)
    errs = []
    for p in (2, 4, 6, 8):
        direct = multipole_eval(kernel, param, p, c2, Z.p2m(kernel, param, p, c2, src, w), x)
        moved = multipole_eval(kernel, param, p, c2,
                               Z.m2m(kernel, param, p, c2 - c1, Z.p2m(kernel, param, p, c1, src, w)), x)
        trunc = np.abs(direct - exact).max()
        err = np.abs(moved - exact).max()
        assert err <= 4.0 * trunc
        errs.append(err)
    assert errs[-1] < 1e-2 * errs[0]


def _far_local(kernel, param, p, c_parent):
    """A local expansion at c_parent of a cluster four box sizes away (P2M then M2L)."""
    g = np.random.Generator(np.random.PCG64(8))
    cs = np.array([4.0, 0.0, 0.0])
    src = cs + g.uniform(-0.5, 0.5, (30, 3))
    w = g.standard_normal(30)
    theta = Z.m2l(kernel, param, p, c_parent - cs, Z.p2m(kernel, param, p, cs, src, w))
    return theta, src, w


@pytest.mark.parametrize("kernel,param", EQUAL_ORDER)
def test_compressed_l2l_is_exact_for_equal_order_pdes(kernel, param):
    cp, cc = np.zeros(3), np.array([0.25, 0.25, -0.25])
    x = cc + np.random.Generator(np.random.PCG64(9)).uniform(-0.25, 0.25, (6, 3))
    for p in (3, 8):
        theta, _, _ = _far_local(kernel, param, p, cp)
        child = Z.l2l(kernel, param, p, cc - cp, theta)
        assert rel(Z.l2p(kernel, param, p, cc, child, x), Z.l2p(kernel, param, p, cp, theta, x)) < 1e-12


@pytest.mark.parametrize("kernel,param", VARYING_ORDER)
def test_compressed_l2l_error_is_at_truncation_level(kernel, param):
    cp, cc = np.zeros(3), np.array([0.25, 0.25, -0.25])
    x = cc + np.random.Generator(np.random.PCG64(9)).uniform(-0.25, 0.25, (6, 3))
    def trunc(p):
        theta, src, w = _far_local(kernel, param, p, cp)
        return np.abs(Z.l2p(kernel, param, p, cp, theta, x) - K.direct_sum(kernel, param, src, w, x)).max()

    errs = []
    for p in (2, 4, 6, 8):
        theta, src, w = _far_local(kernel, param, p, cp)
        exact = K.direct_sum(kernel, param, src, w, x)
        err = np.abs(Z.l2p(kernel, param, p, cc, Z.l2l(kernel, param, p, cc - cp, theta), x) - exact).max()
        # the truncation error is not monotone from one order to the next, so the bound is
        # the larger of orders p and p - 1
        assert err <= 4.0 * max(trunc(p), trunc(p - 1))
        errs.append(err)
    assert errs[-1] < 1e-3 * errs[0]


@pytest.mark.parametrize("kernel,param", EQUAL_ORDER)
def test_scaled_m2m_matches_scaled_p2m(cluster, kernel, param):
    """Children of size h/2 to a parent of size h: the scaled translation of the child's
    scaled moments equals the parent's scaled moments (t = 1/box size)."""
    c1, c2, src, w = cluster
    p = 6
    t_child, t_parent = 1.0 / 0.5, 1.0 / 1.0
    child = Z.scale_multipole(kernel, param, p, Z.p2m(kernel, param, p, c1, src, w), t_child)
    parent = Z.scale_multipole(kernel, param, p, Z.p2m(kernel, param, p, c2, src, w), t_parent)
    assert rel(Z.m2m_scaled(kernel, param, p, c2 - c1, child, t_child, t_parent), parent) < 1e-13
