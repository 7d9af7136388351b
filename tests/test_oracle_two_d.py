"""The 2-D oracle (log r and r^2 log r, Sec. 4.4) pinned to what the mathematics fixes:

  - its derivatives equal SymPy's symbolic derivatives of the two kernels;
  - those derivatives obey the paper's recurrences (eqs. deriv_laplace_2d and
    deriv_biharmonic_2d, in their general (n, m) form) where they apply;
  - the decompression matrix M maps the kept derivatives of a solution of the PDE to all of
    its derivatives;
  - compressed M2L + L2P equals the uncompressed Taylor M2L + L2P to rounding (the kernels
    solve the PDE, so nothing is lost);
  - for log r, the compressed multipole evaluated at a target equals the classical
    complex-variable multipole expansion truncated at the same order;
  - the expansions converge to the direct sum as p grows."""
import math

import mpmath as mp
import numpy as np
import pytest
import sympy as sp

from oracle import two_d as T2

KERNELS = ["laplace2d", "biharmonic2d"]


def sympy_kernel(kernel):
    x, y = sp.symbols("x y", real=True)
    r = sp.sqrt(x ** 2 + y ** 2)
    return x, y, (sp.log(r) if kernel == "laplace2d" else r ** 2 * sp.log(r))


@pytest.mark.parametrize("kernel", KERNELS)
def test_derivatives_match_sympy(kernel):
    x, y, G = sympy_kernel(kernel)
    pts = [(sp.Rational(7, 10), sp.Rational(-13, 10)), (sp.Rational(-3, 1), sp.Rational(1, 4)),
           (sp.Rational(1, 8), sp.Rational(5, 2))]
    for a, b in [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 1), (2, 3), (5, 0), (0, 6), (4, 4), (7, 2)]:
        e = G
        if a:
            e = sp.diff(e, x, a)
        if b:
            e = sp.diff(e, y, b)
        f = sp.lambdify((x, y), e, "mpmath")
        for px, py in pts:
            with mp.workdps(40):
                want = f(mp.mpf(px.p) / px.q, mp.mpf(py.p) / py.q)
                got = T2.deriv_mp(kernel, a, b, mp.mpf(px.p) / px.q, mp.mpf(py.p) / py.q)
                assert abs(got - want) <= mp.mpf(10) ** -30 * (1 + abs(want)), (a, b, px, py)


@pytest.mark.parametrize("kernel", KERNELS)
def test_paper_recurrences_hold(kernel):
    """r^2 G_(n,m) = -A(n) x G_(n-1,m) - B(n) G_(n-2,m) - 2 m y G_(n,m-1) - m (m-1) G_(n,m-2) with
    A = 2(n-1), B = (n-1)(n-2) for log r (n >= 3, or n >= 1 when m >= 1) and A = 2(n-2),
    B = (n-1)(n-4) for r^2 log r (n >= 5; n >= 3 when m >= 1; n >= 1 when m >= 3)."""
    A = (lambda n: 2 * (n - 1)) if kernel == "laplace2d" else (lambda n: 2 * (n - 2))
    B = (lambda n: (n - 1) * (n - 2)) if kernel == "laplace2d" else (lambda n: (n - 1) * (n - 4))

    def first_n(m):
        if kernel == "laplace2d":
            return 3 if m == 0 else 1
        return 5 if m == 0 else (3 if m <= 2 else 1)

    with mp.workdps(40):
        for x, y in ((mp.mpf("0.7"), mp.mpf("-1.3")), (mp.mpf("2.5"), mp.mpf("0.5"))):
            g = lambda a, b: T2.deriv_mp(kernel, a, b, x, y) if a >= 0 and b >= 0 else 0
            r2 = x * x + y * y
            for m in range(7):
                for n in range(first_n(m), 12):
                    lhs = r2 * g(n, m)
                    rhs = -A(n) * x * g(n - 1, m) - B(n) * g(n - 2, m) - 2 * m * y * g(n, m - 1) - m * (m - 1) * g(n, m - 2)
                    assert abs(lhs - rhs) <= mp.mpf(10) ** -28 * (1 + abs(lhs)), (n, m)
            # and where the stated range ends, the recurrence does not hold
            n0 = first_n(0) - 1
            assert abs(r2 * g(n0, 0) + A(n0) * x * g(n0 - 1, 0) + B(n0) * g(n0 - 2, 0)) > 1e-6


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("p", [2, 5, 9])
def test_decompression_maps_kept_derivatives_of_a_solution(kernel, p):
    c = T2.pde_order(kernel)
    M = T2.decompression_matrix(kernel, p)
    J, F = T2.kept_set(p, c), T2.full_set(p)
    assert M.shape == (T2.n_full(p), len(J))
    assert len(J) == (2 * p + 1 if c == 2 else sum(p - b + 1 for b in range(min(4, p + 1))))
    with mp.workdps(40):
        x, y = mp.mpf("1.3"), mp.mpf("-0.4")
        full = np.array([float(T2.deriv_mp(kernel, a, b, x, y)) for a, b in F])
        kept = np.array([float(T2.deriv_mp(kernel, a, b, x, y)) for a, b in J])
    np.testing.assert_allclose(M @ kept, full, rtol=1e-13, atol=1e-13 * np.abs(full).max())
    # a plain polynomial that is not a solution is not reproduced (M uses the PDE)
    if p >= c:
        poly = np.array([1.0 if (a, b) == (0, c) else 0.0 for a, b in F])
        assert np.abs(M @ poly[[F.index(j) for j in J]] - poly).max() > 0.5


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("p", [3, 6])
def test_compressed_m2l_l2p_equals_uncompressed(kernel, p):
    g = np.random.Generator(np.random.PCG64(5))
    h = 0.25
    cs, ct = np.array([0.125, 0.375]), np.array([0.875, -0.375])
    src = cs + h * (g.random((20, 2)) - 0.5)
    tgt = ct + h * (g.random((7, 2)) - 0.5)
    w = g.standard_normal(20)
    beta = T2.p2m(kernel, p, cs, src, w, h)
    theta = T2.m2l(kernel, p, ct - cs, beta, h)
    got = T2.l2p(kernel, p, ct, theta, tgt, h)
    L = T2.m2l_full(kernel, p, ct - cs, src, w, cs, h)
    want = T2.l2p_full(p, ct, L, tgt, h)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("p", [1, 4, 10])
def test_laplace_multipole_equals_complex_expansion(p):
    """log r = Re log z: the compressed multipole of order p evaluated at x equals
    Re(sum_{n <= p} f^(n)(z - c) sum_y w (c - y)^n / n!) with f = log, the classical 2-D
    multipole expansion (complex variables)."""
    g = np.random.Generator(np.random.PCG64(6))
    c = np.array([0.3, 0.6])
    src = c + 0.2 * (g.random((15, 2)) - 0.5)
    w = g.standard_normal(15)
    tgt = np.array([[1.4, 0.2], [-0.8, 1.5], [0.35, -0.9]])
    beta = T2.p2m("laplace2d", p, c, src, w, 1.0)
    got = T2.m2p("laplace2d", p, c, beta, tgt, 1.0)
    zc = complex(*c)
    zs = src[:, 0] + 1j * src[:, 1]
    for k, x in enumerate(tgt):
        u = complex(*x) - zc
        s = np.sum(w) * np.log(u)
        for n in range(1, p + 1):
            s += (-1) ** (n - 1) * math.factorial(n - 1) / u ** n * np.sum(w * (zc - zs) ** n) / math.factorial(n)
        assert abs(got[k] - s.real) <= 1e-12 * (1 + abs(s.real)), (p, k)


@pytest.mark.parametrize("kernel", KERNELS)
def test_expansions_converge_to_the_direct_sum(kernel):
    g = np.random.Generator(np.random.PCG64(7))
    h = 1.0 / 8
    cs, ct = np.array([0.5, 0.5]) * h, np.array([2.5, 1.5]) * h  # offset (2, 1) boxes
    src = cs + h * (g.random((30, 2)) - 0.5)
    tgt = ct + h * (g.random((10, 2)) - 0.5)
    w = g.standard_normal(30)
    ref = T2.direct_sum(kernel, src, w, tgt)
    errs = []
    for p in (2, 4, 8, 12):
        beta = T2.p2m(kernel, p, cs, src, w, h)
        theta = T2.m2l(kernel, p, ct - cs, beta, h)
        errs.append(np.abs(T2.l2p(kernel, p, ct, theta, tgt, h) - ref).max() / np.abs(ref).max())
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6, errs


def test_kept_set_order_and_sizes():
    assert T2.kept_set(3, 2) == [(0, 0), (1, 0), (2, 0), (3, 0), (0, 1), (1, 1), (2, 1)]
    for p in range(0, 17):
        assert len(T2.kept_set(p, 2)) == 2 * p + 1
        assert len(T2.kept_set(p, 4)) == (T2.n_full(p) - T2.n_full(p - 4) if p >= 4 else T2.n_full(p))


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("p", [1, 5, 9])
def test_m2m_equals_p2m_about_the_parent(kernel, p):
    """Both PDEs are homogeneous, so the compressed M2M of a child's P2M is the parent's own
    P2M of the same sources, to rounding (Sec. 4.3 for d = 2)."""
    g = np.random.Generator(np.random.PCG64(21 + p))
    hp, hc = 0.5, 0.25
    cp = np.array([0.25, 0.75])
    for o in ((1, 1), (-1, 1), (1, -1), (-1, -1)):
        cc = cp + 0.5 * hc * np.array(o)
        src = cc + hc * (g.random((25, 2)) - 0.5)
        w = g.standard_normal(25)
        psi = T2.m2m(kernel, p, cp - cc, T2.p2m(kernel, p, cc, src, w, hc), hc, hp)
        want = T2.p2m(kernel, p, cp, src, w, hp)
        assert np.abs(psi - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("p", [1, 5, 9])
def test_l2l_preserves_the_local_expansion(kernel, p):
    """Re-expanding a local's polynomial about a child centre changes nothing (Sec. 4.2 for
    d = 2): the child's local evaluated at its targets equals the parent's."""
    g = np.random.Generator(np.random.PCG64(31 + p))
    J = T2.kept_set(p, T2.pde_order(kernel))
    hp, hc = 0.5, 0.25
    cp = np.array([0.25, 0.75])
    theta = g.standard_normal(len(J)) * 0.6 ** np.array([a + b for a, b in J])
    for o in ((1, 1), (-1, 1), (1, -1), (-1, -1)):
        cc = cp + 0.5 * hc * np.array(o)
        tgt = cc + hc * (g.random((9, 2)) - 0.5)
        got = T2.l2p(kernel, p, cc, T2.l2l(kernel, p, cc - cp, theta, hp, hc), tgt, hc)
        want = T2.l2p(kernel, p, cp, theta, tgt, hp)
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
