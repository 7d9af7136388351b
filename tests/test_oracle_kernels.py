"""Pins for the oracle's kernels, derivative tables and direct sum."""
from math import pi

import mpmath
import numpy as np
import pytest
import sympy as sp

from oracle import kernels as K
from oracle import multiindex as MI

KPARAM = [("laplace", 0.0), ("helmholtz", 1.3), ("yukawa", 2.0), ("biharmonic", 0.0)]


def sympy_kernel(kernel, param):
    x, y, z = sp.symbols("x y z", real=True)
    r = sp.sqrt(x ** 2 + y ** 2 + z ** 2)
    prm = sp.nsimplify(param)
    if kernel == "laplace":
        G = 1 / (4 * sp.pi * r)
    elif kernel == "helmholtz":
        G = sp.exp(sp.I * prm * r) / (4 * sp.pi * r)
    elif kernel == "yukawa":
        G = sp.exp(-prm * r) / (4 * sp.pi * r)
    else:
        G = r
    return G, (x, y, z)


@pytest.mark.parametrize("kernel,param", KPARAM)
def test_mp_table_matches_exact_symbolic_differentiation(kernel, param):
    # Exact differentiation by sympy at a rational point, orders <= 5.
    G, (x, y, z) = sympy_kernel(kernel, param)
    pt = (sp.Rational(3, 7), sp.Rational(-5, 11), sp.Rational(2, 3))
    idx = list(MI.graded_order(5))
    got = K.deriv_table_mp(kernel, param, [float(v) for v in pt], idx)
    for m, g in zip(idx, got):
        e = sp.diff(G, x, m[0], y, m[1], z, m[2]).subs({x: pt[0], y: pt[1], z: pt[2]})
        ev = complex(sp.N(e, 30))
        assert abs(g - ev) <= 1e-14 * max(1.0, abs(ev)), (m, g, ev)


def per_order_rel(a, b, idx):
    worst = 0.0
    for n in sorted({sum(m) for m in idx}):
        sel = [k for k, m in enumerate(idx) if sum(m) == n]
        nb = np.linalg.norm(b[sel])
        worst = max(worst, np.linalg.norm(a[sel] - b[sel]) / nb)
    return worst


OFFSETS = [(2, 0, 0), (3, 3, 3), (2, -3, 1), (0, 0, 2), (3, -2, 0), (-2, 1, 3)]


@pytest.mark.parametrize("kernel,param,h", [("laplace", 0.0, 1 / 16), ("yukawa", 2.0, 1 / 16),
                                            ("yukawa", 2.0, 1 / 4), ("helmholtz", 16.0, 1 / 16),
                                            ("helmholtz", 1.0, 1 / 4), ("biharmonic", 0.0, 1 / 16)])
def test_recurrence_tables_match_mpmath_at_order_24(kernel, param, h):
    p = 12
    idx = K.slab_indices(2 * p, 2 * (K.pde_order(kernel) - 1))
    for o in OFFSETS:
        d = np.array(o) * h
        mp = K.deriv_table_mp(kernel, param, d, idx, dps=40)
        rec = K.deriv_table_rec(kernel, param, d, idx)
        assert per_order_rel(rec, mp, idx) < 2e-14, o


def test_radial_fp64_formula_cancels_near_axis():
    # Documents why the float64 tables do not use the radial product formula.
    idx = K.slab_indices(24, 2)
    d = np.array([2.0, 0.0, 0.0]) / 16
    mp = K.deriv_table_mp("laplace", 0.0, d, idx, dps=40)
    fp = K.deriv_table_fp("laplace", 0.0, d, idx)
    assert per_order_rel(fp, mp, idx) > 1e-11


def test_paper_laplace_recurrence_matches_mpmath():
    # eq. deriv_laplace_3d
    idx = list(MI.graded_order(20))
    for o in OFFSETS:
        d = np.array(o) / 8
        R = K.laplace_recurrence_table(d, 20)
        rec = np.array([R[m] for m in idx])
        mp = K.deriv_table_mp("laplace", 0.0, d, idx, dps=40)
        assert per_order_rel(rec, mp, idx) < 2e-14


@pytest.mark.parametrize("kernel,param", KPARAM)
def test_derivative_parity_and_pde_identity(kernel, param):
    idx = K.slab_indices(10, 10)
    d = np.array([0.31, -0.44, 0.27])
    a = K.deriv_table_rec(kernel, param, d, idx)
    b = K.deriv_table_rec(kernel, param, -d, idx)
    sign = np.array([(-1) ** sum(m) for m in idx])
    assert np.max(np.abs(b - sign * a)) <= 1e-13 * np.max(np.abs(a))
    # L G^(m) = 0 for every derivative (the PDE holds away from the origin)
    pos = {m: k for k, m in enumerate(idx)}
    coef = K.pde_coefficients(kernel, param)
    c = K.pde_order(kernel)
    for m in K.slab_indices(10 - c, 10):
        tot = sum(a_ * a[pos[MI.madd(m, xi)]] for xi, a_ in coef.items())
        scale = max(abs(a[pos[MI.madd(m, xi)]]) for xi in coef)
        assert abs(tot) <= 1e-12 * scale


def test_closed_form_first_derivatives():
    d = np.array([0.3, -0.7, 0.45])
    r = np.linalg.norm(d)
    idx = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    lap = K.deriv_table_rec("laplace", 0.0, d, idx)
    assert np.allclose(lap, -d / (4 * pi * r ** 3), rtol=1e-15, atol=0)
    bih = K.deriv_table_rec("biharmonic", 0.0, d, idx)
    assert np.allclose(bih, d / r, rtol=1e-15, atol=0)
    for kern, prm in (("yukawa", 2.0), ("helmholtz", 1.3)):
        g = K.deriv_table_rec(kern, prm, d, idx)
        assert np.allclose(g, K.grad_green(kern, prm, d), rtol=1e-14, atol=0)


@pytest.mark.parametrize("kernel,param", KPARAM)
def test_direct_sum_brute_force_mpmath(kernel, param):
    g = np.random.Generator(np.random.PCG64(5))
    src = g.random((7, 3))
    tgt = g.random((5, 3)) + np.array([1.5, 0, 0])
    w = g.standard_normal(7)
    got = K.direct_sum(kernel, param, src, w, tgt)
    for i in range(5):
        s = 0
        for j in range(7):
            r = mpmath.sqrt(sum((mpmath.mpf(tgt[i, k]) - mpmath.mpf(src[j, k])) ** 2 for k in range(3)))
            if kernel == "laplace":
                G = 1 / (4 * mpmath.pi * r)
            elif kernel == "helmholtz":
                G = mpmath.exp(1j * param * r) / (4 * mpmath.pi * r)
            elif kernel == "yukawa":
                G = mpmath.exp(-param * r) / (4 * mpmath.pi * r)
            else:
                G = r
            s += G * w[j]
        assert abs(got[i] - complex(s)) <= 1e-14 * abs(complex(s)) + 1e-15


def test_direct_sum_skips_self_and_is_reciprocal():
    g = np.random.Generator(np.random.PCG64(6))
    pts = g.random((40, 3))
    w = g.standard_normal(40)
    c = g.standard_normal(40)
    phi = K.direct_sum("laplace", 0.0, pts, w, pts)
    assert np.all(np.isfinite(phi))
    psi = K.direct_sum("laplace", 0.0, pts, c, pts)
    # G even => <c, phi_w> = <w, psi_c>
    assert abs(c @ phi - w @ psi) <= 1e-13 * abs(c @ phi)
