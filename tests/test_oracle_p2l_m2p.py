"""Pins for the oracle's compressed P2L (Sec. 3.2) and compressed M2P (Sec. 3.5).

Both use only the derivatives of the kept set J.  Since every derivative of G satisfies the PDE,
the compressed forms lose nothing against the full Cartesian Taylor forms (Thm. mult_decompression):
the decompressed P2L local equals the full local expansion of the same sources, and the compressed
multipole evaluation equals the full one, to roundoff.  Independently of that algebra: p = 0 is the
monopole (a closed form), both converge to the direct sum of eq. (1) geometrically in p, and the
mpmath derivatives (the radial formula, no recurrence) give the same coefficients."""
import numpy as np
import pytest

import workloads as W
from oracle import compressed as Z
from oracle import kernels as K
from oracle import multiindex as MI
from oracle import taylor as T

from conftest import rel_err

KPARAM = [("laplace", 0.0), ("helmholtz", 1.0), ("yukawa", 2.0), ("biharmonic", 0.0)]


@pytest.fixture(scope="module")
def two_box():
    return W.small_two_box(0)


@pytest.mark.parametrize("kernel,param", KPARAM)
def test_p0_is_the_monopole(two_box, kernel, param):
    src, tgt, w, c1, c2 = two_box
    # P2L at p = 0: the potential of the sources at the centre
    th = Z.p2l(kernel, param, 0, c2, src, w)
    assert rel_err(th, [K.direct_sum(kernel, param, src, w, c2[None, :])[0]]) < 1e-14
    # M2P at p = 0: total weight times G at the distance from the centre
    beta = Z.p2m(kernel, param, 0, c1, src, w)
    phi = Z.m2p(kernel, param, 0, c1, beta, tgt)
    G = K.green(kernel, param, np.linalg.norm(tgt - c1, axis=1))
    assert rel_err(phi, w.sum() * G) < 1e-14


@pytest.mark.parametrize("kernel,param,p", [("laplace", 0.0, 8), ("helmholtz", 1.0, 6), ("yukawa", 2.0, 6),
                                            ("biharmonic", 0.0, 8)])
def test_compressed_p2l_equals_the_full_local(two_box, kernel, param, p):
    # eq. compressed-local-form: [M theta]_i / i! is the full local coefficient of the same sources
    src, tgt, w, c1, c2 = two_box
    th = Z.p2l(kernel, param, p, c2, src, w)
    full = T.p2l_full(kernel, param, p, c2, src, w)
    assert rel_err(Z.local_full(kernel, param, p, th), full) < 1e-12
    assert rel_err(Z.l2p(kernel, param, p, c2, th, tgt), T.l2p_full(p, c2, full, tgt)) < 1e-12


@pytest.mark.parametrize("kernel,param,p", [("laplace", 0.0, 8), ("helmholtz", 1.0, 6), ("yukawa", 2.0, 6),
                                            ("biharmonic", 0.0, 8)])
def test_compressed_m2p_equals_the_full_evaluation(two_box, kernel, param, p):
    # eq. multipole_eval_beta: [D G(x - c)]_j^T M^T alpha = D G(x - c)^T alpha over all of M(p)
    src, tgt, w, c1, c2 = two_box
    beta = Z.p2m(kernel, param, p, c1, src, w)
    alpha = T.p2m_full(p, c1, src, w)
    order = list(MI.graded_order(p))
    full = np.array([K.deriv_table_rec(kernel, param, x - c1, order) @ alpha for x in tgt])
    assert rel_err(Z.m2p(kernel, param, p, c1, beta, tgt), full) < 1e-12


@pytest.mark.parametrize("kernel,param", KPARAM)
def test_converge_to_the_direct_sum(two_box, kernel, param):
    # truncation errors O((r/R)^(p+1)) for both forms (eqs. local_truncated, mpole_truncated)
    src, tgt, w, c1, c2 = two_box
    exact = K.direct_sum(kernel, param, src, w, tgt)
    e_l, e_m = [], []
    for p in (2, 4, 6, 8):
        th = Z.p2l(kernel, param, p, c2, src, w)
        e_l.append(rel_err(Z.l2p(kernel, param, p, c2, th, tgt), exact))
        beta = Z.p2m(kernel, param, p, c1, src, w)
        e_m.append(rel_err(Z.m2p(kernel, param, p, c1, beta, tgt), exact))
    for errs in (e_l, e_m):
        for a, b in zip(errs, errs[1:]):
            assert b < a, errs  # (Yukawa's low orders decay slowly at first: e^(-lambda r) factor)
        assert errs[-1] < 0.01 * errs[0] and errs[-1] < 2e-4, errs


@pytest.mark.parametrize("kernel,param", [("laplace", 0.0), ("yukawa", 2.0)])
def test_mpmath_derivatives_agree(two_box, kernel, param):
    # the radial formula at 50 digits shares no step with the recurrences
    src, tgt, w, c1, c2 = two_box
    p = 6
    assert rel_err(Z.p2l(kernel, param, p, c2, src[:8], w[:8]),
                   Z.p2l(kernel, param, p, c2, src[:8], w[:8], mp=True)) < 1e-13
    beta = Z.p2m(kernel, param, p, c1, src, w)
    assert rel_err(Z.m2p(kernel, param, p, c1, beta, tgt[:8]), Z.m2p(kernel, param, p, c1, beta, tgt[:8], mp=True)) < 1e-13
