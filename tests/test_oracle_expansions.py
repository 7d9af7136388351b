"""Pins for the oracle's uncompressed and compressed P2M / M2L / L2P."""
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
def test_p0_is_monopole(two_box, kernel, param):
    src, tgt, w, c1, c2 = two_box
    alpha = T.p2m_full(0, c1, src, w)
    assert alpha.shape == (1,) and abs(alpha[0] - w.sum()) <= 1e-14 * np.abs(w).sum()
    beta = Z.p2m(kernel, param, 0, c1, src, w)
    th = Z.m2l(kernel, param, 0, c2 - c1, beta)
    phi = Z.l2p(kernel, param, 0, c2, th, tgt)
    G = K.green(kernel, param, np.linalg.norm(c2 - c1))
    assert np.allclose(phi, w.sum() * G, rtol=1e-14, atol=0)


@pytest.mark.parametrize("kernel,param,pmax", [("laplace", 0.0, 8), ("helmholtz", 1.0, 6),
                                               ("yukawa", 2.0, 6), ("biharmonic", 0.0, 8)])
def test_compressed_equals_full_taylor(two_box, kernel, param, pmax):
    # Compressed P2M/M2L/L2P add no error to Cartesian Taylor (Sec. 1; Secs. 3.3, 3.4, 4.1)
    src, tgt, w, c1, c2 = two_box
    for p in range(1, pmax + 1):
        alpha = T.p2m_full(p, c1, src, w)
        Lf = T.m2l_full(kernel, param, p, c2 - c1, alpha)
        phi_full = T.l2p_full(p, c2, Lf, tgt)
        beta = Z.p2m(kernel, param, p, c1, src, w)
        th = Z.m2l(kernel, param, p, c2 - c1, beta)
        # the compressed local is the kept part of the full local
        J = Z.kept(kernel, param, p)
        pos = [MI.index_of(p)[m] for m in J]
        assert rel_err(th, Lf[pos]) < 1e-13
        phi_c = Z.l2p(kernel, param, p, c2, th, tgt)
        assert rel_err(phi_c, phi_full) < 1e-13


@pytest.mark.parametrize("kernel,param", KPARAM)
def test_geometric_decay_against_direct_sum(two_box, kernel, param):
    # Truncation error O((r/R)^(p+1)) (eqs. local_truncated, mpole_truncated)
    src, tgt, w, c1, c2 = two_box
    exact = K.direct_sum(kernel, param, src, w, tgt)
    errs = []
    for p in (2, 4, 6, 8):
        beta = Z.p2m(kernel, param, p, c1, src, w)
        th = Z.m2l(kernel, param, p, c2 - c1, beta)
        errs.append(rel_err(Z.l2p(kernel, param, p, c2, th, tgt), exact))
    for a, b in zip(errs, errs[1:]):
        assert b < 0.5 * a, errs
    assert errs[-1] < 2e-4


def test_m2l_local_coefficients_converge_to_p2l(two_box):
    # The derivative-form local from M2L approaches the exact local sum_y w D^i G(c2 - y)
    src, tgt, w, c1, c2 = two_box
    errs = []
    for p in (3, 6, 9):
        beta = Z.p2m("laplace", 0.0, p, c1, src, w)
        th = Z.m2l("laplace", 0.0, p, c2 - c1, beta)
        exact = T.p2l_full("laplace", 0.0, p, c2, src, w)
        J = Z.kept("laplace", 0.0, p)
        pos = [MI.index_of(p)[m] for m in J]
        sel = [k for k, m in enumerate(J) if sum(m) <= 2]
        errs.append(rel_err(th[sel], exact[pos][sel]))
    assert errs[1] < 0.1 * errs[0] and errs[2] < 0.1 * errs[1]


def test_single_source_multipole_is_the_monomial():
    c = np.array([0.1, -0.2, 0.3])
    y = np.array([[0.25, 0.05, -0.15]])
    alpha = T.p2m_full(4, c, y, np.array([2.0]))
    v = c - y[0]
    for k, m in enumerate(MI.graded_order(4)):
        expect = 2.0 * v[0] ** m[0] * v[1] ** m[1] * v[2] ** m[2] / MI.mfact(m)
        assert abs(alpha[k] - expect) <= 1e-16


@pytest.mark.parametrize("kernel,param", KPARAM)
def test_scaled_form_is_equivalent(two_box, kernel, param):
    # Sec. 4.1.1: scaling by t preserves the translation
    src, tgt, w, c1, c2 = two_box
    p, t = 6, 4.0
    beta = Z.p2m(kernel, param, p, c1, src, w)
    th = Z.m2l(kernel, param, p, c2 - c1, beta)
    th_s = Z.m2l_scaled(kernel, param, p, c2 - c1, Z.scale_multipole(kernel, param, p, beta, t), t)
    assert rel_err(Z.unscale_local(kernel, param, p, th_s, t), th) < 1e-14


@pytest.mark.parametrize("kernel,param", KPARAM)
def test_fft_form_equals_direct_convolution(two_box, kernel, param):
    # eq. convolution_m2l through the circulant embedding; scaled (Sec. 4.1.1) so that the
    # FFT sees values of similar size
    src, tgt, w, c1, c2 = two_box
    p = 8
    t = p / np.linalg.norm(c2 - c1)
    beta = Z.scale_multipole(kernel, param, p, Z.p2m(kernel, param, p, c1, src, w), t)
    table = Z.slab_table(kernel, param, p, c2 - c1)
    tt = {m: v / t ** sum(m) for m, v in table.items()}
    a = Z.m2l(kernel, param, p, c2 - c1, beta, tt)
    b = Z.m2l_fft(kernel, param, p, c2 - c1, beta, tt)
    assert rel_err(b, a) < 1e-13
    c = K.pde_order(kernel)
    J = Z.kept(kernel, param, p)
    assert (max(m[0] for m in J), max(m[1] for m in J), max(m[2] for m in J)) == (p, p, c - 1)
