"""The oracle's compressed M2M against the errors the paper prints for its M2M accuracy
experiment (tests/golden/m2m_accuracy_helmholtz_3d.txt; Sec. 5.1, Fig. m2m_accuracy).

The sources are the paper's (a 50^3 grid with uniform random strengths, seeded here); the
targets are an 11^3 grid over the paper's target cube instead of 50^3, to keep the test to
seconds.  eps_rel is a ratio of sums over the target grid; with the coarser grid it comes out
at 1.0 to 1.3 times the printed value (1.03 to 1.07 with a 25^3 grid), so the bound is a factor
of 1.5.  Laplace and biharmonic must stay below the paper's 1e-14.
"""
import os

import numpy as np
import pytest

from oracle import compressed as Z
from oracle import kernels as K
from oracle import taylor as T
from oracle.multiindex import graded_order

HERE = os.path.dirname(os.path.abspath(__file__))


def grid(center, side, n):
    t = np.linspace(-0.5, 0.5, n)
    g = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3) * side
    return g + np.asarray(center, dtype=np.float64)


def eps_rel(kernel, param, p, R, n_src=50, n_tgt=11, seed=3):
    """Relative difference at the targets between the compressed and the uncompressed
    translated expansions of the sources (Sec. 5.1)."""
    c1, c2 = np.array([R, R, R]), np.zeros(3)
    src = grid(c1, 2 * R, n_src)
    w = np.random.Generator(np.random.PCG64(seed)).uniform(0.0, 1.0, len(src))
    rho = T.m2m_full(p, c2 - c1, T.p2m_full(p, c1, src, w))
    psi = Z.m2m(kernel, param, p, c2 - c1, Z.p2m(kernel, param, p, c1, src, w))
    full, J = list(graded_order(p)), Z.kept(kernel, param, p)
    num = den = 0.0
    for x in grid([1.0, 1.0, 1.0], 1.0, n_tgt):
        uncompressed = np.dot(rho, K.deriv_table_rec(kernel, param, x - c2, full))
        compressed = np.dot(psi, K.deriv_table_rec(kernel, param, x - c2, J))
        num += abs(compressed - uncompressed) ** 2
        den += abs(uncompressed) ** 2
    return float(np.sqrt(num / den))


def rows():
    with open(os.path.join(HERE, "golden", "m2m_accuracy_helmholtz_3d.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                p, R, v = (s.strip() for s in line.split("|"))
                yield int(p), float(R), float(v)


@pytest.mark.parametrize("p,R,printed", list(rows()))
def test_helmholtz_m2m_error_matches_the_paper(p, R, printed):
    ratio = eps_rel("helmholtz", 1.0, p, R) / printed
    assert 1 / 1.5 < ratio < 1.5, ratio


@pytest.mark.parametrize("kernel", ["laplace", "biharmonic"])
def test_equal_order_m2m_error_below_paper_bound(kernel):
    assert eps_rel(kernel, 0.0, 6, 0.125) < 1e-14


# Fig. m2m_accuracy_compare (Helmholtz 3D): the wavenumber sweep at R = 1e-2.  eps_rel on a 7^3
# target grid, eps_trunc on a 5^3 grid (its direct sum over the 125,000 sources is the cost);
# both come out at 0.92 to 1.13 times the printed values, except eps_trunc at kappa = 1, p = 4,
# where the truncation error varies strongly over the target cube and a coarse grid reads
# 1.8 to 2.2 times the printed value: that row is checked for eps_rel only.
def compare_rows():
    with open(os.path.join(HERE, "golden", "m2m_accuracy_compare_helmholtz_3d.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                p, kappa, rel, trunc = (s.strip() for s in line.split("|"))
                yield int(p), float(kappa), float(rel), float(trunc)


def eps_trunc(kappa, p, R=1e-2, n_src=50, n_tgt=5, seed=3):
    """Relative difference at the targets between the uncompressed translated expansion and
    the direct sum over the sources (Sec. 5.1)."""
    c1, c2 = np.array([R, R, R]), np.zeros(3)
    src = grid(c1, 2 * R, n_src)
    w = np.random.Generator(np.random.PCG64(seed)).uniform(0.0, 1.0, len(src))
    rho = T.m2m_full(p, c2 - c1, T.p2m_full(p, c1, src, w))
    tgt = grid([1.0, 1.0, 1.0], 1.0, n_tgt)
    full = list(graded_order(p))
    expansion = np.array([np.dot(rho, K.deriv_table_rec("helmholtz", kappa, x - c2, full)) for x in tgt])
    exact = K.direct_sum("helmholtz", kappa, src, w, tgt)
    return float(np.sqrt(np.sum(np.abs(expansion - exact) ** 2) / np.sum(np.abs(exact) ** 2)))


@pytest.mark.parametrize("p,kappa,printed,_", list(compare_rows()))
def test_helmholtz_wavenumber_sweep_m2m_error_matches_the_paper(p, kappa, printed, _):
    ratio = eps_rel("helmholtz", kappa, p, 1e-2, n_tgt=7) / printed
    assert 1 / 1.5 < ratio < 1.5, ratio


@pytest.mark.parametrize("p,kappa,printed", [(p, k, t) for p, k, _, t in compare_rows() if (p, k) in
                                             ((2, 50.0), (4, 13.5720880829745), (8, 50.0))])
def test_helmholtz_truncation_error_matches_the_paper(p, kappa, printed):
    ratio = eps_trunc(kappa, p) / printed
    assert 1 / 1.5 < ratio < 1.5, ratio
