"""Pins for the oracle's multi-index sets and the compression matrices (Sec. 3.1)."""
import itertools
from math import comb

import mpmath
import numpy as np
import pytest

from oracle import compression as C
from oracle import kernels as K
from oracle import multiindex as MI

KPARAM = [("laplace", 0.0), ("helmholtz", 1.3), ("yukawa", 2.0), ("biharmonic", 0.0)]


def brute_M(p):
    return [m for m in itertools.product(range(p + 1), repeat=3) if sum(m) <= p]


@pytest.mark.parametrize("p", range(0, 13))
def test_count_and_order(p):
    order = MI.graded_order(p)
    # |M(p)| by brute force, and the closed form C(p+3, 3) (reading of eq. np-count)
    assert sorted(order) == sorted(brute_M(p))
    assert len(order) == comb(p + 3, 3) == MI.n_full(p)
    # Def. bnu: first is zero, degree is non-decreasing
    assert order[0] == (0, 0, 0)
    degs = [sum(m) for m in order]
    assert degs == sorted(degs)


def test_graded_order_compatible_with_addition():
    # Def. bnu (iii): i < j  =>  nu^-1(nu(i) + nu(k)) < nu^-1(nu(j) + nu(k))
    p = 5
    order = MI.graded_order(p)
    big = MI.index_of(2 * p)
    for i, j in itertools.combinations(range(len(order)), 2):
        for k in range(0, len(order), 7):
            a = big[MI.madd(order[i], order[k])]
            b = big[MI.madd(order[j], order[k])]
            assert a < b


@pytest.mark.parametrize("kernel,param", KPARAM)
@pytest.mark.parametrize("p", [0, 1, 3, 4, 6, 8])
def test_kept_set_structure(kernel, param, p):
    c = K.pde_order(kernel)
    P = C.pde_matrix(kernel, param, p)
    assert P.shape == (MI.n_full(p - c), MI.n_full(p))
    M, j, jbar = C.decompression_matrix(kernel, param, p)
    order = MI.graded_order(p)
    # Lemma max_prod_nice: with z slowest, the kept indices are exactly m_z < c
    assert {order[i] for i in j} == {m for m in order if m[2] < c}
    assert len(j) == MI.n_full(p) - MI.n_full(p - c)
    if c == 2:
        assert len(j) == (p + 1) ** 2
    if P.shape[0]:
        h, _, _ = C.h_and_jbar(P)
        # Lemma h_increasing and Lemma h_eq
        assert all(a < b for a, b in zip(h, h[1:]))
        rows = MI.graded_order(p - c)
        for i, n in enumerate(rows):
            assert order[h[i]] == MI.madd(order[h[0]], n)
        assert order[h[0]] == (0, 0, c)
        # Lemma lower_triangular
        A = np.array(P[:, jbar], dtype=float)
        assert np.allclose(A, np.tril(A)) and np.all(np.diag(A) != 0)
    # M restricted to j is the identity
    assert np.array_equal(M[j, :], np.eye(len(j)))


@pytest.mark.parametrize("kernel,param", KPARAM)
def test_exact_and_float_decompression_agree(kernel, param):
    for p in (4, 7):
        Me, _, _ = C.decompression_matrix(kernel, param, p, exact=True)
        Mf, _, _ = C.decompression_matrix(kernel, param, p, exact=False)
        assert np.max(np.abs(Me - Mf)) <= 1e-12 * max(1.0, np.max(np.abs(Me)))


def test_laplace_decompression_small_case_by_hand():
    # p = 2, Laplace: the only dropped index is (0,0,2) and D(0,0,2) = -D(2,0,0) - D(0,2,0)
    M, j, jbar = C.decompression_matrix("laplace", 0.0, 2)
    order = MI.graded_order(2)
    assert [order[i] for i in jbar] == [(0, 0, 2)]
    row = M[jbar[0]]
    kept = [order[i] for i in j]
    expect = np.array([-1.0 if m in ((2, 0, 0), (0, 2, 0)) else 0.0 for m in kept])
    assert np.array_equal(row, expect)


def test_biharmonic_below_pde_order_is_identity():
    for p in range(4):
        M, j, jbar = C.decompression_matrix("biharmonic", 0.0, p)
        assert jbar == [] and np.array_equal(M, np.eye(MI.n_full(p)))


@pytest.mark.parametrize("kernel,param", KPARAM)
def test_pde_nullspace_and_decompression_on_true_derivatives(kernel, param):
    # eq. Pv: P D^p G(x) = 0;  eq. decompression: D^p G = M [D^p G]_j   (mpmath truth)
    p = 6
    order = list(MI.graded_order(p))
    x = np.array([0.37, -0.81, 0.55])
    Dv = K.deriv_table_mp(kernel, param, x, order)
    P = np.array(C.pde_matrix(kernel, param, p), dtype=float)
    assert np.linalg.norm(P @ Dv) <= 1e-13 * np.linalg.norm(Dv)
    M, j, _ = C.decompression_matrix(kernel, param, p)
    assert np.linalg.norm(M @ Dv[j] - Dv) <= 1e-13 * np.linalg.norm(Dv)
