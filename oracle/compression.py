"""Algebraic compression (Sec. 3.1): the PDE-coefficient matrix P, the index maps
h, j-bar and j, and the dense decompression operator M.

Everything is built exactly as the section states, densely:
  b_{n,m} = a_{m-n} if m >= n and m - n in M(c), else 0          (eq. coeff-shift)
  P[i1, i2] = b_{nu(i1), nu(i2)},  P in C^{N(p-c) x N(p)}            (eq. define_P)
  h(i) = last nonzero column of row i,  j-bar = (h(1), ..., h(N(p-c)))  (eqs. define_h,
         define_bar_j)
  j = the remaining columns, in increasing order
  M[j, :] = I,  M[j-bar, :] = -P[:, j-bar]^{-1} P[:, j]              (eq. decompression)

``exact=True`` runs the triangular solve in Python Fractions (exact for every
kernel: float PDE coefficients convert to rationals without rounding) and rounds
M at the end; ``exact=False`` uses a float64 triangular solve.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

import numpy as np
import scipy.linalg

from .kernels import pde_coefficients, pde_order
from .multiindex import graded_order, index_of, mge, morder, msub, n_full


def pde_matrix(kernel: str, param: float, p: int) -> np.ndarray:
    """P (eq. define_P) as a dense object array of Fractions."""
    a = {k: Fraction(v) for k, v in pde_coefficients(kernel, param).items() if v != 0}
    c = pde_order(kernel)
    rows = graded_order(p - c) if p >= c else ()
    cols = graded_order(p)
    P = np.empty((len(rows), len(cols)), dtype=object)
    P[...] = Fraction(0)
    for i1, n in enumerate(rows):
        for i2, m in enumerate(cols):
            if mge(m, n):
                d = msub(m, n)
                if morder(d) <= c and d in a:
                    P[i1, i2] = a[d]
    return P


def h_and_jbar(P: np.ndarray):
    """h(i) for each row (0-based) and the kept columns j (complement of j-bar)."""
    h = []
    for i in range(P.shape[0]):
        nz = [l for l in range(P.shape[1]) if P[i, l] != 0]
        h.append(max(nz))
    jbar = list(h)
    jset = set(jbar)
    j = [l for l in range(P.shape[1]) if l not in jset]
    return h, jbar, j


@lru_cache(maxsize=None)
def _decompression_cached(kernel: str, param: float, p: int, exact: bool):
    P = pde_matrix(kernel, param, p)
    N = n_full(p)
    if P.shape[0] == 0:
        return np.eye(N), list(range(N)), []
    _, jbar, j = h_and_jbar(P)
    A = P[:, jbar]  # lower triangular, nonzero diagonal (Lemma lower_triangular)
    B = P[:, j]
    if exact:
        n = A.shape[0]
        X = np.empty(B.shape, dtype=object)
        for col in range(B.shape[1]):
            for row in range(n):
                s = B[row, col]
                for k in range(row):
                    if A[row, k] != 0:
                        s -= A[row, k] * X[k, col]
                X[row, col] = s / A[row, row]
        Xf = np.array([[float(v) for v in r] for r in X], dtype=np.float64).reshape(B.shape)
    else:
        Af = np.array(A, dtype=np.float64)
        Bf = np.array(B, dtype=np.float64)
        Xf = scipy.linalg.solve_triangular(Af, Bf, lower=True)
    M = np.zeros((N, len(j)))
    M[j, :] = np.eye(len(j))
    M[jbar, :] = -Xf
    return M, j, jbar


def decompression_matrix(kernel: str, param: float, p: int, exact: bool = True):
    """(M, j, jbar): M in R^{N(p) x N_c} with D^p G = M [D^p G]_j (eq. decompression).
    j and jbar are 0-based positions in the graded order of M(p)."""
    M, j, jbar = _decompression_cached(kernel, float(param), int(p), bool(exact))
    return M.copy(), list(j), list(jbar)


def kept_indices(kernel: str, param: float, p: int) -> list:
    """The multi-indices nu(j) in the order of j."""
    _, j, _ = decompression_matrix(kernel, param, p)
    order = graded_order(p)
    return [order[i] for i in j]


def compress(kernel: str, param: float, p: int, alpha: np.ndarray) -> np.ndarray:
    """beta = M^T alpha (eq. define_beta_multipole); alpha in graded order of M(p)."""
    M, _, _ = decompression_matrix(kernel, param, p)
    return M.T @ alpha


def decompress(kernel: str, param: float, p: int, theta: np.ndarray) -> np.ndarray:
    """M theta: the full derivative vector from its kept entries (eq. decompression)."""
    M, _, _ = decompression_matrix(kernel, param, p)
    return M @ theta


def position_map(p: int, indices) -> np.ndarray:
    """Positions of the given multi-indices in the graded order of M(p)."""
    idx = index_of(p)
    return np.array([idx[tuple(m)] for m in indices], dtype=np.int64)
