"""Uncompressed Cartesian Taylor expansions and translations (Sec. 2).

Conventions (the paper's, with the density w restored in every source sum):
  multipole   alpha_q = sum_y w(y) (c - y)^q / q!                 (eq. mpole)
              G(x - y) ~ sum_q G^(q)(x - c) (c - y)^q / q!
  M2L         L[i] = sum_{q in M(p)} G^(i+q)(c2 - c1) alpha_q      (O(p^6) naive M2L)
              (derivative form: L[i] is d^i of the potential at c2)
  L2P         phi(x) = sum_{i in M(p)} L[i] (x - c2)^i / i!        (eq. local)
  M2M         rho_q = sum_{i <= q} h^(q-i) / (q-i)! alpha_i,  h = c_new - c_old
                                                     (eq. mpole_translated_full_coeffs)
  L2L         L'[i] = sum_{q >= i, q in M(p)} L[q] h^(q-i) / (q-i)!,  h = c_new - c_old
              (eq. l2l-expr, written for the derivative form: L'[i] = i! mu_i)
All coefficient vectors are in the graded order of M(p).
"""
from __future__ import annotations

import numpy as np

from .kernels import deriv_table_mp, deriv_table_rec
from .multiindex import graded_order, madd, mfact, mge, mpow, msub


def p2m_full(p: int, center, src, w) -> np.ndarray:
    """alpha_q = sum_s w_s (c - y_s)^q / q!  for q in M(p)."""
    v = np.asarray(center, np.float64)[None, :] - np.asarray(src, np.float64)
    w = np.asarray(w)
    return np.array([np.sum(w * mpow(v, q)) / mfact(q) for q in graded_order(p)])


def full_table(kernel: str, param: float, p: int, d, mp: bool = False) -> dict:
    """{m: G^(m)(d)} for every |m| <= 2p."""
    idx = list(graded_order(2 * p))
    vals = (deriv_table_mp if mp else deriv_table_rec)(kernel, param, d, idx)
    return dict(zip(idx, vals))


def m2l_full(kernel: str, param: float, p: int, d, alpha, table: dict | None = None) -> np.ndarray:
    """L[i] = sum_{q in M(p)} G^(i+q)(d) alpha_q, d = c_target - c_source."""
    if table is None:
        table = full_table(kernel, param, p, d)
    order = graded_order(p)
    T = np.array([[table[madd(i, q)] for q in order] for i in order])
    return T @ np.asarray(alpha)


def l2p_full(p: int, center, L, tgt) -> np.ndarray:
    """phi(x) = sum_i L[i] (x - c)^i / i!."""
    v = np.asarray(tgt, np.float64) - np.asarray(center, np.float64)[None, :]
    out = 0
    for i, m in enumerate(graded_order(p)):
        out = out + L[i] * mpow(v, m) / mfact(m)
    return np.asarray(out)


def p2l_full(kernel: str, param: float, p: int, center, src, w) -> np.ndarray:
    """Local coefficients (derivative form) straight from sources:
    L[i] = sum_y w(y) G^(i)(c - y) (eq. local), for the decay tests."""
    order = list(graded_order(p))
    out = np.zeros(len(order), dtype=np.complex128 if np.iscomplexobj(w) or kernel == "helmholtz"
                   else np.float64)
    for y, wy in zip(np.asarray(src), np.asarray(w)):
        out = out + wy * deriv_table_rec(kernel, param, np.asarray(center) - y, order)
    return out


def _shift_factor(h, m) -> float:
    """h^m / m! for one translation vector h."""
    return float(mpow(np.asarray(h, np.float64)[None, :], m)[0]) / mfact(m)


def m2m_full(p: int, h, alpha) -> np.ndarray:
    """Multipole translation by h = c_new - c_old (eq. mpole_translated_full_coeffs):
    rho_q = sum_{i <= q} h^(q-i)/(q-i)! alpha_i, from the binomial expansion of
    (c_new - y)^q = ((c_new - c_old) + (c_old - y))^q."""
    order = graded_order(p)
    alpha = np.asarray(alpha)
    out = np.zeros(len(order), dtype=alpha.dtype)
    for a, q in enumerate(order):
        for b, i in enumerate(order):
            if mge(q, i):
                out[a] += _shift_factor(h, msub(q, i)) * alpha[b]
    return out


def l2l_full(p: int, h, L) -> np.ndarray:
    """Local translation by h = c_new - c_old (eq. l2l-expr), derivative form: the
    derivatives at c_new of the degree-p polynomial sum_q L[q] (x - c_old)^q / q!."""
    order = graded_order(p)
    L = np.asarray(L)
    out = np.zeros(len(order), dtype=L.dtype)
    for a, i in enumerate(order):
        for b, q in enumerate(order):
            if mge(q, i):
                out[a] += _shift_factor(h, msub(q, i)) * L[b]
    return out
