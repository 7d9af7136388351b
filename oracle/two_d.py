"""Oracle (test infrastructure only): compressed Cartesian Taylor expansions in two dimensions
for the Laplace kernel G = log r and the biharmonic kernel G = r^2 log r (Sec. 4.4, subsections
Laplace 2D and Biharmonic 2D; the expansions are those of Secs. 2-3 written out for d = 2).

Only tests/, the bench's CPU-baseline leg and the smoke check may import this module; the HIP
path never does.  Everything here follows the definitions with no blocking or reordering:

  multi-indices   M(p) = {m = (m_x, m_y) : |m| <= p}; kept set J = {m in M(p) : m_y < c}, c the
                  order of the PDE (Laplace: Delta G = 0 away from 0, c = 2; biharmonic:
                  Delta^2 G = 0, c = 4).  The compressed axis is y (Lemma max_prod_nice's choice
                  of the last axis).  Storage order of J: m_y, then m_x (m_x fastest).
  derivatives     G^(m)(x) by exact complex analysis at 50 digits (mpmath): with z = x + i y,
                  log r = Re log z and r^2 log r = Re(conj(z) z log z), and d/dx = d/dz + d/dzbar,
                  d/dy = i (d/dz - d/dzbar) applied to functions of z and zbar.  Pinned to SymPy's
                  symbolic derivatives of the definitions in the tests.
  decompression   M (|M(p)| x |J|): the derivative D^m u of any solution u of the PDE in terms of
                  its kept derivatives, by replacing d_y^c with the rest of the PDE operator
                  (Laplace: d_y^2 = -d_x^2; biharmonic: d_y^4 = -d_x^4 - 2 d_x^2 d_y^2) until
                  m_y < c (Sec. 3, eqs. define_beta_multipole and compressed-local-form).  The
                  PDEs are homogeneous, so M is the same in the scaled form at every box size.
  P2M             alpha_q = sum_y w (c - y)^q / q!, beta = M^T alpha (eqs. mpole,
                  define_beta_multipole).
  M2L             theta_i = sum_{q in J} G^(i + q)(c_t - c_s) beta_q, i in J (eq. m2l_toeplitz
                  for d = 2).
  L2P             phi(x) = sum_{m in M(p)} (M theta)_m (x - c)^m / m! (eq. compressed-local-form).
  direct sum      phi(x) = sum_y G(x - y) w_y, the term x = y skipped (eq. (1)).
Scaled forms (Sec. 4.1.1, t = 1/h): beta~_q = beta_q / h^|q|, theta~_i = theta_i h^|i|, so that
theta~_i = sum_q [G^(i + q)(d) h^|i + q|] beta~_q.
"""
from __future__ import annotations

from math import factorial

import mpmath as mp
import numpy as np

KERNELS = {"laplace2d": 2, "biharmonic2d": 4}  # kernel -> PDE order c


def pde_order(kernel: str) -> int:
    return KERNELS[kernel]


def full_set(p: int) -> list:
    """M(p) in graded order: by |m|, then by m_y."""
    return [(n - b, b) for n in range(p + 1) for b in range(n + 1)]


def kept_set(p: int, c: int) -> list:
    """J in storage order: m_y = 0, 1, ..., c - 1, m_x = 0 .. p - m_y within each."""
    return [(a, b) for b in range(min(c, p + 1)) for a in range(p - b + 1)]


def n_full(p: int) -> int:
    return (p + 1) * (p + 2) // 2


def green(kernel: str, d) -> np.ndarray:
    """G at the vectors d [..., 2] (float64)."""
    r2 = np.sum(np.asarray(d, dtype=np.float64) ** 2, axis=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        if kernel == "laplace2d":
            return 0.5 * np.log(r2)
        return 0.5 * r2 * np.log(r2)


def deriv_mp(kernel: str, a: int, b: int, x, y):
    """G^(a, b)(x, y) = d_x^a d_y^b G at (x, y), as an mpmath real (current precision)."""
    z = mp.mpc(x, y)
    n = a + b
    if kernel == "laplace2d":
        # d_x^a d_y^b Re f(z) = Re(i^b f^(n)(z)) for holomorphic f = log z
        if n == 0:
            return mp.log(abs(z))
        return mp.re((1j) ** b * (-1) ** (n - 1) * mp.factorial(n - 1) / z ** n)

    # F = conj(z) h(z), h = z log z: d_zbar F = h, d_zbar^2 F = 0, so
    # (d_z + d_zbar)^a (i (d_z - d_zbar))^b F = i^b [conj(z) h^(n) + (a - b) h^(n - 1)]
    def h(k):
        if k == 0:
            return z * mp.log(z)
        if k == 1:
            return mp.log(z) + 1
        return (-1) ** k * mp.factorial(k - 2) / z ** (k - 1)

    F = mp.conj(z) * h(n) + ((a - b) * h(n - 1) if n >= 1 else 0)
    return mp.re((1j) ** b * F)


def table(kernel: str, p: int, d, h: float = 1.0, dps: int = 50) -> dict:
    """Scaled derivatives {(a, b): G^(a, b)(d) h^(a + b)} for a + b <= 2p, b <= 2(c - 1),
    evaluated at the translation vector d (not scaled) in mpmath and rounded to float64."""
    c = pde_order(kernel)
    with mp.workdps(dps):
        x, y, hh = mp.mpf(float(d[0])), mp.mpf(float(d[1])), mp.mpf(float(h))
        return {(a, b): float(deriv_mp(kernel, a, b, x, y) * hh ** (a + b))
                for b in range(2 * c - 1) for a in range(2 * p + 1 - b)}


def decompression_matrix(kernel: str, p: int) -> np.ndarray:
    """M: rows over M(p) (full_set order), columns over J (kept_set order); integer entries."""
    c = pde_order(kernel)
    # d_y^c = sum of (coefficient, x shift, y shift) terms of the same total order
    rule = [(-1, 2, 0)] if c == 2 else [(-1, 4, 0), (-2, 2, 2)]
    J = kept_set(p, c)
    col = {m: k for k, m in enumerate(J)}
    rows = {}

    def row(m):
        if m in rows:
            return rows[m]
        v = np.zeros(len(J))
        if m[1] < c:
            v[col[m]] = 1.0
        else:
            for coef, sx, sy in rule:
                v += coef * row((m[0] + sx, m[1] - c + sy))
        rows[m] = v
        return v

    return np.array([row(m) for m in full_set(p)])


def p2m(kernel: str, p: int, center, src, w, h: float = 1.0) -> np.ndarray:
    """Scaled compressed multipole beta~ [Nc] of the sources src [n, 2] with weights w."""
    M = decompression_matrix(kernel, p)
    X = (np.asarray(center, dtype=np.float64)[None, :] - np.asarray(src, dtype=np.float64)) / h
    alpha = np.array([np.sum(w * X[:, 0] ** a * X[:, 1] ** b) / (factorial(a) * factorial(b))
                      for a, b in full_set(p)])
    return M.T @ alpha


def m2l_matrix(kernel: str, p: int, tab: dict) -> np.ndarray:
    """T~[i, q] = tab[i + q] over i, q in J."""
    J = kept_set(p, pde_order(kernel))
    return np.array([[tab[(i[0] + q[0], i[1] + q[1])] for q in J] for i in J])


def m2l(kernel: str, p: int, d, beta, h: float = 1.0, tab: dict | None = None) -> np.ndarray:
    """Scaled compressed local theta~ from the scaled compressed multipole beta~ across d."""
    if tab is None:
        tab = table(kernel, p, d, h)
    return m2l_matrix(kernel, p, tab) @ np.asarray(beta)


def l2p(kernel: str, p: int, center, theta, tgt, h: float = 1.0) -> np.ndarray:
    """phi at tgt [n, 2] from the scaled compressed local theta~ about center."""
    L = decompression_matrix(kernel, p) @ np.asarray(theta)
    X = (np.asarray(tgt, dtype=np.float64) - np.asarray(center, dtype=np.float64)[None, :]) / h
    out = np.zeros(X.shape[0])
    for (a, b), v in zip(full_set(p), L):
        out += v * X[:, 0] ** a * X[:, 1] ** b / (factorial(a) * factorial(b))
    return out


def direct_sum(kernel: str, src, w, tgt) -> np.ndarray:
    """eq. (1): phi(x) = sum_y G(x - y) w_y, x = y skipped (float64)."""
    src = np.asarray(src, dtype=np.float64)
    out = np.zeros(len(tgt))
    for k, x in enumerate(np.asarray(tgt, dtype=np.float64)):
        g = green(kernel, x[None, :] - src)
        g[~np.isfinite(g)] = 0.0
        out[k] = np.sum(g * w)
    return out


def m2l_full(kernel: str, p: int, d, src, w, center, h: float = 1.0) -> np.ndarray:
    """Uncompressed form for the pins: the full local L~ [|M(p)|] (scaled) at the origin of the
    target box from the full multipole alpha~ of the sources (no PDE used)."""
    X = (np.asarray(center, dtype=np.float64)[None, :] - np.asarray(src, dtype=np.float64)) / h
    F = full_set(p)
    alpha = np.array([np.sum(w * X[:, 0] ** a * X[:, 1] ** b) / (factorial(a) * factorial(b)) for a, b in F])
    with mp.workdps(50):
        x, y, hh = mp.mpf(float(d[0])), mp.mpf(float(d[1])), mp.mpf(float(h))
        G = {}
        for i in F:
            for q in F:
                m = (i[0] + q[0], i[1] + q[1])
                if m not in G:
                    G[m] = float(deriv_mp(kernel, m[0], m[1], x, y) * hh ** (m[0] + m[1]))
    return np.array([sum(G[(i[0] + q[0], i[1] + q[1])] * alpha[k] for k, q in enumerate(F)) for i in F])


def l2p_full(p: int, center, L, tgt, h: float = 1.0) -> np.ndarray:
    X = (np.asarray(tgt, dtype=np.float64) - np.asarray(center, dtype=np.float64)[None, :]) / h
    out = np.zeros(X.shape[0])
    for (a, b), v in zip(full_set(p), L):
        out += v * X[:, 0] ** a * X[:, 1] ** b / (factorial(a) * factorial(b))
    return out


def m2p(kernel: str, p: int, center, beta, tgt, h: float = 1.0) -> np.ndarray:
    """Compressed multipole evaluation phi(x) = sum_{j in J} beta~_j G^(j)(x - c) h^|j|
    (Sec. 3.5, eq. multipole_eval_beta for d = 2), derivatives from deriv_mp."""
    J = kept_set(p, pde_order(kernel))
    out = np.zeros(len(tgt))
    with mp.workdps(50):
        for k, x in enumerate(np.asarray(tgt, dtype=np.float64)):
            dx, dy, hh = (mp.mpf(float(v)) for v in (x[0] - center[0], x[1] - center[1], h))
            out[k] = float(sum(beta[n] * deriv_mp(kernel, j[0], j[1], dx, dy) * hh ** (j[0] + j[1])
                               for n, j in enumerate(J)))
    return out


def m2m(kernel: str, p: int, d, beta, h_child: float = 1.0, h_parent: float = 1.0) -> np.ndarray:
    """Compressed M2M (Sec. 4.3, eq. define_psi, written out for d = 2): the child's scaled kept
    coefficients beta~ are unscaled, embedded with zeros on M(p) \\ J (E), translated from the
    child's centre c1 to the parent's c2, d = c2 - c1, by alpha'_r = sum_{q <= r} alpha_q
    d^(r-q) / (r-q)! (eq. mpole_translated_full_coeffs) (T), compressed (M^T) and scaled by the
    parent's size."""
    c = pde_order(kernel)
    J, F = kept_set(p, c), full_set(p)
    M = decompression_matrix(kernel, p)
    alpha = {q: 0.0 for q in F}
    for k, q in enumerate(J):
        alpha[q] = beta[k] * h_child ** (q[0] + q[1])
    out = np.zeros(len(F))
    for n, r in enumerate(F):
        s = 0.0
        for q in F:
            if q[0] <= r[0] and q[1] <= r[1]:
                a, b = r[0] - q[0], r[1] - q[1]
                s += alpha[q] * d[0] ** a * d[1] ** b / (factorial(a) * factorial(b))
        out[n] = s
    psi = M.T @ out
    return np.array([psi[k] / h_parent ** (q[0] + q[1]) for k, q in enumerate(J)])


def l2l(kernel: str, p: int, d, theta, h_parent: float = 1.0, h_child: float = 1.0) -> np.ndarray:
    """Compressed L2L (Sec. 4.2, eq. l2l-expr, for d = 2): the parent's scaled kept local is
    unscaled and decompressed (L = M theta), the Taylor polynomial is re-expanded about the
    child's centre, d = c_child - c_parent: L'_i = sum_k L_(i+k) d^k / k! over |i + k| <= p, and
    the kept entries are scaled by the child's size."""
    c = pde_order(kernel)
    J, F = kept_set(p, c), full_set(p)
    idx = {q: n for n, q in enumerate(F)}
    L = decompression_matrix(kernel, p) @ np.array([theta[k] / h_parent ** (q[0] + q[1]) for k, q in enumerate(J)])
    out = []
    for i in J:
        s = 0.0
        for kx in range(p + 1):
            for ky in range(p + 1 - kx):
                m = (i[0] + kx, i[1] + ky)
                if m[0] + m[1] <= p:
                    s += L[idx[m]] * d[0] ** kx * d[1] ** ky / (factorial(kx) * factorial(ky))
        out.append(s * h_child ** (i[0] + i[1]))
    return np.array(out)
