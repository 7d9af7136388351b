"""Kernels G, their PDE operators, the direct sum eq. (1), and derivative tables.

Kernels (3-D, r = |x|):
  laplace     G = 1 / (4 pi r)              Delta G = 0
  helmholtz   G = exp(i k r) / (4 pi r)     (Delta + k^2) G = 0
  yukawa      G = exp(-lam r) / (4 pi r)    (Delta - lam^2) G = 0
  biharmonic  G = r                         Delta^2 G = 0

Derivative tables G^(m)(x) follow the radial approach the paper cites for
radially symmetric kernels (Sec. 4.4, eq. tausch-dist-derivatives): with
s = r^2/2 and u_n = ((1/r) d/dr)^n G, a derivative is a finite sum of products of
one-dimensional Hermite-type factors and the u_n.  The u_n come from closed forms
(reverse Bessel polynomials for the exponential kernels, powers for Laplace and
biharmonic), not from the PDE.  The paper's own three-term Cartesian recurrence
for 3-D Laplace (eq. deriv_laplace_3d) is provided as a second, independent
method.  ``deriv_table_mp`` evaluates in mpmath at 50 digits and is the truth the
float64 tables are measured against.

The radial product formula loses up to nine digits in float64 at order 24 for
offsets near a coordinate axis (its terms alternate in sign).  The fast float64
tables therefore use Taylor-coefficient recurrences of the same kind as the
paper's Laplace recurrence, derived here from first-order identities of the
kernels (see ``deriv_table_rec``); tests pin them to the mpmath tables.
"""
from __future__ import annotations

from math import factorial, pi

import mpmath
import numpy as np

from .multiindex import graded_order

KERNELS = ("laplace", "helmholtz", "yukawa", "biharmonic")


def pde_coefficients(kernel: str, param: float = 0.0) -> dict:
    """Coefficients a_m of the operator L = sum a_m d^m (eq. define_pde_op)."""
    lap = {(2, 0, 0): 1.0, (0, 2, 0): 1.0, (0, 0, 2): 1.0}
    if kernel == "laplace":
        return dict(lap)
    if kernel == "helmholtz":
        return {**lap, (0, 0, 0): float(param) ** 2}
    if kernel == "yukawa":
        return {**lap, (0, 0, 0): -float(param) ** 2}
    if kernel == "biharmonic":
        return {(4, 0, 0): 1.0, (0, 4, 0): 1.0, (0, 0, 4): 1.0,
                (2, 2, 0): 2.0, (2, 0, 2): 2.0, (0, 2, 2): 2.0}
    raise ValueError(kernel)


def pde_order(kernel: str) -> int:
    return 4 if kernel == "biharmonic" else 2


def is_complex(kernel: str) -> bool:
    return kernel == "helmholtz"


# ----------------------------------------------------------------------------- G itself

def green(kernel: str, param: float, r: np.ndarray) -> np.ndarray:
    r = np.asarray(r, dtype=np.float64)
    if kernel == "laplace":
        return 1.0 / (4 * pi * r)
    if kernel == "helmholtz":
        return np.exp(1j * param * r) / (4 * pi * r)
    if kernel == "yukawa":
        return np.exp(-param * r) / (4 * pi * r)
    if kernel == "biharmonic":
        return r.copy()
    raise ValueError(kernel)


def direct_sum(kernel: str, param: float, src: np.ndarray, w: np.ndarray,
               tgt: np.ndarray, block: int = 256) -> np.ndarray:
    """phi(x) = sum_y G(x - y) w(y) for every target x (eq. particle-convolution).

    Pairs with x == y exactly are skipped (the sum is over distinct particles)."""
    src = np.asarray(src, np.float64)
    tgt = np.asarray(tgt, np.float64)
    out = np.zeros(tgt.shape[0], dtype=np.complex128 if (is_complex(kernel) or np.iscomplexobj(w))
                   else np.float64)
    for a in range(0, tgt.shape[0], block):
        diff = tgt[a:a + block, None, :] - src[None, :, :]
        r = np.sqrt(np.sum(diff * diff, axis=2))
        same = r == 0.0
        g = green(kernel, param, np.where(same, 1.0, r))
        g = np.where(same, 0.0, g)
        out[a:a + block] = g @ w
    return out


def grad_green(kernel: str, param: float, x: np.ndarray) -> np.ndarray:
    """nabla G at points x [..., 3] (G radial: grad = G'(r) x / r)."""
    x = np.asarray(x, np.float64)
    r = np.sqrt(np.sum(x * x, axis=-1))
    if kernel == "laplace":
        dr = -1.0 / (4 * pi * r * r)
    elif kernel == "helmholtz":
        dr = np.exp(1j * param * r) * (1j * param * r - 1.0) / (4 * pi * r * r)
    elif kernel == "yukawa":
        dr = -np.exp(-param * r) * (param * r + 1.0) / (4 * pi * r * r)
    elif kernel == "biharmonic":
        dr = np.ones_like(r)
    else:
        raise ValueError(kernel)
    return (dr / r)[..., None] * x


# ----------------------------------------------------------------------------- radial derivatives

def _radial_u_mp(kernel: str, param, r, nmax: int) -> list:
    """u_n = ((1/r) d/dr)^n G(r), n = 0..nmax, in mpmath.

    Exponential kernels: with G = exp(-a r)/(4 pi r) (a = lam, or a = -i k),
      u_n = (-1)^n exp(-a r)/(4 pi) * sum_{k=0..n} (n+k)! / (k! (n-k)! 2^k) a^(n-k) r^-(n+k+1),
    which follows by induction on n from (1/r) d/dr applied term by term.
    Laplace is the case a = 0.  Biharmonic G = r: u_0 = r, u_n = (-1)^(n-1) (2n-3)!! r^(1-2n).
    """
    r = mpmath.mpf(r)
    if kernel == "biharmonic":
        u = [r]
        for n in range(1, nmax + 1):
            dfac = mpmath.mpf(1)
            for k in range(2 * n - 3, 0, -2):
                dfac *= k
            u.append((-1) ** (n - 1) * dfac * r ** (1 - 2 * n))
        return u
    if kernel == "laplace":
        a = mpmath.mpf(0)
    elif kernel == "yukawa":
        a = mpmath.mpf(param)
    elif kernel == "helmholtz":
        a = -1j * mpmath.mpf(param)
    else:
        raise ValueError(kernel)
    e = mpmath.exp(-a * r) / (4 * mpmath.pi)
    u = []
    for n in range(nmax + 1):
        s = 0
        for k in range(n + 1):
            coef = mpmath.mpf(factorial(n + k)) / (factorial(k) * factorial(n - k) * 2 ** k)
            s += coef * (a ** (n - k) if n - k > 0 else 1) * r ** (-(n + k + 1))
        u.append((-1) ** n * e * s)
    return u


def _hermite_factor(n: int, i: int, t):
    """h_{n,i}(t) = n! / (i! (n-2i)! 2^i) t^(n-2i): the i-th term of d^n/dt^n f(t^2/2)
    written as sum_i h_{n,i}(t) f^(n-i)(t^2/2)."""
    return factorial(n) / (factorial(i) * factorial(n - 2 * i) * 2 ** i) * t ** (n - 2 * i)


def deriv_mp(kernel: str, param, x, m, u=None):
    """G^(m)(x) in mpmath for one multi-index m = (a, b, c) (radial product formula)."""
    x = [mpmath.mpf(v) for v in x]
    a, b, c = m
    if u is None:
        r = mpmath.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)
        u = _radial_u_mp(kernel, param, r, a + b + c)
    tot = 0
    for i in range(a // 2 + 1):
        hx = mpmath.mpf(factorial(a)) / (factorial(i) * factorial(a - 2 * i) * 2 ** i) * x[0] ** (a - 2 * i)
        for j in range(b // 2 + 1):
            hy = mpmath.mpf(factorial(b)) / (factorial(j) * factorial(b - 2 * j) * 2 ** j) * x[1] ** (b - 2 * j)
            for k in range(c // 2 + 1):
                hz = mpmath.mpf(factorial(c)) / (factorial(k) * factorial(c - 2 * k) * 2 ** k) * x[2] ** (c - 2 * k)
                tot += hx * hy * hz * u[a + b + c - i - j - k]
    return tot


def deriv_table_mp(kernel: str, param, x, indices, dps: int = 50) -> np.ndarray:
    """G^(m)(x) for every m in ``indices``, computed at ``dps`` digits, rounded to
    float64 / complex128."""
    with mpmath.workdps(dps):
        xs = [mpmath.mpf(float(v)) for v in x]
        r = mpmath.sqrt(xs[0] ** 2 + xs[1] ** 2 + xs[2] ** 2)
        nmax = max(sum(m) for m in indices)
        u = _radial_u_mp(kernel, param, r, nmax)
        vals = [deriv_mp(kernel, param, xs, m, u) for m in indices]
    if is_complex(kernel):
        return np.array([complex(v) for v in vals], dtype=np.complex128)
    return np.array([float(v) for v in vals], dtype=np.float64)


def _radial_u_fp(kernel: str, param: float, r: float, nmax: int):
    """float64 / complex128 version of _radial_u_mp (same closed forms)."""
    if kernel == "biharmonic":
        u = [r]
        dfac = 1.0
        for n in range(1, nmax + 1):
            if n >= 2:
                dfac *= (2 * n - 3)
            u.append((-1) ** (n - 1) * dfac * r ** (1 - 2 * n))
        return np.array(u, dtype=np.float64)
    if kernel == "laplace":
        a = 0.0
    elif kernel == "yukawa":
        a = float(param)
    else:
        a = -1j * float(param)
    e = np.exp(-a * r) / (4 * pi)
    u = []
    for n in range(nmax + 1):
        s = 0.0
        for k in range(n + 1):
            coef = factorial(n + k) / (factorial(k) * factorial(n - k) * 2 ** k)
            s = s + coef * (a ** (n - k) if n - k > 0 else 1.0) * r ** (-(n + k + 1))
        u.append((-1) ** n * e * s)
    return np.array(u, dtype=np.complex128 if kernel == "helmholtz" else np.float64)


def deriv_table_fp(kernel: str, param: float, x, indices) -> np.ndarray:
    """G^(m)(x) for every m in ``indices`` by the radial product formula in float64
    (complex128 for Helmholtz).  Pinned against deriv_table_mp by the tests."""
    x = np.asarray(x, dtype=np.float64)
    r = float(np.sqrt(np.sum(x * x)))
    nmax = max(sum(m) for m in indices)
    u = _radial_u_fp(kernel, param, r, nmax)
    out = np.zeros(len(indices), dtype=u.dtype)
    for idx, (a, b, c) in enumerate(indices):
        tot = 0.0
        for i in range(a // 2 + 1):
            hx = _hermite_factor(a, i, x[0])
            for j in range(b // 2 + 1):
                hy = _hermite_factor(b, j, x[1])
                for k in range(c // 2 + 1):
                    hz = _hermite_factor(c, k, x[2])
                    tot = tot + hx * hy * hz * u[a + b + c - i - j - k]
        out[idx] = tot
    return out


def laplace_recurrence_table(x, order: int, zmax: int | None = None) -> dict:
    """All derivatives of 1/r up to total order ``order`` (and m_z <= zmax) by the
    paper's 3-D Laplace recurrence (eq. deriv_laplace_3d), float64, then times
    1/(4 pi).  For n = 0 (no x derivative) the same recurrence is used with the
    roles of the axes rotated (y leading, then z), as the formula is symmetric
    under relabelling of the axes.  Returns {m: value}."""
    xx, yy, zz = (float(v) for v in x)
    r2 = xx * xx + yy * yy + zz * zz
    if zmax is None:
        zmax = order
    D = {}

    def get(n, m, l):
        if n < 0 or m < 0 or l < 0:
            return 0.0
        return D[(n, m, l)]

    for tot in range(order + 1):
        for l in range(min(tot, zmax) + 1):
            for m in range(tot - l + 1):
                n = tot - m - l
                if tot == 0:
                    D[(0, 0, 0)] = 1.0 / np.sqrt(r2)
                    continue
                if n >= 1:
                    v = (-(2 * n - 1) * xx * get(n - 1, m, l) - (n - 1) ** 2 * get(n - 2, m, l)
                         - 2 * m * yy * get(n, m - 1, l) - m * (m - 1) * get(n, m - 2, l)
                         - 2 * l * zz * get(n, m, l - 1) - l * (l - 1) * get(n, m, l - 2))
                elif m >= 1:
                    v = (-(2 * m - 1) * yy * get(0, m - 1, l) - (m - 1) ** 2 * get(0, m - 2, l)
                         - 2 * l * zz * get(0, m, l - 1) - l * (l - 1) * get(0, m, l - 2))
                else:
                    v = -(2 * l - 1) * zz * get(0, 0, l - 1) - (l - 1) ** 2 * get(0, 0, l - 2)
                D[(n, m, l)] = v / r2
    return {k: v / (4 * pi) for k, v in D.items()}


def deriv_table_rec(kernel: str, param: float, x, indices) -> np.ndarray:
    """G^(m)(x) for every m in ``indices`` by Taylor-coefficient recurrences, float64.

    Write a_k = G^(k)(x0) / k! for the Taylor coefficients of G about x0, so that
    sum_j h_j d_j G has coefficient |k| a_k at h^k and |x0 + h|^2 = r0^2 + 2 x0.h + |h|^2.
    Multiplying a first-order identity  r^2 grad G = (polynomial in x) * (...)  by h and
    matching coefficients of h^k gives a recurrence that reaches order n from orders
    n-1 and n-2 only, in the style of the paper's Laplace recurrence (eq. deriv_laplace_3d):

      G = r^nu (nu = -1 Laplace, nu = 1 biharmonic):  r^2 grad G = nu x G  =>
        n r0^2 a_k + (2n - 2 - nu) S1(a) + (n - 2 - nu) S2(a) = 0
      G = psi / r, psi = exp(-s r) (s = lam Yukawa, s = -i k Helmholtz):
        r^2 grad G = -x G - s x psi,  grad psi = -s x G  =>
        n r0^2 a_k + (2n - 1) S1(a) + (n - 1) S2(a) + s (S1(b) + S2(b)) = 0
        n b_k + s (S1(a) + S2(a)) = 0
    with n = |k|, S1(a) = sum_j x0_j a_{k - e_j}, S2(a) = sum_j a_{k - 2 e_j} (terms with a
    negative index are zero) and b the Taylor coefficients of psi.  Only lower indices of k
    are read, so any downward-closed index set (such as the slab m_z <= 2(c-1)) is closed
    under the recurrence.  Constant factors 1/(4 pi) are applied at the end.
    """
    x0 = np.asarray(x, dtype=np.float64)
    r02 = float(x0 @ x0)
    r0 = float(np.sqrt(r02))
    need = set()
    for m in indices:
        for a in range(m[0] + 1):
            for b in range(m[1] + 1):
                for c in range(m[2] + 1):
                    need.add((a, b, c))
    order = sorted(need, key=lambda m: (sum(m), m[2], m[1], m[0]))
    cplx = kernel == "helmholtz"
    s = (-1j * float(param)) if kernel == "helmholtz" else float(param)
    A, B = {}, {}

    def get(d, m):
        return d.get(m, 0.0) if min(m) >= 0 else 0.0

    def sums(d, m):
        s1 = sum(x0[j] * get(d, tuple(m[i] - (i == j) for i in range(3))) for j in range(3))
        s2 = sum(get(d, tuple(m[i] - 2 * (i == j) for i in range(3))) for j in range(3))
        return s1, s2

    for m in order:
        n = sum(m)
        if n == 0:
            if kernel == "laplace":
                A[m] = 1.0 / r0
            elif kernel == "biharmonic":
                A[m] = r0
            else:
                B[m] = np.exp(-s * r0)
                A[m] = B[m] / r0
            continue
        s1, s2 = sums(A, m)
        if kernel in ("laplace", "biharmonic"):
            nu = -1 if kernel == "laplace" else 1
            A[m] = -((2 * n - 2 - nu) * s1 + (n - 2 - nu) * s2) / (n * r02)
        else:
            t1, t2 = sums(B, m)
            A[m] = -((2 * n - 1) * s1 + (n - 1) * s2 + s * (t1 + t2)) / (n * r02)
            B[m] = -s * (s1 + s2) / n
    norm = 1.0 if kernel == "biharmonic" else 1.0 / (4 * pi)
    out = np.array([A[tuple(m)] * factorial(m[0]) * factorial(m[1]) * factorial(m[2]) * norm
                    for m in indices])
    return out.astype(np.complex128 if cplx else np.float64)


def all_indices(order: int) -> list:
    return list(graded_order(order))


def slab_indices(order: int, zmax: int) -> list:
    """Multi-indices of total order <= order with m_z <= zmax: the derivatives the
    compressed M2L needs (|i + q| <= 2p and (i + q)_z <= 2(c - 1) for i, q in J)."""
    return [m for m in graded_order(order) if m[2] <= zmax]
