"""Compressed expansions and translations (Secs. 3.3, 3.4, 4.1, 4.1.1).

  P2M   beta = M^T alpha                                  (eq. define_beta_multipole)
  M2L   theta_i = sum_{q in j} G^(i+q)(c2 - c1) beta_q,  i in j   (eq. m2l_toeplitz,
        kept in derivative form: the 1/i! of the local coefficient is applied at
        evaluation, as the stored local of eq. stored_local_coeffs carries none)
  L2P   phi(x) = sum_i [M theta]_i / i! (x - c)^i         (eq. compressed-local-form)
  M2M   psi = M^T T E beta                                (eq. define_psi: embed with
        zeros at the indices not kept, translate uncompressed, compress again)
  L2L   theta' = [T_L M theta]_j                          (Sec. 4.2: decompress, translate
        with eq. l2l-expr, keep the entries of j)
  P2L   theta = sum_y w(y) [D^p G(c - y)]_j              (Sec. 3.2, eq. stored_local_coeffs)
  M2P   phi(x) = [D^p G(x - c)]_j^T beta                  (Sec. 3.5, eq. multipole_eval_beta)

Scaled form (Sec. 4.1.1) with parameter t:
  beta~_q = beta_q t^|q|,  table~_m = G^(m) / t^|m|,  theta~_i = theta_i / t^|i|,
  theta~ = sum_q table~_{i+q} beta~_q.

FFT form (eq. convolution_m2l): the sum over q is a 3-D correlation of the
derivative grid g[m] = G^(m), m in [0, 2M], M = (max_j nu_x, max_j nu_y, max_j nu_z),
with the kept coefficients; embedding in a circulant of size 2M + 1 per axis turns it
into one FFT product.

Coefficient vectors are in the order of the kept positions j of Sec. 3.1 (which,
for the graded order used here, is the graded order restricted to m_z < c).
"""
from __future__ import annotations

import numpy as np

from .compression import decompression_matrix, kept_indices, position_map
from .kernels import deriv_table_mp, deriv_table_rec, pde_order, slab_indices
from .multiindex import graded_order, madd, mfact, morder, mpow
from .taylor import l2l_full, l2p_full, m2m_full, p2m_full


def kept(kernel: str, param: float, p: int) -> list:
    return kept_indices(kernel, param, p)


def p2m(kernel: str, param: float, p: int, center, src, w) -> np.ndarray:
    M, _, _ = decompression_matrix(kernel, param, p)
    return M.T @ p2m_full(p, center, src, w)


def slab_table(kernel: str, param: float, p: int, d, mp: bool = False) -> dict:
    """{m: G^(m)(d)} for |m| <= 2p, m_z <= 2(c-1): all the compressed M2L reads."""
    idx = slab_indices(2 * p, 2 * (pde_order(kernel) - 1))
    vals = (deriv_table_mp if mp else deriv_table_rec)(kernel, param, d, idx)
    return dict(zip(idx, vals))


def m2l_matrix(kernel: str, param: float, p: int, d, table: dict | None = None) -> np.ndarray:
    """T[i, q] = G^(i+q)(d) for i, q in j."""
    if table is None:
        table = slab_table(kernel, param, p, d)
    J = kept(kernel, param, p)
    return np.array([[table[madd(i, q)] for q in J] for i in J])


def m2l(kernel: str, param: float, p: int, d, beta, table: dict | None = None) -> np.ndarray:
    return m2l_matrix(kernel, param, p, d, table) @ np.asarray(beta)


def local_full(kernel: str, param: float, p: int, theta) -> np.ndarray:
    """M theta: the full derivative-form local vector in graded order of M(p)."""
    M, _, _ = decompression_matrix(kernel, param, p)
    return M @ np.asarray(theta)


def l2p(kernel: str, param: float, p: int, center, theta, tgt) -> np.ndarray:
    return l2p_full(p, center, local_full(kernel, param, p, theta), tgt)


def embed(kernel: str, param: float, p: int, beta) -> np.ndarray:
    """E beta: the kept coefficients placed in the graded order of M(p), zero elsewhere
    (the embedding operator E of Sec. 4.3)."""
    beta = np.asarray(beta)
    out = np.zeros(len(graded_order(p)), dtype=beta.dtype)
    out[position_map(p, kept(kernel, param, p))] = beta
    return out


def m2m(kernel: str, param: float, p: int, h, beta) -> np.ndarray:
    """Compressed multipole translation by h = c_new - c_old: psi = M^T T E beta
    (eq. define_psi)."""
    M, _, _ = decompression_matrix(kernel, param, p)
    return M.T @ m2m_full(p, h, embed(kernel, param, p, beta))


def l2l(kernel: str, param: float, p: int, h, theta) -> np.ndarray:
    """Compressed local translation by h = c_new - c_old: decompress, translate
    (eq. l2l-expr), keep the entries of j (Sec. 4.2)."""
    full = l2l_full(p, h, local_full(kernel, param, p, theta))
    return full[position_map(p, kept(kernel, param, p))]


# ----------------------------------------------------------------------------- from and to points

def p2l(kernel: str, param: float, p: int, center, src, w, mp: bool = False) -> np.ndarray:
    """Compressed local expansion straight from the sources (Sec. 3.2, eq. stored_local_coeffs,
    with the density restored): theta = sum_y w(y) [D^p G(c - y)]_j, derivative form like the
    M2L's output (the 1/i! comes after decompression, eq. compressed-local-form)."""
    J = kept(kernel, param, p)
    deriv = deriv_table_mp if mp else deriv_table_rec
    src = np.asarray(src, np.float64)
    w = np.asarray(w)
    out = np.zeros(len(J), dtype=np.complex128 if np.iscomplexobj(w) or kernel == "helmholtz" else np.float64)
    for y, wy in zip(src, w):
        out = out + wy * deriv(kernel, param, np.asarray(center, np.float64) - y, J)
    return out


def m2p(kernel: str, param: float, p: int, center, beta, tgt, mp: bool = False) -> np.ndarray:
    """Compressed multipole evaluation (Sec. 3.5, eq. multipole_eval_beta):
    phi(x) = [D^p G(x - c)]_j^T beta for every target x."""
    J = kept(kernel, param, p)
    deriv = deriv_table_mp if mp else deriv_table_rec
    beta = np.asarray(beta)
    return np.array([deriv(kernel, param, np.asarray(x, np.float64) - np.asarray(center, np.float64), J) @ beta
                     for x in np.asarray(tgt, np.float64)])


# ----------------------------------------------------------------------------- scaled form

def scale_multipole(kernel, param, p, beta, t):
    J = kept(kernel, param, p)
    return np.asarray(beta) * np.array([float(t) ** morder(q) for q in J])


def unscale_multipole(kernel, param, p, beta_s, t):
    J = kept(kernel, param, p)
    return np.asarray(beta_s) / np.array([float(t) ** morder(q) for q in J])


def scale_local(kernel, param, p, theta, t):
    J = kept(kernel, param, p)
    return np.asarray(theta) / np.array([float(t) ** morder(i) for i in J])


def unscale_local(kernel, param, p, theta_s, t):
    J = kept(kernel, param, p)
    return np.asarray(theta_s) * np.array([float(t) ** morder(i) for i in J])


def m2l_scaled(kernel, param, p, d, beta_s, t, table: dict | None = None):
    """theta~ = sum_q (G^(i+q)/t^|i+q|) beta~_q  (Sec. 4.1.1)."""
    if table is None:
        table = slab_table(kernel, param, p, d)
    tt = {m: v / float(t) ** morder(m) for m, v in table.items()}
    return m2l(kernel, param, p, d, beta_s, tt)


def m2m_scaled(kernel, param, p, h, beta_s, t_old, t_new):
    """m2m on scaled coefficients: beta~ at parameter t_old in, psi~ at t_new out."""
    beta = unscale_multipole(kernel, param, p, beta_s, t_old)
    return scale_multipole(kernel, param, p, m2m(kernel, param, p, h, beta), t_new)


def l2l_scaled(kernel, param, p, h, theta_s, t_old, t_new):
    """l2l on scaled coefficients: theta~ at parameter t_old in, at t_new out."""
    theta = unscale_local(kernel, param, p, theta_s, t_old)
    return scale_local(kernel, param, p, l2l(kernel, param, p, h, theta), t_new)


# ----------------------------------------------------------------------------- FFT form

def fft_grid(kernel: str, param: float, p: int) -> tuple:
    """Sizes (2 M_x + 1, 2 M_y + 1, 2 M_z + 1) of the circulant embedding of the convolution
    (eq. convolution_m2l and the complexity argument after it), M the largest index of J
    along each axis."""
    J = kept(kernel, param, p)
    return tuple(2 * max(m[k] for m in J) + 1 for k in range(3))


def m2l_fft(kernel: str, param: float, p: int, d, beta, table: dict | None = None) -> np.ndarray:
    """eq. convolution_m2l evaluated by a circulant embedding and numpy FFTs."""
    if table is None:
        table = slab_table(kernel, param, p, d)
    J = kept(kernel, param, p)
    L = fft_grid(kernel, param, p)
    Mx, My, Mz = [(n - 1) // 2 for n in L]
    cplx = np.iscomplexobj(beta) or any(np.iscomplexobj(v) for v in table.values())
    g = np.zeros(L, dtype=np.complex128)
    for m, v in table.items():
        if m[0] <= 2 * Mx and m[1] <= 2 * My and m[2] <= 2 * Mz:
            g[m] = v
    b = np.zeros(L, dtype=np.complex128)
    for q, v in zip(J, beta):
        b[(-q[0]) % L[0], (-q[1]) % L[1], (-q[2]) % L[2]] = v
    conv = np.fft.ifftn(np.fft.fftn(g) * np.fft.fftn(b))
    out = np.array([conv[i] for i in J])
    return out if cplx else out.real


# ----------------------------------------------------------------------------- batched helpers

def p2m_boxes(kernel, param, p, centers, pt_range, src, w, boxes, t=None):
    """beta (scaled by t^|q| per box when t is given) for the listed boxes."""
    out = []
    for k, b in enumerate(boxes):
        lo, hi = pt_range[b]
        beta = p2m(kernel, param, p, centers[b], src[lo:hi], w[lo:hi])
        if t is not None:
            beta = scale_multipole(kernel, param, p, beta, t[k])
        out.append(beta)
    return np.array(out)


def l2p_boxes(kernel, param, p, centers, pt_range, tgt, theta, boxes, n_tgt, t=None):
    """phi at every target of the listed boxes (theta scaled by 1/t^|i| when t given)."""
    dtype = np.complex128 if np.iscomplexobj(theta) else np.float64
    phi = np.zeros(n_tgt, dtype=dtype)
    for k, b in enumerate(boxes):
        lo, hi = pt_range[b]
        th = theta[k]
        if t is not None:
            th = unscale_local(kernel, param, p, th, t[k])
        phi[lo:hi] += l2p(kernel, param, p, centers[b], th, tgt[lo:hi])
    return phi
