"""Shared test helpers: seeded inputs on the device and oracle references in the library's
coefficient order.  Oracle values are computed here with ``oracle`` only."""
from __future__ import annotations

from functools import lru_cache

import numpy as np

import workloads as W
from oracle import compressed as Z
from oracle import kernels as K


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb else 1.0))


def perm_to_lib(kernel, param, p, lib_index_table):
    """Positions in the oracle's kept order of each library coefficient."""
    J = Z.kept(kernel, param, p)
    pos = {m: k for k, m in enumerate(J)}
    return np.array([pos[tuple(int(v) for v in r)] for r in lib_index_table])


@lru_cache(maxsize=None)
def oracle_scaled_table(kernel, param, p, o, h, mp=False):
    """{m: G^(m)(h o) h^|m|} for the compressed slab.  mp=False: the oracle's float64
    Taylor-coefficient recurrences; mp=True: the radial product formula of the paper's Sec. 4.4
    (eq. tausch-dist-derivatives) evaluated in mpmath at 50 digits and rounded once, which shares
    no step with the recurrence the GPU tables use."""
    d = np.array(o, dtype=np.float64) * h
    tab = Z.slab_table(kernel, param, p, d, mp=mp)
    return {m: v * h ** sum(m) for m, v in tab.items()}


def per_order_rel(got, ref, index_table):
    """{n: normwise relative error over the coefficients of total order n} (columns are the
    coefficients in the library's order given by index_table [Nc][3])."""
    order = np.asarray(index_table).sum(axis=1)
    out = {}
    for n in sorted(set(order.tolist())):
        sel = order == n
        out[n] = rel(np.asarray(got)[:, sel], np.asarray(ref)[:, sel])
    return out


def decaying_multipoles(index_table, n_box, seed):
    """Scaled multipoles with the decay of physical ones: N(0,1) * 0.6^|q| / q!."""
    from math import factorial
    g = np.random.Generator(np.random.PCG64(seed))
    f = np.array([0.6 ** sum(q) / (factorial(q[0]) * factorial(q[1]) * factorial(q[2])) for q in index_table])
    return g.standard_normal((n_box, len(f))) * f


def oracle_m2l_scaled(kernel, param, p, tree_ijk, tree_level, level_h, t, s, beta_s, transpose_of=None,
                      mp=False):
    """theta~ for every box from scaled multipoles beta_s [n_box, Nc] (oracle kept order),
    grouped by (level, offset) and applied with the oracle's dense T~ matrices (tables from the
    float64 recurrences, or from mpmath with mp=True).

    transpose_of=(t0, s0): apply T~(ijk_t0 - ijk_s0)^T for each pair instead (t, s given reversed),
    i.e. the transpose of the M2L over the pairs (t0, s0)."""
    nb, nc = beta_s.shape
    out = np.zeros((nb, nc), dtype=np.result_type(beta_s.dtype, np.complex128 if kernel == "helmholtz"
                                                  else np.float64))
    if transpose_of is not None:
        t0, s0 = transpose_of
        off = tree_ijk[t0] - tree_ijk[s0]
    else:
        off = tree_ijk[t] - tree_ijk[s]
    lev = tree_level[t]
    keys = np.concatenate([lev[:, None], off], axis=1)
    uk, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.ravel()
    for g, key in enumerate(uk):
        sel = np.nonzero(inv == g)[0]
        h = level_h[int(key[0])]
        tab = oracle_scaled_table(kernel, param, p, tuple(int(v) for v in key[1:]), h, mp)
        T = Z.m2l_matrix(kernel, param, p, None, tab)
        if transpose_of is not None:
            T = T.T
        contrib = beta_s[s[sel]] @ T.T
        np.add.at(out, t[sel], contrib)
    return out


def tree_inputs(n_pts, depth, seed, kind="uniform", max_leaf=64, complex_w=False):
    if kind == "uniform":
        pts = W.uniform_points(n_pts, seed)
        tr = W.uniform_tree(pts, depth)
    elif kind == "plummer":
        tr = W.adaptive_tree(W.plummer_points(n_pts, seed, 0.1), max_leaf)
    else:
        tr = W.adaptive_tree(W.gaussian_mixture_points(n_pts, seed), max_leaf)
    w = W.normal_weights(tr.points.shape[0], seed + 100, complex_=complex_w)
    return tr, w
