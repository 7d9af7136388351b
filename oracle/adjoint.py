"""Reference gradients (test infrastructure).

  direct sum eq. (1), L = sum_x c(x) phi(x):
    d L / d w_s = sum_x c(x) G(x - y_s)
    d L / d y_s = -w_s sum_x c(x) grad G(x - y_s)
    d L / d x   = c(x) sum_y w_y grad G(x - y)
  the far field built from the compressed operators (every level's List-2 pairs, P2M from the
  points of each source box, L2P at each level's target boxes), evaluated plainly per pair, and
  its gradients by brute-force transposes (unit vectors) and central differences;
  the same three gradients of the direct sum restricted to the far field's box pairs (the limit
  of the far field's gradients as p grows).
"""
from __future__ import annotations

import numpy as np

from . import compressed as Z
from . import kernels as K


def direct_gradients(kernel, param, src, w, tgt, c):
    """(d L/d w, d L/d src, d L/d tgt) of L = sum_x c(x) sum_y G(x - y) w_y, x == y skipped."""
    src = np.asarray(src, np.float64)
    tgt = np.asarray(tgt, np.float64)
    dw = np.zeros(src.shape[0])
    dy = np.zeros_like(src)
    dx = np.zeros_like(tgt)
    for a in range(tgt.shape[0]):
        diff = tgt[a][None, :] - src
        r = np.sqrt(np.sum(diff * diff, axis=1))
        ok = r > 0
        G = np.zeros(src.shape[0])
        G[ok] = K.green(kernel, param, r[ok])
        gG = np.zeros_like(src)
        gG[ok] = K.grad_green(kernel, param, diff[ok])
        dw += c[a] * G
        dy -= c[a] * w[:, None] * gG
        dx[a] = c[a] * (w @ gG)
    return dw, dy, dx


def far_field(kernel, param, p, tree_s, tree_t, pairs, w, src, tgt):
    """phi(x) = sum over pairs (t, s) of L2P_t(M2L(P2M_s)) evaluated per pair, FP64."""
    t_all, s_all = pairs
    out = np.zeros(tgt.shape[0], dtype=np.complex128 if kernel == "helmholtz" else np.float64)
    betas = {}
    for s in np.unique(s_all):
        lo, hi = tree_s.pt_range[s]
        betas[s] = Z.p2m(kernel, param, p, tree_s.center[s], src[lo:hi], w[lo:hi])
    tables = {}
    for t in np.unique(t_all):
        theta = 0
        for s in s_all[t_all == t]:
            d = tree_s.center[t] - tree_s.center[s]
            key = (int(tree_s.level[t]),) + tuple(int(v) for v in (tree_s.ijk[t] - tree_s.ijk[s]))
            if key not in tables:
                tables[key] = Z.slab_table(kernel, param, p, d)
            theta = theta + Z.m2l(kernel, param, p, d, betas[s], tables[key])
        lo, hi = tree_t.pt_range[t]
        out[lo:hi] += Z.l2p(kernel, param, p, tree_s.center[t], theta, tgt[lo:hi])
    return out


def far_field_direct(kernel, param, tree_s, tree_t, pairs, w, src, tgt):
    """The same far field by the direct sum over the points of each (target, source) box pair."""
    t_all, s_all = pairs
    out = np.zeros(tgt.shape[0], dtype=np.complex128 if kernel == "helmholtz" else np.float64)
    for t, s in zip(t_all, s_all):
        a, b = tree_t.pt_range[t]
        c, d = tree_s.pt_range[s]
        if b > a and d > c:
            out[a:b] += K.direct_sum(kernel, param, src[c:d], w[c:d], tgt[a:b])
    return out


def far_field_direct_gradients(kernel, param, tree_s, tree_t, pairs, w, src, tgt, c):
    """(d L/d w, d L/d src, d L/d tgt) of L = sum_x c(x) phi_far(x), phi_far the direct sum of
    eq. (1) over the points of each (target box, source box) pair (far_field_direct): for every
    target box, direct_gradients over the points of all its source boxes at once, accumulated."""
    t_all, s_all = (np.asarray(a) for a in pairs)
    src = np.asarray(src, np.float64)
    tgt = np.asarray(tgt, np.float64)
    dw = np.zeros(src.shape[0])
    dy = np.zeros_like(src)
    dx = np.zeros_like(tgt)
    for t in np.unique(t_all):
        a, b = tree_t.pt_range[t]
        if b <= a:
            continue
        idx = np.concatenate([np.arange(*tree_s.pt_range[s]) for s in s_all[t_all == t]])
        if idx.size == 0:
            continue
        gw, gy, gx = direct_gradients(kernel, param, src[idx], w[idx], tgt[a:b], c[a:b])
        np.add.at(dw, idx, gw)
        np.add.at(dy, idx, gy)
        dx[a:b] += gx
    return dw, dy, dx
