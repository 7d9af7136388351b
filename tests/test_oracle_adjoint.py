"""Pins for the oracle's reference gradients."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as A
from oracle import kernels as K

from conftest import rel_err


@pytest.mark.parametrize("kernel,param", [("laplace", 0.0), ("yukawa", 2.0), ("biharmonic", 0.0)])
def test_direct_gradients_match_central_differences(kernel, param):
    g = np.random.Generator(np.random.PCG64(8))
    src = g.random((9, 3))
    tgt = g.random((7, 3)) + np.array([1.2, 0, 0])
    w = g.standard_normal(9)
    c = g.standard_normal(7)
    L = lambda w_, s_, t_: c @ K.direct_sum(kernel, param, s_, w_, t_)
    dw, dy, dx = A.direct_gradients(kernel, param, src, w, tgt, c)
    eps = 1e-6
    fw = np.array([(L(w + eps * e, src, tgt) - L(w - eps * e, src, tgt)) / (2 * eps) for e in np.eye(9)])
    assert rel_err(dw, fw) < 1e-8
    fy = np.zeros_like(src)
    for i in range(9):
        for k in range(3):
            d = np.zeros_like(src)
            d[i, k] = eps
            fy[i, k] = (L(w, src + d, tgt) - L(w, src - d, tgt)) / (2 * eps)
    assert rel_err(dy, fy) < 1e-7
    fx = np.zeros_like(tgt)
    for i in range(7):
        for k in range(3):
            d = np.zeros_like(tgt)
            d[i, k] = eps
            fx[i, k] = (L(w, src, tgt + d) - L(w, src, tgt - d)) / (2 * eps)
    assert rel_err(dx, fx) < 1e-7


def test_far_field_converges_to_direct_far_field():
    pts = W.uniform_points(600, 2)
    tr = W.uniform_tree(pts, 2)
    w = W.normal_weights(600, 3)
    pairs = W.interaction_pairs(tr, [2])
    ref = A.far_field_direct("laplace", 0.0, tr, tr, pairs, w, tr.points, tr.points)
    errs = [rel_err(A.far_field("laplace", 0.0, p, tr, tr, pairs, w, tr.points, tr.points), ref) for p in (2, 4, 6)]
    assert errs[1] < 0.3 * errs[0] and errs[2] < 0.3 * errs[1] and errs[2] < 1e-3


def test_far_field_direct_gradients_pins():
    """The restricted direct-sum gradients: equal to the unrestricted ones when the pairs cover
    every (target box, source box) combination, and to central differences of
    far_field_direct when they do not."""
    src = W.uniform_points(80, 21)
    tgt = W.uniform_points(70, 22)
    ts = W.uniform_tree(src, 1)
    tt = W.uniform_tree(tgt, 1)
    w = W.normal_weights(80, 23)
    c = W.normal_weights(70, 24)
    boxes = ts.boxes_at(1)
    every = (np.repeat(boxes, len(boxes)), np.tile(boxes, len(boxes)))
    got = A.far_field_direct_gradients("laplace", 0.0, ts, tt, every, w, ts.points, tt.points, c)
    ref = A.direct_gradients("laplace", 0.0, ts.points, w, tt.points, c)
    for a, b in zip(got, ref):
        assert rel_err(a, b) < 1e-13
    # a restricted set: pairs of non-adjacent level-1 boxes only
    ijk = ts.ijk
    keep = [(t, s) for t in boxes for s in boxes if np.abs(ijk[t] - ijk[s]).max() >= 1 and (t + s) % 3]
    pairs = (np.array([k[0] for k in keep]), np.array([k[1] for k in keep]))
    dw, dy, dx = A.far_field_direct_gradients("yukawa", 2.0, ts, tt, pairs, w, ts.points, tt.points, c)
    L = lambda w_, s_, t_: c @ A.far_field_direct("yukawa", 2.0, ts, tt, pairs, w_, s_, t_)
    eps = 1e-6
    e = np.zeros(80)
    e[5] = 1.0
    assert abs(dw[5] - (L(w + eps * e, ts.points, tt.points) - L(w - eps * e, ts.points, tt.points)) / (2 * eps)) < 1e-7
    for i, k in ((7, 0), (31, 2)):
        d = np.zeros_like(ts.points)
        d[i, k] = eps
        fd = (L(w, ts.points + d, tt.points) - L(w, ts.points - d, tt.points)) / (2 * eps)
        assert abs(dy[i, k] - fd) <= 1e-6 * max(1.0, abs(fd))
        d = np.zeros_like(tt.points)
        d[i, k] = eps
        fd = (L(w, ts.points, tt.points + d) - L(w, ts.points, tt.points - d)) / (2 * eps)
        assert abs(dx[i, k] - fd) <= 1e-6 * max(1.0, abs(fd))
