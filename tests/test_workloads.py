"""The shared geometry: trees and List-2 interaction pairs."""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def uniform4():
    pts = W.uniform_points(1 << 16, 1)
    return W.uniform_tree(pts, 4)


def test_uniform_pair_counts(uniform4):
    tr = uniform4
    counts = {lev: len(W.interaction_pairs(tr, [lev])[0]) for lev in (2, 3, 4)}
    assert counts == {2: 3096, 3: 53352, 4: 584136}
    t, s = W.interaction_pairs(tr, [4])
    off = tr.ijk[t] - tr.ijk[s]
    u, c = np.unique(off, axis=0, return_counts=True)
    assert len(u) == 316 and c.min() == 343 and c.max() == 3584
    per_t = np.bincount(t - tr.level_start[4], minlength=4096)
    assert per_t.max() == 189


def test_list2_matches_definition_by_brute_force(uniform4):
    tr = uniform4
    ids = tr.boxes_at(3)
    ijk = tr.ijk[ids].astype(int)
    expect = set()
    for a in range(len(ids)):
        d = ijk - ijk[a]
        par = (ijk // 2) - (ijk[a] // 2)
        ok = (np.max(np.abs(d), axis=1) >= 2) & (np.max(np.abs(par), axis=1) <= 1)
        for b in np.nonzero(ok)[0]:
            expect.add((int(ids[a]), int(ids[b])))
    t, s = W.interaction_pairs(tr, [3])
    assert set(zip(t.tolist(), s.tolist())) == expect


def test_offsets_per_parity():
    allo = {tuple(o) for o in W.all_list2_offsets()}
    assert len(allo) == 316
    union = set()
    for par in np.ndindex(2, 2, 2):
        o = {tuple(v) for v in W.list2_offsets(par)}
        assert len(o) == 189 and o <= allo
        union |= o
    assert union == allo


def test_points_sorted_into_boxes(uniform4):
    tr = uniform4
    for b in tr.boxes_at(4)[::97]:
        lo, hi = tr.pt_range[b]
        h = tr.box_size(4)
        x = tr.points[lo:hi]
        assert np.all(np.abs(x - tr.center[b]) <= h / 2 + 1e-15)
    assert tr.counts()[tr.boxes_at(4)].sum() == tr.points.shape[0]


def test_adaptive_tree_leaf_bound():
    pts = W.plummer_points(50000, 3)
    tr = W.adaptive_tree(pts, 64)
    c = tr.counts()
    assert c[tr.is_leaf].max() <= 64
    assert np.all(c[~tr.is_leaf] > 64)
    for lev in range(1, tr.n_levels):
        ids = tr.boxes_at(lev)
        assert c[ids].sum() <= pts.shape[0]
    t, s = W.interaction_pairs(tr)
    assert np.all(tr.level[t] == tr.level[s])
    d = np.max(np.abs(tr.ijk[t] - tr.ijk[s]), axis=1)
    assert d.min() >= 2 and d.max() <= 3


def test_generators_are_seeded():
    a = W.plummer_points(1000, 9)
    b = W.plummer_points(1000, 9)
    assert np.array_equal(a, b)
    g = W.gaussian_mixture_points(2000, 4)
    assert np.all((g >= 0) & (g < 1))
