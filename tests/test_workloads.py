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


@pytest.mark.parametrize("points,max_leaf,max_src", [("plummer", 16, None), ("mixture", 24, None), ("uniform", 40, None),
                                                     ("plummer", 16, 100), ("mixture", 24, 60)])
def test_near_lists_and_list2_partition_every_leaf_pair(points, max_leaf, max_src):
    """Every (target leaf, source leaf) pair of an adaptive tree is counted exactly once: by
    the near list of the target leaf (one list box containing the source leaf), or by exactly
    one List-2 pair of their ancestors on a level >= 2.  Checked by brute force over all leaf
    pairs against the definition: near iff the ancestors on the level min(l_t, l_s) are
    adjacent or equal."""
    pts = {"plummer": lambda: W.plummer_points(3000, 11),
           "mixture": lambda: W.gaussian_mixture_points(3000, 12),
           "uniform": lambda: W.uniform_points(3000, 13)}[points]()
    tr = W.adaptive_tree(pts, max_leaf)
    assert len(set(tr.level[tr.is_leaf].tolist())) > 1 or points == "uniform"
    owner, ptr, src = W.near_lists(tr, max_src)
    leaves = np.flatnonzero(tr.is_leaf)
    assert np.array_equal(np.unique(owner), leaves)
    counts = tr.counts()
    if max_src is None:
        assert np.array_equal(owner, leaves)
    else:
        assert len(owner) > len(leaves)  # some lists were split
        for k in range(len(owner)):  # each entry within the cap, or a single box that is a leaf
            part = src[ptr[k]:ptr[k + 1]]
            assert counts[part].sum() <= max_src or (len(part) == 1 and tr.is_leaf[part[0]])
    # the entries of one leaf, concatenated
    per_leaf = {int(b): [] for b in leaves}
    for k, b in enumerate(owner):
        per_leaf[int(b)].append(src[ptr[k]:ptr[k + 1]])
    t, s = W.interaction_pairs(tr)
    pair_keys = np.sort(t.astype(np.int64) * tr.n_box + s)
    lv = tr.level.astype(np.int64)
    ijk = tr.ijk.astype(np.int64)
    # box id from (level, coords): boxes sorted by a key of level and Morton code
    box_key = (lv << 58) + W.morton_keys(ijk).astype(np.int64)
    order = np.argsort(box_key)

    def box_at(level, coords):
        pos = np.searchsorted(box_key[order], (level << 58) + W.morton_keys(coords).astype(np.int64))
        return order[np.minimum(pos, len(order) - 1)]  # entries off the tree are masked by the caller

    S = leaves.astype(np.int64)
    for b in leaves:
        lst = np.concatenate(per_leaf[int(b)]).astype(np.int64)
        assert len(np.unique(lst)) == len(lst)
        lstar = np.minimum(lv[b], lv[S])
        anc_b = ijk[b][None, :] >> (lv[b] - lstar)[:, None]
        anc_s = ijk[S] >> (lv[S] - lstar)[:, None]
        near = np.max(np.abs(anc_b - anc_s), axis=1) <= 1
        n_in = np.zeros(len(S), dtype=np.int64)
        for n in lst:
            inside = lv[n] <= lv[S]
            shift = np.where(inside, lv[S] - lv[n], 0)
            n_in += inside & np.all((ijk[S] >> shift[:, None]) == ijk[n], axis=1)
        n_far = np.zeros(len(S), dtype=np.int64)
        for l in range(2, int(lv[b]) + 1):
            ok = lstar >= l
            a_b = box_at(np.int64(l), (ijk[b] >> (lv[b] - l))[None, :])[0]
            a_s = box_at(np.int64(l), ijk[S] >> np.where(ok, lv[S] - l, 0)[:, None])
            key = a_b * tr.n_box + a_s
            pos = np.minimum(np.searchsorted(pair_keys, key), len(pair_keys) - 1)
            n_far += ok & (pair_keys[pos] == key)
        assert np.array_equal(n_in, near.astype(np.int64)), b
        assert np.array_equal(n_far, (~near).astype(np.int64)), b


def test_near_lists_of_a_uniform_tree_are_the_neighbour_lists():
    tr = W.uniform_tree(W.uniform_points(500, 14), 2)
    a = W.near_lists(tr)
    b = W.neighbours(tr, 2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("points,max_leaf", [("plummer", 16), ("mixture", 24), ("uniform", 40)])
def test_adaptive_lists_partition_every_leaf_pair(points, max_leaf):
    """U (direct sum), W (multipole at the targets), X (sources into a local) and the List-2
    pairs of every level count every (target leaf, source leaf) pair exactly once, and W and X
    boxes are separated from the box they serve: a W box does not touch its leaf but its parent
    does; an X leaf does not touch its box but touches the box's parent.  Brute force over all
    leaf pairs."""
    pts = {"plummer": lambda: W.plummer_points(3000, 11),
           "mixture": lambda: W.gaussian_mixture_points(3000, 12),
           "uniform": lambda: W.uniform_points(3000, 13)}[points]()
    tr = W.adaptive_tree(pts, max_leaf)
    (ub, up, ul), (wb, wp, wl), (xb, xp, xl) = W.adaptive_lists(tr)
    leaves = np.flatnonzero(tr.is_leaf).astype(np.int64)
    lv = tr.level.astype(np.int64)
    ijk = tr.ijk.astype(np.int64)
    parent = {}
    for l in range(tr.n_levels - 1):
        par, ch = W.children(tr, l)
        for k, pb in enumerate(par):
            for c in ch[k]:
                if c >= 0:
                    parent[int(c)] = int(pb)

    def anc_or_self(b):
        out = [int(b)]
        while out[-1] in parent:
            out.append(parent[out[-1]])
        return out

    # separation of W and X
    for k, b in enumerate(wb):
        for w_ in wl[wp[k]:wp[k + 1]]:
            assert not W._touch(tr, int(w_), int(b)) and W._touch(tr, parent[int(w_)], int(b))
    for k, a in enumerate(xb):
        for x_ in xl[xp[k]:xp[k + 1]]:
            assert tr.is_leaf[x_] and lv[x_] < lv[a]
            assert not W._touch(tr, int(x_), int(a)) and W._touch(tr, int(x_), parent[int(a)])
    U = {int(b): set(ul[up[k]:up[k + 1]].tolist()) for k, b in enumerate(ub)}
    Wd = {int(b): set(wl[wp[k]:wp[k + 1]].tolist()) for k, b in enumerate(wb)}
    Xd = {int(a): set(xl[xp[k]:xp[k + 1]].tolist()) for k, a in enumerate(xb)}
    t, s = W.interaction_pairs(tr)
    V = set(zip(t.tolist(), s.tolist()))
    anc = {int(b): anc_or_self(b) for b in leaves}
    for b in leaves:
        b = int(b)
        for sl in leaves:
            sl = int(sl)
            n = int(sl in U.get(b, ()))
            n += sum((ta, sa) in V for ta in anc[b] for sa in anc[sl] if lv[ta] == lv[sa])
            n += sum(a in Wd.get(b, ()) for a in anc[sl])
            n += sum(sl in Xd.get(a, ()) for a in anc[b])
            assert n == 1, (b, sl, n)


def test_quadtree_ranges_and_list2_partition_every_leaf_pair():
    """Uniform quadtree: every box's range holds exactly its points, and the List-2 pairs of
    all levels with the leaf neighbours count every (target, source) leaf pair exactly once."""
    import numpy as np
    import workloads as W
    pts = W.uniform_points2d(3000, 3)
    tr = W.uniform_quadtree(pts, 4)
    for b in range(tr.n_box):
        lo, hi = tr.pt_range[b]
        h = tr.box_size(int(tr.level[b]))
        inside = np.all((tr.points >= tr.ij[b] * h) & (tr.points < (tr.ij[b] + 1) * h), axis=1)
        assert inside.sum() == hi - lo and inside[lo:hi].all()
    t, s = W.quad_list2(tr)
    assert np.all(np.diff(t.astype(np.int64) * tr.n_box + s) > 0)
    offs = {tuple(tr.ij[a] - tr.ij[b]) for a, b in zip(t, s) if tr.level[a] == 4}
    assert len(offs) == 40
    leaves = tr.boxes_at(4)
    pos = {int(b): k for k, b in enumerate(leaves)}
    cover = np.zeros((len(leaves), len(leaves)), dtype=np.int64)
    for a, b in zip(t, s):
        sh = 4 - int(tr.level[a])
        la = [k for k, c in enumerate(leaves) if np.all(tr.ij[c] >> sh == tr.ij[a])]
        lb = [k for k, c in enumerate(leaves) if np.all(tr.ij[c] >> sh == tr.ij[b])]
        cover[np.ix_(la, lb)] += 1
    bx, ptr, nbr = W.quad_neighbours(tr, 4)
    for k, b in enumerate(bx):
        for n in nbr[ptr[k]:ptr[k + 1]]:
            cover[pos[int(b)], pos[int(n)]] += 1
    assert np.all(cover == 1)
