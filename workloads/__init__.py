"""Seeded synthetic workloads: point clouds, weights, octrees and interaction lists.

This module is shared by the CPU oracle and the GPU path.  It holds no arithmetic
of the expansion method itself (no derivatives, moments, translations or
compression): only the geometry that every FMM pass needs as input --

* point distributions (uniform cube, Plummer sphere, Gaussian mixture) drawn from
  NumPy's PCG64 with an explicit seed;
* octrees over the unit cube, uniform or adaptive, with points sorted in Morton
  order so that the points of every box (at every level) are one contiguous range;
* "List 2" (interaction list) pairs: boxes of the same level whose parents are
  adjacent or equal but which are not adjacent themselves (the well-separated
  pairs an FMM translates by multipole-to-local);
* near-field lists: the neighbour boxes of the leaves of a uniform tree and, for
  adaptive trees, the boxes holding the sources that no List-2 pair of any level
  separates from a leaf, so that near lists and List 2 together count every leaf
  pair once.

Box ids are global across levels.  For every box: ``level``, integer grid
coordinates ``ijk`` at its level, ``center`` (float64), ``pt_range`` (int64
(begin, end) into the Morton-sorted points).  A box at level l has side 2**-l.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MAX_DEPTH = 20  # Morton keys use 3 * MAX_DEPTH = 60 bits of a uint64


# --------------------------------------------------------------------------- points

def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_points(n: int, seed: int, low=0.0, high=1.0) -> np.ndarray:
    """n points uniform in [low, high)^3 (per-axis bounds allowed), float64 [n, 3]."""
    g = rng(seed)
    low = np.broadcast_to(np.asarray(low, dtype=np.float64), (3,))
    high = np.broadcast_to(np.asarray(high, dtype=np.float64), (3,))
    return low + (high - low) * g.random((n, 3))


def normal_weights(n: int, seed: int, complex_: bool = False) -> np.ndarray:
    """Weights with N(0,1) entries; complex weights have N(0,1) real and imaginary parts."""
    g = rng(seed)
    if complex_:
        w = g.standard_normal((n, 2))
        return w[:, 0] + 1j * w[:, 1]
    return g.standard_normal(n)


def plummer_points(n: int, seed: int, scale: float = 0.1, center=(0.5, 0.5, 0.5)) -> np.ndarray:
    """Plummer-sphere radii r = a (u^(-2/3) - 1)^(-1/2), isotropic directions,
    points outside the unit cube rejected and redrawn."""
    g = rng(seed)
    center = np.asarray(center, dtype=np.float64)
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = max(1024, int((n - out.shape[0]) * 1.3))
        u = g.random(m)
        u = np.clip(u, 1e-300, 1.0)
        r = scale / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        v = g.standard_normal((m, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        x = center + r[:, None] * v
        ok = np.all((x >= 0.0) & (x < 1.0), axis=1)
        out = np.concatenate([out, x[ok]], axis=0)
    return out[:n]


def gaussian_mixture_points(n: int, seed: int, k: int = 4, sigma: float = 0.05,
                            mean_low: float = 0.2, mean_high: float = 0.8) -> np.ndarray:
    """k equal-weight isotropic Gaussians (std sigma), means uniform in
    [mean_low, mean_high]^3; points outside the unit cube rejected and redrawn."""
    g = rng(seed)
    means = mean_low + (mean_high - mean_low) * g.random((k, 3))
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = max(1024, int((n - out.shape[0]) * 1.2))
        comp = g.integers(0, k, m)
        x = means[comp] + sigma * g.standard_normal((m, 3))
        ok = np.all((x >= 0.0) & (x < 1.0), axis=1)
        out = np.concatenate([out, x[ok]], axis=0)
    return out[:n]


# --------------------------------------------------------------------------- morton

def _spread_bits(v: np.ndarray) -> np.ndarray:
    """Insert two zero bits between each of the low 20 bits of v (uint64), by the usual
    shift-and-mask steps (each step moves groups of bits to their places at once)."""
    v = v.astype(np.uint64) & np.uint64(0xFFFFF)
    for shift, mask in ((32, 0x1F00000000FFFF), (16, 0x1F0000FF0000FF), (8, 0x100F00F00F00F00F),
                        (4, 0x10C30C30C30C30C3), (2, 0x1249249249249249)):
        v = (v | (v << np.uint64(shift))) & np.uint64(mask)
    return v


def morton_keys(ijk: np.ndarray) -> np.ndarray:
    """Interleaved key (x bit highest within each triple) for integer coords [n, 3]."""
    ijk = np.asarray(ijk)
    return (_spread_bits(ijk[:, 0]) << np.uint64(2)) | (_spread_bits(ijk[:, 1]) << np.uint64(1)) \
        | _spread_bits(ijk[:, 2])


def _compact_bits(k: np.ndarray) -> np.ndarray:
    out = np.zeros_like(k)
    for b in range(MAX_DEPTH):
        out |= ((k >> np.uint64(3 * b)) & np.uint64(1)) << np.uint64(b)
    return out


def morton_decode(keys: np.ndarray) -> np.ndarray:
    keys = np.asarray(keys, dtype=np.uint64)
    return np.stack([_compact_bits(keys >> np.uint64(2)), _compact_bits(keys >> np.uint64(1)),
                     _compact_bits(keys)], axis=1).astype(np.int64)


# --------------------------------------------------------------------------- trees

@dataclass
class Tree:
    """Octree over [0,1)^3 with Morton-sorted points.

    perm:      original index of each sorted point
    points:    sorted points [n, 3]
    level, ijk, center, pt_range: per box (global ids, level-major order);
               pt_range[b] = (begin, end) into the sorted points
    level_start: first box id of each level (len n_levels + 1)
    is_leaf:   per box
    """
    points: np.ndarray
    perm: np.ndarray
    level: np.ndarray
    ijk: np.ndarray
    center: np.ndarray
    pt_range: np.ndarray
    level_start: np.ndarray
    is_leaf: np.ndarray
    kind: str = "uniform"
    meta: dict = field(default_factory=dict)

    @property
    def n_box(self) -> int:
        return int(self.level.shape[0])

    @property
    def n_levels(self) -> int:
        return int(self.level_start.shape[0] - 1)

    def boxes_at(self, lev: int) -> np.ndarray:
        return np.arange(self.level_start[lev], self.level_start[lev + 1])

    def box_size(self, lev: int) -> float:
        return 2.0 ** (-lev)

    def counts(self) -> np.ndarray:
        return self.pt_range[:, 1] - self.pt_range[:, 0]


def children(tree: Tree, lev: int) -> tuple[np.ndarray, np.ndarray]:
    """Boxes of level lev and their children on level lev + 1: (parent [n] int32,
    child [n][8] int32, -1 where a child box does not exist).  Octant o of a parent with
    integer coordinates ijk is the box 2 ijk + (o & 1, (o >> 1) & 1, (o >> 2) & 1)."""
    parents = tree.boxes_at(lev)
    nxt = tree.boxes_at(lev + 1)
    index = {tuple(int(v) for v in tree.ijk[b]): int(b) for b in nxt}
    child = np.full((parents.shape[0], 8), -1, dtype=np.int32)
    for k, b in enumerate(parents):
        base = 2 * tree.ijk[b]
        for o in range(8):
            key = (int(base[0]) + (o & 1), int(base[1]) + ((o >> 1) & 1), int(base[2]) + ((o >> 2) & 1))
            child[k, o] = index.get(key, -1)
    return parents.astype(np.int32), child


def neighbours(tree: Tree, lev: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Near-field lists of the boxes of level lev: every existing box of the same level whose
    integer coordinates differ by at most one in each axis, the box itself included (the
    U list of a uniform tree at its leaf level).  Returns (box [n] int32, ptr [n + 1] int32,
    nbr int32) in CSR form."""
    boxes = tree.boxes_at(lev)
    index = {tuple(int(v) for v in tree.ijk[b]): int(b) for b in boxes}
    ptr, nbr = [0], []
    for b in boxes:
        i, j, k = (int(v) for v in tree.ijk[b])
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for dk in (-1, 0, 1):
                    n = index.get((i + di, j + dj, k + dk))
                    if n is not None:
                        nbr.append(n)
        ptr.append(len(nbr))
    return boxes.astype(np.int32), np.asarray(ptr, dtype=np.int32), np.asarray(nbr, dtype=np.int32)


def near_lists(tree: Tree, max_src: int | None = None) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Near-field lists of the leaves of any octree (uniform or adaptive), in CSR form
    (leaf [n] int32, ptr [n + 1] int32, src int32).

    A source leaf s is near a target leaf b when their ancestors on the level min(level b,
    level s) are adjacent or equal; every other pair is well separated on some level >= 2 at
    which both ancestors exist, and is then in exactly one List-2 pair of those ancestors
    (``interaction_pairs``).  The list of b holds
      - the existing boxes of b's level adjacent to b, b included, whose point ranges cover
        all their descendant leaves, and
      - on every coarser level, the leaves adjacent to b's ancestor there.
    No box appears twice, and together with the List-2 pairs of all levels every (target,
    source) leaf pair is counted exactly once.

    With max_src, a list whose boxes hold more than max_src points in all is split into
    several entries of the same leaf: boxes above max_src points are replaced by their
    children (depth first, children in box order, i.e. by Morton key; down to leaves), and the
    boxes are packed in order into entries of at most max_src points (a single leaf above the
    cap is an entry of its own).  A coarse leaf next
    to a densely refined region would otherwise leave one workgroup with most of the work."""
    count = tree.pt_range[:, 1] - tree.pt_range[:, 0]
    index = {}  # (level, i, j, k) -> box, built on first use by split()

    def split(n):
        if count[n] <= max_src or tree.is_leaf[n]:
            return [n]
        if not index:
            index.update({(int(tree.level[b]),) + tuple(int(v) for v in tree.ijk[b]): int(b) for b in range(tree.n_box)})
        lev, base = int(tree.level[n]) + 1, 2 * tree.ijk[n].astype(np.int64)
        out = []
        for o in range(8):  # Morton order of the children: x bit highest
            c = index.get((lev, int(base[0]) + ((o >> 2) & 1), int(base[1]) + ((o >> 1) & 1), int(base[2]) + (o & 1)))
            if c is not None:
                out += split(c)
        return out

    # candidates of every leaf, found level by level with sorted Morton keys: (leaf position,
    # level, offset) -> box, kept in the order leaf, level, offset (di, dj, dk lexicographic)
    leaves = np.flatnonzero(tree.is_leaf)
    lb = tree.level[leaves].astype(np.int64)
    ijk = tree.ijk[leaves].astype(np.int64)
    offs = np.array([(di, dj, dk) for di in (-1, 0, 1) for dj in (-1, 0, 1) for dk in (-1, 0, 1)], dtype=np.int64)
    parts = []  # (leaf position, level, offset index, box)
    for lev in range(tree.n_levels):
        sel = np.flatnonzero(lb >= lev)
        ids = tree.boxes_at(lev)
        if sel.size == 0 or ids.size == 0:
            continue
        keys = morton_keys(tree.ijk[ids].astype(np.int64))  # sorted: boxes are stored in Morton order
        anc = ijk[sel] >> (lb[sel] - lev)[:, None]
        cand = anc[:, None, :] + offs[None, :, :]
        inside = np.all((cand >= 0) & (cand < (1 << lev)), axis=2)
        ck = morton_keys(np.where(inside[..., None], cand, 0).reshape(-1, 3)).reshape(cand.shape[:2])
        pos = np.minimum(np.searchsorted(keys, ck), keys.shape[0] - 1)
        found = inside & (keys[pos] == ck)
        box = ids[pos]
        keep = found & ((lb[sel] == lev)[:, None] | tree.is_leaf[box])
        li, oi = np.nonzero(keep)
        parts.append(np.stack([sel[li], np.full(li.shape, lev), oi, box[li, oi]], axis=1))
    allp = np.concatenate(parts) if parts else np.zeros((0, 4), dtype=np.int64)
    allp = allp[np.lexsort((allp[:, 2], allp[:, 1], allp[:, 0]))]
    per_leaf = np.bincount(allp[:, 0], minlength=leaves.shape[0])
    lst_ptr = np.concatenate([[0], np.cumsum(per_leaf)])
    src_all = allp[:, 3]
    if max_src is None:
        return leaves.astype(np.int32), lst_ptr.astype(np.int32), src_all.astype(np.int32)
    total = np.add.reduceat(count[src_all], lst_ptr[:-1]) if src_all.size else np.zeros(0, dtype=np.int64)
    owner, ptr, src = [], [0], []
    for k, b in enumerate(leaves):
        lst = src_all[lst_ptr[k]:lst_ptr[k + 1]]
        if per_leaf[k] == 0 or total[k] <= max_src:
            owner.append(b)
            src += lst.tolist()
            ptr.append(len(src))
            continue
        run = 0
        for n in [m for x in lst for m in split(int(x))]:
            if run and run + count[n] > max_src:
                owner.append(b)
                ptr.append(len(src))
                run = 0
            src.append(n)
            run += count[n]
        owner.append(b)
        ptr.append(len(src))
    return np.asarray(owner, dtype=np.int32), np.asarray(ptr, dtype=np.int32), np.asarray(src, dtype=np.int32)


def _touch(tree: Tree, a: int, b: int) -> bool:
    """Whether the closed cubes of boxes a and b (any levels) intersect."""
    la, lb = int(tree.level[a]), int(tree.level[b])
    L = max(la, lb)
    lo_a = tree.ijk[a].astype(np.int64) << (L - la)
    lo_b = tree.ijk[b].astype(np.int64) << (L - lb)
    hi_a = lo_a + (1 << (L - la))
    hi_b = lo_b + (1 << (L - lb))
    return bool(np.all((lo_a <= hi_b) & (lo_b <= hi_a)))


def adaptive_lists(tree: Tree, max_src: int | None = None):
    """The near-field lists of an adaptive octree split by what each interaction needs, in
    CSR form (box [n] int32, ptr [n + 1] int32, list int32):

      U  per leaf b: the leaves touching b (b included): the direct sum (P2P);
      W  per leaf b: boxes w whose parent touches b but which do not touch b themselves, the
         children of b's colleagues (same-level boxes touching b) found by descending while
         boxes touch b: w's multipole is evaluated at b's targets (M2P);
      X  per box a (any level): leaves x coarser than a that touch a's parent but not a:
         x's sources form a's local expansion directly (P2L), which L2L carries to the leaves.

    These are the interactions that ``near_lists`` gives to the direct sum; with the List-2
    pairs of every level (``interaction_pairs``) every (target leaf, source leaf) pair is
    counted exactly once.  With max_src, U lists are split as in ``near_lists``."""
    leaves0, ptr0, src0 = near_lists(tree)
    kid = {}
    for b in range(tree.n_box):
        kid[(int(tree.level[b]),) + tuple(int(v) for v in tree.ijk[b])] = b

    def children(n):
        lev, base = int(tree.level[n]) + 1, 2 * tree.ijk[n].astype(np.int64)
        out = []
        for o in range(8):
            c = kid.get((lev, int(base[0]) + (o & 1), int(base[1]) + ((o >> 1) & 1), int(base[2]) + ((o >> 2) & 1)))
            if c is not None:
                out.append(c)
        return out

    def ancestor(b, lev):
        lb = int(tree.level[b])
        return kid[(lev,) + tuple(int(v) >> (lb - lev) for v in tree.ijk[b])]

    u_lists, w_lists, x_sets = {}, {}, {}
    for k, b in enumerate(leaves0):
        b = int(b)
        lb = int(tree.level[b])
        u, w = [], []
        for n in src0[ptr0[k]:ptr0[k + 1]]:
            n = int(n)
            if int(tree.level[n]) == lb:  # b itself or a colleague: descend while touching b
                stack = [n]
                while stack:
                    m = stack.pop()
                    if tree.is_leaf[m]:
                        u.append(m)
                        continue
                    for c in children(m):
                        (stack if _touch(tree, c, b) else w).append(c)
            elif _touch(tree, n, b):  # a coarser leaf touching b
                u.append(n)
            else:  # a coarser leaf: X of the first ancestor of b it does not touch
                for lev in range(int(tree.level[n]) + 1, lb + 1):
                    a = ancestor(b, lev)
                    if not _touch(tree, n, a):
                        x_sets.setdefault(a, set()).add(n)
                        break
        u_lists[b] = sorted(u)
        w_lists[b] = sorted(w)

    def csr(d, keys):
        box, ptr, lst = [], [0], []
        for key in keys:
            if not d.get(key):
                continue
            box.append(key)
            lst += list(d[key])
            ptr.append(len(lst))
        return np.asarray(box, np.int32), np.asarray(ptr, np.int32), np.asarray(lst, np.int32)

    leaves = [int(b) for b in leaves0]
    U = csr(u_lists, leaves)
    if max_src is not None:
        count = tree.pt_range[:, 1] - tree.pt_range[:, 0]
        owner, ptr, src = [], [0], []
        for k, b in enumerate(U[0]):
            run = 0
            for n in U[2][U[1][k]:U[1][k + 1]]:
                if run and run + count[n] > max_src:
                    owner.append(b)
                    ptr.append(len(src))
                    run = 0
                src.append(int(n))
                run += count[n]
            owner.append(b)
            ptr.append(len(src))
        U = (np.asarray(owner, np.int32), np.asarray(ptr, np.int32), np.asarray(src, np.int32))
    Wl = csr(w_lists, leaves)
    X = csr({a: sorted(v) for a, v in x_sets.items()}, sorted(x_sets))
    return U, Wl, X


def _point_keys(points: np.ndarray) -> np.ndarray:
    scale = float(1 << MAX_DEPTH)
    ijk = np.floor(points * scale).astype(np.int64)
    ijk = np.clip(ijk, 0, (1 << MAX_DEPTH) - 1)
    return morton_keys(ijk)


def _assemble(points, perm, keys_sorted, level_keys, is_leaf_lists, kind, meta) -> Tree:
    """level_keys[l] = sorted unique Morton prefixes (level-l keys) of existing boxes."""
    levels, ijks, centers, ranges, leaves, level_start = [], [], [], [], [], [0]
    for lev, lk in enumerate(level_keys):
        shift = np.uint64(3 * (MAX_DEPTH - lev))
        lo = np.searchsorted(keys_sorted, lk << shift, side="left")
        hi = np.searchsorted(keys_sorted, (lk + np.uint64(1)) << shift, side="left") if lev > 0 \
            else np.array([keys_sorted.shape[0]])
        ijk = morton_decode(lk)
        h = 2.0 ** (-lev)
        levels.append(np.full(lk.shape[0], lev, dtype=np.int32))
        ijks.append(ijk.astype(np.int32))
        centers.append((ijk + 0.5) * h)
        ranges.append(np.stack([lo, hi], axis=1).astype(np.int64))
        leaves.append(is_leaf_lists[lev])
        level_start.append(level_start[-1] + lk.shape[0])
    return Tree(points=points, perm=perm, level=np.concatenate(levels), ijk=np.concatenate(ijks),
                center=np.concatenate(centers), pt_range=np.concatenate(ranges),
                level_start=np.asarray(level_start, dtype=np.int64),
                is_leaf=np.concatenate(leaves), kind=kind, meta=meta)


def uniform_tree(points: np.ndarray, depth: int) -> Tree:
    """All 8**l boxes at every level l <= depth (empty boxes included)."""
    keys = _point_keys(points)
    perm = np.argsort(keys, kind="stable")
    ks = keys[perm]
    level_keys, leaf = [], []
    for lev in range(depth + 1):
        lk = np.arange(8 ** lev, dtype=np.uint64)
        level_keys.append(lk)
        leaf.append(np.full(lk.shape[0], lev == depth))
    return _assemble(points[perm], perm, ks, level_keys, leaf, "uniform", {"depth": depth})


def adaptive_tree(points: np.ndarray, max_leaf: int, max_depth: int = 16) -> Tree:
    """Refine every box holding more than max_leaf points; empty children are dropped."""
    keys = _point_keys(points)
    perm = np.argsort(keys, kind="stable")
    ks = keys[perm]
    level_keys, leaf = [np.zeros(1, dtype=np.uint64)], []
    active = ks  # keys of points inside boxes that get refined
    lev = 0
    while True:
        lk = level_keys[-1]
        shift = np.uint64(3 * (MAX_DEPTH - lev))
        counts = (np.searchsorted(ks, (lk + np.uint64(1)) << shift) - np.searchsorted(ks, lk << shift)) \
            if lev > 0 else np.array([ks.shape[0]])
        refine = (counts > max_leaf) & (lev < max_depth)
        leaf.append(~refine)
        if not np.any(refine):
            break
        # points of refined boxes -> unique child keys
        box_of_pt = ks >> shift
        sel = np.isin(box_of_pt, lk[refine])
        active = ks[sel]
        child = np.unique(active >> np.uint64(3 * (MAX_DEPTH - lev - 1)))
        level_keys.append(child)
        lev += 1
    return _assemble(points[perm], perm, ks, level_keys, leaf, "adaptive", {"max_leaf": max_leaf})


# --------------------------------------------------------------------------- interaction lists

def list2_offsets(parity) -> np.ndarray:
    """Integer offsets o = ijk_t - ijk_s of List 2 for a target with the given child parity
    (ijk mod 2): sources are children of the parent's neighbours (parent included) that are
    not adjacent to the target.  189 offsets per parity, 316 distinct over all parities."""
    per_axis = []
    for par in parity:
        # source child coords span [2P-2, 2P+3]; target is at 2P + par
        lo, hi = -2 - par, 3 - par  # o_src = s - t in [lo, hi]
        per_axis.append(np.arange(lo, hi + 1))
    g = np.stack(np.meshgrid(*per_axis, indexing="ij"), axis=-1).reshape(-1, 3)
    g = g[np.max(np.abs(g), axis=1) >= 2]
    return -g  # o = t - s


def all_list2_offsets() -> np.ndarray:
    r = np.arange(-3, 4)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    return g[np.max(np.abs(g), axis=1) >= 2]


def interaction_pairs(tree: Tree, levels=None) -> tuple[np.ndarray, np.ndarray]:
    """All List-2 pairs (target box, source box) at the given levels (default: all levels >= 2).
    Both boxes must exist in the tree.  Returns int32 arrays, sorted by (target, source)."""
    if levels is None:
        levels = range(2, tree.n_levels)
    tgts, srcs = [], []
    for lev in levels:
        ids = tree.boxes_at(lev)
        if ids.size == 0:
            continue
        ijk = tree.ijk[ids].astype(np.int64)
        n_side = 1 << lev
        keys = morton_keys(ijk)  # sorted, since boxes are stored in Morton order
        for par in np.ndindex(2, 2, 2):
            sel = np.all((ijk & 1) == np.asarray(par), axis=1)
            if not np.any(sel):
                continue
            t_ids = ids[sel]
            offs = list2_offsets(par)  # o = t - s  =>  s = t - o
            cand = ijk[sel][:, None, :] - offs[None, :, :]
            inside = np.all((cand >= 0) & (cand < n_side), axis=2)
            ti = np.broadcast_to(t_ids[:, None], inside.shape)[inside]
            cs = cand[inside]
            ck = morton_keys(cs)
            pos = np.searchsorted(keys, ck)
            pos_c = np.minimum(pos, keys.shape[0] - 1)
            found = keys[pos_c] == ck
            tgts.append(ti[found])
            srcs.append(ids[pos_c[found]])
    if not tgts:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    t = np.concatenate(tgts).astype(np.int32)
    s = np.concatenate(srcs).astype(np.int32)
    order = np.lexsort((s, t))
    return t[order], s[order]


# --------------------------------------------------------------------------- quadtrees (2-D)

def uniform_points2d(n: int, seed: int, low=0.0, high=1.0) -> np.ndarray:
    """n points uniform in [low, high)^2."""
    return rng(seed).uniform(low, high, size=(n, 2))


def _spread2(v: np.ndarray) -> np.ndarray:
    """Insert one zero bit between each of the low 20 bits of v (uint64)."""
    v = v.astype(np.uint64) & np.uint64(0xFFFFF)
    for shift, mask in ((16, 0x0000FFFF0000FFFF), (8, 0x00FF00FF00FF00FF), (4, 0x0F0F0F0F0F0F0F0F),
                        (2, 0x3333333333333333), (1, 0x5555555555555555)):
        v = (v | (v << np.uint64(shift))) & np.uint64(mask)
    return v


def morton2(ij: np.ndarray) -> np.ndarray:
    """Interleaved key (x bit higher within each pair) for integer coords [n, 2]."""
    ij = np.asarray(ij)
    return (_spread2(ij[:, 0]) << np.uint64(1)) | _spread2(ij[:, 1])


@dataclass
class QuadTree:
    """Uniform quadtree over [0,1)^2: every box of every level <= depth, level-major, Morton
    order within a level (box id = level_start[l] + Morton key); points sorted by key."""
    points: np.ndarray
    perm: np.ndarray
    level: np.ndarray
    ij: np.ndarray
    center: np.ndarray
    pt_range: np.ndarray
    level_start: np.ndarray
    depth: int

    @property
    def n_box(self) -> int:
        return int(self.level.shape[0])

    @property
    def n_levels(self) -> int:
        return self.depth + 1

    def boxes_at(self, lev: int) -> np.ndarray:
        return np.arange(self.level_start[lev], self.level_start[lev + 1])

    def box_size(self, lev: int) -> float:
        return 2.0 ** (-lev)


def uniform_quadtree(points: np.ndarray, depth: int) -> QuadTree:
    scale = float(1 << MAX_DEPTH)
    ij = np.clip(np.floor(points * scale).astype(np.int64), 0, (1 << MAX_DEPTH) - 1)
    keys = morton2(ij)
    perm = np.argsort(keys, kind="stable")
    ks = keys[perm]
    levels, ijs, centers, ranges, level_start = [], [], [], [], [0]
    for lev in range(depth + 1):
        lk = np.arange(4 ** lev, dtype=np.uint64)
        shift = np.uint64(2 * (MAX_DEPTH - lev))
        lo = np.searchsorted(ks, lk << shift)
        hi = np.searchsorted(ks, (lk + np.uint64(1)) << shift) if lev > 0 else np.array([ks.shape[0]])
        # decode: even bits are y, odd bits x
        bij = np.zeros((lk.shape[0], 2), dtype=np.int64)
        for b in range(lev):
            bij[:, 0] |= ((lk >> np.uint64(2 * b + 1)) & np.uint64(1)).astype(np.int64) << b
            bij[:, 1] |= ((lk >> np.uint64(2 * b)) & np.uint64(1)).astype(np.int64) << b
        levels.append(np.full(lk.shape[0], lev, dtype=np.int32))
        ijs.append(bij.astype(np.int32))
        centers.append((bij + 0.5) * 2.0 ** (-lev))
        ranges.append(np.stack([lo, hi], axis=1).astype(np.int64))
        level_start.append(level_start[-1] + lk.shape[0])
    return QuadTree(points=points[perm], perm=perm, level=np.concatenate(levels), ij=np.concatenate(ijs),
                    center=np.concatenate(centers), pt_range=np.concatenate(ranges),
                    level_start=np.asarray(level_start, dtype=np.int64), depth=depth)


def quad_list2(tree: QuadTree, levels=None) -> tuple[np.ndarray, np.ndarray]:
    """List-2 pairs (target, source) of a uniform quadtree: the children of the parent's
    neighbours (parent included) that are not adjacent to the target; at most 27 per box,
    40 distinct offsets per level (7^2 - 3^2).  Sorted by (target, source)."""
    if levels is None:
        levels = range(2, tree.n_levels)
    tg, sr = [], []
    for lev in levels:
        ids = tree.boxes_at(lev)
        ij = tree.ij[ids].astype(np.int64)
        side = 1 << lev
        base = 2 * (ij >> 1)
        d = np.arange(-2, 4)
        cand = base[:, None, None, :] + np.stack(np.meshgrid(d, d, indexing="ij"), axis=-1)[None]
        cand = cand.reshape(len(ids), 36, 2)
        far = np.max(np.abs(cand - ij[:, None, :]), axis=2) >= 2
        inside = np.all((cand >= 0) & (cand < side), axis=2)
        keep = far & inside
        ti = np.broadcast_to(ids[:, None], keep.shape)[keep]
        si = tree.level_start[lev] + morton2(cand[keep]).astype(np.int64)
        tg.append(ti)
        sr.append(si)
    if not tg:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    t, s = np.concatenate(tg).astype(np.int32), np.concatenate(sr).astype(np.int32)
    order = np.lexsort((s, t))
    return t[order], s[order]


def quad_neighbours(tree: QuadTree, lev: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Boxes of level lev and their adjacent boxes (themselves included), CSR (box, ptr, nbr)."""
    ids = tree.boxes_at(lev)
    ij = tree.ij[ids].astype(np.int64)
    side = 1 << lev
    ptr, nbr = [0], []
    for b, (i, j) in zip(ids, ij):
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                if 0 <= i + di < side and 0 <= j + dj < side:
                    nbr.append(int(tree.level_start[lev] + morton2(np.array([[i + di, j + dj]]))[0]))
        ptr.append(len(nbr))
    return ids.astype(np.int32), np.asarray(ptr, np.int32), np.asarray(nbr, np.int32)


# --------------------------------------------------------------------------- configs

def small_two_box(seed: int = 0):
    """64 sources uniform in [-0.5,0.5]^3 (expansion centre 0) and 64 targets uniform in a
    unit box centred at (3,0,0), weights N(0,1)."""
    src = uniform_points(64, seed, -0.5, 0.5)
    tgt = uniform_points(64, seed + 1, (2.5, -0.5, -0.5), (3.5, 0.5, 0.5))
    w = normal_weights(64, seed + 2)
    return src, tgt, w, np.zeros(3), np.array([3.0, 0.0, 0.0])
