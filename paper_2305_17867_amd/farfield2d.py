"""Far field of a uniform quadtree in two dimensions (kernels log r and r^2 log r, Sec. 4.4) from
the 2-D operators, in one of two forms:
  - per level (default): P2M of every box of the M2L levels, one M2L launch over the List-2
    pairs of every level, L2P of every level's locals at its boxes' points;
  - tree pass (tree_pass=True): P2M at the leaves, compressed M2M up the levels (Sec. 4.3), the
    same M2L, compressed L2L down the levels (Sec. 4.2) and L2P at the leaves.  Both kernels'
    PDEs are homogeneous, so M2M and L2L are exact and the two forms agree to rounding.

Set-up (host): the pairs are grouped by target box (CSR), and one scaled derivative table is
made on the device per distinct (level, offset); at most 40 offsets occur per level (7^2 - 3^2).
"""
from __future__ import annotations

import numpy as np
import torch

import workloads as W

from . import fmm


class FarField2D:
    def __init__(self, kernel: str, order: int, tree: "W.QuadTree", levels=None, device="cuda",
                 tree_pass: bool = False):
        self.desc = fmm.Desc(kernel, order, "f64")
        self.tree_pass = tree_pass
        self.levels = list(range(2, tree.n_levels)) if levels is None else list(levels)
        dev = torch.device(device)
        t, s = W.quad_list2(tree, self.levels)
        self.n_pair = len(t)
        lev = tree.level[t].astype(np.int64)
        off = (tree.ij[t] - tree.ij[s]).astype(np.int64)
        keys, pair_tab = np.unique(np.stack([lev, off[:, 0], off[:, 1]], axis=1), axis=0, return_inverse=True)
        h = 2.0 ** (-keys[:, 0].astype(np.float64))
        self.tables = fmm.deriv_tables2d(self.desc, torch.as_tensor(keys[:, 1:].astype(np.float64), device=dev),
                                         torch.as_tensor(h, device=dev))
        # targets in box (Morton) order: neighbouring targets share most of their sources, whose
        # multipoles the caches then serve to several lanes
        tb, first = np.unique(t, return_index=True)
        ptr = np.concatenate([first, [len(t)]]).astype(np.int32)
        i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.int32, device=dev)
        self.tbox, self.pair_ptr, self.pair_src, self.pair_tab = i32(tb), i32(ptr), i32(s), i32(pair_tab.ravel())
        self.n_box = tree.n_box
        self.center = torch.as_tensor(tree.center, dtype=torch.float64, device=dev)
        self.box_h = torch.as_tensor(2.0 ** (-tree.level.astype(np.float64)), device=dev)
        self.rng = torch.as_tensor(tree.pt_range, dtype=torch.int64, device=dev)
        self.level_boxes = {l: (int(tree.level_start[l]), int(tree.level_start[l + 1])) for l in self.levels}
        self.box_lo = self.level_boxes[self.levels[0]][0]
        counts = tree.pt_range[:, 1] - tree.pt_range[:, 0]
        self.max_count = {l: max(1, int(counts[a:b].max())) for l, (a, b) in self.level_boxes.items()}
        self.leaf = tree.depth
        self.family = {}
        if tree_pass:
            assert self.levels == list(range(self.levels[0], tree.n_levels)), \
                "the tree pass needs every level from the first M2L level to the leaves"
            # parents of level l and their four children (Morton key 4 key + octant) on level l + 1
            for l in range(self.levels[0], self.leaf):
                a, b = self.level_boxes[l]
                par = np.arange(a, b, dtype=np.int64)
                ch = tree.level_start[l + 1] + 4 * (par - a)[:, None] + np.arange(4)[None, :]
                self.family[l] = (i32(par), i32(ch))

    def p2m(self, w, src):
        """Multipoles of every box of the M2L levels (the boxes' chunks of points are added
        atomically, so rows of boxes above 256 points may differ in the last bits between runs)."""
        nc = self.desc.nc
        mpole = torch.zeros((self.n_box, nc), dtype=torch.float64, device=w.device)
        self.p2m_into(w, src, mpole)
        return mpole

    def p2m_into(self, w, src, mpole):
        """mpole += the multipoles, one launch per level (each sized for its level's largest box)."""
        for l in self.levels:
            a, b = self.level_boxes[l]
            fmm.p2m2d(self.desc, self.center[a:b], self.box_h[a:b], self.rng[a:b], src, w, out=mpole[a:b],
                      max_per_box=self.max_count[l])

    def m2l(self, mpole, local=None):
        if local is None:
            local = torch.zeros_like(mpole)
        fmm.m2l2d(self.desc, self.tbox, self.pair_ptr, self.pair_src, self.pair_tab, self.tables, mpole, local)
        return local

    def l2p(self, local, tgt, pot):
        for l in self.levels:  # the boxes of one level hold disjoint point ranges
            a, b = self.level_boxes[l]
            fmm.l2p2d(self.desc, self.center[a:b], self.box_h[a:b], self.rng[a:b], tgt, local[a:b], pot,
                      max_per_box=self.max_count[l])
        return pot

    def upward(self, w, src, mpole):
        """Tree pass: P2M at the leaves, then M2M level by level up to the first M2L level."""
        a, b = self.level_boxes[self.leaf]
        fmm.p2m2d(self.desc, self.center[a:b], self.box_h[a:b], self.rng[a:b], src, w, out=mpole[a:b],
                  max_per_box=self.max_count[self.leaf])
        for l in range(self.leaf - 1, self.levels[0] - 1, -1):
            par, ch = self.family[l]
            fmm.m2m2d(self.desc, par, ch, self.center, self.box_h, mpole)

    def downward(self, local, tgt, pot):
        """Tree pass: L2L level by level down to the leaves, then L2P at the leaves."""
        for l in range(self.levels[0], self.leaf):
            par, ch = self.family[l]
            fmm.l2l2d(self.desc, par, ch, self.center, self.box_h, local)
        a, b = self.level_boxes[self.leaf]
        fmm.l2p2d(self.desc, self.center[a:b], self.box_h[a:b], self.rng[a:b], tgt, local[a:b], pot,
                  max_per_box=self.max_count[self.leaf])

    def forward(self, w, src, tgt):
        pot = torch.zeros(tgt.shape[0], dtype=torch.float64, device=w.device)
        if self.tree_pass:
            mpole = torch.zeros((self.n_box, self.desc.nc), dtype=torch.float64, device=w.device)
            self.upward(w, src, mpole)
            local = self.m2l(mpole)
            self.downward(local, tgt, pot)
            return pot, mpole, local
        mpole = self.p2m(w, src)
        local = self.m2l(mpole)
        return self.l2p(local, tgt, pot), mpole, local
