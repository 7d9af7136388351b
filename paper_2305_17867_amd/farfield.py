"""The far field of a tree pass built from the hot-path operators, with a hand-written adjoint.

For a uniform octree the far field of every target box is the sum over its List-2 source
boxes at every level >= 2.  Two ways to form it:
  - per level (default): each box's multipole is formed by P2M straight from its points (every
    box's points are one Morton range at every level) and each level's local expansion is
    evaluated by L2P at that level's boxes;
  - tree pass (tree_pass=True): P2M at the leaves, compressed M2M up the tree (Sec. 4.3),
    M2L at every level, compressed L2L down the tree (Sec. 4.2) and L2P at the leaves.  For
    Laplace and biharmonic the two agree to roundoff; for Helmholtz and Yukawa they differ at
    the truncation level.
``FarField`` sets this up once (plans, prepared M2L batches and their transposes) and
``apply`` runs it as a torch.autograd.Function:

    phi = FarField(...).apply(w, src_xyz, tgt_xyz)

whose backward calls only the HIP adjoints (L2P^T, L2L^T, M2L^T, M2M^T, P2M^T) and returns
d L / d w, d L / d src_xyz and d L / d tgt_xyz for the frozen tree (box membership of the
points is fixed when FarField is built).
"""
from __future__ import annotations

import numpy as np
import torch

import workloads as W

from . import fmm


class FarField:
    def __init__(self, kernel: str, order: int, dtype: str, src_tree: "W.Tree", tgt_tree: "W.Tree",
                 param: float = 0.0, levels=None, device="cuda", tree_pass: bool = False, wx_lists=None,
                 pairs=None):
        """wx_lists: (W, X) of ``workloads.adaptive_lists`` for one tree (sources and targets the
        same boxes): the forward then also evaluates the multipoles of each leaf's W boxes at
        its targets (compressed M2P, Sec. 3.5) and forms the locals of each X box from its X
        leaves' sources (compressed P2L, Sec. 3.2), the interactions that the near lists of
        ``near_lists`` would otherwise leave to the direct sum (use the U lists for the near
        field then).  Forward only.
        pairs: (target, source) List-2 pairs of the M2L levels (host int32 arrays, e.g. from the
        device tree build); default: ``workloads.interaction_pairs`` of src_tree."""
        assert src_tree.n_levels == tgt_tree.n_levels and np.array_equal(src_tree.ijk, tgt_tree.ijk), \
            "source and target trees must share the box grid (one tree, or uniform trees of one depth)"
        self.desc = fmm.Desc(kernel, order, dtype, param)
        n_lev = src_tree.n_levels
        self.levels = list(range(2, n_lev)) if levels is None else list(levels)
        self.plan = fmm.Plan(self.desc, [src_tree.box_size(l) for l in range(n_lev)])
        t, s = W.interaction_pairs(src_tree, self.levels) if pairs is None else \
            (np.asarray(pairs[0], dtype=np.int32), np.asarray(pairs[1], dtype=np.int32))
        self.n_pair = len(t)
        self.batch = self.plan.prepare(t, s, src_tree.ijk, src_tree.level)
        # the adjoints are implemented for real dtypes; a complex far field runs forward only
        self.batch_t = None if dtype in ("c128", "c64") else \
            self.plan.prepare_adjoint(t, s, src_tree.ijk, src_tree.level)
        self.n_box = src_tree.n_box
        dev = torch.device(device)
        i64 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.int64, device=dev)
        self.center = torch.as_tensor(src_tree.center, dtype=torch.float64, device=dev)
        self.level = torch.as_tensor(src_tree.level, dtype=torch.int32, device=dev)
        self.src_rng = i64(src_tree.pt_range)
        self.tgt_rng = i64(tgt_tree.pt_range)
        self.level_boxes = {l: (int(src_tree.level_start[l]), int(src_tree.level_start[l + 1])) for l in self.levels}
        lo, hi = self.level_boxes[self.levels[0]][0], self.level_boxes[self.levels[-1]][1]
        self.box_lo, self.box_hi = lo, hi  # boxes with multipoles / locals
        self.tree_pass = tree_pass
        self.wx = None
        if wx_lists is not None:
            i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.int32, device=dev)
            (wb, wp, wl), (xb, xp, xl) = wx_lists
            self.wx = ((i32(wb), i32(wp), i32(wl)), (i32(xb), i32(xp), i32(xl)))
        if tree_pass:
            self.leaf = n_lev - 1
            assert self.levels == list(range(self.levels[0], n_lev)), \
                "the tree pass needs every level from the first M2L level to the deepest level"
            assert np.array_equal(src_tree.is_leaf, tgt_tree.is_leaf), "source and target trees must share their leaves"
            # P2M and L2P run on every level that holds leaves (only the deepest one for a uniform
            # tree), over the level's boxes with the point ranges of non-leaf boxes emptied: their
            # multipoles come from M2M and their locals go down by L2L
            leaf = src_tree.is_leaf
            self.leaf_levels = [l for l in self.levels if leaf[slice(*self.level_boxes[l])].any()]
            self.src_leaf_rng = i64(np.where(leaf[:, None], src_tree.pt_range, 0))
            self.tgt_leaf_rng = i64(np.where(leaf[:, None], tgt_tree.pt_range, 0))
            # parents on level l that have children, and their children on level l + 1
            self.family = {}
            for l in range(self.levels[0], self.leaf):
                par, ch = W.children(src_tree, l)
                keep = np.any(ch >= 0, axis=1)
                if np.any(keep):
                    self.family[l] = (torch.as_tensor(par[keep], device=dev),
                                      torch.as_tensor(np.ascontiguousarray(ch[keep]), device=dev))

    def _sl(self, a):
        return a[self.box_lo:self.box_hi]

    def forward_raw(self, w, src, tgt):
        if self.tree_pass:
            return self._forward_tree(w, src, tgt)
        d = self.desc
        nc = self.plan.nc
        mpole = torch.zeros((self.n_box, nc), dtype=d.value_dtype, device=w.device)
        # one call per level: the boxes of a level have similar point counts, so the large boxes
        # of coarse levels are spread over several workgroups
        for l in self.levels:
            a, b = self.level_boxes[l]
            self.plan.p2m(self.center[a:b], self.level[a:b], self.src_rng[a:b], src, w, out=mpole[a:b])
        local = torch.zeros_like(mpole)
        self.batch(mpole, local)
        self._p2l(w, src, local)
        pot = torch.zeros(tgt.shape[0], dtype=d.value_dtype, device=w.device)
        for l in self.levels:
            a, b = self.level_boxes[l]
            self.plan.l2p(self.center[a:b], self.level[a:b], self.tgt_rng[a:b], tgt, local[a:b], pot)
        self._m2p(tgt, mpole, pot)
        return pot, mpole, local

    def _p2l(self, w, src, local):
        """X lists: locals of the X boxes straight from the sources of their X leaves."""
        if self.wx is not None and self.wx[1][0].shape[0]:
            xb, xp, xl = self.wx[1]
            self.plan.p2l(xb, xp, xl, self.center, self.level, self.src_rng, src, w, local)

    def _m2p(self, tgt, mpole, pot):
        """W lists: multipoles of the W boxes at the targets of their leaves."""
        if self.wx is not None and self.wx[0][0].shape[0]:
            wb, wp, wl = self.wx[0]
            self.plan.m2p(wb, wp, wl, self.center, self.level, self.tgt_rng, tgt, mpole, pot)

    def _forward_tree(self, w, src, tgt):
        d = self.desc
        mpole = torch.zeros((self.n_box, self.plan.nc), dtype=d.value_dtype, device=w.device)
        for l in self.leaf_levels:
            a, b = self.level_boxes[l]
            self.plan.p2m(self.center[a:b], self.level[a:b], self.src_leaf_rng[a:b], src, w, out=mpole[a:b])
        for l in reversed(range(self.levels[0], self.leaf)):  # children before parents
            if l in self.family:
                self.plan.m2m(*self.family[l], self.center, self.level, mpole)
        local = torch.zeros_like(mpole)
        self.batch(mpole, local)
        self._p2l(w, src, local)
        for l in range(self.levels[0], self.leaf):  # parents before children
            if l in self.family:
                self.plan.l2l(*self.family[l], self.center, self.level, local)
        pot = torch.zeros(tgt.shape[0], dtype=d.value_dtype, device=w.device)
        for l in self.leaf_levels:
            a, b = self.level_boxes[l]
            self.plan.l2p(self.center[a:b], self.level[a:b], self.tgt_leaf_rng[a:b], tgt, local[a:b], pot)
        self._m2p(tgt, mpole, pot)
        return pot, mpole, local

    def _backward_tree(self, g, w, src, tgt, local, need_w, need_src, need_tgt):
        local_grad = torch.zeros_like(local)
        tgt_grad = torch.zeros_like(tgt) if need_tgt else None
        for l in self.leaf_levels:
            a, b = self.level_boxes[l]
            self.plan.l2p_adjoint(self.center[a:b], self.level[a:b], self.tgt_leaf_rng[a:b], tgt, g,
                                  local_grad=local_grad[a:b], local=local[a:b] if need_tgt else None,
                                  tgt_grad=tgt_grad)
        for l in reversed(range(self.levels[0], self.leaf)):  # L2L^T: children before parents
            if l in self.family:
                self.plan.l2l_adjoint(*self.family[l], self.center, self.level, local_grad)
        mpole_grad = torch.zeros_like(local)
        self.batch_t(local_grad, mpole_grad)
        for l in range(self.levels[0], self.leaf):  # M2M^T: parents before children
            if l in self.family:
                self.plan.m2m_adjoint(*self.family[l], self.center, self.level, mpole_grad)
        w_grad = torch.zeros_like(w) if need_w else None
        src_grad = torch.zeros_like(src) if need_src else None
        for l in self.leaf_levels:
            a, b = self.level_boxes[l]
            self.plan.p2m_adjoint(self.center[a:b], self.level[a:b], self.src_leaf_rng[a:b], src, w,
                                  mpole_grad[a:b], w_grad=w_grad, src_grad=src_grad)
        return w_grad, src_grad, tgt_grad

    def backward_raw(self, g, w, src, tgt, local, need_w=True, need_src=True, need_tgt=True):
        if self.wx is not None:
            raise NotImplementedError("the adjoint of the W / X interactions (M2P, P2L) is not implemented")
        if self.batch_t is None:
            raise NotImplementedError("the far-field adjoint is implemented for real dtypes (f64, f32)")
        if self.tree_pass:
            return self._backward_tree(g, w, src, tgt, local, need_w, need_src, need_tgt)
        local_grad = torch.zeros_like(local)
        tgt_grad = torch.zeros_like(tgt) if need_tgt else None
        # L2P^T level by level (point ranges of one call are disjoint): local gradients of the
        # level's boxes and, when asked, the target-position gradients
        for l in self.levels:
            a, b = self.level_boxes[l]
            self.plan.l2p_adjoint(self.center[a:b], self.level[a:b], self.tgt_rng[a:b], tgt, g,
                                  local_grad=local_grad[a:b], local=local[a:b] if need_tgt else None,
                                  tgt_grad=tgt_grad)
        mpole_grad = torch.zeros_like(local)
        self.batch_t(local_grad, mpole_grad)
        w_grad = torch.zeros_like(w) if need_w else None
        src_grad = torch.zeros_like(src) if need_src else None
        for l in self.levels:
            a, b = self.level_boxes[l]
            self.plan.p2m_adjoint(self.center[a:b], self.level[a:b], self.src_rng[a:b], src, w,
                                  mpole_grad[a:b], w_grad=w_grad, src_grad=src_grad)
        return w_grad, src_grad, tgt_grad

    def apply(self, w, src, tgt):
        return _FarFieldFn.apply(w, src, tgt, self)


class _FarFieldFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, src, tgt, ff: FarField):
        w, src, tgt = w.detach().contiguous(), src.detach().contiguous(), tgt.detach().contiguous()
        pot, _, local = ff.forward_raw(w, src, tgt)
        ctx.ff = ff
        ctx.save_for_backward(w, src, tgt, local)
        return pot

    @staticmethod
    def backward(ctx, g):
        w, src, tgt, local = ctx.saved_tensors
        ff = ctx.ff
        need = ctx.needs_input_grad
        wg, sg, tg = ff.backward_raw(g.contiguous(), w, src, tgt, local, need_w=need[0], need_src=need[1],
                                     need_tgt=need[2])
        return wg, sg, tg, None
