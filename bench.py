"""Benchmark of the compressed-Taylor FMM hot path on one MI355X.

Workload (the metric's configuration): 3-D Laplace, 1,048,576 uniform random points in
the unit cube (one set serving as sources and targets), weights N(0,1), uniform octree of
depth 4 (4,096 leaves, ~256 points each), M2L over all 584,136 List-2 pairs of level 4
(316 distinct offsets).  One step = compressed P2M of every leaf -> batched M2L -> L2P at
every point (plus clearing the local and potential arrays).  Inputs are resident in HBM
before the timed region.  The step's launches are issued with their arguments marshalled once
(bound calls); the same step captured in a HIP graph and replayed is reported beside it.  The headline line is FP64 at p = 8; FP32 and p = 12 are reported
as variants in the same line.

value = M2L box-pairs per second of the whole step (pairs / step time).
roofline: the M2L kernel (the dominant one), algorithmic FLOPs 2 Nc^2 per pair over its
average launch time measured with HIP events on its stream.  traffic: HBM bytes per launch from
the rocprofv3 FETCH_SIZE / WRITE_SIZE passes recorded in profiles/ (scaled by the factors a
plain copy gives), or null when the kernel sources changed since they were taken.
Supplementary fields: the FFT form of the same M2L, and the mixed Yukawa + biharmonic workload
(524,288 points, orders per level) as one graph-captured persistent launch.
cpu_baseline: the CPU oracle (NumPy) on a bounded sample of the same workload, scaled.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6e12, "f32": 157.3e12}  # dense matrix-core peaks, FLOP/s (equal to the vector peaks)
HBM_PEAK = 8.0e12  # bytes/s
# FLOP per point of the Laplace moments (uncompressed P2M), from the paper's operation counts
# (Fig. "Laplace P2M 3D" of the operation-count section); L2P has very similar counts
POINT_FLOPS = {8: 276, 12: 788}
DEPTH, NPTS, SEED = 4, 1 << 20, 1
COPY_BYTES = 256 << 20  # plain copy used to calibrate the FETCH_SIZE / WRITE_SIZE counters
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "m2l_kernel_laplace_p8_f64_traffic.txt")
# sources that decide the M2L kernel's memory traffic at the headline configuration
TRAFFIC_SOURCES = ["paper_2305_17867_amd/csrc/m2l.hip", "paper_2305_17867_amd/csrc/kernels.hpp",
                   "paper_2305_17867_amd/csrc/capi.cpp", "paper_2305_17867_amd/m2l_tuned.json"]


def sources_hash() -> str:
    h = hashlib.sha256()
    for rel_path in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel_path), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per M2L launch from the recorded counter passes, or None if absent or stale."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_sources_sha256") != sources_hash():
        return None
    return float(kv["m2l_traffic_bytes"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload():
    import workloads as W
    pts = W.uniform_points(NPTS, SEED)
    tr = W.uniform_tree(pts, DEPTH)
    w = W.normal_weights(NPTS, SEED + 1)
    t, s = W.interaction_pairs(tr, [DEPTH])
    return tr, w, t, s


class Case:
    """Device state for one (order, dtype) variant."""

    def __init__(self, fmm, torch, tr, w, t, s, p, dtype):
        self.torch, self.p, self.dtype = torch, p, dtype
        self.desc = fmm.Desc("laplace", p, dtype)
        lh = [tr.box_size(l) for l in range(tr.n_levels)]
        self.plan = fmm.Plan(self.desc, lh)
        self.batch = self.plan.prepare(t, s, tr.ijk, tr.level)
        self.info = self.batch.info()
        dev = "cuda"
        rd, vd = self.desc.real_dtype, self.desc.value_dtype
        leaves = tr.boxes_at(DEPTH)
        self.n_leaf = len(leaves)
        self.leaf0 = int(leaves[0])
        self.center = torch.as_tensor(tr.center[leaves], dtype=torch.float64, device=dev)
        self.level = torch.as_tensor(tr.level[leaves], dtype=torch.int32, device=dev)
        self.rng = torch.as_tensor(tr.pt_range[leaves], dtype=torch.int64, device=dev)
        self.pts = torch.as_tensor(tr.points, dtype=rd, device=dev)
        self.w = torch.as_tensor(w, dtype=vd, device=dev)
        nc = self.plan.nc
        self.mpole = torch.zeros((tr.n_box, nc), dtype=vd, device=dev)
        self.local = torch.zeros((tr.n_box, nc), dtype=vd, device=dev)
        self.pot = torch.zeros(NPTS, dtype=vd, device=dev)
        self.n_pair = len(t)
        self.nc = nc
        # launches with their arguments marshalled once (the step repeats them unchanged)
        self.run_p2m = self.plan.bind_p2m(self.center, self.level, self.rng, self.pts, self.w,
                                          self.mpole[self.leaf0:self.leaf0 + self.n_leaf])
        self.run_m2l = self.batch.bind(self.mpole, self.local)
        self.run_l2p = self.plan.bind_l2p(self.center, self.level, self.rng, self.pts,
                                          self.local[self.leaf0:self.leaf0 + self.n_leaf], self.pot)

    def p2m(self):
        self.plan.p2m(self.center, self.level, self.rng, self.pts, self.w,
                      out=self.mpole[self.leaf0:self.leaf0 + self.n_leaf])

    def m2l(self):
        self.batch(self.mpole, self.local)

    def l2p(self):
        self.plan.l2p(self.center, self.level, self.rng, self.pts,
                      self.local[self.leaf0:self.leaf0 + self.n_leaf], self.pot)

    def step(self):
        self.local.zero_()
        self.pot.zero_()
        self.run_p2m()
        self.run_m2l()
        self.run_l2p()


def point_rooflines(case, dt, p, t_p2m, t_l2p):
    """P2M and L2P against both ceilings: algorithmic HBM bytes per launch (P2M: x, y, z, w in
    and the box coefficients out; L2P: x, y, z and the potential in, the potential out, and
    the box coefficients in) over HBM bandwidth, and the paper's FLOP count per point over
    the vector peak.  frac is taken against the lower ceiling (the larger of the two)."""
    rb = 8 if dt == "f64" else 4
    coef = case.n_leaf * case.nc * rb
    b_p2m = NPTS * 4 * rb + coef
    b_l2p = NPTS * 5 * rb + coef
    fl = POINT_FLOPS.get(p)
    out = {}
    for name, b, t in (("p2m", b_p2m, t_p2m), ("l2p", b_l2p, t_l2p)):
        hbm = b / t / HBM_PEAK
        valu = NPTS * fl / t / PEAK[dt] if fl else None
        out[f"{name}_hbm_gbps"] = b / t / 1e9
        out[f"{name}_hbm_frac"] = hbm
        out[f"{name}_valu_frac"] = valu
        out[f"{name}_frac"] = max(hbm, valu or 0.0)
    return out


def time_step(torch, case, steps, warmup, graph=False):
    """Seconds per step: eager launches, or (graph=True) the whole step (fills, P2M, M2L, L2P)
    captured once in a HIP graph after the warm-up and replayed."""
    for _ in range(warmup):
        case.step()
    torch.cuda.synchronize()
    run = case.step
    if graph:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                case.step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        run = g.replay
        run()
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    if graph:
        del g
    return sec


def time_kernel(torch, fn, reps=20):
    """Average duration of one launch, HIP events on the launching (current) stream."""
    st = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    fn()
    for a, b in evs:
        a.record(st)
        fn()
        b.record(st)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs])) * 1e-3


def cpu_baseline(tr, w, t, s, p=8, budget_s=12.0):
    """The FP64 oracle on a bounded sample: P2M and L2P of sampled leaves and the full M2L of
    sampled target boxes (all their pairs), each rate scaled to the whole workload."""
    import resource
    from oracle import compressed as Z
    leaves = tr.boxes_at(DEPTH)
    h = tr.box_size(DEPTH)
    g = np.random.Generator(np.random.PCG64(0))
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    wall0 = time.perf_counter()
    # P2M
    n_p2m, t_p2m, pts_p2m = 0, 0.0, 0
    betas = {}
    while t_p2m < budget_s / 3:
        b = int(g.choice(leaves))
        lo, hi = tr.pt_range[b]
        a = time.perf_counter()
        betas[b] = Z.scale_multipole("laplace", 0.0, p, Z.p2m("laplace", 0.0, p, tr.center[b], tr.points[lo:hi],
                                                                w[lo:hi]), 1 / h)
        t_p2m += time.perf_counter() - a
        n_p2m += 1
        pts_p2m += hi - lo
    # M2L: whole target boxes
    n_pairs_done, t_m2l = 0, 0.0
    beta_any = next(iter(betas.values()))
    while t_m2l < budget_s / 3:
        tb = int(g.choice(leaves))
        sel = np.nonzero(t == tb)[0]
        a = time.perf_counter()
        acc = np.zeros_like(beta_any)
        for k in sel:
            d = (tr.center[tb] - tr.center[s[k]])
            acc = acc + Z.m2l("laplace", 0.0, p, d, beta_any)
        t_m2l += time.perf_counter() - a
        n_pairs_done += len(sel)
    # L2P
    n_l2p, t_l2p, pts_l2p = 0, 0.0, 0
    while t_l2p < budget_s / 3:
        b = int(g.choice(leaves))
        lo, hi = tr.pt_range[b]
        a = time.perf_counter()
        Z.l2p("laplace", 0.0, p, tr.center[b], beta_any, tr.points[lo:hi])
        t_l2p += time.perf_counter() - a
        pts_l2p += hi - lo
    wall = time.perf_counter() - wall0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    full = (t_p2m / pts_p2m) * NPTS + (t_m2l / n_pairs_done) * len(t) + (t_l2p / pts_l2p) * NPTS
    return {"value": len(t) / full, "unit": "box-pairs/s", "cores": max(1, int(round(cpu / wall))),
            "kind": "oracle",
            "sample": (f"Laplace p={p} FP64 oracle: P2M of {n_p2m} leaves ({pts_p2m} pts), M2L of "
                       f"{n_pairs_done} pairs (whole target boxes), L2P of {pts_l2p} pts; per-unit times "
                       f"scaled to {NPTS} pts and {len(t)} pairs"),
            "p2m_pts_per_s": pts_p2m / t_p2m, "m2l_pairs_per_s": n_pairs_done / t_m2l,
            "l2p_pts_per_s": pts_l2p / t_l2p}


def translation_flops(p, c, rec_terms):
    """Algorithmic FLOPs (2 per multiply-add) of the separable M2M per child, of the compression
    (or, for L2L, the decompression) per parent, and of the L2L per child."""
    full = [(x, y, z) for z in range(p + 1) for x in range(p + 1 - z) for y in range(p + 1 - z - x)]
    kept = [m for m in full if m[2] < c]
    m2m_child = 2 * (sum(x + 1 for x, y, z in kept) + sum(y + 1 for x, y, z in kept)
                     + sum(min(z, c - 1) + 1 for x, y, z in full))
    l2l_child = 2 * 3 * sum(p - x - y - z + 1 for x, y, z in kept)  # three passes, p - |m| + 1 terms
    recompress = 2 * rec_terms * (len(full) - len(kept))
    return m2m_child, recompress, l2l_child


def translations(torch, fmm, tr, reps=20):
    """Compressed M2M (levels 4 -> 3 -> 2) and L2L (2 -> 3 -> 4) on the headline octree,
    Laplace p = 8, FP64 and FP32: launch times and child translations per second."""
    import workloads as W
    out = []
    dev = "cuda"
    cen = torch.as_tensor(tr.center, dtype=torch.float64, device=dev)
    lev = torch.as_tensor(tr.level, dtype=torch.int32, device=dev)
    fam = {}
    for l in (3, 2):
        par, ch = W.children(tr, l)
        fam[l] = (torch.as_tensor(par, device=dev), torch.as_tensor(ch, device=dev), int((ch >= 0).sum()))
    m2m_child, recompress, l2l_child = translation_flops(8, 2, 2)
    for dt in ("f64", "f32"):
        desc = fmm.Desc("laplace", 8, dt)
        plan = fmm.Plan(desc, [tr.box_size(l) for l in range(tr.n_levels)])
        coef = torch.randn((tr.n_box, plan.nc), dtype=desc.value_dtype, device=dev)
        row = {"dtype": dt}
        for l in (3, 2):
            par, ch, nch = fam[l]
            t = time_kernel(torch, lambda: plan.m2m(par, ch, cen, lev, coef), reps)
            row[f"m2m_l{l + 1}_to_l{l}_us"] = t * 1e6
            row[f"m2m_l{l + 1}_to_l{l}_children_per_s"] = nch / t
            row[f"m2m_l{l + 1}_to_l{l}_gflops"] = (nch * m2m_child + par.shape[0] * recompress) / t / 1e9
        for l in (2, 3):
            par, ch, nch = fam[l]
            t = time_kernel(torch, lambda: plan.l2l(par, ch, cen, lev, coef), reps)
            row[f"l2l_l{l}_to_l{l + 1}_us"] = t * 1e6
            row[f"l2l_l{l}_to_l{l + 1}_children_per_s"] = nch / t
            row[f"l2l_l{l}_to_l{l + 1}_gflops"] = (nch * l2l_child + par.shape[0] * recompress) / t / 1e9
        out.append(row)
    return {"workload": "uniform octree depth 4 (2^20 points), laplace p8: M2M 4->3->2, L2L 2->3->4",
            "flops_per_child_m2m": m2m_child, "flops_per_child_l2l": l2l_child,
            "flops_per_parent_compression": recompress,
            "variants": out}


def full_fmm(torch, fmm, tr, w, reps=5, sample=512):
    """The complete FMM potential of the headline point set (Laplace p = 8, FP64): far field as
    a tree pass (P2M at the leaves, M2M up, M2L on levels 2-4, L2L down, L2P at the leaves) plus
    the near field of the leaves (P2P over the 27 neighbour boxes); its error against the GPU
    direct sum at sampled targets."""
    import workloads as W
    from paper_2305_17867_amd.farfield import FarField
    dev = "cuda"
    ff = FarField("laplace", 8, "f64", tr, tr, tree_pass=True)
    pts = torch.as_tensor(tr.points, dtype=torch.float64, device=dev)
    wd = torch.as_tensor(w, dtype=torch.float64, device=dev)
    boxes, ptr, nbr = W.neighbours(tr, DEPTH)
    d = fmm.Desc("laplace", 8, "f64")
    lists = [torch.as_tensor(a, device=dev) for a in (boxes, ptr, nbr)]
    rng = torch.as_tensor(tr.pt_range, dtype=torch.int64, device=dev)
    out = {}

    def far():
        with torch.no_grad():
            out["pot"] = ff.forward_raw(wd, pts, pts)[0]

    def near():
        fmm.p2p(d, *lists, rng, rng, pts, wd, pts, out["pot"])

    t_far = time_kernel(torch, far, reps)
    t_near = time_kernel(torch, near, reps)
    far()
    near()
    idx = np.sort(np.random.Generator(np.random.PCG64(SEED + 7)).choice(len(w), sample, replace=False))
    ref = fmm.direct(d, pts, wd, pts[torch.as_tensor(idx, device=dev)].contiguous())
    # the direct sum of eq. (1) itself: 4,096 targets against all 2^20 sources
    sub = pts[torch.as_tensor(np.sort(np.random.Generator(np.random.PCG64(SEED + 8)).choice(len(w), 4096, replace=False)),
                              device=dev)].contiguous()
    phi_sub = torch.empty(4096, dtype=torch.float64, device=dev)
    t_direct = time_kernel(torch, lambda: fmm.direct(d, pts, wd, sub, out=phi_sub), reps)
    got = out["pot"][torch.as_tensor(idx, device=dev)]
    err = float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref))
    counts = tr.pt_range[:, 1] - tr.pt_range[:, 0]
    inter = int(sum(int(counts[b]) * int(counts[nbr[ptr[k]:ptr[k + 1]]].sum()) for k, b in enumerate(boxes)))
    # the same potential in FP32 (FP64 tables, FP32 products), against the same FP64 reference
    ff32 = FarField("laplace", 8, "f32", tr, tr, tree_pass=True)
    d32 = fmm.Desc("laplace", 8, "f32")
    pts32, w32 = pts.float(), wd.float()

    def far32():
        with torch.no_grad():
            out["pot32"] = ff32.forward_raw(w32, pts32, pts32)[0]

    def near32():
        fmm.p2p(d32, *lists, rng, rng, pts32, w32, pts32, out["pot32"])

    t_far32 = time_kernel(torch, far32, reps)
    t_near32 = time_kernel(torch, near32, reps)
    far32()
    near32()
    got32 = out["pot32"][torch.as_tensor(idx, device=dev)].double()
    err32 = float(torch.linalg.norm(got32 - ref) / torch.linalg.norm(ref))
    return {"workload": "uniform 2^20 points, depth 4, laplace p8 f64: far field (tree pass) + near field",
            "far_ms": t_far * 1e3, "near_ms": t_near * 1e3, "near_interactions": inter,
            "near_interactions_per_s": inter / t_near, "rel_error_vs_direct": err, "error_sample": sample,
            "direct_4096_targets_ms": t_direct * 1e3, "direct_interactions_per_s": 4096 * len(w) / t_direct,
            "f32": {"far_ms": t_far32 * 1e3, "near_ms": t_near32 * 1e3, "rel_error_vs_direct": err32,
                    "speedup_vs_f64": (t_far + t_near) / (t_far32 + t_near32)}}


def full_fmm_adaptive(torch, fmm, reps=5, sample=512):
    """The complete FMM potential on an adaptive octree (524,288 Gaussian-mixture points, <= 64
    per leaf, leaves on several levels), Laplace p = 8, FP64: far field as a tree pass (P2M at
    the leaves of every level, M2M up, M2L over the List-2 pairs of every level, L2L down, L2P
    at the leaves; the per-level form is timed beside it) plus the near field over the adaptive
    near lists; error against the GPU direct sum at sampled targets."""
    import workloads as W
    from paper_2305_17867_amd.farfield import FarField
    dev = "cuda"
    tr = W.adaptive_tree(W.gaussian_mixture_points(1 << 19, 4), 64)
    w = W.normal_weights(tr.points.shape[0], SEED + 9)
    ff = FarField("laplace", 8, "f64", tr, tr, tree_pass=True)
    ff_level = FarField("laplace", 8, "f64", tr, tr)
    pts = torch.as_tensor(tr.points, dtype=torch.float64, device=dev)
    wd = torch.as_tensor(w, dtype=torch.float64, device=dev)
    leaves, ptr, nbr = W.near_lists(tr, max_src=2048)  # long lists split into parallel entries
    d = fmm.Desc("laplace", 8, "f64")
    lists = [torch.as_tensor(a, device=dev) for a in (leaves, ptr, nbr)]
    rng = torch.as_tensor(tr.pt_range, dtype=torch.int64, device=dev)
    out = {}

    def far():
        with torch.no_grad():
            out["pot"] = ff.forward_raw(wd, pts, pts)[0]

    def near():
        fmm.p2p(d, *lists, rng, rng, pts, wd, pts, out["pot"])

    def far_level():
        with torch.no_grad():
            ff_level.forward_raw(wd, pts, pts)

    t_far = time_kernel(torch, far, reps)
    t_far_level = time_kernel(torch, far_level, reps)
    t_near = time_kernel(torch, near, reps)
    far()
    near()
    idx = np.sort(np.random.Generator(np.random.PCG64(SEED + 10)).choice(len(w), sample, replace=False))
    ref = fmm.direct(d, pts, wd, pts[torch.as_tensor(idx, device=dev)].contiguous())
    got = out["pot"][torch.as_tensor(idx, device=dev)]
    err = float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref))
    counts = tr.pt_range[:, 1] - tr.pt_range[:, 0]
    inter = int(sum(int(counts[b]) * int(counts[nbr[ptr[k]:ptr[k + 1]]].sum()) for k, b in enumerate(leaves)))
    leaf_levels = np.bincount(tr.level[tr.is_leaf])
    return {"workload": "adaptive octree, 524288 Gaussian-mixture points, <= 64 per leaf, laplace p8 f64: "
                        "far field (tree pass) + near field",
            "leaves": int(tr.is_leaf.sum()), "near_entries": int(len(leaves)), "leaf_levels": {int(l): int(c) for l, c in enumerate(leaf_levels) if c},
            "m2l_pairs": ff.n_pair, "far_ms": t_far * 1e3, "far_per_level_ms": t_far_level * 1e3,
            "near_ms": t_near * 1e3, "near_interactions": inter,
            "near_interactions_per_s": inter / t_near, "rel_error_vs_direct": err, "error_sample": sample}


def mixed_batch(torch, fmm, reps=10):
    """Yukawa (lambda = 2) + biharmonic far field of 524,288 Gaussian-mixture points (adaptive
    octree, <= 64 per leaf), orders 6/8/10 by level, FP32: one batch per (kernel, order), all
    drained by one persistent launch, captured in a HIP graph and replayed."""
    import workloads as W
    tr = W.adaptive_tree(W.gaussian_mixture_points(1 << 19, 4), 64)
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    tuning = {"rows_per_wave": 2, "col_tiles_per_wave": 2, "col_groups": 1, "lds_buffers": 1}
    batches, mps, flops, pairs = [], [], 0.0, 0
    for kernel, param in (("yukawa", 2.0), ("biharmonic", 0.0)):
        for p in (6, 8, 10):
            levels = [l for l in range(2, tr.n_levels) if 6 + 2 * ((l - 2) % 3) == p]
            t, s = W.interaction_pairs(tr, levels)
            if len(t) == 0:
                continue
            d = fmm.Desc(kernel, p, "f32", param)
            plan = fmm.Plan(d, lh)
            batches.append(plan.prepare(t, s, tr.ijk, tr.level, tuning=tuning))
            mps.append(torch.randn((tr.n_box, d.nc), dtype=torch.float32, device="cuda"))
            flops += 2.0 * d.nc ** 2 * len(t)
            pairs += len(t)
    locs = [torch.zeros_like(m) for m in mps]
    multi = fmm.Multi(batches)
    seq = time_kernel(torch, lambda: [b(m, l) for b, m, l in zip(batches, mps, locs)], reps)
    one = time_kernel(torch, lambda: multi(mps, locs), reps)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            multi(mps, locs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    replay = time_kernel(torch, graph.replay, reps)
    out = {"workload": "mixture 524288 pts, adaptive <=64, yukawa+biharmonic p 6/8/10 by level, f32",
           "batches": len(batches), "pairs": pairs, "gflop": flops / 1e9,
           "sequential_ms": seq * 1e3, "persistent_ms": one * 1e3, "graph_replay_ms": replay * 1e3,
           "pairs_per_s": pairs / replay, "tflops": flops / replay / 1e12,
           "frac": flops / replay / PEAK["f32"]}
    del graph
    multi.close()
    return out


def plummer_helmholtz(torch, fmm, dt, reps=5):
    """Helmholtz p = 12 far field of 2^21 Plummer points (adaptive octree <= 64 per leaf,
    k = 1 / largest leaf side): every level's List-2 pairs in one prepared batch, one launch."""
    import workloads as W
    tr = W.adaptive_tree(W.plummer_points(1 << 21, 3, 0.1), 64)
    leaf_side = max(tr.box_size(int(tr.level[b])) for b in np.nonzero(tr.is_leaf)[0])
    t, s = W.interaction_pairs(tr, list(range(2, tr.n_levels)))
    d = fmm.Desc("helmholtz", 12, dt, 1.0 / leaf_side)
    plan = fmm.Plan(d, [tr.box_size(l) for l in range(tr.n_levels)])
    batch = plan.prepare(t, s, tr.ijk, tr.level)
    mp = torch.randn((tr.n_box, d.nc), dtype=d.value_dtype, device="cuda")
    loc = torch.zeros_like(mp)
    sec = time_kernel(torch, lambda: batch(mp, loc), reps)
    flops = 8.0 * d.nc ** 2 * len(t)
    batch.close()
    # the FFT form of the same M2L (None where its working set exceeds a workgroup's LDS)
    try:
        fft = plan.prepare_fft(t, s, tr.ijk, tr.level)
    except fmm._lib.FmmError:
        fft_ms = None
    else:
        fft_ms = time_kernel(torch, lambda: fft(mp, loc), reps) * 1e3
        fft.close()
    return {"workload": "plummer 2097152 pts, adaptive <=64, helmholtz p12 k*h_leaf=1, all levels one launch",
            "dtype": dt, "pairs": int(len(t)), "m2l_ms": sec * 1e3, "pairs_per_s": len(t) / sec,
            "tflops": flops / sec / 1e12, "frac": flops / sec / PEAK["f64" if dt == "c128" else "f32"],
            "m2l_fft_ms": fft_ms}


def plummer_helmholtz_fmm(torch, fmm, reps=3, sample=256):
    """The complete Helmholtz potential (complex128, p = 12) of 2^21 Plummer points on their
    adaptive octree (<= 64 per leaf, k = 1 / largest leaf side): far field as a tree pass plus
    the near field over the adaptive near lists; error against the GPU direct sum at sampled
    targets."""
    import workloads as W
    from paper_2305_17867_amd.farfield import FarField
    dev = "cuda"
    tr = W.adaptive_tree(W.plummer_points(1 << 21, 3, 0.1), 64)
    leaf_side = max(tr.box_size(int(tr.level[b])) for b in np.nonzero(tr.is_leaf)[0])
    k = 1.0 / leaf_side
    w = W.normal_weights(tr.points.shape[0], SEED + 11, complex_=True)
    ff = FarField("helmholtz", 12, "c128", tr, tr, param=k, tree_pass=True)
    d = ff.desc
    pts = torch.as_tensor(tr.points, dtype=torch.float64, device=dev)
    wd = torch.as_tensor(w, dtype=torch.complex128, device=dev)
    owner, ptr, nbr = W.near_lists(tr, max_src=2048)
    lists = [torch.as_tensor(a, device=dev) for a in (owner, ptr, nbr)]
    rng = torch.as_tensor(tr.pt_range, dtype=torch.int64, device=dev)
    out = {}

    def far():
        with torch.no_grad():
            out["pot"] = ff.forward_raw(wd, pts, pts)[0]

    def near():
        fmm.p2p(d, *lists, rng, rng, pts, wd, pts, out["pot"])

    t_far = time_kernel(torch, far, reps)
    t_near = time_kernel(torch, near, reps)
    far()
    near()
    idx = np.sort(np.random.Generator(np.random.PCG64(SEED + 12)).choice(len(w), sample, replace=False))
    ref = fmm.direct(d, pts, wd, pts[torch.as_tensor(idx, device=dev)].contiguous())
    got = out["pot"][torch.as_tensor(idx, device=dev)]
    err = float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref))
    counts = tr.pt_range[:, 1] - tr.pt_range[:, 0]
    inter = int(sum(int(counts[b]) * int(counts[nbr[ptr[j]:ptr[j + 1]]].sum()) for j, b in enumerate(owner)))
    return {"workload": "plummer 2097152 pts, adaptive <=64, helmholtz p12 c128 k*h_leaf=1: far field (tree pass) "
                        "+ near field",
            "k": k, "leaves": int(tr.is_leaf.sum()), "m2l_pairs": ff.n_pair, "far_ms": t_far * 1e3,
            "near_ms": t_near * 1e3, "near_interactions": inter, "near_interactions_per_s": inter / t_near,
            "rel_error_vs_direct": err, "error_sample": sample}


def gradient_pass(torch, dt, reps=10, tree_pass=False):
    """Laplace p = 10 far field of 2^21 sources at 2^21 targets (depth-4 octrees) and its
    adjoint: forward and forward + backward times (per level, or as a tree pass with M2M and
    L2L)."""
    import workloads as W
    from paper_2305_17867_amd.farfield import FarField
    n = 1 << 21
    ts = W.uniform_tree(W.uniform_points(n, 5), 4)
    tt = W.uniform_tree(W.uniform_points(n, 6), 4)
    ff = FarField("laplace", 10, dt, ts, tt, tree_pass=tree_pass)
    tdt = torch.float64 if dt == "f64" else torch.float32
    w = torch.as_tensor(W.normal_weights(n, 7), dtype=tdt, device="cuda").requires_grad_(True)
    S = torch.as_tensor(ts.points, dtype=tdt, device="cuda").requires_grad_(True)
    T = torch.as_tensor(tt.points, dtype=tdt, device="cuda").requires_grad_(True)
    c = torch.as_tensor(W.normal_weights(n, 8), dtype=tdt, device="cuda")

    def fwd():
        with torch.no_grad():
            ff.apply(w, S, T)

    def fwd_bwd():
        (ff.apply(w, S, T) * c).sum().backward()

    # the first two backward passes load kernels lazily (the second is the first to add into
    # existing gradients); keep them out of the timed passes
    for _ in range(2):
        fwd_bwd()
    return {"workload": "uniform 2^21 sources + 2^21 targets, depth 4, laplace p10, far field",
            "form": "tree pass (M2M / L2L)" if tree_pass else "per level (P2M / L2P at every level)", "dtype": dt,
            "forward_ms": time_kernel(torch, fwd, reps) * 1e3, "forward_backward_ms": time_kernel(torch, fwd_bwd, reps) * 1e3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--only", default=None, help="run one variant, e.g. f64:8 (for profiling)")
    ap.add_argument("--no-extras", action="store_true", help="skip the FFT path and the mixed workload")
    ap.add_argument("--full-fmm", action="store_true",
                    help="also time the complete FMM potential when --only or --no-extras is given")
    ap.add_argument("--translations", action="store_true",
                    help="also time M2M / L2L when --only or --no-extras is given")
    ap.add_argument("--extended", action="store_true",
                    help="also time the Plummer Helmholtz launch and the far-field gradient pass")
    ap.add_argument("--gradient", action="store_true",
                    help="also time the far-field gradient pass (part of --extended)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy three times, to calibrate HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding is a "
              "design note, not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2305_17867_amd import fmm
    assert torch.cuda.is_available(), "needs a GPU"

    log("building workload")
    tr, w, t, s = build_workload()
    variants = [("f64", 8), ("f32", 8), ("f64", 12), ("f32", 12)]
    if args.only:
        dt, p = args.only.split(":")
        variants = [(dt, int(p))]
    elif args.no_variants:
        variants = variants[:1]
    results = []
    for dt, p in variants:
        log(f"variant {dt} p={p}: prepare")
        case = Case(fmm, torch, tr, w, t, s, p, dt)
        log(f"variant {dt} p={p}: time {args.steps} steps")
        sec = time_step(torch, case, args.steps, args.warmup, graph=False)
        sec_graph = time_step(torch, case, args.steps, 1, graph=True)
        t_p2m = time_kernel(torch, case.p2m)
        t_m2l = time_kernel(torch, case.m2l)
        t_l2p = time_kernel(torch, case.l2p)
        flops = 2.0 * case.nc ** 2 * case.n_pair
        achieved = flops / t_m2l
        t_fft = None
        if not (args.only or args.no_extras) and dt == "f64":
            fb = case.plan.prepare_fft(t, s, tr.ijk, tr.level)
            t_fft = time_kernel(torch, lambda: fb(case.mpole, case.local))
            fb.close()
        results.append({
            "dtype": dt, "order": p, "nc": case.nc, "ms_per_step": sec * 1e3,
            "ms_per_step_graph": sec_graph * 1e3,
            "pairs_per_s": case.n_pair / sec,
            "p2m_pts_per_s": NPTS / t_p2m, "m2l_pairs_per_s": case.n_pair / t_m2l,
            "l2p_pts_per_s": NPTS / t_l2p,
            **point_rooflines(case, dt, p, t_p2m, t_l2p),
            "p2m_ms": t_p2m * 1e3, "m2l_ms": t_m2l * 1e3, "l2p_ms": t_l2p * 1e3,
            "m2l_tflops": achieved / 1e12, "m2l_frac": achieved / PEAK[dt],
            "m2l_fft_ms": None if t_fft is None else t_fft * 1e3,
            "m2l_batch": case.info,
        })
        log(json.dumps(results[-1]))
        del case
        torch.cuda.empty_cache()
    head = results[0]
    out = {
        "metric": "M2L box-pairs/sec + P2M/L2P pts/sec, 3D Laplace p=8/12, FP32 vs FP64",
        "value": head["pairs_per_s"], "unit": "box-pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head["dtype"], "data": "synthetic",
        "config": {"workload": f"laplace3d-p{head['order']}-uniform-depth{DEPTH}-{NPTS}pts",
                   "kernel": "laplace", "order": head["order"], "points": NPTS, "tree_depth": DEPTH,
                   "m2l_level": DEPTH, "m2l_pairs": len(t), "offsets": 316},
        "p2m_pts_per_s": head["p2m_pts_per_s"], "m2l_pairs_per_s": head["m2l_pairs_per_s"],
        "l2p_pts_per_s": head["l2p_pts_per_s"],
        "roofline": {"bound": "mfma", "kernel": "m2l_kernel",
                     "achieved": head["m2l_tflops"], "peak": PEAK[head["dtype"]] / 1e12, "unit": "TFLOP/s",
                     "frac": head["m2l_frac"], "traffic": recorded_traffic(),
                     "algorithmic": f"2*Nc^2 FLOP per pair, Nc={head['nc']}, {len(t)} pairs per launch"},
        "variants": results,
    }
    if args.translations or not (args.only or args.no_extras):
        log("M2M / L2L")
        out["translations"] = translations(torch, fmm, tr)
    if args.full_fmm or not (args.only or args.no_extras):
        log("complete FMM (far field + near field)")
        out["full_fmm"] = full_fmm(torch, fmm, tr, w)
        log("complete FMM on an adaptive tree (far field + near field)")
        out["full_fmm_adaptive"] = full_fmm_adaptive(torch, fmm)
    if not (args.only or args.no_extras):
        log("mixed workload (persistent, graph-captured launch)")
        out["mixed_batch"] = mixed_batch(torch, fmm)
    if args.extended:
        log("Plummer Helmholtz, one launch over all levels")
        out["plummer_helmholtz"] = [plummer_helmholtz(torch, fmm, dt) for dt in ("c128", "c64")]
        log("Plummer Helmholtz, complete FMM (tree pass + near field)")
        out["plummer_helmholtz_fmm"] = plummer_helmholtz_fmm(torch, fmm)
    if args.extended or args.gradient:
        log("far-field gradient pass")
        out["gradient"] = [gradient_pass(torch, dt, tree_pass=tp) for tp in (False, True) for dt in ("f32", "f64")]
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = COPY_BYTES
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(tr, w, t, s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
