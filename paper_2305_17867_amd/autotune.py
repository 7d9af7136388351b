"""Autotuner for the batched M2L launch shape.

For one (kernel, order, dtype) and one set of interaction pairs it prepares the batch with
every candidate launch shape (the streaming form with its wavefronts and workgroups per launch;
the tiled form with rows per wavefront, column tiles per wavefront, column groups, K splits,
LDS buffers, workgroups per launch; see fmm_m2l_tuning in include/fmm.h), times the launches
with HIP events on the current stream, and keeps the fastest.  Results are cached in a JSON
file keyed by device, kernel, order, dtype and problem size, so later runs reuse them.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np
import torch

from . import fmm

SHAPES = [(1, 1), (1, 2), (2, 1), (2, 2), (3, 1), (3, 2), (4, 1), (5, 1)]  # tiled (rows, col tiles) per wave
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "fmm_m2l_autotune.json")
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "m2l_tuned.json")


def candidates(nc: int, n_cu: int, max_waves: int = 8, full: bool = False):
    """Streaming-form candidates (wavefronts per workgroup, workgroups per launch) first, then
    tiled-form candidates: all of them with full=True, else the shapes that have won on the
    Laplace workloads (2-3 row tiles of 2 column tiles per wavefront, no column groups)."""
    out = [{"form": "stream", "waves": w, "workgroups": g}
           for w in (16, 8, 4, 2) for g in (n_cu, n_cu // 2) if w <= 16]
    rem = nc % 16
    rtiles = nc // 16 if (nc > 16 and 1 <= rem <= 2) else (nc + 15) // 16  # matrix-core row tiles
    for rt, ctw in (SHAPES if full else [(2, 2), (3, 2)]):
        nrg = -(-rtiles // rt)
        for ncg in ((1, 2, 4) if full else (1,)):
            for nks in ((1, 2, 3, 4) if full else (1, 2)):
                waves = nrg * ncg * nks
                if waves > max_waves or ncg * ctw > 4:
                    continue
                for items in ((2 * n_cu, 3 * n_cu, 4 * n_cu) if full else (2 * n_cu, 4 * n_cu)):
                    for nbuf in ((1, 2) if full else (1,)):
                        out.append({"form": "tiled", "rows_per_wave": rt, "col_tiles_per_wave": ctw,
                                    "col_groups": ncg, "target_items": items, "lds_buffers": nbuf,
                                    "k_splits": nks})
    return out


def _key(desc, n_pair: int) -> str:
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return f"{name}|hip{torch.version.hip}|{desc.kernel}|p{desc.order}|{desc.dtype}|pairs{n_pair}"


def time_batch(batch, mpole, local, reps: int = 5) -> float:
    batch(mpole, local)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        batch(mpole, local)
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def tune(plan: "fmm.Plan", tgt_box, src_box, box_ijk, box_level, reps: int = 5,
         cache: str | None = DEFAULT_CACHE, max_candidates: int | None = None, log=None,
         full: bool = False) -> dict:
    """Returns {"tuning": best tuning dict, "ms": its time, "results": [(tuning, ms | error)]}."""
    desc = plan.desc
    key = _key(desc, len(tgt_box))
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                db = json.load(f)
            if key in db:
                return db[key]
        except (OSError, ValueError):
            pass
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    n_box = int(np.asarray(box_level).shape[0])
    mpole = torch.randn((n_box, plan.nc), dtype=desc.value_dtype, device="cuda")
    local = torch.zeros_like(mpole)
    cands = candidates(plan.nc, n_cu, full=full)
    if max_candidates:
        cands = cands[:max_candidates]
    results = []
    best = None
    t0 = time.time()
    for tun in cands:
        try:
            b = plan.prepare(tgt_box, src_box, box_ijk, box_level, tuning=tun)
        except fmm._lib.FmmError as e:
            results.append((tun, str(e).split(":")[1].strip()))
            continue
        ms = time_batch(b, mpole, local, reps)
        b.close()
        results.append((tun, ms))
        if log:
            log(f"  {tun} -> {ms:.3f} ms")
        if best is None or ms < best[1]:
            best = (tun, ms)
    out = {"tuning": best[0] if best else None, "ms": best[1] if best else None, "results": results,
           "seconds": time.time() - t0}
    if cache and best:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        db = {}
        if os.path.exists(cache):
            try:
                with open(cache) as f:
                    db = json.load(f)
            except (OSError, ValueError):
                db = {}
        db[key] = out
        with open(cache, "w") as f:
            json.dump(db, f, indent=1)
    return out


def _merge(path: str, entries: dict) -> dict:
    table = {}
    if os.path.exists(path):
        try:
            with open(path) as fh:
                table = json.load(fh)
        except (OSError, ValueError):
            table = {}
    table.update(entries)
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    return table


def _entry(r, n_pair, workload):
    return {"tuning": r["tuning"], "ms": round(r["ms"], 4), "pairs": int(n_pair),
            "device": torch.cuda.get_device_name(0), "hip": torch.version.hip, "workload": workload}


def write_table(path: str = TABLE, cases=((8, "f64"), (8, "f32"), (12, "f64"), (12, "f32")), reps: int = 5,
                log=print) -> dict:
    """Tune the Laplace M2L of the uniform workload (2^20 random points in the unit cube,
    octree depth 4, all List-2 pairs of level 4) for each (order, dtype) and add the launch
    shapes to the table read by fmm.tuned_m2l_shape()."""
    import workloads as W
    pts = W.uniform_points(1 << 20, 1)
    tr = W.uniform_tree(pts, 4)
    t, s = W.interaction_pairs(tr, [4])
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    entries = {}
    for p, dt in cases:
        plan = fmm.Plan(fmm.Desc("laplace", p, dt), lh)
        r = tune(plan, t, s, tr.ijk, tr.level, reps=reps, cache=None)
        log(f"laplace p={p} {dt}: {r['ms']:.4f} ms {r['tuning']} ({len(r['results'])} candidates, "
            f"{r['seconds']:.0f} s)")
        entries[f"laplace|p{p}|{dt}"] = _entry(r, len(t), "uniform 2^20 points, depth 4, level-4 List-2 pairs")
        plan.close()
    return _merge(path, entries)


def write_mixture_table(path: str = TABLE, reps: int = 5, log=print) -> dict:
    """Tune each (kernel, order) batch of the mixed workload: Yukawa (lambda = 2) and
    biharmonic far fields of 524,288 Gaussian-mixture points (adaptive octree, <= 64 per leaf),
    order p(l) = 6 + 2 ((l - 2) mod 3) on M2L level l, FP32; add the shapes to the table."""
    import workloads as W
    tr = W.adaptive_tree(W.gaussian_mixture_points(1 << 19, 4), 64)
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    entries = {}
    for kernel, param in (("yukawa", 2.0), ("biharmonic", 0.0)):
        for p in (6, 8, 10):
            levels = [l for l in range(2, tr.n_levels) if 6 + 2 * ((l - 2) % 3) == p]
            t, s = W.interaction_pairs(tr, levels)
            plan = fmm.Plan(fmm.Desc(kernel, p, "f32", param), lh)
            r = tune(plan, t, s, tr.ijk, tr.level, reps=reps, cache=None)
            log(f"{kernel} p={p} f32: {r['ms']:.4f} ms {r['tuning']} ({len(r['results'])} candidates, "
                f"{r['seconds']:.0f} s)")
            entries[f"{kernel}|p{p}|f32"] = _entry(
                r, len(t), f"mixture 524288 points, adaptive <= 64 per leaf, levels {levels}")
            plan.close()
    return _merge(path, entries)


if __name__ == "__main__":
    import sys
    if "--mixture" in sys.argv:
        write_mixture_table()
    else:
        write_table()
