"""GPU: several M2L batches enqueued as one unit (fmm_m2l_multi_*), and its capture into a HIP
graph.

Workload: a mixed far field on an adaptive Gaussian-mixture tree (8192 points, at most 32
per leaf, levels 2..6), Yukawa (lambda = 2) and biharmonic, with the order depending on the
level as p(l) = 6 + 2 ((l - 2) mod 3), FP32.  One batch per (kernel, order), six in all,
prepared three ways: with one tiled shape (one persistent launch drains all six), with each
batch's own streaming shape (six launches), and mixed (tiled shapes differing per batch, and
streaming batches beside them).

Checks: every batch of the multi launch against the oracle (normwise relative 2e-5, the FP32
M2L tolerance), the multi launch bit-identical to the per-batch launches (same work items,
same per-item arithmetic, split tiles reduced in part order), with and without split tiles,
two launches in a row, and graph replays bit-identical to the eager launch.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import compressed as Z

from helpers import oracle_m2l_scaled, perm_to_lib, rel, tree_inputs

pytestmark = pytest.mark.gpu

TUNING = {"rows_per_wave": 2, "col_tiles_per_wave": 2, "col_groups": 1, "lds_buffers": 1}
KERNELS = (("yukawa", 2.0), ("biharmonic", 0.0))
ORDERS = (6, 8, 10)


def order_of_level(l):
    return 6 + 2 * ((l - 2) % 3)


@pytest.fixture(scope="module")
def mixed():
    tr, _ = tree_inputs(8192, 0, 5, kind="gmm", max_leaf=32)
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    groups = []
    for kernel, param in KERNELS:
        for p in ORDERS:
            levels = [l for l in range(2, tr.n_levels) if order_of_level(l) == p]
            t, s = W.interaction_pairs(tr, levels)
            nc = len(Z.kept(kernel, param, p))
            g = np.random.Generator(np.random.PCG64(1000 + 10 * p + len(kernel)))
            beta = g.standard_normal((tr.n_box, nc))
            groups.append(dict(kernel=kernel, param=param, p=p, levels=levels, t=t, s=s, beta=beta))
    return tr, lh, groups


@pytest.fixture(scope="module")
def oracle_refs(mixed):
    """Oracle theta~ of every group, in the oracle's kept order."""
    tr, lh, groups = mixed
    return [oracle_m2l_scaled(g["kernel"], g["param"], g["p"], tr.ijk.astype(np.int64), tr.level, lh,
                              g["t"], g["s"], g["beta"]) for g in groups]


# per-batch tunings of the "mixed" preparation: two tiled shapes and streaming batches
MIXED_TUNINGS = [TUNING, {"form": "stream", "waves": 4}, dict(TUNING, col_tiles_per_wave=1),
                 {"form": "stream"}, TUNING, dict(TUNING, col_tiles_per_wave=1)]


def build(fmm, mixed, monkeypatch, items, how="tiled"):
    if items is not None:
        monkeypatch.setenv("FMM_M2L_ITEMS", str(items))
    tr, lh, groups = mixed
    plans, batches, mp, perms = [], [], [], []
    for k, g in enumerate(groups):
        d = fmm.Desc(g["kernel"], g["p"], "f32", g["param"])
        plan = fmm.Plan(d, lh)
        perm = perm_to_lib(g["kernel"], g["param"], g["p"], d.index_table())
        inv = np.argsort(perm)
        plans.append(plan)
        tuning = {"tiled": TUNING, "stream": "library", "mixed": MIXED_TUNINGS[k % len(MIXED_TUNINGS)]}[how]
        batches.append(plan.prepare(g["t"], g["s"], tr.ijk, tr.level, tuning=tuning))
        # library order: coefficient k is the oracle's coefficient perm[k]
        mp.append(torch.as_tensor(np.ascontiguousarray(g["beta"][:, perm]), dtype=torch.float32, device="cuda"))
        perms.append((perm, inv))
    return plans, batches, mp, perms


@pytest.mark.parametrize("items,how", [(None, "tiled"), (4096, "tiled"), (None, "stream"), (None, "mixed"),
                                       (4096, "mixed")])
def test_multi_matches_oracle_and_single(gpu_lib, mixed, oracle_refs, items, how, monkeypatch):
    fmm = gpu_lib
    tr, lh, groups = mixed
    plans, batches, mp, perms = build(fmm, mixed, monkeypatch, items, how)
    forms = [b.info()["stream_form"] for b in batches]
    assert forms == ([0] * 6 if how == "tiled" else [1] * 6 if how == "stream" else [0, 1, 0, 1, 0, 0])
    if items is not None:
        assert any(b.info()["n_items"] > b.info()["n_tiles"] for b in batches if not b.info()["stream_form"])
    single = [torch.zeros_like(m) for m in mp]
    for b, m, l in zip(batches, mp, single):
        b(m, l)
    multi = fmm.Multi(batches)
    out = [torch.zeros_like(m) for m in mp]
    multi(mp, out)
    torch.cuda.synchronize()
    for k, g in enumerate(groups):
        perm, _ = perms[k]
        got = out[k].cpu().numpy().astype(np.float64)
        ref = oracle_refs[k][:, perm]
        assert rel(got, ref) < 2e-5, (g["kernel"], g["p"], rel(got, ref))
        assert torch.equal(out[k], single[k]), (g["kernel"], g["p"])
    # a second launch into the same outputs adds the same values again, bit for bit
    again = [torch.zeros_like(m) for m in mp]
    multi(mp, again)
    multi(mp, again)
    for k in range(len(groups)):
        twice = single[k].clone()
        batches[k](mp[k], twice)
        assert torch.equal(again[k], twice)
    multi.close()


@pytest.mark.parametrize("how", ["tiled", "mixed"])
def test_multi_graph_replay(gpu_lib, mixed, monkeypatch, how):
    fmm = gpu_lib
    plans, batches, mp, perms = build(fmm, mixed, monkeypatch, None, how)
    multi = fmm.Multi(batches)
    eager = [torch.zeros_like(m) for m in mp]
    multi(mp, eager)  # also the warm-up before capture
    torch.cuda.synchronize()
    out = [torch.zeros_like(m) for m in mp]
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for o in out:
                o.zero_()
            multi(mp, out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        for o in out:
            o.fill_(float(rep + 1))  # eager work between replays; the graph must clear it
        graph.replay()
        torch.cuda.synchronize()
        for k in range(len(mp)):
            assert torch.equal(out[k], eager[k]), (rep, k)
        scratch = torch.randn(1 << 16, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        assert torch.isfinite(scratch)
    del graph
    multi.close()


def test_multi_validation(gpu_lib, mixed, monkeypatch):
    fmm = gpu_lib
    from paper_2305_17867_amd._lib import FmmError
    tr, lh, groups = mixed
    g = groups[0]
    p32 = fmm.Plan(fmm.Desc(g["kernel"], g["p"], "f32", g["param"]), lh)
    p64 = fmm.Plan(fmm.Desc(g["kernel"], g["p"], "f64", g["param"]), lh)
    b32 = p32.prepare(g["t"], g["s"], tr.ijk, tr.level, tuning=TUNING)
    b64 = p64.prepare(g["t"], g["s"], tr.ijk, tr.level, tuning=TUNING)
    adj = p32.prepare_adjoint(g["t"], g["s"], tr.ijk, tr.level, tuning=TUNING)
    fft = p32.prepare_fft(g["t"], g["s"], tr.ijk, tr.level)
    for bad in ([b32, b64], [b32, adj], [b32, fft], []):
        with pytest.raises((FmmError, ValueError)):
            fmm.Multi(bad)
    with pytest.raises(FmmError):
        fmm.Multi([b32] * 33)
    with pytest.raises(FmmError):
        fmm.Multi([b32, b32])  # split tiles keep partials in the batch's own scratch
