"""fmm_m2l_batched_static (split-tile partials and part counters in the library's fixed device
array, no allocation) against fmm_m2l_batched through the C ABI: two calls in a row, the
second on a smaller batch, for the streaming and the tiled form; bit-identical results are
expected since both run the same kernels over the same work in the same order."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _run(fmm, batch, fn_name, mp, loc0):
    from paper_2305_17867_amd import _lib
    loc = loc0.clone()
    fn = getattr(_lib.load(), fn_name)
    st = fn(batch._h, C.c_void_p(mp.data_ptr()), C.c_void_p(loc.data_ptr()),
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, (fn_name, st, _lib.load().fmm_last_error())
    torch.cuda.synchronize()
    return loc


@pytest.mark.parametrize("form", ["stream", "tiled"])
def test_static_scratch_matches_batched(gpu_lib, form):
    fmm = gpu_lib
    pts = W.uniform_points(1 << 15, 31)
    tr = W.uniform_tree(pts, 4)
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    d = fmm.Desc("laplace", 8, "f64")
    plan = fmm.Plan(d, lh)
    if form == "stream":
        tun = {"form": "stream", "workgroups": 64}  # chunk boundaries cut tiles: partials are used
    else:
        tun = {"form": "tiled", "rows_per_wave": 3, "col_tiles_per_wave": 2, "col_groups": 1,
               "lds_buffers": 1, "k_splits": 2, "target_items": 256}
    g = torch.Generator(device="cuda").manual_seed(5)
    # first call: levels 3 and 4; second call: level 3 only (a smaller batch)
    for levels in ([3, 4], [3]):
        t, s = W.interaction_pairs(tr, levels)
        batch = plan.prepare(t, s, tr.ijk, tr.level, tuning=tun)
        info = batch.info()
        assert info["n_pair"] == len(t)
        if form == "stream":
            assert info["stream_form"] == 1
        mp = torch.randn((tr.n_box, d.nc), dtype=torch.float64, device="cuda", generator=g)
        loc0 = torch.randn((tr.n_box, d.nc), dtype=torch.float64, device="cuda", generator=g)
        ref = _run(fmm, batch, "fmm_m2l_batched", mp, loc0)
        got = _run(fmm, batch, "fmm_m2l_batched_static", mp, loc0)
        assert torch.equal(got, ref), float((got - ref).abs().max())
        # and again: the array keeps the previous call's contents
        got2 = _run(fmm, batch, "fmm_m2l_batched_static", mp, loc0)
        assert torch.equal(got2, ref)
        batch.close()
    plan.close()


def test_static_scratch_rejects_large_batches(gpu_lib):
    """A batch whose partials exceed the fixed array is refused before anything is enqueued."""
    fmm = gpu_lib
    from paper_2305_17867_amd import _lib
    pts = W.uniform_points(1 << 14, 32)
    tr = W.uniform_tree(pts, 4)
    d = fmm.Desc("laplace", 12, "f64")
    plan = fmm.Plan(d, [tr.box_size(l) for l in range(tr.n_levels)])
    t, s = W.interaction_pairs(tr, [4])
    # many parts per tile: thousands of items, each with FP64 partials of its tile
    batch = plan.prepare(t, s, tr.ijk, tr.level, tuning={"form": "tiled", "target_items": 8192})
    assert batch.info()["scratch_bytes"] > (16 << 20)
    mp = torch.zeros((tr.n_box, d.nc), dtype=torch.float64, device="cuda")
    st = _lib.load().fmm_m2l_batched_static(batch._h, C.c_void_p(mp.data_ptr()), C.c_void_p(mp.data_ptr()), None)
    assert st == _lib.FMM_EUNSUPPORTED
    assert b"static array" in _lib.load().fmm_last_error()
    batch.close()
    plan.close()
