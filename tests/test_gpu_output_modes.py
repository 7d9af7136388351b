"""GPU: the output modes of fmm_m2l_batched_ex and fmm_l2p_ex.  FMM_OVERWRITE stores into the
targets' rows (M2L) or the targets' potentials (L2P) and leaves every other entry unchanged;
the stored values are bit for bit those of accumulating into zeroed arrays, and storing twice
gives the same arrays again.  The tiled and FFT M2L forms refuse FMM_OVERWRITE."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

CASES = [("laplace", 8, "f64", 0.0), ("laplace", 8, "f32", 0.0), ("helmholtz", 6, "c128", 1.0),
         ("biharmonic", 8, "f64", 0.0)]


def setup(fmm, kernel, p, dt, param):
    tr = W.uniform_tree(W.uniform_points(4096, 41), 3)
    d = fmm.Desc(kernel, p, dt, param)
    plan = fmm.Plan(d, [tr.box_size(l) for l in range(tr.n_levels)])
    return tr, d, plan


def coeffs(d, n_box, seed, fill=None):
    g = np.random.Generator(np.random.PCG64(seed))
    x = g.standard_normal((n_box, d.nc)) if fill is None else np.full((n_box, d.nc), fill)
    if d.value_dtype.is_complex:
        x = x + 1j * (g.standard_normal((n_box, d.nc)) if fill is None else fill)
    return torch.as_tensor(x).to(device="cuda", dtype=d.value_dtype)


@pytest.mark.parametrize("kernel,p,dt,param", CASES)
@pytest.mark.parametrize("workgroups", [None, 48])
def test_m2l_overwrite_matches_accumulating_into_zeros(gpu_lib, kernel, p, dt, param, workgroups):
    """workgroups = 48: chunk boundaries cut target tiles, so the split-tile finisher stores too."""
    fmm = gpu_lib
    tr, d, plan = setup(fmm, kernel, p, dt, param)
    t, s = W.interaction_pairs(tr, [2, 3])
    tun = {"form": "stream"}
    if workgroups:
        tun["workgroups"] = workgroups
    batch = plan.prepare(t, s, tr.ijk, tr.level, tuning=tun)
    assert batch.info()["stream_form"] == 1
    mp = coeffs(d, tr.n_box, 42)
    ref = torch.zeros_like(mp)
    batch(mp, ref)
    before = coeffs(d, tr.n_box, 0, fill=7.0)
    got = before.clone()
    batch(mp, got, overwrite=True)
    targets = np.unique(t)
    others = np.setdiff1d(np.arange(tr.n_box), targets)
    assert torch.equal(got[targets], ref[targets])
    assert torch.equal(got[others], before[others])
    bound = batch.bind(mp, got, overwrite=True)
    bound()  # storing again gives the same rows
    assert torch.equal(got[targets], ref[targets])
    tiled = plan.prepare(t, s, tr.ijk, tr.level, tuning={"form": "tiled"})
    with pytest.raises(fmm._lib.FmmError) as e:
        tiled(mp, got, overwrite=True)
    assert e.value.status == fmm._lib.FMM_EUNSUPPORTED


@pytest.mark.parametrize("kernel,p,dt,param", CASES)
def test_l2p_overwrite_matches_accumulating_into_zeros(gpu_lib, kernel, p, dt, param):
    """The call covers every other leaf: their points are stored, the rest keep their values."""
    fmm = gpu_lib
    tr, d, plan = setup(fmm, kernel, p, dt, param)
    leaves = tr.boxes_at(3)[::2]
    center = torch.as_tensor(tr.center[leaves], dtype=torch.float64, device="cuda")
    level = torch.as_tensor(tr.level[leaves], dtype=torch.int32, device="cuda")
    rng = torch.as_tensor(tr.pt_range[leaves], dtype=torch.int64, device="cuda")
    pts = torch.as_tensor(tr.points, device="cuda", dtype=d.real_dtype)
    loc = coeffs(d, len(leaves), 43) * 1e-2
    ref = torch.zeros(len(pts), dtype=d.value_dtype, device="cuda")
    plan.l2p(center, level, rng, pts, loc, ref)
    before = torch.full_like(ref, 5.0)
    got = before.clone()
    plan.l2p(center, level, rng, pts, loc, got, overwrite=True)
    inside = np.zeros(len(pts), dtype=bool)
    for b in leaves:
        inside[slice(*tr.pt_range[b])] = True
    ins = torch.as_tensor(inside, device="cuda")
    assert torch.equal(got[ins], ref[ins])
    assert torch.equal(got[~ins], before[~ins])
    plan.l2p(center, level, rng, pts, loc, got, overwrite=True)
    assert torch.equal(got[ins], ref[ins])
