"""GPU parity: every entry point of the C ABI against the CPU oracle on seeded inputs.

Tolerances (normwise relative l2 over the whole output array unless stated):
  FP64 / complex128: 1e-12 (P2M, M2L, L2P, direct, end to end); derivative tables 1e-13.
  FP32 / complex64: P2M and L2P 2e-6, direct 1e-5 (700-term sums), M2L 2e-5 (FP32 products of
  entries that span many orders of magnitude, FP64 accumulation across offset groups).
Derivative tables and M2L outputs are checked per derivative order |i| (the normwise error over
each order on its own), so that the small low-order coefficients are held to the same relative
bound as the large high-order ones; M2L is fed both unit-variance multipoles and multipoles
with the decay of physical ones.  The derivative tables are compared with the mpmath (50-digit)
radial product formula, which shares no step with the recurrences of the GPU tables.
"""
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import compressed as Z
from oracle import kernels as K
from oracle import multiindex as MI

from helpers import (decaying_multipoles, oracle_m2l_scaled, oracle_scaled_table, per_order_rel, perm_to_lib, rel,
                     tree_inputs)

pytestmark = pytest.mark.gpu

CASES = {  # kernel -> (param, real dtype, complex?)
    "laplace": 0.0, "yukawa": 2.0, "helmholtz": 1.0, "biharmonic": 0.0}


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def desc_for(fmm, kernel, p, single, param=None):
    cplx = kernel == "helmholtz"
    dt = ("c64" if single else "c128") if cplx else ("f32" if single else "f64")
    return fmm.Desc(kernel, p, dt, CASES[kernel] if param is None else param)


# ----------------------------------------------------------------------------- derivative tables

# offsets of the interaction list, including ones on and near the coordinate axes, where the
# radial product formula's terms cancel most
DERIV_OFFSETS = [(2, 0, 0), (0, 0, 3), (0, -2, 0), (3, 3, 3), (2, -3, 1), (-3, 1, -2), (2, 2, 0), (-1, 3, -3),
                 (0, 2, -3), (3, -2, 2)]


@pytest.mark.parametrize("kernel,param,p,h", [
    ("laplace", 0.0, 8, 1 / 16), ("laplace", 0.0, 12, 1 / 16), ("yukawa", 2.0, 8, 1 / 16),
    ("yukawa", 2.0, 12, 1 / 4), ("helmholtz", 16.0, 8, 1 / 16), ("helmholtz", 16.0, 12, 1 / 16),
    ("helmholtz", 1.0, 6, 1.0), ("biharmonic", 0.0, 8, 1 / 8), ("biharmonic", 0.0, 12, 1 / 8)])
def test_deriv_tables(gpu_lib, kernel, param, p, h):
    """GPU tables (Taylor-coefficient recurrences in FP64) against the mpmath tables of the
    radial product formula (Sec. 4.4, eq. tausch-dist-derivatives), per derivative order."""
    fmm = gpu_lib
    d = fmm.Desc(kernel, p, "c128" if kernel == "helmholtz" else "f64", param)
    offs = np.array(DERIV_OFFSETS, dtype=np.float64)
    got = host(fmm.deriv_tables(d, dev(offs, torch.float64), dev(np.full(len(offs), h), torch.float64)))
    for k, o in enumerate(DERIV_OFFSETS):
        ref = oracle_scaled_table(kernel, param, p, o, h, True)
        for n in range(2 * p + 1):
            ms = [m for m in ref if sum(m) == n]
            a = np.array([got[k][m[2], m[0], m[1]] for m in ms])
            b = np.array([ref[m] for m in ms])
            assert rel(a, b) < 1e-13, (o, n, rel(a, b))
        # unused corner (|m| > 2p) is zero
        assert got[k][0, 2 * p, 2 * p] == 0


# ----------------------------------------------------------------------------- P2M / L2P

def small_tree(seed=3, complex_w=False):
    tr, w = tree_inputs(1 << 13, 3, seed, complex_w=complex_w)
    return tr, w


@pytest.mark.parametrize("kernel", list(CASES))
@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("p", [0, 4, 8])
def test_p2m(gpu_lib, kernel, single, p):
    fmm = gpu_lib
    d = desc_for(fmm, kernel, p, single)
    tr, w = small_tree(complex_w=kernel == "helmholtz")
    param = CASES[kernel]
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    plan = fmm.Plan(d, lh)
    # boxes of levels 2 and 3 in one call (different h), plus an empty and a one-point range
    boxes = np.concatenate([tr.boxes_at(2), tr.boxes_at(3)])
    rng = tr.pt_range[boxes].copy()
    rng[3] = [rng[3][0], rng[3][0]]
    rng[5] = [rng[5][0], rng[5][0] + 1]
    rd = d.real_dtype
    out = plan.p2m(dev(tr.center[boxes], torch.float64), dev(tr.level[boxes], torch.int32),
                   dev(rng, torch.int64), dev(tr.points, rd), dev(w, d.value_dtype))
    got = host(out)[:, :]
    perm = perm_to_lib(kernel, param, p, d.index_table())
    ref = []
    for k, b in enumerate(boxes):
        lo, hi = rng[k]
        beta = Z.p2m(kernel, param, p, tr.center[b], tr.points[lo:hi], w[lo:hi])
        ref.append(Z.scale_multipole(kernel, param, p, beta, 1.0 / lh[tr.level[b]])[perm])
    ref = np.array(ref)
    assert np.all(got[3] == 0)
    tol = 2e-6 if single else 1e-12
    assert rel(got, ref) < tol, rel(got, ref)


@pytest.mark.parametrize("kernel", list(CASES))
@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("p", [0, 5, 8])
def test_l2p(gpu_lib, kernel, single, p):
    fmm = gpu_lib
    d = desc_for(fmm, kernel, p, single)
    tr, _ = small_tree(seed=4)
    param = CASES[kernel]
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    plan = fmm.Plan(d, lh)
    boxes = tr.boxes_at(3)
    nc = d.nc
    g = np.random.Generator(np.random.PCG64(11))
    theta = g.standard_normal((len(boxes), nc))
    if kernel == "helmholtz":
        theta = theta + 1j * g.standard_normal((len(boxes), nc))
    pot0 = g.standard_normal(tr.points.shape[0])
    if kernel == "helmholtz":
        pot0 = pot0 + 0j
    pot = dev(pot0, d.value_dtype)
    plan.l2p(dev(tr.center[boxes], torch.float64), dev(tr.level[boxes], torch.int32),
             dev(tr.pt_range[boxes], torch.int64), dev(tr.points, d.real_dtype),
             dev(theta, d.value_dtype), pot)
    got = host(pot) - pot0
    perm = perm_to_lib(kernel, param, p, d.index_table())
    inv = np.argsort(perm)
    th_or = theta[:, inv]  # oracle kept order
    ref = np.zeros_like(pot0)
    for k, b in enumerate(boxes):
        lo, hi = tr.pt_range[b]
        th = Z.unscale_local(kernel, param, p, th_or[k], 1.0 / lh[3])
        ref[lo:hi] += Z.l2p(kernel, param, p, tr.center[b], th, tr.points[lo:hi])
    tol = 2e-6 if single else 1e-12
    assert rel(got, ref) < tol, rel(got, ref)


# ----------------------------------------------------------------------------- M2L

M2L_CASES = [("laplace", 8, False), ("laplace", 8, True), ("laplace", 12, False), ("yukawa", 6, True),
             ("biharmonic", 6, False), ("helmholtz", 6, False), ("helmholtz", 4, True),
             ("laplace", 16, False), ("biharmonic", 12, True)]


@pytest.fixture(scope="module")
def m2l_tree():
    pts = W.uniform_points(4096, 7)
    return W.uniform_tree(pts, 3)


def _multipoles(kind, kernel, index_table, n_box, seed):
    """Unit-variance or physically decaying scaled multipoles (complex for Helmholtz)."""
    g = np.random.Generator(np.random.PCG64(seed))
    if kind == "unit":
        beta = g.standard_normal((n_box, len(index_table)))
        if kernel == "helmholtz":
            beta = beta + 1j * g.standard_normal((n_box, len(index_table)))
    else:
        beta = decaying_multipoles(index_table, n_box, seed)
        if kernel == "helmholtz":
            beta = beta + 1j * decaying_multipoles(index_table, n_box, seed + 1)
    return beta


def assert_per_order(got, ref, index_table, tol, what):
    errs = per_order_rel(got, ref, index_table)
    worst = max(errs, key=errs.get)
    assert errs[worst] < tol, (what, "order", worst, errs[worst])


@pytest.mark.parametrize("kernel,p,single", M2L_CASES)
@pytest.mark.parametrize("items", [1, 4096])
def test_m2l(gpu_lib, m2l_tree, kernel, p, single, items, monkeypatch):
    fmm = gpu_lib
    monkeypatch.setenv("FMM_M2L_ITEMS", str(items))
    monkeypatch.setenv("FMM_M2LS_WG", str(items))  # streaming form: one workgroup, or many with split tiles
    tr = m2l_tree
    param = CASES[kernel]
    d = desc_for(fmm, kernel, p, single)
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    plan = fmm.Plan(d, lh)
    levels = [3] if p >= 12 else [2, 3]
    t, s = W.interaction_pairs(tr, levels)
    batch = plan.prepare(t, s, tr.ijk, tr.level)
    info = batch.info()
    assert info["n_pair"] == len(t)
    it = d.index_table()
    perm = perm_to_lib(kernel, param, p, it)
    inv = np.argsort(perm)
    tol = 2e-5 if single else 1e-12
    for kind, seed in (("unit", 21), ("decaying", 22)):
        beta = _multipoles(kind, kernel, it, tr.n_box, seed)
        g = np.random.Generator(np.random.PCG64(seed + 100))
        loc0 = g.standard_normal(beta.shape) + (1j * g.standard_normal(beta.shape) if kernel == "helmholtz" else 0)
        mp = dev(beta, d.value_dtype)
        loc = dev(loc0, d.value_dtype)
        batch(mp, loc)
        got = host(loc) - host(dev(loc0, d.value_dtype))
        ref = oracle_m2l_scaled(kernel, param, p, tr.ijk.astype(np.int64), tr.level, lh, t, s, beta[:, inv])
        ref = ref[:, perm]
        targets = np.unique(t)
        assert rel(got, ref) < tol, (kind, rel(got, ref))
        assert_per_order(got[targets], ref[targets], it, tol, kind)
        # deterministic: a second launch on the same input gives bit-identical output
        loc2 = dev(loc0, d.value_dtype)
        batch(mp, loc2)
        assert np.array_equal(host(loc2), host(loc))


# each kernel once with mpmath derivative tables (a few offsets, so that the 50-digit tables stay
# cheap): the M2L output against the oracle's dense T~ built from the mpmath tables, per order,
# in the streaming and the tiled form
MP_CASES = [("laplace", 8, "f64"), ("yukawa", 8, "f64"), ("helmholtz", 6, "c128"), ("biharmonic", 8, "f64"),
            ("laplace", 12, "f64")]


@pytest.mark.parametrize("kernel,p,dt", MP_CASES)
@pytest.mark.parametrize("form", ["stream", "tiled"])
def test_m2l_against_mpmath_tables(gpu_lib, m2l_tree, kernel, p, dt, form):
    fmm = gpu_lib
    tr = m2l_tree
    param = CASES[kernel]
    d = fmm.Desc(kernel, p, dt, param)
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    plan = fmm.Plan(d, lh)
    t, s = W.interaction_pairs(tr, [3])
    off = tr.ijk[t] - tr.ijk[s]
    keep = np.zeros(len(t), bool)
    for o in DERIV_OFFSETS[:6]:
        keep |= np.all(off == np.array(o), axis=1)
    t, s = t[keep], s[keep]
    assert len(np.unique(tr.ijk[t] - tr.ijk[s], axis=0)) == 6
    if form == "stream":
        tun = {"form": "stream", "workgroups": 4}
    else:
        tun = {"form": "tiled"}
    try:
        batch = plan.prepare(t, s, tr.ijk, tr.level, tuning=tun)
    except fmm._lib.FmmError as e:
        assert form == "stream" and e.status == fmm._lib.FMM_EUNSUPPORTED
        pytest.skip(f"streaming form not instantiated for {kernel} p={p} {dt}")
    it = d.index_table()
    perm = perm_to_lib(kernel, param, p, it)
    inv = np.argsort(perm)
    for kind, seed in (("unit", 31), ("decaying", 32)):
        beta = _multipoles(kind, kernel, it, tr.n_box, seed)
        loc = torch.zeros((tr.n_box, d.nc), dtype=d.value_dtype, device="cuda")
        batch(dev(beta, d.value_dtype), loc)
        ref = oracle_m2l_scaled(kernel, param, p, tr.ijk.astype(np.int64), tr.level, lh, t, s, beta[:, inv],
                                mp=True)[:, perm]
        targets = np.unique(t)
        assert_per_order(host(loc)[targets], ref[targets], it, 1e-12, kind)


# tiled launch shapes (rows per wavefront, column tiles per wavefront, column groups) with at
# most two row groups, so that three K ranges still fit the eight wavefronts of a workgroup
KSPLIT_CASES = [("laplace", 8, False, (3, 2, 1)), ("laplace", 8, True, (3, 2, 1)), ("helmholtz", 6, False, (2, 1, 1)),
                ("biharmonic", 8, True, (4, 1, 1)), ("yukawa", 10, True, (4, 1, 1)), ("laplace", 6, False, (3, 1, 2))]


@pytest.mark.parametrize("kernel,p,single,shape", KSPLIT_CASES)
@pytest.mark.parametrize("nks", [2, 3])
@pytest.mark.parametrize("items", [None, 4096])
def test_m2l_k_split(gpu_lib, m2l_tree, kernel, p, single, shape, nks, items):
    """Contraction split over several wavefronts of a workgroup (fmm_m2l_tuning.k_splits),
    against the oracle at the M2L tolerance, with and without split tiles."""
    fmm = gpu_lib
    tr = m2l_tree
    param = CASES[kernel]
    d = desc_for(fmm, kernel, p, single)
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    plan = fmm.Plan(d, lh)
    t, s = W.interaction_pairs(tr, [3])
    rt, ct, ncg = shape
    tun = dict(rows_per_wave=rt, col_tiles_per_wave=ct, col_groups=ncg, lds_buffers=1, k_splits=nks)
    if items:
        tun["target_items"] = items
    batch = plan.prepare(t, s, tr.ijk, tr.level, tuning=tun)
    assert batch.info()["k_splits"] == nks and batch.info()["stream_form"] == 0
    it = d.index_table()
    perm = perm_to_lib(kernel, param, p, it)
    inv = np.argsort(perm)
    tol = 2e-5 if single else 1e-12
    targets = np.unique(t)
    for kind, seed in (("unit", 23), ("decaying", 24)):
        beta = _multipoles(kind, kernel, it, tr.n_box, seed)
        mp = dev(beta, d.value_dtype)
        loc = torch.zeros_like(mp)
        batch(mp, loc)
        ref = oracle_m2l_scaled(kernel, param, p, tr.ijk.astype(np.int64), tr.level, lh, t, s, beta[:, inv])[:, perm]
        assert rel(host(loc), ref) < tol, (kind, rel(host(loc), ref))
        assert_per_order(host(loc)[targets], ref[targets], it, tol, kind)


def test_m2l_empty_and_validation(gpu_lib):
    fmm = gpu_lib
    d = fmm.Desc("laplace", 4, "f64")
    plan = fmm.Plan(d, [1.0, 0.5])
    b = plan.prepare(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((2, 3), np.int32),
                     np.zeros(2, np.int32))
    z = torch.zeros((2, d.nc), dtype=torch.float64, device="cuda")
    b(z, z)
    with pytest.raises(fmm._lib.FmmError):
        plan.prepare([0], [1], [[0, 0, 0], [1, 0, 0]], [1, 0])  # different levels
    with pytest.raises(fmm._lib.FmmError):
        plan.prepare([0], [0], [[0, 0, 0]], [0])  # zero offset
    with pytest.raises(fmm._lib.FmmError):
        plan.prepare([0, 0], [1, 1], [[0, 0, 0], [2, 0, 0]], [0, 0])  # duplicate pair


# ----------------------------------------------------------------------------- direct, end to end

@pytest.mark.parametrize("kernel", list(CASES))
@pytest.mark.parametrize("single", [False, True])
def test_direct(gpu_lib, kernel, single):
    fmm = gpu_lib
    d = desc_for(fmm, kernel, 2, single)
    g = np.random.Generator(np.random.PCG64(2))
    src = g.random((700, 3))
    tgt = np.concatenate([g.random((300, 3)), src[:5]])  # includes coincident points
    w = W.normal_weights(700, 4, complex_=kernel == "helmholtz")
    got = host(fmm.direct(d, dev(src, d.real_dtype), dev(w, d.value_dtype), dev(tgt, d.real_dtype)))
    ref = K.direct_sum(kernel, CASES[kernel], src, w, tgt)
    tol = 1e-5 if single else 1e-12
    assert rel(got, ref) < tol


def test_end_to_end_two_box_laplace_p4(gpu_lib):
    """64 sources in [-0.5,0.5]^3, 64 targets in the unit box at (3,0,0), Laplace p=4, FP64."""
    fmm = gpu_lib
    src, tgt, w, c1, c2 = W.small_two_box(0)
    p = 4
    d = fmm.Desc("laplace", p, "f64")
    plan = fmm.Plan(d, [1.0])
    cen = np.array([c1, c2])
    lev = np.zeros(2, np.int32)
    rng_s = np.array([[0, 64], [0, 0]])
    mp = plan.p2m(dev(cen, torch.float64), dev(lev, torch.int32), dev(rng_s, torch.int64),
                  dev(src, torch.float64), dev(w, torch.float64))
    batch = plan.prepare([1], [0], [[0, 0, 0], [3, 0, 0]], [0, 0])
    loc = torch.zeros_like(mp)
    batch(mp, loc)
    pot = torch.zeros(64, dtype=torch.float64, device="cuda")
    plan.l2p(dev(cen[1:], torch.float64), dev(lev[1:], torch.int32), dev(np.array([[0, 64]]), torch.int64),
             dev(tgt, torch.float64), loc[1:].contiguous(), pot)
    got = host(pot)
    beta = Z.p2m("laplace", 0.0, p, c1, src, w)
    th = Z.m2l("laplace", 0.0, p, c2 - c1, beta)
    ref = Z.l2p("laplace", 0.0, p, c2, th, tgt)
    assert rel(got, ref) < 1e-12
    exact = K.direct_sum("laplace", 0.0, src, w, tgt)
    e = rel(got, exact)
    assert 1e-5 < e < 1e-3  # the truncation error of p = 4, not roundoff


def test_bound_launches_match_calls(gpu_lib, m2l_tree):
    """Plan.bind_p2m / bind_l2p and Batch.bind enqueue the same work as the plain calls."""
    fmm = gpu_lib
    tr = m2l_tree
    d = fmm.Desc("laplace", 6, "f64")
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    plan = fmm.Plan(d, lh)
    boxes = tr.boxes_at(3)
    cen, lev, rng = dev(tr.center[boxes], torch.float64), dev(tr.level[boxes], torch.int32), dev(tr.pt_range[boxes], torch.int64)
    pts = dev(tr.points, torch.float64)
    w = dev(W.normal_weights(tr.points.shape[0], 5), torch.float64)
    a = plan.p2m(cen, lev, rng, pts, w)
    b = torch.zeros_like(a)
    plan.bind_p2m(cen, lev, rng, pts, w, b)()
    assert torch.equal(a, b)
    t, s = W.interaction_pairs(tr, [3])
    batch = plan.prepare(t, s, tr.ijk, tr.level)
    mp = torch.randn((tr.n_box, d.nc), dtype=torch.float64, device="cuda")
    l1, l2 = torch.zeros_like(mp), torch.zeros_like(mp)
    batch(mp, l1)
    batch.bind(mp, l2)()
    assert torch.equal(l1, l2)
    th = torch.randn((len(boxes), d.nc), dtype=torch.float64, device="cuda")
    p1 = torch.zeros(tr.points.shape[0], dtype=torch.float64, device="cuda")
    p2 = torch.zeros_like(p1)
    plan.l2p(cen, lev, rng, pts, th, p1)
    plan.bind_l2p(cen, lev, rng, pts, th, p2)()
    assert torch.equal(p1, p2)


@pytest.mark.parametrize("kernel", ["laplace", "biharmonic", "yukawa"])
@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("p", [3, 8, 12])
def test_p2m_several_boxes_per_workgroup(gpu_lib, kernel, single, p):
    """Real P2M of boxes that are not split takes several boxes per workgroup: boxes of
    different sizes (empty, one point, one tile, a tile and one more point, several tiles) and
    levels share workgroups, and the number of boxes is not a multiple of the boxes per
    workgroup.  Every box is checked on its own against the oracle, per derivative order."""
    fmm = gpu_lib
    tr, w = tree_inputs(1 << 15, 3, 21)
    d = desc_for(fmm, kernel, p, single)
    param = CASES[kernel]
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    plan = fmm.Plan(d, lh)
    l2, l3 = tr.boxes_at(2), tr.boxes_at(3)
    sizes = [300, 0, 1, 129, 256, 17, 5, 511, 128, 127, 255, 257, 64]
    boxes = np.array([l2[i] if s > 64 or i % 2 else l3[i] for i, s in enumerate(sizes)])
    rng = tr.pt_range[boxes].copy()
    for k, s in enumerate(sizes):
        rng[k, 1] = rng[k, 0] + min(s, rng[k, 1] - rng[k, 0])
    got = host(plan.p2m(dev(tr.center[boxes], torch.float64), dev(tr.level[boxes], torch.int32),
                        dev(rng, torch.int64), dev(tr.points, d.real_dtype), dev(w, d.value_dtype)))
    perm = perm_to_lib(kernel, param, p, d.index_table())
    orders = np.array([sum(m) for m in d.index_table()])
    tol = (2e-6 if p <= 8 else 1e-5) if single else 1e-12
    assert np.all(got[1] == 0)
    for k, b in enumerate(boxes):
        lo, hi = rng[k]
        if hi == lo:
            continue
        beta = Z.p2m(kernel, param, p, tr.center[b], tr.points[lo:hi], w[lo:hi])
        ref = Z.scale_multipole(kernel, param, p, beta, 1.0 / lh[tr.level[b]])[perm]
        assert rel(got[k], ref) < tol, (k, hi - lo, rel(got[k], ref))
        for n in range(p + 1):
            sel = orders == n
            assert rel(got[k][sel], ref[sel]) < 50 * tol, (k, n, rel(got[k][sel], ref[sel]))


@pytest.mark.parametrize("kernel,single", [("laplace", False), ("helmholtz", False), ("yukawa", True)])
def test_p2m_large_boxes_split_over_workgroups(gpu_lib, kernel, single):
    """Boxes with tens of thousands of points are spread over several workgroups whose results
    are added in chunk order; the multipoles still match the oracle."""
    fmm = gpu_lib
    pts = W.uniform_points(200_000, 12)
    tr = W.uniform_tree(pts, 2)
    p = 8
    d = desc_for(fmm, kernel, p, single)
    param = CASES[kernel]
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    plan = fmm.Plan(d, lh)
    boxes = tr.boxes_at(1)  # 8 boxes of ~25,000 points
    w = W.normal_weights(tr.points.shape[0], 13, complex_=kernel == "helmholtz")
    got = host(plan.p2m(dev(tr.center[boxes], torch.float64), dev(tr.level[boxes], torch.int32),
                        dev(tr.pt_range[boxes], torch.int64), dev(tr.points, d.real_dtype), dev(w, d.value_dtype)))
    perm = perm_to_lib(kernel, param, p, d.index_table())
    ref = []
    for b in boxes[:3]:
        lo, hi = tr.pt_range[b]
        beta = Z.p2m(kernel, param, p, tr.center[b], tr.points[lo:hi], w[lo:hi])
        ref.append(Z.scale_multipole(kernel, param, p, beta, 1.0 / lh[1])[perm])
    tol = 2e-6 if single else 1e-12
    assert rel(got[:3], np.array(ref)) < tol, rel(got[:3], np.array(ref))
