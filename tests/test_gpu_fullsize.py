"""GPU parity at the full workload sizes, in the launch configuration the benchmark times,
checked on sampled outputs that the oracle computes one by one.

Workloads (recipes in the workloads module, seeds below):
  uniform   2^20 uniform points, depth-4 octree, level-4 List-2 pairs (584,136), Laplace
            p = 8 and 12, FP64 and FP32 (the benchmark's workload and launch shapes).
  plummer   2^21 Plummer points (a = 0.1), adaptive octree <= 64 per leaf, complex weights,
            Helmholtz p = 12 with k = 1 / (largest leaf side), List-2 pairs of every level in one
            prepared batch, complex128 and complex64.
  mixture   2^19 points from 4 Gaussians (sigma 0.05), adaptive <= 64, Yukawa (lambda = 2) and
            biharmonic with p(l) = 6 + 2 ((l - 2) mod 3), FP32, the six batches as one multi
            launch (tuned per-(kernel, order) shapes, or one shared tiled shape drained by one
            persistent launch) captured in a HIP graph.
  gradient  2^21 sources and 2^21 targets uniform, depth-4 octrees, Laplace p = 10: the far field
            and its adjoint (d L / d weights, source and target positions).

Inputs to each operator are seeded arrays (never outputs of the GPU path).  Tolerances are the
per-operator ones (normwise relative over the sampled rows): FP64 / complex128 1e-12; FP32
P2M and L2P 2e-6 up to p = 8 and 1e-5 above (every moment X^q / q! is a product of |q| rounded
factors, so the FP32 error grows with the order: about |q| + log2(points per box) roundings of
6e-8 before the compression sums), M2L 2e-5; complex64 Helmholtz p = 12 M2L 1e-4 (products of
entries that span many orders of magnitude).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import compressed as Z

from helpers import decaying_multipoles, oracle_m2l_scaled, per_order_rel, perm_to_lib, rel

pytestmark = pytest.mark.gpu


def tol_pts(single, p):
    """P2M / L2P tolerance (see the module docstring)."""
    return (2e-6 if p <= 8 else 1e-5) if single else 1e-12


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def pick(seed, arr, k):
    g = np.random.Generator(np.random.PCG64(seed))
    arr = np.asarray(arr)
    return np.sort(g.choice(arr, size=min(k, len(arr)), replace=False))


def check_p2m(fmm, plan, kernel, param, p, tr, boxes, w, seed, tol, n_sample=4):
    """P2M of every box in `boxes` (one launch), sampled rows against the oracle."""
    d = plan.desc
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    out = plan.p2m(dev(tr.center[boxes], torch.float64), dev(tr.level[boxes], torch.int32),
                   dev(tr.pt_range[boxes], torch.int64), dev(tr.points, d.real_dtype), dev(w, d.value_dtype))
    got = host(out)
    perm = perm_to_lib(kernel, param, p, d.index_table())
    sel = pick(seed, np.arange(len(boxes)), n_sample)
    ref = []
    for k in sel:
        b = boxes[k]
        lo, hi = tr.pt_range[b]
        h = lh[tr.level[b]]
        beta = Z.p2m(kernel, param, p, tr.center[b], tr.points[lo:hi], w[lo:hi])
        ref.append(Z.scale_multipole(kernel, param, p, beta, 1.0 / h)[perm])
    err = rel(got[sel], np.array(ref))
    assert err < tol, ("p2m", err)


def check_l2p(fmm, plan, kernel, param, p, tr, boxes, seed, tol, cplx, n_sample=4):
    """L2P of seeded locals at every box in `boxes`, sampled boxes' points against the oracle."""
    d = plan.desc
    nc = d.nc
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    g = np.random.Generator(np.random.PCG64(seed))
    theta = g.standard_normal((len(boxes), nc))
    if cplx:
        theta = theta + 1j * g.standard_normal((len(boxes), nc))
    pot = torch.zeros(tr.points.shape[0], dtype=d.value_dtype, device="cuda")
    plan.l2p(dev(tr.center[boxes], torch.float64), dev(tr.level[boxes], torch.int32),
             dev(tr.pt_range[boxes], torch.int64), dev(tr.points, d.real_dtype), dev(theta, d.value_dtype), pot)
    got = host(pot)
    perm = perm_to_lib(kernel, param, p, d.index_table())
    inv = np.argsort(perm)
    sel = pick(seed + 1, np.arange(len(boxes)), n_sample)
    got_s, ref_s = [], []
    for k in sel:
        b = boxes[k]
        lo, hi = tr.pt_range[b]
        th = Z.unscale_local(kernel, param, p, theta[k][inv], 1.0 / lh[tr.level[b]])
        ref_s.append(Z.l2p(kernel, param, p, tr.center[b], th, tr.points[lo:hi]))
        got_s.append(got[lo:hi])
    err = rel(np.concatenate(got_s), np.concatenate(ref_s))
    assert err < tol, ("l2p", err)


def check_m2l(plan, kernel, param, p, tr, t, s, batch, seed, tol, cplx, targets):
    """Batched M2L of seeded multipoles over all pairs (unit-variance ones, then ones with the
    decay of physical multipoles); the sampled targets against the oracle, normwise and per
    derivative order."""
    d = plan.desc
    nc = d.nc
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    it = d.index_table()
    perm = perm_to_lib(kernel, param, p, it)
    inv = np.argsort(perm)
    m = np.isin(t, targets)
    for kind in ("unit", "decaying"):
        if kind == "unit":
            g = np.random.Generator(np.random.PCG64(seed))
            beta = g.standard_normal((tr.n_box, nc))
            if cplx:
                beta = beta + 1j * g.standard_normal((tr.n_box, nc))
        else:
            beta = decaying_multipoles(it, tr.n_box, seed + 1)
            if cplx:
                beta = beta + 1j * decaying_multipoles(it, tr.n_box, seed + 2)
        mp = dev(beta, d.value_dtype)
        loc = torch.zeros_like(mp)
        batch(mp, loc)
        got = host(loc)[targets]
        ref = oracle_m2l_scaled(kernel, param, p, tr.ijk.astype(np.int64), tr.level, lh, t[m], s[m],
                                beta[:, inv])[targets][:, perm]
        err = rel(got, ref)
        assert err < tol, ("m2l", kind, err)
        errs = per_order_rel(got, ref, it)
        worst = max(errs, key=errs.get)
        assert errs[worst] < tol, ("m2l per order", kind, worst, errs[worst])


# ----------------------------------------------------------------------------- uniform (benchmark)

@pytest.fixture(scope="module")
def uniform():
    pts = W.uniform_points(1 << 20, 1)
    tr = W.uniform_tree(pts, 4)
    w = W.normal_weights(1 << 20, 2)
    t, s = W.interaction_pairs(tr, [4])
    return tr, w, t, s


@pytest.mark.parametrize("p,dt", [(8, "f64"), (8, "f32"), (12, "f64"), (12, "f32")])
def test_uniform_full_size(gpu_lib, uniform, p, dt):
    fmm = gpu_lib
    tr, w, t, s = uniform
    single = dt == "f32"
    plan = fmm.Plan(fmm.Desc("laplace", p, dt), [tr.box_size(l) for l in range(tr.n_levels)])
    leaves = tr.boxes_at(4)
    check_p2m(fmm, plan, "laplace", 0.0, p, tr, leaves, w, 10 + p, tol_pts(single, p))
    batch = plan.prepare(t, s, tr.ijk, tr.level)  # the benchmark's (tuned) launch shape
    check_m2l(plan, "laplace", 0.0, p, tr, t, s, batch, 20 + p, 2e-5 if single else 1e-12, False,
              pick(30 + p, leaves, 3))
    check_l2p(fmm, plan, "laplace", 0.0, p, tr, leaves, 40 + p, tol_pts(single, p), False)


_E2E_REF = {}


def _oracle_far_potential(p, tr, w, t, s, leaf):
    """The oracle's far-field potential at the points of target leaf `leaf` from its List-2
    sources: uncompressed geometry, compressed P2M of each source box, M2L by the translation
    vector of the pair, L2P (Secs. 3.3, 3.4, 4.1)."""
    key = (p, int(leaf))
    if key not in _E2E_REF:
        theta = 0.0
        for sb in s[t == leaf]:
            lo, hi = tr.pt_range[sb]
            beta = Z.p2m("laplace", 0.0, p, tr.center[sb], tr.points[lo:hi], w[lo:hi])
            theta = theta + Z.m2l("laplace", 0.0, p, tr.center[leaf] - tr.center[sb], beta)
        lo, hi = tr.pt_range[leaf]
        _E2E_REF[key] = Z.l2p("laplace", 0.0, p, tr.center[leaf], theta, tr.points[lo:hi])
    return _E2E_REF[key]


@pytest.mark.parametrize("p,dt", [(8, "f64"), (8, "f32"), (12, "f64"), (12, "f32")])
def test_uniform_end_to_end_potential(gpu_lib, uniform, p, dt):
    """P2M of every leaf -> batched M2L of level 4 -> L2P at every point, in the benchmark's
    launch shapes; the potential at the points of sampled target leaves against the oracle's
    P2M -> M2L -> L2P over the same List-2 pairs.  FP64 at 1e-12; FP32 (FP32 points, weights,
    products and potentials) at 2e-5, the FP32 M2L bound."""
    fmm = gpu_lib
    tr, w, t, s = uniform
    single = dt == "f32"
    d = fmm.Desc("laplace", p, dt)
    plan = fmm.Plan(d, [tr.box_size(l) for l in range(tr.n_levels)])
    leaves = tr.boxes_at(4)
    l0, nl = int(leaves[0]), len(leaves)
    assert np.array_equal(leaves, np.arange(l0, l0 + nl))  # leaves are one contiguous box range
    rd, vd = d.real_dtype, d.value_dtype
    cen = dev(tr.center[leaves], torch.float64)
    lev = dev(tr.level[leaves], torch.int32)
    rng = dev(tr.pt_range[leaves], torch.int64)
    pts = dev(tr.points, rd)
    mp = torch.zeros((tr.n_box, d.nc), dtype=vd, device="cuda")
    loc = torch.zeros_like(mp)
    pot = torch.zeros(tr.points.shape[0], dtype=vd, device="cuda")
    plan.p2m(cen, lev, rng, pts, dev(w, vd), out=mp[l0:l0 + nl])
    batch = plan.prepare(t, s, tr.ijk, tr.level)  # the benchmark's (tuned) launch shape
    batch(mp, loc)
    plan.l2p(cen, lev, rng, pts, loc[l0:l0 + nl].contiguous(), pot)
    got_all = host(pot).astype(np.float64)
    sample = pick(200 + p, leaves, 2 if p <= 8 else 1)
    got = np.concatenate([got_all[tr.pt_range[b][0]:tr.pt_range[b][1]] for b in sample])
    ref = np.concatenate([_oracle_far_potential(p, tr, w, t, s, b) for b in sample])
    err = rel(got, ref)
    assert err < (2e-5 if single else 1e-12), err


# ----------------------------------------------------------------------------- Plummer, Helmholtz

@pytest.fixture(scope="module")
def plummer():
    tr = W.adaptive_tree(W.plummer_points(1 << 21, 3, 0.1), 64)
    w = W.normal_weights(tr.points.shape[0], 4, complex_=True)
    leaf_side = max(tr.box_size(int(tr.level[b])) for b in np.nonzero(tr.is_leaf)[0])
    t, s = W.interaction_pairs(tr, list(range(2, tr.n_levels)))
    return tr, w, t, s, 1.0 / leaf_side


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_plummer_helmholtz_full_size(gpu_lib, plummer, dt):
    fmm = gpu_lib
    tr, w, t, s, k = plummer
    p = 12
    single = dt == "c64"
    plan = fmm.Plan(fmm.Desc("helmholtz", p, dt, k), [tr.box_size(l) for l in range(tr.n_levels)])
    leaves = np.nonzero(tr.is_leaf)[0]
    check_p2m(fmm, plan, "helmholtz", k, p, tr, leaves, w, 50, tol_pts(single, p))
    batch = plan.prepare(t, s, tr.ijk, tr.level)  # every level in one launch
    assert batch.info()["n_pair"] == len(t)
    # two targets on each of three levels (the deepest ones carry most pairs)
    lev_t = tr.level[t]
    levels = sorted(set(lev_t.tolist()))[-3:]
    targets = np.concatenate([pick(60 + l, np.unique(t[lev_t == l]), 2) for l in levels])
    check_m2l(plan, "helmholtz", k, p, tr, t, s, batch, 70, 1e-4 if single else 1e-12, True, np.sort(targets))
    check_l2p(fmm, plan, "helmholtz", k, p, tr, leaves, 80, tol_pts(single, p), True)


# ----------------------------------------------------------------------------- mixture, one graph

def order_of_level(l):
    return 6 + 2 * ((l - 2) % 3)


@pytest.mark.parametrize("shapes", ["tuned", "one_tiled_shape"])
def test_mixture_full_size_one_captured_launch(gpu_lib, shapes):
    """The mixed workload at full size (524,288 mixture points, Yukawa and biharmonic, p = 6/8/10
    by level, FP32): the six batches in their tuned per-(kernel, order) shapes, or in one shared
    tiled shape (one persistent launch), enqueued as one multi launch and captured in a graph;
    replays bit-identical to the eager launch, sampled targets against the oracle."""
    fmm = gpu_lib
    tr = W.adaptive_tree(W.gaussian_mixture_points(1 << 19, 4), 64)
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    tuning = None if shapes == "tuned" else {"rows_per_wave": 2, "col_tiles_per_wave": 2, "col_groups": 1,
                                              "lds_buffers": 1}
    groups, batches, mps = [], [], []
    for kernel, param in (("yukawa", 2.0), ("biharmonic", 0.0)):
        for p in (6, 8, 10):
            levels = [l for l in range(2, tr.n_levels) if order_of_level(l) == p]
            t, s = W.interaction_pairs(tr, levels)
            if len(t) == 0:
                continue
            d = fmm.Desc(kernel, p, "f32", param)
            plan = fmm.Plan(d, lh)
            g = np.random.Generator(np.random.PCG64(90 + p + len(kernel)))
            beta = g.standard_normal((tr.n_box, d.nc))
            groups.append((kernel, param, p, plan, t, s, beta))
            batches.append(plan.prepare(t, s, tr.ijk, tr.level, tuning=tuning))
            mps.append(dev(beta, torch.float32))
    multi = fmm.Multi(batches)
    outs = [torch.zeros_like(m) for m in mps]
    multi(mps, outs)  # warm-up (and the eager result)
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for o in outs:
                o.zero_()
            multi(mps, outs)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(2):
        for o in outs:
            o.fill_(float(rep + 7))
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs, eager):
            assert torch.equal(a, b), rep
    for (kernel, param, p, plan, t, s, beta), out in zip(groups, outs):
        targets = pick(100 + p + len(kernel), np.unique(t), 2)
        perm = perm_to_lib(kernel, param, p, plan.desc.index_table())
        inv = np.argsort(perm)
        m = np.isin(t, targets)
        ref = oracle_m2l_scaled(kernel, param, p, tr.ijk.astype(np.int64), tr.level, lh, t[m], s[m],
                                beta[:, inv])[targets][:, perm]
        err = rel(host(out)[targets].astype(np.float64), ref)
        assert err < 2e-5, (kernel, p, err)
    del graph
    multi.close()


# ----------------------------------------------------------------------------- gradient

def test_gradient_full_size(gpu_lib):
    """Laplace p = 10 far field of 2^21 sources at 2^21 targets: the FP32 adjoint against the
    FP64 adjoint, and the FP64 adjoint against fourth-order central differences of the FP64
    forward along seeded directions supported on a 4,096-point subset."""
    from paper_2305_17867_amd.farfield import FarField
    n, depth, p = 1 << 21, 4, 10
    ts = W.uniform_tree(W.uniform_points(n, 5), depth)
    tt = W.uniform_tree(W.uniform_points(n, 6), depth)
    w = W.normal_weights(n, 7)
    c = W.normal_weights(n, 8)
    sub = pick(9, np.arange(n), 4096)
    grads = {}
    ffs = {}
    for dt, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        ff = FarField("laplace", p, dt, ts, tt)
        ffs[dt] = ff
        W_ = dev(w, tdt).requires_grad_(True)
        S_ = dev(ts.points, tdt).requires_grad_(True)
        T_ = dev(tt.points, tdt).requires_grad_(True)
        (ff.apply(W_, S_, T_) * dev(c, tdt)).sum().backward()
        grads[dt] = [host(x.grad).astype(np.float64)[sub] for x in (W_, S_, T_)]
    for a, b in zip(grads["f32"], grads["f64"]):
        assert rel(a, b) < 2e-5, rel(a, b)
    ff = ffs["f64"]
    base = [dev(w, torch.float64), dev(ts.points, torch.float64), dev(tt.points, torch.float64)]
    C_ = dev(c, torch.float64)
    g = np.random.Generator(np.random.PCG64(10))
    eps = 1e-4
    for which in range(3):
        dirn = np.zeros(tuple(base[which].shape))
        dirn[sub] = g.standard_normal(dirn[sub].shape)
        dirn_t = dev(dirn, torch.float64)

        def at(k):
            args = list(base)
            args[which] = (base[which] + k * eps * dirn_t).contiguous()
            with torch.no_grad():
                return float((ff.apply(*args) * C_).sum())

        fd = (-at(2) + 8 * at(1) - 8 * at(-1) + at(-2)) / (12 * eps)
        an = float((grads["f64"][which] * dirn[sub]).sum())
        assert abs(fd - an) <= 1e-6 * abs(an), (which, fd, an)
