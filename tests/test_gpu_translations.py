"""GPU parity of the compressed M2M and L2L (fmm_m2m, fmm_l2l) against the CPU oracle.

Inputs are seeded: random scaled coefficients on the boxes of uniform and adaptive
(Plummer) octrees, so that every parent has eight, some or no children.  Tolerances,
normwise relative l2 over all outputs: FP64 / complex128 1e-12; FP32 / complex64 2e-6
(inputs and outputs rounded to single precision, arithmetic in double).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import compressed as Z

from helpers import perm_to_lib, rel

pytestmark = pytest.mark.gpu

CASES = [("laplace", 0.0), ("yukawa", 2.0), ("helmholtz", 1.0), ("biharmonic", 0.0)]


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def make(fmm, kernel, param, p, single, tree):
    cplx = kernel == "helmholtz"
    dt = ("c64" if single else "c128") if cplx else ("f32" if single else "f64")
    d = fmm.Desc(kernel, p, dt, param)
    plan = fmm.Plan(d, [tree.box_size(l) for l in range(tree.n_levels)])
    perm = perm_to_lib(kernel, param, p, d.index_table())
    return d, plan, perm


def random_coefs(tree, nc, cplx, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    v = g.standard_normal((tree.n_box, nc))
    return v + 1j * g.standard_normal((tree.n_box, nc)) if cplx else v


def oracle_m2m(kernel, param, p, tree, parents, child, coef_lib, perm):
    """Scaled psi~ of each parent (library order) from the children's scaled beta~."""
    out = {}
    for k, pb in enumerate(parents):
        tp = 1.0 / tree.box_size(int(tree.level[pb]))
        acc = 0
        for cb in child[k]:
            if cb < 0:
                continue
            tc = 1.0 / tree.box_size(int(tree.level[cb]))
            beta = np.empty_like(coef_lib[cb])
            beta[perm] = coef_lib[cb]
            acc = acc + Z.m2m_scaled(kernel, param, p, tree.center[pb] - tree.center[cb], beta, tc, tp)
        psi = np.zeros(coef_lib.shape[1], dtype=coef_lib.dtype) if np.isscalar(acc) else acc
        out[int(pb)] = np.asarray(psi)[perm]
    return out


def oracle_l2l(kernel, param, p, tree, parents, child, coef_lib, perm):
    """Scaled theta~ added to each child (library order) from its parent's scaled theta~."""
    out = {}
    for k, pb in enumerate(parents):
        tp = 1.0 / tree.box_size(int(tree.level[pb]))
        theta = np.empty_like(coef_lib[pb])
        theta[perm] = coef_lib[pb]
        for cb in child[k]:
            if cb < 0:
                continue
            tc = 1.0 / tree.box_size(int(tree.level[cb]))
            out[int(cb)] = np.asarray(
                Z.l2l_scaled(kernel, param, p, tree.center[cb] - tree.center[pb], theta, tp, tc))[perm]
    return out


@pytest.fixture(scope="module")
def uniform3():
    return W.uniform_tree(W.uniform_points(4096, 31), 3)


@pytest.fixture(scope="module")
def plummer():
    return W.adaptive_tree(W.plummer_points(20000, 32, 0.1), 64)


def run_m2m(fmm, kernel, param, p, single, tree, lev, seed, sample=None):
    d, plan, perm = make(fmm, kernel, param, p, single, tree)
    parents, child = W.children(tree, lev)
    if sample is not None:
        parents, child = parents[sample], child[sample]
    coef = random_coefs(tree, plan.nc, d.value_dtype.is_complex, seed)
    mp = dev(coef, d.value_dtype)
    plan.m2m(dev(parents, torch.int32), dev(child, torch.int32), dev(tree.center, torch.float64),
             dev(tree.level, torch.int32), mp)
    got = host(mp)
    ref = oracle_m2m(kernel, param, p, tree, parents, child, host(dev(coef, d.value_dtype)).astype(coef.dtype), perm)
    a = np.array([got[b] for b in ref])
    b = np.array([ref[b] for b in ref])
    # boxes that are not parents keep their values
    others = np.setdiff1d(np.arange(tree.n_box), parents)
    assert np.array_equal(got[others], host(dev(coef, d.value_dtype))[others])
    return rel(a, b)


def run_l2l(fmm, kernel, param, p, single, tree, lev, seed, sample=None):
    d, plan, perm = make(fmm, kernel, param, p, single, tree)
    parents, child = W.children(tree, lev)
    if sample is not None:
        parents, child = parents[sample], child[sample]
    coef = random_coefs(tree, plan.nc, d.value_dtype.is_complex, seed)
    start = host(dev(coef, d.value_dtype))
    loc = dev(coef, d.value_dtype)
    plan.l2l(dev(parents, torch.int32), dev(child, torch.int32), dev(tree.center, torch.float64),
             dev(tree.level, torch.int32), loc)
    got = host(loc)
    ref = oracle_l2l(kernel, param, p, tree, parents, child, start.astype(coef.dtype), perm)
    a = np.array([got[b] - start[b] for b in ref])
    b = np.array([ref[b] for b in ref])
    touched = np.array(sorted(ref))
    others = np.setdiff1d(np.arange(tree.n_box), touched)
    assert np.array_equal(got[others], start[others])
    return rel(a, b)


@pytest.mark.parametrize("kernel,param", CASES)
@pytest.mark.parametrize("single", [False, True])
def test_m2m_uniform(gpu_lib, uniform3, kernel, param, single):
    err = run_m2m(gpu_lib, kernel, param, 4, single, uniform3, 2, 41)
    assert err < (2e-6 if single else 1e-12), err


@pytest.mark.parametrize("kernel,param", CASES)
@pytest.mark.parametrize("single", [False, True])
def test_l2l_uniform(gpu_lib, uniform3, kernel, param, single):
    err = run_l2l(gpu_lib, kernel, param, 4, single, uniform3, 2, 42)
    assert err < (2e-6 if single else 1e-12), err


@pytest.mark.parametrize("kernel,param,p", [("laplace", 0.0, 8), ("helmholtz", 1.0, 8), ("yukawa", 2.0, 12),
                                            ("biharmonic", 0.0, 10)])
def test_m2m_l2l_high_order_sampled(gpu_lib, uniform3, kernel, param, p):
    sample = np.array([0, 21, 42, 63])
    assert run_m2m(gpu_lib, kernel, param, p, False, uniform3, 2, 43, sample) < 1e-12
    assert run_l2l(gpu_lib, kernel, param, p, False, uniform3, 2, 44, sample) < 1e-12


@pytest.mark.parametrize("kernel,param", [("laplace", 0.0), ("helmholtz", 1.0)])
def test_ragged_children_adaptive_tree(gpu_lib, plummer, kernel, param):
    """Parents with fewer than eight children (and parents without any: M2M writes zeros)."""
    parents, child = W.children(plummer, 3)
    assert (child < 0).any()
    assert run_m2m(gpu_lib, kernel, param, 6, False, plummer, 3, 45) < 1e-12
    assert run_l2l(gpu_lib, kernel, param, 6, False, plummer, 3, 46) < 1e-12


def test_parent_without_children_gets_zero_and_bad_indices_are_skipped(gpu_lib, uniform3):
    fmm = gpu_lib
    d, plan, _ = make(fmm, "laplace", 0.0, 4, False, uniform3)
    coef = random_coefs(uniform3, plan.nc, False, 47)
    mp = dev(coef, torch.float64)
    parents = np.array([0, 1, uniform3.n_box + 5, -3], dtype=np.int32)
    child = np.full((4, 8), -1, dtype=np.int32)
    child[1, 0] = uniform3.n_box + 100  # out of range: no child
    plan.m2m(dev(parents, torch.int32), dev(child, torch.int32), dev(uniform3.center, torch.float64),
             dev(uniform3.level, torch.int32), mp)
    got = host(mp)
    assert np.all(got[0] == 0) and np.all(got[1] == 0)
    assert np.array_equal(got[2:], coef[2:])
    # zero parents: nothing happens
    plan.m2m(dev(np.zeros(0, np.int32), torch.int32), dev(np.zeros((0, 8), np.int32), torch.int32),
             dev(uniform3.center, torch.float64), dev(uniform3.level, torch.int32), mp)
    assert np.array_equal(host(mp), got)


@pytest.mark.parametrize("kernel,param", [("laplace", 0.0), ("biharmonic", 0.0)])
def test_m2m_of_leaf_moments_equals_parent_moments(gpu_lib, uniform3, kernel, param):
    """For PDEs whose terms have one order the compressed M2M is exact (Sec. 4.3): P2M at
    the leaves then M2M equals P2M at the parents, on the GPU end to end."""
    fmm = gpu_lib
    tr = uniform3
    d, plan, _ = make(fmm, kernel, param, 8, False, tr)
    w = W.normal_weights(tr.points.shape[0], 48)
    pts, wd = dev(tr.points, torch.float64), dev(w, torch.float64)
    cen, lev, rng = dev(tr.center, torch.float64), dev(tr.level, torch.int32), dev(tr.pt_range, torch.int64)
    direct = plan.p2m(cen, lev, rng, pts, wd)
    moved = torch.zeros_like(direct)
    leaves = tr.boxes_at(3)
    moved[leaves] = direct[leaves]
    parents, child = W.children(tr, 2)
    plan.m2m(dev(parents, torch.int32), dev(child, torch.int32), cen, lev, moved)
    assert rel(host(moved[parents]), host(direct[parents])) < 1e-12


@pytest.mark.parametrize("kernel,param", CASES)
def test_adjoints_are_the_transposes(gpu_lib, uniform3, kernel, param):
    """<M2M b, g> = <b, M2M^T g> and <L2L t, g> = <t, L2L^T g> (bilinear, no conjugation), with
    M2M / L2L and their transposes all run on the GPU."""
    fmm = gpu_lib
    tr = uniform3
    d, plan, _ = make(fmm, kernel, param, 6, False, tr)
    cplx = d.value_dtype.is_complex
    parents, child = W.children(tr, 2)
    par, ch = dev(parents, torch.int32), dev(child, torch.int32)
    cen, lev = dev(tr.center, torch.float64), dev(tr.level, torch.int32)
    kids = child.ravel()
    for seed, fwd, adj, out_boxes, in_boxes in (
            (51, plan.m2m, plan.m2m_adjoint, parents, kids),
            (52, plan.l2l, plan.l2l_adjoint, kids, parents)):
        x = random_coefs(tr, plan.nc, cplx, seed)
        g = random_coefs(tr, plan.nc, cplx, seed + 10)
        # forward applied to x on the input boxes only
        xin = np.zeros_like(x)
        xin[in_boxes] = x[in_boxes]
        y = dev(xin, d.value_dtype)
        fwd(par, ch, cen, lev, y)
        y = host(y)
        if fwd == plan.l2l:
            y[in_boxes] = 0  # L2L accumulates into the children: keep only what it added
        lhs = np.sum(y[out_boxes] * g[out_boxes])
        gin = np.zeros_like(g)
        gin[out_boxes] = g[out_boxes]
        z = dev(gin, d.value_dtype)
        adj(par, ch, cen, lev, z)
        z = host(z)
        rhs = np.sum(x[in_boxes] * (z[in_boxes] - gin[in_boxes]))
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0), (kernel, fwd, lhs, rhs)


def _tree_far_field(dtype, tree_pass, kernel="laplace", param=0.0, p=8, n=3000, depth=4):
    from paper_2305_17867_amd.farfield import FarField
    ts = W.uniform_tree(W.uniform_points(n, 61), depth)
    tt = W.uniform_tree(W.uniform_points(n, 62), depth)
    ff = FarField(kernel, p, dtype, ts, tt, param=param, tree_pass=tree_pass)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    w = dev(W.normal_weights(n, 63), tdt).requires_grad_(True)
    s = dev(ts.points, tdt).requires_grad_(True)
    t = dev(tt.points, tdt).requires_grad_(True)
    c = dev(W.normal_weights(n, 64), tdt)
    phi = ff.apply(w, s, t)
    (phi * c).sum().backward()
    return [host(v) for v in (phi.detach(), w.grad, s.grad, t.grad)]


@pytest.mark.parametrize("kernel,param,tol", [("laplace", 0.0, 1e-12), ("biharmonic", 0.0, 1e-12),
                                              ("yukawa", 2.0, 1e-4)])
def test_tree_pass_far_field_matches_per_level(gpu_lib, kernel, param, tol):
    """P2M + M2M up + M2L + L2L down + L2P at the leaves, forward and backward, against P2M and
    L2P at every level: equal to roundoff for Laplace and biharmonic (M2M and L2L exact), at
    truncation level for Yukawa."""
    tree = _tree_far_field("f64", True, kernel, param)
    per_level = _tree_far_field("f64", False, kernel, param)
    for a, b in zip(tree, per_level):
        assert rel(a, b) < tol


def test_tree_pass_fp32_gradients_agree_with_fp64(gpu_lib):
    """The tree pass in FP32 (M2M / L2L and their transposes in single precision) against the
    same pass in FP64, at the FP32 adjoint tolerance."""
    f32 = _tree_far_field("f32", True)
    f64 = _tree_far_field("f64", True)
    for a, b in zip(f32, f64):
        assert rel(a.astype(np.float64), b) < 2e-5


def _adaptive_far_field(dtype, tree_pass, kernel="laplace", param=0.0, p=8, n=4000):
    """Far field of an adaptive octree (Plummer points, leaves on several levels), one point
    set as sources and targets (separate tensors, so that both position gradients are formed)."""
    from paper_2305_17867_amd.farfield import FarField
    tr = W.adaptive_tree(W.plummer_points(n, 65), 24)
    assert len(set(tr.level[tr.is_leaf].tolist())) >= 3
    ff = FarField(kernel, p, dtype, tr, tr, param=param, tree_pass=tree_pass)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    w = dev(W.normal_weights(n, 66), tdt).requires_grad_(True)
    s = dev(tr.points, tdt).requires_grad_(True)
    t = dev(tr.points, tdt).requires_grad_(True)
    c = dev(W.normal_weights(n, 67), tdt)
    phi = ff.apply(w, s, t)
    (phi * c).sum().backward()
    return [host(v) for v in (phi.detach(), w.grad, s.grad, t.grad)]


@pytest.mark.parametrize("kernel,param,tol", [("laplace", 0.0, 1e-12), ("biharmonic", 0.0, 1e-12),
                                              ("yukawa", 2.0, 1e-4)])
def test_tree_pass_on_adaptive_tree_matches_per_level(gpu_lib, kernel, param, tol):
    """On an adaptive tree the tree pass forms multipoles by P2M at leaves of every level and M2M
    from the parents that have children, and evaluates locals by L2L down to the leaves and L2P
    there; against P2M and L2P of every box at every level, forward and backward: equal to
    roundoff for Laplace and biharmonic, at truncation level for Yukawa."""
    tree = _adaptive_far_field("f64", True, kernel, param)
    per_level = _adaptive_far_field("f64", False, kernel, param)
    for a, b in zip(tree, per_level):
        assert rel(a, b) < tol, rel(a, b)


def test_tree_pass_on_adaptive_tree_fp32_agrees_with_fp64(gpu_lib):
    """The adaptive tree pass in FP32, forward and all gradients, against FP64 at the FP32
    adjoint tolerance."""
    f32 = _adaptive_far_field("f32", True)
    f64 = _adaptive_far_field("f64", True)
    for a, b in zip(f32, f64):
        assert rel(a.astype(np.float64), b) < 2e-5, rel(a.astype(np.float64), b)
