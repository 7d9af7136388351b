"""FFT form of the M2L (eq. convolution_m2l) against the oracle's dense translation and against
the matrix-core path, with decaying multipoles (the decay of physical ones, so that the low
orders carry their share of the norm).  Tolerances: FP64 / complex128 at 1e-12 for every order
(measured 6e-15 at p = 4, 5e-14 at p = 8, 3.4e-13 at p = 12: the rescaling by tau keeps the
transformed grids within a few orders of magnitude, and the dense per-axis DFTs reduce their
twiddle angles exactly); FP32 / complex64 at 5e-5."""
from math import factorial

import numpy as np
import pytest
import torch

import workloads as W

from helpers import oracle_m2l_scaled, perm_to_lib, rel

pytestmark = pytest.mark.gpu


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def decaying_multipoles(index_table, n_box, seed):
    """Scaled multipoles with the decay of physical ones: N(0,1) * 0.6^|q| / q!."""
    g = np.random.Generator(np.random.PCG64(seed))
    f = np.array([0.6 ** sum(q) / (factorial(q[0]) * factorial(q[1]) * factorial(q[2])) for q in index_table])
    return g.standard_normal((n_box, len(f))) * f


@pytest.mark.parametrize("kernel,param,p,dt,tol", [
    ("laplace", 0.0, 4, "f64", 1e-12), ("laplace", 0.0, 8, "f64", 1e-12), ("laplace", 0.0, 12, "f64", 1e-12),
    ("yukawa", 2.0, 6, "f64", 1e-12), ("biharmonic", 0.0, 6, "f64", 1e-12), ("laplace", 0.0, 8, "f32", 5e-5),
    ("biharmonic", 0.0, 8, "f32", 5e-5), ("helmholtz", 1.0, 6, "c128", 1e-12), ("helmholtz", 1.0, 8, "c128", 1e-12),
    ("helmholtz", 4.0, 8, "c64", 5e-5)])
def test_fft_m2l_matches_oracle_and_gemm(gpu_lib, kernel, param, p, dt, tol):
    fmm = gpu_lib
    tr = W.uniform_tree(W.uniform_points(4096, 7), 3)
    d = fmm.Desc(kernel, p, dt, param)
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    plan = fmm.Plan(d, lh)
    t, s = W.interaction_pairs(tr, [2, 3])
    it = d.index_table()
    beta = decaying_multipoles(it, tr.n_box, 3)
    td = d.value_dtype
    if td.is_complex:
        beta = beta + 1j * decaying_multipoles(it, tr.n_box, 4)
    fft = plan.prepare_fft(t, s, tr.ijk, tr.level)
    out = dev(np.zeros_like(beta), td)
    fft(dev(beta, td), out)
    perm = perm_to_lib(kernel, param, p, it)
    inv = np.argsort(perm)
    ref = oracle_m2l_scaled(kernel, param, p, tr.ijk.astype(np.int64), tr.level, lh, t, s, beta[:, inv])[:, perm]
    got = out.cpu().numpy().astype(np.complex128 if td.is_complex else np.float64)
    assert rel(got, ref) < tol, rel(got, ref)
    gemm = plan.prepare(t, s, tr.ijk, tr.level)
    out2 = dev(np.zeros_like(beta), td)
    gemm(dev(beta, td), out2)
    assert rel(got, out2.cpu().numpy().astype(got.dtype)) < tol


def test_fft_complex_high_order_runs(gpu_lib):
    """complex128 at p = 12 needs 90 KB of LDS per workgroup, which gfx950 grants (160 KB per
    CU): prepare must succeed and the result match the oracle at 1e-12."""
    fmm = gpu_lib
    tr = W.uniform_tree(W.uniform_points(4096, 7), 3)
    d = fmm.Desc("helmholtz", 12, "c128", 1.0)
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    plan = fmm.Plan(d, lh)
    t, s = W.interaction_pairs(tr, [3])
    fft = plan.prepare_fft(t, s, tr.ijk, tr.level)
    it = d.index_table()
    beta = decaying_multipoles(it, tr.n_box, 5) + 1j * decaying_multipoles(it, tr.n_box, 6)
    out = dev(np.zeros_like(beta), d.value_dtype)
    fft(dev(beta, d.value_dtype), out)
    perm = perm_to_lib("helmholtz", 1.0, 12, it)
    ref = oracle_m2l_scaled("helmholtz", 1.0, 12, tr.ijk.astype(np.int64), tr.level, lh, t, s,
                            beta[:, np.argsort(perm)])[:, perm]
    assert rel(out.cpu().numpy(), ref) < 1e-12
