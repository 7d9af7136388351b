"""FFT form of the M2L (eq. convolution_m2l) against the oracle's dense translation and against
the matrix-core path.  Tolerances: the FFT's rounding error grows with p (the oracle's own FFT
form measures 8e-14 at p = 8 and 4e-11 at p = 12 with the same scaling), so FP64 is checked at
1e-10 for p <= 8 and 1e-9 for p = 12; FP32 at 5e-5."""
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
    ("laplace", 0.0, 4, "f64", 1e-10), ("laplace", 0.0, 8, "f64", 1e-10), ("laplace", 0.0, 12, "f64", 1e-9),
    ("yukawa", 2.0, 6, "f64", 1e-10), ("biharmonic", 0.0, 6, "f64", 1e-10), ("laplace", 0.0, 8, "f32", 5e-5),
    ("biharmonic", 0.0, 8, "f32", 5e-5), ("helmholtz", 1.0, 6, "c128", 1e-10), ("helmholtz", 1.0, 8, "c128", 1e-10),
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


def test_fft_complex_high_order_runs_or_reports_lds(gpu_lib):
    """complex128 at p = 12 needs 90 KB of LDS per workgroup: where the device grants it the
    result matches the oracle; otherwise prepare reports FMM_EUNSUPPORTED (never a launch)."""
    fmm = gpu_lib
    tr = W.uniform_tree(W.uniform_points(4096, 7), 3)
    d = fmm.Desc("helmholtz", 12, "c128", 1.0)
    lh = [tr.box_size(l) for l in range(tr.n_levels)]
    plan = fmm.Plan(d, lh)
    t, s = W.interaction_pairs(tr, [3])
    try:
        fft = plan.prepare_fft(t, s, tr.ijk, tr.level)
    except fmm._lib.FmmError as e:
        assert e.status == fmm._lib.FMM_EUNSUPPORTED and "LDS" in str(e)
        return
    it = d.index_table()
    beta = decaying_multipoles(it, tr.n_box, 5) + 1j * decaying_multipoles(it, tr.n_box, 6)
    out = dev(np.zeros_like(beta), d.value_dtype)
    fft(dev(beta, d.value_dtype), out)
    perm = perm_to_lib("helmholtz", 1.0, 12, it)
    ref = oracle_m2l_scaled("helmholtz", 1.0, 12, tr.ijk.astype(np.int64), tr.level, lh, t, s,
                            beta[:, np.argsort(perm)])[:, perm]
    assert rel(out.cpu().numpy(), ref) < 1e-9
