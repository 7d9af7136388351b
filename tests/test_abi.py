"""The C-ABI library loads, exports every symbol include/fmm.h declares, and its host-only
entry points agree with the oracle (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import compression as OC
from oracle import multiindex as MI

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2305_17867_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libfmm.so not built")
    return _lib


def test_every_declared_symbol_is_exported(lib):
    L = lib.load()
    names = declared_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    # and the binding declares a signature for each
    assert set(names) <= set(lib.SIGNATURES), set(names) - set(lib.SIGNATURES)
    assert L.fmm_abi_version() == 2


@pytest.mark.parametrize("kernel,c", [("laplace", 2), ("helmholtz", 2), ("yukawa", 2), ("biharmonic", 4)])
@pytest.mark.parametrize("p", [0, 1, 3, 8, 12, 16])
def test_sizes_and_index_table_match_oracle(lib, kernel, c, p):
    dt = "c128" if kernel == "helmholtz" else "f64"
    d = lib.make_desc(kernel, p, dt, 1.0)
    nf, nc = C.c_int32(), C.c_int32()
    lib.check(lib.load().fmm_sizes(C.byref(d), C.byref(nf), C.byref(nc)), "sizes")
    assert nf.value == MI.n_full(p)
    kept = [m for m in MI.graded_order(p) if m[2] < c]
    assert nc.value == len(kept)
    tab = np.zeros((nc.value, 3), np.int32)
    lib.check(lib.load().fmm_index_table(C.byref(d), tab.ctypes.data_as(lib.I32P)), "index")
    assert {tuple(r) for r in tab.tolist()} == set(kept)
    # storage order: lexicographic in (m_z, m_x, m_y)
    keys = [(r[2], r[0], r[1]) for r in tab.tolist()]
    assert keys == sorted(keys)
    if kernel in ("laplace", "biharmonic") and p <= 6:
        # the kept set the oracle's Gaussian elimination of the PDE relations selects (Sec. 3.1)
        _, j, _ = OC.decompression_matrix(kernel, 0.0, p)
        order = MI.graded_order(p)
        assert {tuple(order[i]) for i in j} == {tuple(r) for r in tab.tolist()}


@pytest.mark.parametrize("bad,status", [
    (dict(kernel=7), -1), (dict(dtype=9), -1), (dict(order=-1), -2), (dict(order=17), -2),
    (dict(flags=1), -1), (dict(kernel=1, dtype=0), -2), (dict(kernel=0, dtype=2), -2),
    (dict(kernel=2, param=0.0), -1), (dict(kernel=1, dtype=2, param=float("nan")), -1),
])
def test_descriptor_validation(lib, bad, status):
    d = lib.FmmDesc(0, 4, 0, 0, 1.0)
    for k, v in bad.items():
        setattr(d, k, v)
    nf, nc = C.c_int32(), C.c_int32()
    assert lib.load().fmm_sizes(C.byref(d), C.byref(nf), C.byref(nc)) == status
    assert lib.load().fmm_last_error()


@pytest.mark.parametrize("kernel,c", [("laplace2d", 2), ("biharmonic2d", 4)])
@pytest.mark.parametrize("p", [0, 1, 3, 8, 16])
def test_two_d_sizes_and_index_table_match_oracle(lib, kernel, c, p):
    from oracle import two_d as T2
    L = lib.load()
    d = lib.make_desc(kernel, p, "f64")
    nf, nc = C.c_int32(), C.c_int32()
    assert L.fmm2d_sizes(C.byref(d), C.byref(nf), C.byref(nc)) == 0
    J = T2.kept_set(p, c)
    assert (nf.value, nc.value) == (T2.n_full(p), len(J))
    out = (C.c_int32 * (2 * nc.value))()
    assert L.fmm2d_index_table(C.byref(d), out) == 0
    assert [(out[2 * k], out[2 * k + 1]) for k in range(nc.value)] == J
    # 2-D kernels are refused by the 3-D calls and 3-D kernels by the 2-D calls; FP64 only
    assert L.fmm_sizes(C.byref(d), C.byref(nf), C.byref(nc)) == -1
    assert L.fmm2d_sizes(C.byref(lib.make_desc("laplace", p, "f64")), C.byref(nf), C.byref(nc)) == -1
    assert L.fmm2d_sizes(C.byref(lib.make_desc(kernel, p, "f32")), C.byref(nf), C.byref(nc)) == -2
    assert L.fmm2d_sizes(C.byref(lib.make_desc(kernel, 17, "f64")), C.byref(nf), C.byref(nc)) == -2


def test_null_arguments_are_rejected_before_any_launch(lib):
    L = lib.load()
    assert L.fmm_sizes(None, None, None) == -1
    d = lib.make_desc("laplace", 4, "f64")
    assert L.fmm_index_table(C.byref(d), None) == -1
    assert L.fmm_plan_create(C.byref(d), 1, None, C.byref(C.c_void_p())) == -1
    lv = (C.c_double * 1)(-1.0)
    assert L.fmm_plan_create(C.byref(d), 1, lv, C.byref(C.c_void_p())) == -1
    assert L.fmm_p2m(None, 1, None, None, None, 0, None, None, None, None) == -1
    assert L.fmm_m2l_batched(None, None, None, None) == -1
    assert L.fmm_m2m(None, 1, None, None, 0, None, None, None, None) == -1
    assert L.fmm_l2l(None, 1, None, None, 0, None, None, None, None) == -1
    assert L.fmm_m2m_adjoint(None, 1, None, None, 0, None, None, None, None) == -1
    assert L.fmm_p2p(C.byref(d), 1, None, None, 0, None, 0, None, None, 0, None, None, 0, None, None, None) == -1
    assert L.fmm_p2p(C.byref(d), 0, None, None, 0, None, 0, None, None, 0, None, None, 0, None, None, None) == 0
    assert L.fmm_l2l_adjoint(None, 1, None, None, 0, None, None, None, None) == -1
    assert L.fmm_batch_info(None, None, 0) == -1
    assert L.fmm_direct(C.byref(d), -1, None, None, 0, None, None, None) == -1
    assert L.fmm_m2l_batched_multi(-1, None, None, None, None) == -1
    h = C.c_void_p()
    assert L.fmm_m2l_multi_prepare(0, None, C.byref(h)) == -1 and not h.value
    assert L.fmm_m2l_multi_prepare(33, None, C.byref(h)) == -1
    assert L.fmm_m2l_multi_prepare(1, None, None) == -1
    assert L.fmm_m2l_multi_launch(None, None, None, None) == -1
    L.fmm_m2l_multi_destroy(None)
    t = C.c_void_p()
    assert L.fmm_tree_build(-1, None, 0, 2, C.byref(t), None) == -1 and not t.value
    assert L.fmm_tree_build(8, None, 0, 2, C.byref(t), None) == -1
    assert L.fmm_tree_build(0, None, 0, 11, C.byref(t), None) == -1  # uniform depth above 10
    assert L.fmm_tree_build(0, None, 4, 21, C.byref(t), None) == -1  # adaptive depth above 20
    assert L.fmm_tree_build(0, None, -1, 2, C.byref(t), None) == -1
    assert L.fmm_tree_build(0, None, 0, 2, None, None) == -1
    n64 = C.c_int64()
    assert L.fmm_tree_size(None, None, None, None) == -1
    assert L.fmm_tree_export(None, None, None, None, None, None, None, None, None, None) == -1
    assert L.fmm_tree_list2(None, 2, 3, C.byref(n64), None, None, None) == -1
    assert L.fmm_tree_lists(None, 0, 0, C.byref(n64), C.byref(n64), None, None, None, None) == -1
    L.fmm_tree_destroy(None)
    d2 = lib.make_desc("laplace2d", 4, "f64")
    assert L.fmm2d_p2m(C.byref(d2), 1, None, None, None, 0, None, None, None, 1, None) == -1
    assert L.fmm2d_m2l(C.byref(d2), 1, None, None, 0, None, None, 0, None, 0, None, None, None) == -1
    assert L.fmm2d_l2p(C.byref(d2), 1, None, None, None, 0, None, None, None, 1, None) == -1
    assert L.fmm2d_direct(C.byref(d2), 0, None, None, 1, None, None, None) == -1
    assert L.fmm2d_p2p(C.byref(d2), 1, None, None, 0, None, 0, None, None, 0, None, None, 0, None, None, 1, None) == -1
    assert L.fmm2d_deriv_tables(C.byref(d2), 1, None, None, None, None) == -1
    assert L.fmm2d_m2l(C.byref(d2), 0, None, None, 0, None, None, 0, None, 0, None, None, None) == 0
    # zero-size work is a no-op that needs no GPU
    assert L.fmm_direct(C.byref(d), 0, None, None, 0, None, None, None) == 0
    assert L.fmm_deriv_tables(C.byref(d), 0, None, None, None, None) == 0
