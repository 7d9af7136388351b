"""ctypes loader for libfmm.so with the signatures of include/fmm.h.

There is no fallback: if the shared library is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmm.so")

FMM_OK, FMM_EINVAL, FMM_EUNSUPPORTED, FMM_EHIP, FMM_ENOMEM, FMM_ESTATE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "FMM_OK", -1: "FMM_EINVAL", -2: "FMM_EUNSUPPORTED", -3: "FMM_EHIP",
                -4: "FMM_ENOMEM", -5: "FMM_ESTATE"}
KERNELS = {"laplace": 0, "helmholtz": 1, "yukawa": 2, "biharmonic": 3, "laplace2d": 4, "biharmonic2d": 5}
DTYPES = {"f64": 0, "f32": 1, "c128": 2, "c64": 3}
MAX_ORDER = 16


class FmmDesc(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("order", C.c_int32), ("dtype", C.c_int32),
                ("flags", C.c_int32), ("param", C.c_double)]


class FmmM2LTuning(C.Structure):
    _fields_ = [("rows_per_wave", C.c_int32), ("col_tiles_per_wave", C.c_int32),
                ("col_groups", C.c_int32), ("target_items", C.c_int32), ("lds_buffers", C.c_int32),
                ("k_splits", C.c_int32), ("form", C.c_int32), ("waves", C.c_int32), ("workgroups", C.c_int32)]


class FmmError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


P = C.c_void_p
I32P = C.POINTER(C.c_int32)
I64P = C.POINTER(C.c_int64)
F64P = C.POINTER(C.c_double)

# name -> (restype, argtypes)
SIGNATURES = {
    "fmm_abi_version": (C.c_int32, []),
    "fmm_last_error": (C.c_char_p, []),
    "fmm_sizes": (C.c_int, [C.POINTER(FmmDesc), I32P, I32P]),
    "fmm_index_table": (C.c_int, [C.POINTER(FmmDesc), I32P]),
    "fmm_deriv_tables": (C.c_int, [C.POINTER(FmmDesc), C.c_int64, P, P, P, P]),
    "fmm_plan_create": (C.c_int, [C.POINTER(FmmDesc), C.c_int32, F64P, C.POINTER(P)]),
    "fmm_plan_destroy": (None, [P]),
    "fmm_p2m": (C.c_int, [P, C.c_int64, P, P, P, C.c_int64, P, P, P, P]),
    "fmm_l2p": (C.c_int, [P, C.c_int64, P, P, P, C.c_int64, P, P, P, P]),
    "fmm_m2m": (C.c_int, [P, C.c_int64, P, P, C.c_int64, P, P, P, P]),
    "fmm_l2l": (C.c_int, [P, C.c_int64, P, P, C.c_int64, P, P, P, P]),
    "fmm_m2m_adjoint": (C.c_int, [P, C.c_int64, P, P, C.c_int64, P, P, P, P]),
    "fmm_l2l_adjoint": (C.c_int, [P, C.c_int64, P, P, C.c_int64, P, P, P, P]),
    "fmm_m2l_prepare": (C.c_int, [P, C.c_int64, I32P, I32P, C.c_int64, I32P, I32P, C.POINTER(P)]),
    "fmm_m2l_prepare_ex": (C.c_int, [P, C.c_int64, I32P, I32P, C.c_int64, I32P, I32P,
                                     C.POINTER(FmmM2LTuning), C.POINTER(P)]),
    "fmm_batch_destroy": (None, [P]),
    "fmm_batch_info": (C.c_int, [P, I64P, C.c_int32]),
    "fmm_m2l_batched": (C.c_int, [P, P, P, P]),
    "fmm_m2l_batched_static": (C.c_int, [P, P, P, P]),
    "fmm_m2l_batched_multi": (C.c_int, [C.c_int32, C.POINTER(P), C.POINTER(P), C.POINTER(P), P]),
    "fmm_direct": (C.c_int, [C.POINTER(FmmDesc), C.c_int64, P, P, C.c_int64, P, P, P]),
    "fmm_p2p": (C.c_int, [C.POINTER(FmmDesc), C.c_int64, P, P, C.c_int64, P, C.c_int64, P, P, C.c_int64, P, P,
                          C.c_int64, P, P, P]),
    "fmm_m2p": (C.c_int, [P, C.c_int64, P, P, C.c_int64, P, C.c_int64, P, P, P, C.c_int64, P, P, P, P]),
    "fmm_p2l": (C.c_int, [P, C.c_int64, P, P, C.c_int64, P, C.c_int64, P, P, P, C.c_int64, P, P, P, P]),
    "fmm_l2p_adjoint": (C.c_int, [P, C.c_int64, P, P, P, C.c_int64, P, P, P, P, P, P]),
    "fmm_p2m_adjoint": (C.c_int, [P, C.c_int64, P, P, P, C.c_int64, P, P, P, P, P, P]),
    "fmm_m2l_prepare_adjoint": (C.c_int, [P, C.c_int64, I32P, I32P, C.c_int64, I32P, I32P,
                                          C.POINTER(FmmM2LTuning), C.POINTER(P)]),
    "fmm_m2l_batched_adjoint": (C.c_int, [P, P, P, P]),
    "fmm_m2l_prepare_fft": (C.c_int, [P, C.c_int64, I32P, I32P, C.c_int64, I32P, I32P, C.POINTER(P)]),
    "fmm_m2l_multi_prepare": (C.c_int, [C.c_int32, C.POINTER(P), C.POINTER(P)]),
    "fmm_m2l_multi_launch": (C.c_int, [P, C.POINTER(P), C.POINTER(P), P]),
    "fmm_m2l_multi_destroy": (None, [P]),
    "fmm_l2p_ex": (C.c_int, [P, C.c_int64, P, P, P, C.c_int64, P, P, P, C.c_int32, P]),
    "fmm_m2l_batched_ex": (C.c_int, [P, P, P, C.c_int32, P]),
    "fmm2d_sizes": (C.c_int, [C.POINTER(FmmDesc), I32P, I32P]),
    "fmm2d_index_table": (C.c_int, [C.POINTER(FmmDesc), I32P]),
    "fmm2d_deriv_tables": (C.c_int, [C.POINTER(FmmDesc), C.c_int64, P, P, P, P]),
    "fmm2d_p2m": (C.c_int, [C.POINTER(FmmDesc), C.c_int64, P, P, P, C.c_int64, P, P, P, C.c_int32, P]),
    "fmm2d_m2l": (C.c_int, [C.POINTER(FmmDesc), C.c_int64, P, P, C.c_int64, P, P, C.c_int64, P, C.c_int64, P, P, P]),
    "fmm2d_l2p": (C.c_int, [C.POINTER(FmmDesc), C.c_int64, P, P, P, C.c_int64, P, P, P, C.c_int32, P]),
    "fmm2d_m2m": (C.c_int, [C.POINTER(FmmDesc), C.c_int64, P, P, C.c_int64, P, P, P, P]),
    "fmm2d_l2l": (C.c_int, [C.POINTER(FmmDesc), C.c_int64, P, P, C.c_int64, P, P, P, P]),
    "fmm2d_direct": (C.c_int, [C.POINTER(FmmDesc), C.c_int64, P, P, C.c_int64, P, P, P]),
    "fmm2d_p2p": (C.c_int, [C.POINTER(FmmDesc), C.c_int64, P, P, C.c_int64, P, C.c_int64, P, P, C.c_int64, P, P,
                            C.c_int64, P, P, C.c_int32, P]),
    "fmm_tree_build": (C.c_int, [C.c_int64, P, C.c_int32, C.c_int32, C.POINTER(P), P]),
    "fmm_tree_size": (C.c_int, [P, I64P, I32P, I64P]),
    "fmm_tree_export": (C.c_int, [P, P, P, P, P, P, P, P, I64P, P]),
    "fmm_tree_list2": (C.c_int, [P, C.c_int32, C.c_int32, I64P, P, P, P]),
    "fmm_tree_lists": (C.c_int, [P, C.c_int32, C.c_int64, I64P, I64P, P, P, P, P]),
    "fmm_tree_destroy": (None, [P]),
}
LIST_KINDS = {"near": 0, "u": 1, "w": 2, "x": 3}
TREE_MAX_DEPTH, TREE_MAX_UNIFORM_DEPTH = 20, 10

_LIB = None


def load() -> C.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "or python paper_2305_17867_amd/build.py")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def check(status: int, where: str):
    if status != FMM_OK:
        msg = load().fmm_last_error()
        raise FmmError(status, where, msg.decode() if msg else "")


def make_desc(kernel: str, order: int, dtype: str, param: float = 0.0) -> FmmDesc:
    return FmmDesc(KERNELS[kernel], int(order), DTYPES[dtype], 0, float(param))
