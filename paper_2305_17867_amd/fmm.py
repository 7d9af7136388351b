"""Python binding of the C ABI: torch tensors in, kernel launches out.

Every function here only checks and marshals arguments and calls libfmm.so; all
arithmetic of the method runs in the HIP kernels.  Device tensors must live on
the current CUDA (HIP) device; work is enqueued on torch's current stream.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np
import torch

from . import _lib
from ._lib import check, make_desc

_TUNED = None


def tuned_m2l_shape(kernel: str, order: int, dtype: str):
    """Launch shape chosen by the autotuner for (kernel, p, dtype) on MI355X, or None.
    The table (m2l_tuned.json) is written by paper_2305_17867_amd.autotune."""
    global _TUNED
    if _TUNED is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "m2l_tuned.json")
        try:
            with open(path) as fh:
                _TUNED = json.load(fh)
        except (OSError, ValueError):
            _TUNED = {}
    ent = _TUNED.get(f"{kernel}|p{order}|{dtype}")
    return dict(ent["tuning"]) if ent else None

REAL = {"f64": torch.float64, "f32": torch.float32, "c128": torch.float64, "c64": torch.float32}
VALUE = {"f64": torch.float64, "f32": torch.float32, "c128": torch.complex128, "c64": torch.complex64}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _dev(t: torch.Tensor, dtype, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


class Desc:
    """(kernel, order p, dtype, param): kernel in laplace/helmholtz/yukawa/biharmonic,
    dtype in f64/f32/c128/c64, param = k (Helmholtz) or lambda (Yukawa)."""

    def __init__(self, kernel: str, order: int, dtype: str = "f64", param: float = 0.0):
        self.kernel, self.order, self.dtype, self.param = kernel, int(order), dtype, float(param)
        self.c = make_desc(kernel, order, dtype, param)

    @property
    def two_d(self) -> bool:
        return self.kernel.endswith("2d")

    def sizes(self) -> tuple[int, int]:
        nf, nc = C.c_int32(), C.c_int32()
        name = "fmm2d_sizes" if self.two_d else "fmm_sizes"
        check(getattr(_lib.load(), name)(C.byref(self.c), C.byref(nf), C.byref(nc)), name)
        return nf.value, nc.value

    @property
    def nc(self) -> int:
        return self.sizes()[1]

    def index_table(self) -> np.ndarray:
        nc = self.nc
        out = np.zeros((nc, 3), dtype=np.int32)
        check(_lib.load().fmm_index_table(C.byref(self.c), out.ctypes.data_as(_lib.I32P)),
              "fmm_index_table")
        return out

    @property
    def real_dtype(self):
        return REAL[self.dtype]

    @property
    def value_dtype(self):
        return VALUE[self.dtype]


def deriv_tables(desc: Desc, offsets: torch.Tensor, h: torch.Tensor) -> torch.Tensor:
    """Scaled FP64 derivative tables [n, 2c-1, 2p+1, 2p+1] (complex128 for Helmholtz)."""
    n = offsets.shape[0]
    _dev(offsets, torch.float64, "offsets", (n, 3))
    _dev(h, torch.float64, "h", (n,))
    p, c = desc.order, (4 if desc.kernel == "biharmonic" else 2)
    dt = torch.complex128 if desc.kernel == "helmholtz" else torch.float64
    out = torch.empty((n, 2 * c - 1, 2 * p + 1, 2 * p + 1), dtype=dt, device=offsets.device)
    check(_lib.load().fmm_deriv_tables(C.byref(desc.c), n, _ptr(offsets), _ptr(h), _ptr(out), _stream()),
          "fmm_deriv_tables")
    return out


class Plan:
    """A plan for one (kernel, p, dtype) and the box sizes of the tree levels."""

    def __init__(self, desc: Desc, level_box_size):
        self.desc = desc
        lv = np.ascontiguousarray(np.asarray(level_box_size, dtype=np.float64))
        self.n_levels = int(lv.shape[0])
        self._h = C.c_void_p()
        check(_lib.load().fmm_plan_create(C.byref(desc.c), self.n_levels, lv.ctypes.data_as(_lib.F64P),
                                          C.byref(self._h)), "fmm_plan_create")
        self.nf, self.nc = desc.sizes()

    def close(self):
        if self._h:
            _lib.load().fmm_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _boxes(self, center, level, rng):
        nb = center.shape[0]
        _dev(center, torch.float64, "box_center", (nb, 3))
        _dev(level, torch.int32, "box_level", (nb,))
        _dev(rng, torch.int64, "pt_range", (nb, 2))
        return nb

    def p2m(self, center, level, rng, src, w, out=None) -> torch.Tensor:
        nb = self._boxes(center, level, rng)
        n = src.shape[0]
        _dev(src, self.desc.real_dtype, "src_xyz", (n, 3))
        _dev(w, self.desc.value_dtype, "weight", (n,))
        if out is None:
            out = torch.empty((nb, self.nc), dtype=self.desc.value_dtype, device=src.device)
        _dev(out, self.desc.value_dtype, "mpole", (nb, self.nc))
        check(_lib.load().fmm_p2m(self._h, nb, _ptr(center), _ptr(level), _ptr(rng), n, _ptr(src),
                                  _ptr(w), _ptr(out), _stream()), "fmm_p2m")
        return out

    def bind_p2m(self, center, level, rng, src, w, out):
        """A zero-argument callable that enqueues this P2M on the current stream.  The tensors
        are checked and their pointers taken once here; the caller keeps them alive and
        unmoved.  For loops that launch the same step many times."""
        self.p2m(center, level, rng, src, w, out=out)  # validates the arguments
        fn = _lib.load().fmm_p2m
        args = (self._h, center.shape[0], _ptr(center), _ptr(level), _ptr(rng), src.shape[0], _ptr(src),
                _ptr(w), _ptr(out))
        return lambda: check(fn(*args, _stream()), "fmm_p2m")

    def bind_l2p(self, center, level, rng, tgt, local, pot, overwrite: bool = False):
        """Like bind_p2m, for L2P (the potentials keep accumulating on every call; with
        overwrite, the targets' potentials are stored instead)."""
        nb = self._boxes(center, level, rng)
        n = tgt.shape[0]
        _dev(tgt, self.desc.real_dtype, "tgt_xyz", (n, 3))
        _dev(local, self.desc.value_dtype, "local", (nb, self.nc))
        _dev(pot, self.desc.value_dtype, "potential", (n,))
        fn = _lib.load().fmm_l2p_ex
        args = (self._h, nb, _ptr(center), _ptr(level), _ptr(rng), n, _ptr(tgt), _ptr(local), _ptr(pot),
                1 if overwrite else 0)
        return lambda: check(fn(*args, _stream()), "fmm_l2p_ex")

    def l2p(self, center, level, rng, tgt, local, pot, overwrite: bool = False) -> torch.Tensor:
        """pot += the boxes' local expansions at their targets (overwrite: stored instead)."""
        nb = self._boxes(center, level, rng)
        n = tgt.shape[0]
        _dev(tgt, self.desc.real_dtype, "tgt_xyz", (n, 3))
        _dev(local, self.desc.value_dtype, "local", (nb, self.nc))
        _dev(pot, self.desc.value_dtype, "potential", (n,))
        check(_lib.load().fmm_l2p_ex(self._h, nb, _ptr(center), _ptr(level), _ptr(rng), n, _ptr(tgt),
                                     _ptr(local), _ptr(pot), 1 if overwrite else 0, _stream()), "fmm_l2p_ex")
        return pot

    def _lists(self, tbox, list_ptr, lst, center, level, rng, xyz):
        nt, nb = tbox.shape[0], center.shape[0]
        _dev(tbox, torch.int32, "tbox", (nt,))
        _dev(list_ptr, torch.int32, "list_ptr", (nt + 1,))
        _dev(lst, torch.int32, "list", (lst.shape[0],))
        _dev(center, torch.float64, "box_center", (nb, 3))
        _dev(level, torch.int32, "box_level", (nb,))
        _dev(rng, torch.int64, "range", (nb, 2))
        _dev(xyz, self.desc.real_dtype, "xyz", (xyz.shape[0], 3))
        return nt, nb

    def m2p(self, tbox, list_ptr, lst, center, level, tgt_range, tgt, mpole, pot) -> torch.Tensor:
        """pot[targets of tbox[k]] += compressed multipoles mpole[s] of the boxes s in
        lst[list_ptr[k] : list_ptr[k + 1]] evaluated at the targets (fmm_m2p)."""
        nt, nb = self._lists(tbox, list_ptr, lst, center, level, tgt_range, tgt)
        _dev(mpole, self.desc.value_dtype, "mpole", (nb, self.nc))
        _dev(pot, self.desc.value_dtype, "potential", (tgt.shape[0],))
        check(_lib.load().fmm_m2p(self._h, nt, _ptr(tbox), _ptr(list_ptr), lst.shape[0], _ptr(lst), nb, _ptr(center),
                                  _ptr(level), _ptr(tgt_range), tgt.shape[0], _ptr(tgt), _ptr(mpole), _ptr(pot),
                                  _stream()), "fmm_m2p")
        return pot

    def p2l(self, tbox, list_ptr, lst, center, level, src_range, src, w, local) -> torch.Tensor:
        """local[tbox[k]] += compressed locals formed straight from the sources of the boxes in
        lst[list_ptr[k] : list_ptr[k + 1]] (fmm_p2l)."""
        nt, nb = self._lists(tbox, list_ptr, lst, center, level, src_range, src)
        _dev(w, self.desc.value_dtype, "weight", (src.shape[0],))
        _dev(local, self.desc.value_dtype, "local", (nb, self.nc))
        check(_lib.load().fmm_p2l(self._h, nt, _ptr(tbox), _ptr(list_ptr), lst.shape[0], _ptr(lst), nb, _ptr(center),
                                  _ptr(level), _ptr(src_range), src.shape[0], _ptr(src), _ptr(w), _ptr(local),
                                  _stream()), "fmm_p2l")
        return local

    def _tree(self, parent, child, center, level, coef, name):
        npar = parent.shape[0]
        nb = center.shape[0]
        _dev(parent, torch.int32, "parent", (npar,))
        _dev(child, torch.int32, "child", (npar, 8))
        _dev(center, torch.float64, "box_center", (nb, 3))
        _dev(level, torch.int32, "box_level", (nb,))
        _dev(coef, self.desc.value_dtype, name, (nb, self.nc))
        return npar, nb

    def m2m(self, parent, child, center, level, mpole) -> torch.Tensor:
        """mpole[parent[k]] (overwritten) = compressed M2M of its children mpole[child[k, :]]
        (child < 0: none).  One tree level per call."""
        npar, nb = self._tree(parent, child, center, level, mpole, "mpole")
        check(_lib.load().fmm_m2m(self._h, npar, _ptr(parent), _ptr(child), nb, _ptr(center), _ptr(level),
                                  _ptr(mpole), _stream()), "fmm_m2m")
        return mpole

    def l2l(self, parent, child, center, level, local) -> torch.Tensor:
        """local[child[k, :]] += compressed L2L of local[parent[k]] (child < 0: none).  One tree
        level per call."""
        npar, nb = self._tree(parent, child, center, level, local, "local")
        check(_lib.load().fmm_l2l(self._h, npar, _ptr(parent), _ptr(child), nb, _ptr(center), _ptr(level),
                                  _ptr(local), _stream()), "fmm_l2l")
        return local

    def m2m_adjoint(self, parent, child, center, level, mpole_grad) -> torch.Tensor:
        """mpole_grad[child[k, :]] += M2M^T of mpole_grad[parent[k]]."""
        npar, nb = self._tree(parent, child, center, level, mpole_grad, "mpole_grad")
        check(_lib.load().fmm_m2m_adjoint(self._h, npar, _ptr(parent), _ptr(child), nb, _ptr(center),
                                          _ptr(level), _ptr(mpole_grad), _stream()), "fmm_m2m_adjoint")
        return mpole_grad

    def l2l_adjoint(self, parent, child, center, level, local_grad) -> torch.Tensor:
        """local_grad[parent[k]] += L2L^T of local_grad[child[k, :]]."""
        npar, nb = self._tree(parent, child, center, level, local_grad, "local_grad")
        check(_lib.load().fmm_l2l_adjoint(self._h, npar, _ptr(parent), _ptr(child), nb, _ptr(center),
                                          _ptr(level), _ptr(local_grad), _stream()), "fmm_l2l_adjoint")
        return local_grad

    def l2p_adjoint(self, center, level, rng, tgt, pot_grad, local_grad=None, local=None, tgt_grad=None):
        """local_grad (overwritten) = L2P^T(pot_grad); tgt_grad (accumulated) += pot_grad * grad phi
        when given (needs the forward local expansions `local`)."""
        nb = self._boxes(center, level, rng)
        n = tgt.shape[0]
        d = self.desc
        _dev(tgt, d.real_dtype, "tgt_xyz", (n, 3))
        _dev(pot_grad, d.value_dtype, "potential_grad", (n,))
        if local_grad is None:
            local_grad = torch.empty((nb, self.nc), dtype=d.value_dtype, device=tgt.device)
        _dev(local_grad, d.value_dtype, "local_grad", (nb, self.nc))
        if tgt_grad is not None:
            _dev(tgt_grad, d.real_dtype, "tgt_xyz_grad", (n, 3))
            _dev(local, d.value_dtype, "local", (nb, self.nc))
        check(_lib.load().fmm_l2p_adjoint(self._h, nb, _ptr(center), _ptr(level), _ptr(rng), n, _ptr(tgt),
                                          _ptr(local), _ptr(pot_grad), _ptr(local_grad), _ptr(tgt_grad),
                                          _stream()), "fmm_l2p_adjoint")
        return local_grad

    def p2m_adjoint(self, center, level, rng, src, w, mpole_grad, w_grad=None, src_grad=None):
        """w_grad += P2M^T(mpole_grad); src_grad += w * d/dy of it (both accumulated, optional)."""
        nb = self._boxes(center, level, rng)
        n = src.shape[0]
        d = self.desc
        _dev(src, d.real_dtype, "src_xyz", (n, 3))
        _dev(w, d.value_dtype, "weight", (n,))
        _dev(mpole_grad, d.value_dtype, "mpole_grad", (nb, self.nc))
        if w_grad is not None:
            _dev(w_grad, d.value_dtype, "weight_grad", (n,))
        if src_grad is not None:
            _dev(src_grad, d.real_dtype, "src_xyz_grad", (n, 3))
        check(_lib.load().fmm_p2m_adjoint(self._h, nb, _ptr(center), _ptr(level), _ptr(rng), n, _ptr(src),
                                          _ptr(w), _ptr(mpole_grad), _ptr(w_grad), _ptr(src_grad), _stream()),
              "fmm_p2m_adjoint")

    def prepare_adjoint(self, tgt_box, src_box, box_ijk, box_level, tuning=None) -> "Batch":
        """Transpose of the M2L over the same pairs (see fmm_m2l_prepare_adjoint)."""
        if tuning is None:
            tuning = tuned_m2l_shape(self.desc.kernel, self.desc.order, self.desc.dtype)
        elif tuning == "library":
            tuning = None
        return Batch(self, tgt_box, src_box, box_ijk, box_level, tuning, adjoint=True)

    def prepare_fft(self, tgt_box, src_box, box_ijk, box_level) -> "Batch":
        """The FFT form of the batched M2L over the same pairs (fmm_m2l_prepare_fft)."""
        return Batch(self, tgt_box, src_box, box_ijk, box_level, None, fft=True)

    def prepare(self, tgt_box, src_box, box_ijk, box_level, tuning=None) -> "Batch":
        """tuning: None (the autotuned shape for this kernel, order and dtype if there is one,
        else the library's own choice), "library" (the library's choice), or a dict with
        rows_per_wave, col_tiles_per_wave, col_groups, target_items, lds_buffers
        (see fmm_m2l_tuning)."""
        if tuning is None:
            tuning = tuned_m2l_shape(self.desc.kernel, self.desc.order, self.desc.dtype)
        elif tuning == "library":
            tuning = None
        return Batch(self, tgt_box, src_box, box_ijk, box_level, tuning)


class Batch:
    """A prepared M2L batch (host arrays in, device work lists and tables owned)."""

    INFO = ("n_pair", "n_tables", "n_tiles", "n_entries", "n_items", "useful_columns",
            "computed_columns", "nc", "nc_pad", "scratch_bytes", "rows_per_wave", "col_tiles_per_wave",
            "waves", "col_groups", "lds_bytes", "lds_buffers", "k_splits", "valu_rows", "stream_form",
            "workgroups")

    def __init__(self, plan: Plan, tgt_box, src_box, box_ijk, box_level, tuning=None, adjoint=False,
                 fft=False):
        self.plan = plan
        self.adjoint = adjoint
        self.fft = fft
        t = np.ascontiguousarray(np.asarray(tgt_box, dtype=np.int32))
        s = np.ascontiguousarray(np.asarray(src_box, dtype=np.int32))
        ijk = np.ascontiguousarray(np.asarray(box_ijk, dtype=np.int32))
        lev = np.ascontiguousarray(np.asarray(box_level, dtype=np.int32))
        if t.shape != s.shape or ijk.ndim != 2 or ijk.shape[1] != 3 or lev.shape[0] != ijk.shape[0]:
            raise ValueError("pair / box array shapes do not match")
        self.n_box = int(ijk.shape[0])
        self._h = C.c_void_p()
        tun = None
        if tuning is not None:
            form = tuning.get("form", 0)
            form = {"auto": 0, "tiled": 1, "stream": 2}.get(form, form)
            tun = _lib.FmmM2LTuning(int(tuning.get("rows_per_wave", 0)), int(tuning.get("col_tiles_per_wave", 0)),
                                    int(tuning.get("col_groups", 0)), int(tuning.get("target_items", 0)),
                                    int(tuning.get("lds_buffers", 0)), int(tuning.get("k_splits", 0)),
                                    int(form), int(tuning.get("waves", 0)), int(tuning.get("workgroups", 0)))
        args = (plan._h, int(t.shape[0]), t.ctypes.data_as(_lib.I32P), s.ctypes.data_as(_lib.I32P), self.n_box,
                ijk.ctypes.data_as(_lib.I32P), lev.ctypes.data_as(_lib.I32P))
        if fft:
            check(_lib.load().fmm_m2l_prepare_fft(*args, C.byref(self._h)), "fmm_m2l_prepare_fft")
        else:
            fn = _lib.load().fmm_m2l_prepare_adjoint if adjoint else _lib.load().fmm_m2l_prepare_ex
            check(fn(*args, None if tun is None else C.byref(tun), C.byref(self._h)),
                  "fmm_m2l_prepare_adjoint" if adjoint else "fmm_m2l_prepare_ex")

    def info(self) -> dict:
        v = np.zeros(len(self.INFO), dtype=np.int64)
        check(_lib.load().fmm_batch_info(self._h, v.ctypes.data_as(_lib.I64P), len(self.INFO)),
              "fmm_batch_info")
        return dict(zip(self.INFO, v.tolist()))

    def __call__(self, mpole: torch.Tensor, local: torch.Tensor, overwrite: bool = False) -> torch.Tensor:
        """Forward batch: local += M2L(mpole) (overwrite: local = M2L(mpole) for the target rows,
        streaming-form batches only).  Adjoint batch: mpole_grad (2nd) += M2L^T(local_grad)."""
        d = self.plan.desc
        _dev(mpole, d.value_dtype, "input", (self.n_box, self.plan.nc))
        _dev(local, d.value_dtype, "output", (self.n_box, self.plan.nc))
        if overwrite:
            check(_lib.load().fmm_m2l_batched_ex(self._h, _ptr(mpole), _ptr(local), 1, _stream()),
                  "fmm_m2l_batched_ex")
        elif self.adjoint:
            check(_lib.load().fmm_m2l_batched_adjoint(self._h, _ptr(mpole), _ptr(local), _stream()),
                  "fmm_m2l_batched_adjoint")
        else:
            check(_lib.load().fmm_m2l_batched(self._h, _ptr(mpole), _ptr(local), _stream()), "fmm_m2l_batched")
        return local

    def bind(self, mpole: torch.Tensor, local: torch.Tensor, overwrite: bool = False):
        """A zero-argument callable that enqueues this batch on the current stream with the
        given (checked once) tensors; see Plan.bind_p2m.  overwrite (forward streaming-form
        batches): the targets' rows are stored instead of added to."""
        d = self.plan.desc
        _dev(mpole, d.value_dtype, "input", (self.n_box, self.plan.nc))
        _dev(local, d.value_dtype, "output", (self.n_box, self.plan.nc))
        lib = _lib.load()
        h, a, b = self._h, _ptr(mpole), _ptr(local)
        if overwrite:
            fn = lib.fmm_m2l_batched_ex
            return lambda: check(fn(h, a, b, 1, _stream()), "fmm_m2l_batched_ex")
        fn, name = ((lib.fmm_m2l_batched_adjoint, "fmm_m2l_batched_adjoint") if self.adjoint
                    else (lib.fmm_m2l_batched, "fmm_m2l_batched"))
        return lambda: check(fn(h, a, b, _stream()), name)

    def close(self):
        if self._h:
            _lib.load().fmm_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def m2l_multi(batches, mpoles, locals_):
    n = len(batches)
    for b, m, l in zip(batches, mpoles, locals_):
        d = b.plan.desc
        _dev(m, d.value_dtype, "mpole", (b.n_box, b.plan.nc))
        _dev(l, d.value_dtype, "local", (b.n_box, b.plan.nc))
    hb = (C.c_void_p * n)(*[b._h for b in batches])
    hm = (C.c_void_p * n)(*[m.data_ptr() for m in mpoles])
    hl = (C.c_void_p * n)(*[l.data_ptr() for l in locals_])
    check(_lib.load().fmm_m2l_batched_multi(n, hb, hm, hl, _stream()), "fmm_m2l_batched_multi")


def direct(desc: Desc, src, w, tgt, out=None) -> torch.Tensor:
    ns, nt = src.shape[0], tgt.shape[0]
    _dev(src, desc.real_dtype, "src_xyz", (ns, 3))
    _dev(w, desc.value_dtype, "weight", (ns,))
    _dev(tgt, desc.real_dtype, "tgt_xyz", (nt, 3))
    if out is None:
        out = torch.empty(nt, dtype=desc.value_dtype, device=tgt.device)
    _dev(out, desc.value_dtype, "potential", (nt,))
    check(_lib.load().fmm_direct(C.byref(desc.c), ns, _ptr(src), _ptr(w), nt, _ptr(tgt), _ptr(out),
                                 _stream()), "fmm_direct")
    return out


def p2p(desc: Desc, tbox, nbr_ptr, nbr, tgt_range, src_range, src, w, tgt, pot) -> torch.Tensor:
    """Near field: pot[targets of tbox[k]] += direct sum over the sources of the boxes
    nbr[nbr_ptr[k] : nbr_ptr[k + 1]] (fmm_p2p).  Point ranges are per box id.  A target box may
    be listed several times (a long list split into parts that run in parallel; the parts are
    added atomically, in no fixed order)."""
    nt_box, nb = tbox.shape[0], tgt_range.shape[0]
    ns, nt = src.shape[0], tgt.shape[0]
    _dev(tbox, torch.int32, "tbox", (nt_box,))
    _dev(nbr_ptr, torch.int32, "nbr_ptr", (nt_box + 1,))
    _dev(nbr, torch.int32, "nbr", (nbr.shape[0],))
    _dev(tgt_range, torch.int64, "tgt_range", (nb, 2))
    _dev(src_range, torch.int64, "src_range", (nb, 2))
    _dev(src, desc.real_dtype, "src_xyz", (ns, 3))
    _dev(w, desc.value_dtype, "weight", (ns,))
    _dev(tgt, desc.real_dtype, "tgt_xyz", (nt, 3))
    _dev(pot, desc.value_dtype, "potential", (nt,))
    check(_lib.load().fmm_p2p(C.byref(desc.c), nt_box, _ptr(tbox), _ptr(nbr_ptr), nbr.shape[0], _ptr(nbr), nb,
                              _ptr(tgt_range), _ptr(src_range), ns, _ptr(src), _ptr(w), nt, _ptr(tgt), _ptr(pot),
                              _stream()), "fmm_p2p")
    return pot


class Multi:
    """Several prepared forward batches of one dtype enqueued as one unit (fmm_m2l_multi_*):
    streaming-form batches each in their own tuned launch, tiled-form batches that share a
    tile shape drained by one persistent launch."""

    def __init__(self, batches):
        self.batches = list(batches)
        n = len(self.batches)
        hb = (C.c_void_p * n)(*[b._h for b in self.batches])
        self._h = C.c_void_p()
        check(_lib.load().fmm_m2l_multi_prepare(n, hb, C.byref(self._h)), "fmm_m2l_multi_prepare")

    def __call__(self, mpoles, locals_):
        n = len(self.batches)
        for b, m, l in zip(self.batches, mpoles, locals_):
            d = b.plan.desc
            _dev(m, d.value_dtype, "mpole", (b.n_box, b.plan.nc))
            _dev(l, d.value_dtype, "local", (b.n_box, b.plan.nc))
        hm = (C.c_void_p * n)(*[m.data_ptr() for m in mpoles])
        hl = (C.c_void_p * n)(*[l.data_ptr() for l in locals_])
        check(_lib.load().fmm_m2l_multi_launch(self._h, hm, hl, _stream()), "fmm_m2l_multi_launch")

    def close(self):
        if self._h:
            _lib.load().fmm_m2l_multi_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    """Octree and interaction lists built on the device (fmm_tree_*).

    max_leaf == 0: uniform tree of the given depth (every box of every level); max_leaf > 0:
    adaptive tree, boxes above max_leaf points refined down to level `depth` at most, empty
    children not created.  Box order: level by level, Morton order within a level; each box's
    points are one range of the sorted points.  Arrays come back as device tensors."""

    def __init__(self, points: torch.Tensor, max_leaf: int = 0, depth: int = 3):
        _dev(points, torch.float64, "points")
        if points.dim() != 2 or points.shape[1] != 3:
            raise ValueError("points: expected shape (n, 3)")
        self.n = points.shape[0]
        self.max_leaf, self.depth = int(max_leaf), int(depth)
        self.device = points.device
        self._h = C.c_void_p()
        L = _lib.load()
        check(L.fmm_tree_build(self.n, _ptr(points), self.max_leaf, self.depth, C.byref(self._h), _stream()),
              "fmm_tree_build")
        nb, nl, nleaf = C.c_int64(), C.c_int32(), C.c_int64()
        check(L.fmm_tree_size(self._h, C.byref(nb), C.byref(nl), C.byref(nleaf)), "fmm_tree_size")
        self.n_box, self.n_levels, self.n_leaf = nb.value, nl.value, nleaf.value

    def arrays(self) -> dict:
        """perm, points (sorted), level, ijk, center, pt_range, is_leaf (device tensors) and
        level_start (numpy)."""
        dev, n, nb = self.device, self.n, self.n_box
        out = {"perm": torch.empty(n, dtype=torch.int64, device=dev),
               "points": torch.empty((n, 3), dtype=torch.float64, device=dev),
               "level": torch.empty(nb, dtype=torch.int32, device=dev),
               "ijk": torch.empty((nb, 3), dtype=torch.int32, device=dev),
               "center": torch.empty((nb, 3), dtype=torch.float64, device=dev),
               "pt_range": torch.empty((nb, 2), dtype=torch.int64, device=dev),
               "is_leaf": torch.empty(nb, dtype=torch.uint8, device=dev)}
        ls = np.zeros(self.n_levels + 1, dtype=np.int64)
        o = out
        check(_lib.load().fmm_tree_export(self._h, _ptr(o["perm"]), _ptr(o["points"]), _ptr(o["level"]),
                                          _ptr(o["ijk"]), _ptr(o["center"]), _ptr(o["pt_range"]),
                                          _ptr(o["is_leaf"]), ls.ctypes.data_as(_lib.I64P), _stream()),
              "fmm_tree_export")
        out["level_start"] = ls
        return out

    def to_host(self):
        """The tree as a workloads.Tree (numpy arrays), for the host-side set-up calls."""
        import workloads as W
        a = {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in self.arrays().items()}
        kind = "uniform" if self.max_leaf == 0 else "adaptive"
        meta = {"depth": self.depth} if self.max_leaf == 0 else {"max_leaf": self.max_leaf}
        return W.Tree(points=a["points"], perm=a["perm"], level=a["level"], ijk=a["ijk"], center=a["center"],
                      pt_range=a["pt_range"], level_start=a["level_start"], is_leaf=a["is_leaf"].astype(bool),
                      kind=kind, meta=meta)

    def list2(self, level_lo: int = 2, level_hi: int | None = None):
        """List-2 pairs (target, source) of the target boxes on levels [level_lo, level_hi),
        sorted by (target, source): two int32 device tensors.  The range is clipped to the
        tree's levels (levels 0 and 1 have no List-2 pairs)."""
        hi = self.n_levels if level_hi is None else min(int(level_hi), self.n_levels)
        level_lo = min(max(int(level_lo), 0), hi)
        L, n = _lib.load(), C.c_int64()
        check(L.fmm_tree_list2(self._h, int(level_lo), hi, C.byref(n), None, None, _stream()), "fmm_tree_list2")
        t = torch.empty(n.value, dtype=torch.int32, device=self.device)
        s = torch.empty_like(t)
        check(L.fmm_tree_list2(self._h, int(level_lo), hi, C.byref(n), _ptr(t), _ptr(s), _stream()),
              "fmm_tree_list2")
        return t, s

    def lists(self, kind: str, max_src: int | None = None):
        """Rows (box, ptr, item) of the near, U, W or X lists (int32 device tensors); max_src cuts
        long near / U rows as fmm_tree_lists describes."""
        L, nr, ni = _lib.load(), C.c_int64(), C.c_int64()
        k, ms = _lib.LIST_KINDS[kind], int(max_src or 0)
        check(L.fmm_tree_lists(self._h, k, ms, C.byref(nr), C.byref(ni), None, None, None, _stream()),
              "fmm_tree_lists")
        box = torch.empty(nr.value, dtype=torch.int32, device=self.device)
        ptr = torch.empty(nr.value + 1, dtype=torch.int32, device=self.device)
        item = torch.empty(ni.value, dtype=torch.int32, device=self.device)
        check(L.fmm_tree_lists(self._h, k, ms, C.byref(nr), C.byref(ni), _ptr(box), _ptr(ptr), _ptr(item),
                               _stream()), "fmm_tree_lists")
        return box, ptr, item

    def close(self):
        if self._h:
            _lib.load().fmm_tree_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- two dimensions

def index_table2d(desc: Desc) -> np.ndarray:
    """J of a 2-D descriptor in storage order, [Nc, 2] (a, b)."""
    out = np.zeros((desc.nc, 2), dtype=np.int32)
    check(_lib.load().fmm2d_index_table(C.byref(desc.c), out.ctypes.data_as(_lib.I32P)), "fmm2d_index_table")
    return out


def deriv_tables2d(desc: Desc, offsets: torch.Tensor, h: torch.Tensor) -> torch.Tensor:
    """Scaled 2-D tables [n, 2c - 1, 2p + 1] at offsets [n, 2] (units of h) and sizes h [n]."""
    n = offsets.shape[0]
    _dev(offsets, torch.float64, "offset", (n, 2))
    _dev(h, torch.float64, "h", (n,))
    c = 4 if desc.kernel == "biharmonic2d" else 2
    out = torch.empty((n, 2 * c - 1, 2 * desc.order + 1), dtype=torch.float64, device=offsets.device)
    check(_lib.load().fmm2d_deriv_tables(C.byref(desc.c), n, _ptr(offsets), _ptr(h), _ptr(out), _stream()),
          "fmm2d_deriv_tables")
    return out


def _max_count(rng, given):
    if given is not None:
        return int(given)
    return int((rng[:, 1] - rng[:, 0]).max().item()) if rng.shape[0] else 1


def p2m2d(desc: Desc, center, box_h, rng, src, w, out=None, max_per_box=None) -> torch.Tensor:
    """out += compressed scaled multipoles of the boxes (zeros when out is None).  max_per_box:
    the largest point count of a box (sets the launch width; read from rng when None)."""
    nb, ns = center.shape[0], src.shape[0]
    _dev(center, torch.float64, "box_center", (nb, 2))
    _dev(box_h, torch.float64, "box_h", (nb,))
    _dev(rng, torch.int64, "pt_range", (nb, 2))
    _dev(src, torch.float64, "src_xy", (ns, 2))
    _dev(w, torch.float64, "weight", (ns,))
    if out is None:
        out = torch.zeros((nb, desc.nc), dtype=torch.float64, device=center.device)
    _dev(out, torch.float64, "mpole", (nb, desc.nc))
    check(_lib.load().fmm2d_p2m(C.byref(desc.c), nb, _ptr(center), _ptr(box_h), _ptr(rng), ns, _ptr(src), _ptr(w),
                                _ptr(out), max(1, _max_count(rng, max_per_box)), _stream()), "fmm2d_p2m")
    return out


def m2l2d(desc: Desc, tbox, pair_ptr, pair_src, pair_tab, tables, mpole, local) -> torch.Tensor:
    nt, npair, ntab, nb = tbox.shape[0], pair_src.shape[0], tables.shape[0], mpole.shape[0]
    _dev(tbox, torch.int32, "tbox", (nt,))
    _dev(pair_ptr, torch.int32, "pair_ptr", (nt + 1,))
    _dev(pair_src, torch.int32, "pair_src", (npair,))
    _dev(pair_tab, torch.int32, "pair_tab", (npair,))
    _dev(tables, torch.float64, "tables")
    _dev(mpole, torch.float64, "mpole", (nb, desc.nc))
    _dev(local, torch.float64, "local", (nb, desc.nc))
    check(_lib.load().fmm2d_m2l(C.byref(desc.c), nt, _ptr(tbox), _ptr(pair_ptr), npair, _ptr(pair_src),
                                _ptr(pair_tab), ntab, _ptr(tables), nb, _ptr(mpole), _ptr(local), _stream()),
          "fmm2d_m2l")
    return local


def l2p2d(desc: Desc, center, box_h, rng, tgt, local, pot, max_per_box=None) -> torch.Tensor:
    nb, nt = center.shape[0], tgt.shape[0]
    _dev(center, torch.float64, "box_center", (nb, 2))
    _dev(box_h, torch.float64, "box_h", (nb,))
    _dev(rng, torch.int64, "pt_range", (nb, 2))
    _dev(tgt, torch.float64, "tgt_xy", (nt, 2))
    _dev(local, torch.float64, "local", (nb, desc.nc))
    _dev(pot, torch.float64, "potential", (nt,))
    check(_lib.load().fmm2d_l2p(C.byref(desc.c), nb, _ptr(center), _ptr(box_h), _ptr(rng), nt, _ptr(tgt),
                                _ptr(local), _ptr(pot), max(1, _max_count(rng, max_per_box)), _stream()),
          "fmm2d_l2p")
    return pot


def _tree2d(desc: Desc, name, parent, child, center, box_h, coef):
    npar, nb = parent.shape[0], center.shape[0]
    _dev(parent, torch.int32, "parent", (npar,))
    _dev(child, torch.int32, "child", (npar, 4))
    _dev(center, torch.float64, "box_center", (nb, 2))
    _dev(box_h, torch.float64, "box_h", (nb,))
    _dev(coef, torch.float64, "coefficients", (nb, desc.nc))
    check(getattr(_lib.load(), name)(C.byref(desc.c), npar, _ptr(parent), _ptr(child), nb, _ptr(center),
                                     _ptr(box_h), _ptr(coef), _stream()), name)
    return coef


def m2m2d(desc: Desc, parent, child, center, box_h, mpole) -> torch.Tensor:
    """mpole[parent] = compressed M2M of its (up to four) children (overwrites the parents' rows)."""
    return _tree2d(desc, "fmm2d_m2m", parent, child, center, box_h, mpole)


def l2l2d(desc: Desc, parent, child, center, box_h, local) -> torch.Tensor:
    """local[children] += compressed L2L of their parent's local."""
    return _tree2d(desc, "fmm2d_l2l", parent, child, center, box_h, local)


def direct2d(desc: Desc, src, w, tgt, out=None) -> torch.Tensor:
    ns, nt = src.shape[0], tgt.shape[0]
    _dev(src, torch.float64, "src_xy", (ns, 2))
    _dev(w, torch.float64, "weight", (ns,))
    _dev(tgt, torch.float64, "tgt_xy", (nt, 2))
    if out is None:
        out = torch.empty(nt, dtype=torch.float64, device=tgt.device)
    _dev(out, torch.float64, "potential", (nt,))
    check(_lib.load().fmm2d_direct(C.byref(desc.c), ns, _ptr(src), _ptr(w), nt, _ptr(tgt), _ptr(out), _stream()),
          "fmm2d_direct")
    return out


def p2p2d(desc: Desc, tbox, nbr_ptr, nbr, tgt_range, src_range, src, w, tgt, pot, max_tgt_per_box: int):
    nt_box, nb = tbox.shape[0], tgt_range.shape[0]
    ns, nt = src.shape[0], tgt.shape[0]
    _dev(tbox, torch.int32, "tbox", (nt_box,))
    _dev(nbr_ptr, torch.int32, "nbr_ptr", (nt_box + 1,))
    _dev(nbr, torch.int32, "nbr", (nbr.shape[0],))
    _dev(tgt_range, torch.int64, "tgt_range", (nb, 2))
    _dev(src_range, torch.int64, "src_range", (nb, 2))
    _dev(src, torch.float64, "src_xy", (ns, 2))
    _dev(w, torch.float64, "weight", (ns,))
    _dev(tgt, torch.float64, "tgt_xy", (nt, 2))
    _dev(pot, torch.float64, "potential", (nt,))
    check(_lib.load().fmm2d_p2p(C.byref(desc.c), nt_box, _ptr(tbox), _ptr(nbr_ptr), nbr.shape[0], _ptr(nbr), nb,
                                _ptr(tgt_range), _ptr(src_range), ns, _ptr(src), _ptr(w), nt, _ptr(tgt), _ptr(pot),
                                max(1, int(max_tgt_per_box)), _stream()), "fmm2d_p2p")
    return pot
