"""ctypes binding of libdefmm.so (include/defmm.h).

Argument marshalling only: every step of the matvec runs in the library's HIP
kernels.  torch provides device buffers and streams.  If the library is not
built, importing this module raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdefmm.so")

C128, C64 = 0, 1
M2L_AUTO, M2L_FFT, M2L_DENSE = 0, 1, 2
SAME_POINTS = 1
COMPRESS_SPECTRA = 2
YUKAWA = 4  # screened kernel exp(-kappa r) / (4 pi r); every level low-frequency
NUM_PASSES = 12


class DefmmError(RuntimeError):
    pass


class _Params(ctypes.Structure):
    _fields_ = [("order_L", ctypes.c_int32), ("ncrit", ctypes.c_int32), ("eta", ctypes.c_double),
                ("hf_threshold", ctypes.c_double), ("dir_refine", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("m2l_mode", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Tuning(ctypes.Structure):
    _fields_ = [("overlap", ctypes.c_int32), ("p2p_waves_per_cu", ctypes.c_int32), ("m2l_variant", ctypes.c_int32),
                ("dense_levels", ctypes.c_uint32), ("updown_variant", ctypes.c_int32),
                ("fourier_items", ctypes.c_int32), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("hf_levels", ctypes.c_int32), ("cells", ctypes.c_int64),
                ("leaves", ctypes.c_int64), ("m2l_pairs", ctypes.c_int64),
                ("p2p_cell_pairs", ctypes.c_int64), ("p2p_point_pairs", ctypes.c_int64),
                ("eff_expansions", ctypes.c_int64), ("m2l_expansions", ctypes.c_int64),
                ("unique_offsets", ctypes.c_int64), ("m2l_mode_per_level", ctypes.c_int32 * 32),
                ("spectra", ctypes.c_int64), ("compressed_spectra", ctypes.c_int32)]


EXPORTS = ["defmm_default_params", "defmm_plan_create", "defmm_plan_inspect_create", "defmm_plan_footprint", "defmm_plan_stats",
           "defmm_workspace_create", "defmm_matvec", "defmm_matvec_graph", "defmm_workspace_destroy", "defmm_plan_destroy",
           "defmm_status_string", "defmm_last_error", "defmm_plan_geometry", "defmm_plan_export_tree",
           "defmm_plan_export_m2l", "defmm_plan_export_p2p", "defmm_plan_export_marks",
           "defmm_workspace_export_expansions",
           "defmm_workspace_set_timing", "defmm_workspace_set_overlap", "defmm_workspace_pass_times",
           "defmm_workspace_autotune", "defmm_workspace_get_tuning", "defmm_workspace_set_tuning",
           "defmm_pass_name",
           "defmm_workspace_pass_work", "defmm_fourier_layout", "defmm_canonical_offset",
           "defmm_directions", "defmm_matvec_noalloc", "defmm_matvec_noalloc_capacity"]

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise DefmmError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, f64, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    L.defmm_default_params.argtypes = [P]
    L.defmm_plan_create.argtypes = [P, i64, P, i64, f64, P, P, P]
    L.defmm_plan_inspect_create.argtypes = [P, i64, P, i64, f64, P, P]
    L.defmm_plan_footprint.argtypes = [P, P, P]
    L.defmm_plan_stats.argtypes = [P, P]
    L.defmm_workspace_create.argtypes = [P, P]
    L.defmm_matvec.argtypes = [P, P, P, P, P]
    L.defmm_matvec_graph.argtypes = [P, P, P, P, P]
    L.defmm_workspace_destroy.argtypes = [P]
    L.defmm_plan_destroy.argtypes = [P]
    L.defmm_status_string.argtypes = [st]
    L.defmm_status_string.restype = ctypes.c_char_p
    L.defmm_last_error.restype = ctypes.c_char_p
    L.defmm_plan_geometry.argtypes = [P, P, P]
    L.defmm_plan_export_tree.argtypes = [P, i32, P, P, P, P, P, P, P]
    L.defmm_plan_export_m2l.argtypes = [P, P, P, P, P, P, P]
    L.defmm_plan_export_p2p.argtypes = [P, P, P, P]
    L.defmm_plan_export_marks.argtypes = [P, i32, P, P, P]
    L.defmm_workspace_export_expansions.argtypes = [P, i32, i32, P, P, P, P]
    L.defmm_workspace_set_timing.argtypes = [P, i32]
    L.defmm_workspace_set_overlap.argtypes = [P, i32]
    L.defmm_workspace_autotune.argtypes = [P, P, P, P, P, i32, P]
    L.defmm_workspace_get_tuning.argtypes = [P, P]
    L.defmm_workspace_set_tuning.argtypes = [P, P]
    L.defmm_workspace_pass_times.argtypes = [P, P, P]
    L.defmm_pass_name.argtypes = [i32]
    L.defmm_pass_name.restype = ctypes.c_char_p
    L.defmm_workspace_pass_work.argtypes = [P, P, P]
    L.defmm_fourier_layout.argtypes = [i32, P, P, P, P, P]
    L.defmm_canonical_offset.argtypes = [P, P, P]
    L.defmm_directions.argtypes = [i32, P, P, P]
    L.defmm_matvec_noalloc.argtypes = [P, P, P, P]
    L.defmm_matvec_noalloc_capacity.argtypes = []
    for name in EXPORTS:
        if name not in ("defmm_status_string", "defmm_last_error", "defmm_pass_name",
                        "defmm_matvec_noalloc_capacity"):
            getattr(L, name).restype = st
    L.defmm_matvec_noalloc_capacity.restype = ctypes.c_size_t
    _lib = L
    return L


def _check(status):
    if status != 0:
        L = lib()
        raise DefmmError(f"{L.defmm_status_string(status).decode()}: {L.defmm_last_error().decode()}")


def fourier_layout(L: int):
    """Storage order of the Fourier-domain rows for order L (host only):
    (slices, cap, freq [row] int32, perm [slices, 48, 64] uint8)."""
    sl, cap, row = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().defmm_fourier_layout(L, ctypes.byref(sl), ctypes.byref(cap), ctypes.byref(row), None, None))
    freq = np.zeros(row.value, np.int32)
    perm = np.zeros((sl.value, 48, 64), np.uint8)
    _check(lib().defmm_fourier_layout(L, ctypes.byref(sl), ctypes.byref(cap), ctypes.byref(row),
                                      _np_ptr(freq), _np_ptr(perm)))
    return sl.value, cap.value, freq, perm


def canonical_offset(d):
    """(sorted |d|, symmetry code) of an M2L offset (host only)."""
    a = np.ascontiguousarray(d, dtype=np.int32)
    d0 = np.zeros(3, np.int32)
    code = ctypes.c_int32()
    _check(lib().defmm_canonical_offset(_np_ptr(a), _np_ptr(d0), ctypes.byref(code)))
    return d0, code.value


def directions(E: int):
    """The library's direction set at direction level E (host only): unit
    vectors [6 * 4^E, 3] and father indices (-1 at E = 0)."""
    n = ctypes.c_int64()
    _check(lib().defmm_directions(E, ctypes.byref(n), None, None))
    d = np.zeros((n.value, 3))
    f = np.zeros(n.value, np.int64)
    _check(lib().defmm_directions(E, ctypes.byref(n), _np_ptr(d), _np_ptr(f)))
    return d, f


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Params:
    order_L: int = 5
    ncrit: int = 64
    eta: float = 1.0
    hf_threshold: float = 2.0
    dir_refine: int = 0
    precision: int = C64
    m2l_mode: int = M2L_FFT
    flags: int = 0

    def c(self):
        return _Params(self.order_L, self.ncrit, self.eta, self.hf_threshold, self.dir_refine,
                       self.precision, self.m2l_mode, self.flags)


def pass_name(i: int) -> str:
    return lib().defmm_pass_name(i).decode()


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A plan over target points X and source points Y (None: Y is X)."""

    def __init__(self, X, Y=None, kappa=0.0, params: Params | None = None, stream=None):
        import torch
        self.params = params or Params()
        same = Y is None
        if same:
            self.params.flags |= SAME_POINTS
        X = torch.as_tensor(X, dtype=torch.float64, device="cuda").contiguous()
        Yt = X if same else torch.as_tensor(Y, dtype=torch.float64, device="cuda").contiguous()
        self.nx, self.ny = X.shape[0], Yt.shape[0]
        self.kappa = float(kappa)
        self.cdtype = torch.complex128 if self.params.precision == C128 else torch.complex64
        self._prm = self.params.c()
        h = ctypes.c_void_p()
        _check(lib().defmm_plan_create(ctypes.c_void_p(X.data_ptr()), self.nx,
                                       None if same else ctypes.c_void_p(Yt.data_ptr()), self.ny,
                                       self.kappa, ctypes.byref(self._prm), _stream_handle(stream),
                                       ctypes.byref(h)))
        self.h = h

    @classmethod
    def inspect(cls, X, Y=None, kappa=0.0, params: Params | None = None):
        """Host-only plan (no device use): stats and exported lists only."""
        self = cls.__new__(cls)
        self.params = params or Params()
        same = Y is None
        if same:
            self.params.flags |= SAME_POINTS
        X = np.ascontiguousarray(X, dtype=np.float64)
        Yn = X if same else np.ascontiguousarray(Y, dtype=np.float64)
        self.nx, self.ny = X.shape[0], Yn.shape[0]
        self.kappa = float(kappa)
        self.cdtype = None
        self._prm = self.params.c()
        h = ctypes.c_void_p()
        _check(lib().defmm_plan_inspect_create(_np_ptr(X), self.nx, None if same else _np_ptr(Yn), self.ny,
                                               self.kappa, ctypes.byref(self._prm), ctypes.byref(h)))
        self.h = h
        return self

    def close(self):
        if getattr(self, "h", None):
            lib().defmm_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> dict:
        s = _Stats()
        _check(lib().defmm_plan_stats(self.h, ctypes.byref(s)))
        d = {k: getattr(s, k) for k, _ in _Stats._fields_ if k != "m2l_mode_per_level"}
        d["m2l_mode_per_level"] = list(s.m2l_mode_per_level)[: max(d["levels"], 0)]
        return d

    def footprint(self):
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().defmm_plan_footprint(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def geometry(self):
        D = ctypes.c_double()
        o = np.zeros(3)
        _check(lib().defmm_plan_geometry(self.h, ctypes.byref(D), _np_ptr(o)))
        return D.value, o

    def tree(self, which=0):
        n = ctypes.c_int64()
        _check(lib().defmm_plan_export_tree(self.h, which, ctypes.byref(n), None, None, None, None, None,
                                            None))
        n = n.value
        lev = np.zeros(n, np.int32)
        ijk = np.zeros((n, 3), np.int32)
        first = np.zeros(n, np.int32)
        count = np.zeros(n, np.int32)
        leaf = np.zeros(n, np.int32)
        perm = np.zeros(self.nx if which == 0 else self.ny, np.int32)
        nn = ctypes.c_int64()
        _check(lib().defmm_plan_export_tree(self.h, which, ctypes.byref(nn), _np_ptr(lev), _np_ptr(ijk),
                                            _np_ptr(first), _np_ptr(count), _np_ptr(leaf), _np_ptr(perm)))
        return dict(level=lev, ijk=ijk, first=first, count=count, is_leaf=leaf, perm=perm)

    def m2l(self):
        n = ctypes.c_int64()
        _check(lib().defmm_plan_export_m2l(self.h, ctypes.byref(n), None, None, None, None, None))
        n = n.value
        lev, t, s, u = (np.zeros(n, np.int32) for _ in range(4))
        d = np.zeros((n, 3), np.int32)
        _check(lib().defmm_plan_export_m2l(self.h, ctypes.byref(ctypes.c_int64()), _np_ptr(lev), _np_ptr(t),
                                           _np_ptr(s), _np_ptr(d), _np_ptr(u)))
        return dict(level=lev, t=t, s=s, delta=d, dir=u)

    def marks(self, which=0):
        """Effective expansions of tree `which` (0 = X, 1 = Y): cell ids and
        direction indices (-1 = non-directional), ordered by cell, direction."""
        n = ctypes.c_int64()
        _check(lib().defmm_plan_export_marks(self.h, which, ctypes.byref(n), None, None))
        cell = np.zeros(n.value, np.int32)
        d = np.zeros(n.value, np.int32)
        _check(lib().defmm_plan_export_marks(self.h, which, ctypes.byref(ctypes.c_int64()), _np_ptr(cell),
                                             _np_ptr(d)))
        return dict(cell=cell, dir=d)

    def p2p(self):
        n = ctypes.c_int64()
        _check(lib().defmm_plan_export_p2p(self.h, ctypes.byref(n), None, None))
        t = np.zeros(n.value, np.int32)
        s = np.zeros(n.value, np.int32)
        _check(lib().defmm_plan_export_p2p(self.h, ctypes.byref(n), _np_ptr(t), _np_ptr(s)))
        return dict(t=t, s=s)



def matvec_noalloc(plan: "Plan", q, p, stream=None):
    """p = G q through the allocation-free entry point: the workspace lives in
    the library's static device array (defmm_matvec_noalloc_capacity() bytes per
    GPU), nothing is allocated, so p must be given.  Calls on one GPU must not
    overlap."""
    if q.dtype != plan.cdtype or not q.is_cuda or q.shape != (plan.ny,) or not q.is_contiguous():
        raise DefmmError(f"q must be a contiguous cuda {plan.cdtype} tensor of shape ({plan.ny},)")
    if p.dtype != plan.cdtype or not p.is_cuda or p.shape != (plan.nx,) or not p.is_contiguous():
        raise DefmmError(f"p must be a contiguous cuda {plan.cdtype} tensor of shape ({plan.nx},)")
    _check(lib().defmm_matvec_noalloc(plan.h, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(p.data_ptr()),
                                      _stream_handle(stream)))
    return p


def noalloc_capacity() -> int:
    """Bytes of the allocation-free matvec's static device workspace."""
    return int(lib().defmm_matvec_noalloc_capacity())


def torch_empty_like_out(plan, q):
    import torch
    return torch.empty(plan.nx, dtype=plan.cdtype, device=q.device)


class Workspace:
    def __init__(self, plan: Plan):
        self.plan = plan
        h = ctypes.c_void_p()
        _check(lib().defmm_workspace_create(plan.h, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().defmm_workspace_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matvec(self, q, p=None, stream=None, graph=False):
        """p = G q on the device; q: complex tensor on cuda (caller order).
        graph=True replays a HIP graph captured for this (q, p) pair (refill q
        in place; a created stream is needed)."""
        import torch
        pl = self.plan
        if q.dtype != pl.cdtype or not q.is_cuda or q.shape != (pl.ny,):
            raise DefmmError(f"q must be a cuda {pl.cdtype} tensor of shape ({pl.ny},)")
        q = q.contiguous()
        if p is None:
            p = torch.empty(pl.nx, dtype=pl.cdtype, device=q.device)
        elif p.dtype != pl.cdtype or not p.is_cuda or p.shape != (pl.nx,) or not p.is_contiguous():
            raise DefmmError(f"p must be a contiguous cuda {pl.cdtype} tensor of shape ({pl.nx},)")
        fn = lib().defmm_matvec_graph if graph else lib().defmm_matvec
        _check(fn(pl.h, self.h, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(p.data_ptr()),
                  _stream_handle(stream)))
        return p

    def set_timing(self, on: bool):
        _check(lib().defmm_workspace_set_timing(self.h, 1 if on else 0))

    def autotune(self, q, reps=3, stream=None):
        """Time the execution choices on charges q and keep the fastest."""
        pl = self.plan
        q = q.contiguous()
        p = torch_empty_like_out(pl, q)
        t = Tuning()
        _check(lib().defmm_workspace_autotune(pl.h, self.h, ctypes.c_void_p(q.data_ptr()),
                                              ctypes.c_void_p(p.data_ptr()), _stream_handle(stream), reps,
                                              ctypes.byref(t)))
        return t.as_dict()

    def tuning(self):
        t = Tuning()
        _check(lib().defmm_workspace_get_tuning(self.h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, overlap=2, p2p_waves_per_cu=2, m2l_variant=2, dense_levels=0, updown_variant=1,
                   fourier_items=0, **_):
        t = Tuning(overlap, p2p_waves_per_cu, m2l_variant, dense_levels, updown_variant, fourier_items, 0.0)
        _check(lib().defmm_workspace_set_tuning(self.h, ctypes.byref(t)))

    def set_overlap(self, on: bool):
        _check(lib().defmm_workspace_set_overlap(self.h, 1 if on else 0))

    def pass_work(self):
        """Compulsory HBM bytes and flops of one matvec per pass, under the
        workspace's current execution choices."""
        b = np.zeros(NUM_PASSES)
        f = np.zeros(NUM_PASSES)
        _check(lib().defmm_workspace_pass_work(self.h, _np_ptr(b), _np_ptr(f)))
        return b, f

    def pass_times(self):
        ms = np.zeros(NUM_PASSES)
        calls = np.zeros(NUM_PASSES, np.int64)
        _check(lib().defmm_workspace_pass_times(self.h, _np_ptr(ms), _np_ptr(calls)))
        return ms, calls

    def expansions(self, which=0, kind=0):
        pl = self.plan
        n = ctypes.c_int64()
        _check(lib().defmm_workspace_export_expansions(self.h, which, kind, ctypes.byref(n), None, None,
                                                       None))
        n = n.value
        L3 = pl.params.order_L ** 3
        cell = np.zeros(n, np.int32)
        d = np.zeros(n, np.int32)
        vals = np.zeros((n, L3), np.complex128 if pl.params.precision == C128 else np.complex64)
        _check(lib().defmm_workspace_export_expansions(self.h, which, kind, ctypes.byref(ctypes.c_int64()),
                                                       _np_ptr(cell), _np_ptr(d), _np_ptr(vals)))
        return dict(cell=cell, dir=d, values=vals)
