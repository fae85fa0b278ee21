"""defmm oracle -- TEST INFRASTRUCTURE ONLY.

ctypes binding over ``liboracle.so`` (built from ``defmm_oracle.c`` by
``oracle.build()``): a plain FP64 CPU implementation of the directional
equispaced-interpolation FMM and of the direct sum it approximates.  Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package; the product path never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "defmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, no FP contraction)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           _SRC, "-o", _LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.oracle_direct_sum.argtypes = [P, i64, P, i64, P, f64, f64, P, i64, P, i32]
        L.oracle_direct_sum.restype = None
        L.oracle_lagrange_1d.argtypes = [i32, f64, P]
        L.oracle_directions.argtypes = [i32, P, P]
        L.oracle_directions.restype = i64
        L.oracle_spectrum.argtypes = [f64, f64, i32, P, P, i32]
        L.oracle_m2l_fft.argtypes = [f64, f64, i32, P, P, P, i32]
        L.oracle_m2l_dense.argtypes = [f64, f64, i32, P, P, P, i32]
        L.oracle_dft3.argtypes = [i32, P, P, i32]
        L.oracle_p2m.argtypes = [f64, i32, P, f64, P, i64, P, P, P]
        L.oracle_m2m.argtypes = [f64, i32, P, f64, P, P, f64, P, P]
        L.oracle_l2l.argtypes = [f64, i32, P, f64, P, P, f64, P, P]
        L.oracle_l2p.argtypes = [f64, i32, P, f64, P, P, i64, P, P]
        L.oracle_fmm_create.argtypes = [P, i64, P, i64, i32, f64, P]
        L.oracle_fmm_create.restype = P
        L.oracle_fmm_destroy.argtypes = [P]
        L.oracle_fmm_apply.argtypes = [P, P, P]
        L.oracle_fmm_apply.restype = f64
        L.oracle_fmm_info.argtypes = [P, P]
        L.oracle_fmm_geometry.argtypes = [P, P]
        L.oracle_fmm_geometry.restype = f64
        L.oracle_fmm_perm.argtypes = [P, i32, P]
        L.oracle_fmm_perm.restype = i64
        L.oracle_fmm_cells.argtypes = [P, i32, P, P, P, P, P]
        L.oracle_fmm_cells.restype = i64
        L.oracle_fmm_m2l.argtypes = [P, P, P, P, P, P]
        L.oracle_fmm_m2l.restype = i64
        L.oracle_fmm_p2p.argtypes = [P, P, P]
        L.oracle_fmm_p2p.restype = i64
        L.oracle_fmm_expansions.argtypes = [P, i32, P, P, P, P]
        L.oracle_fmm_expansions.restype = i64
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# The kernel G(r), r = |x - y|: HELMHOLTZ = exp(i kappa r) / (4 pi r) (the paper's),
# YUKAWA = exp(-kappa r) / (4 pi r) (screened, non-oscillatory: every level is
# low-frequency).
HELMHOLTZ, YUKAWA = 0, 1


class _Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("ncrit", ctypes.c_int32), ("eta", ctypes.c_double),
                ("hf_threshold", ctypes.c_double), ("dir_refine", ctypes.c_int32),
                ("kernel", ctypes.c_int32)]


@dataclass
class Params:
    L: int = 4
    ncrit: int = 32
    eta: float = 1.0
    hf_threshold: float = 2.0
    dir_refine: int = 0
    kernel: int = HELMHOLTZ

    def c(self):
        return _Params(self.L, self.ncrit, self.eta, self.hf_threshold, self.dir_refine, self.kernel)


def direct_sum(X, Y, q, kappa, tau, targets=None, kernel=HELMHOLTZ):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.complex128)
    if targets is None:
        nt = X.shape[0]
        tg = None
    else:
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tg.shape[0]
    p = np.zeros(nt, dtype=np.complex128)
    lib().oracle_direct_sum(_ptr(X), X.shape[0], _ptr(Y), Y.shape[0], _ptr(q), float(kappa),
                            float(tau), _ptr(tg), nt, _ptr(p), int(kernel))
    return p


def lagrange_1d(L, t):
    out = np.zeros(L)
    lib().oracle_lagrange_1d(L, float(t), _ptr(out))
    return out


def directions(E):
    n = lib().oracle_directions(E, None, None)
    d = np.zeros((n, 3))
    f = np.zeros(n, dtype=np.int64)
    lib().oracle_directions(E, _ptr(d), _ptr(f))
    return d, f


def spectrum(kappa, h, L, delta, kernel=HELMHOLTZ):
    P = 2 * L - 1
    D = np.zeros(P ** 3, dtype=np.complex128)
    dl = np.ascontiguousarray(delta, dtype=np.int32)
    lib().oracle_spectrum(float(kappa), float(h), L, _ptr(dl), _ptr(D), int(kernel))
    return D.reshape(P, P, P)  # index [mz, my, mx]


def m2l_fft(kappa, h, L, delta, M, kernel=HELMHOLTZ):
    M = np.ascontiguousarray(M, dtype=np.complex128)
    out = np.zeros(L ** 3, dtype=np.complex128)
    dl = np.ascontiguousarray(delta, dtype=np.int32)
    lib().oracle_m2l_fft(float(kappa), float(h), L, _ptr(dl), _ptr(M), _ptr(out), int(kernel))
    return out


def m2l_dense(kappa, h, L, delta, M, kernel=HELMHOLTZ):
    M = np.ascontiguousarray(M, dtype=np.complex128)
    out = np.zeros(L ** 3, dtype=np.complex128)
    dl = np.ascontiguousarray(delta, dtype=np.int32)
    lib().oracle_m2l_dense(float(kappa), float(h), L, _ptr(dl), _ptr(M), _ptr(out), int(kernel))
    return out


def dft3(a, sign=-1):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    P = a.shape[0]
    out = np.zeros_like(a)
    lib().oracle_dft3(P, _ptr(a), _ptr(out), sign)
    return out


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def p2m(kappa, L, alpha, h, u, y, q):
    """Single-expansion P2M; u = unit direction or None (non-directional)."""
    y, q, alpha, u = _f64(y), _c128(q), _f64(alpha), _f64(u)
    M = np.zeros(L ** 3, dtype=np.complex128)
    lib().oracle_p2m(float(kappa), L, _ptr(alpha), float(h), _ptr(u), y.shape[0], _ptr(y),
                     _ptr(q), _ptr(M))
    return M


def m2m(kappa, L, alpha, h, v, calpha, ch, Mc):
    """One son's contribution to the father's multipole expansion."""
    alpha, v, calpha, Mc = _f64(alpha), _f64(v), _f64(calpha), _c128(Mc)
    M = np.zeros(L ** 3, dtype=np.complex128)
    lib().oracle_m2m(float(kappa), L, _ptr(alpha), float(h), _ptr(v), _ptr(calpha), float(ch),
                     _ptr(Mc), _ptr(M))
    return M


def l2l(kappa, L, alpha, h, v, calpha, ch, Lp):
    """One father expansion's contribution to a son's local expansion."""
    alpha, v, calpha, Lp = _f64(alpha), _f64(v), _f64(calpha), _c128(Lp)
    Lc = np.zeros(L ** 3, dtype=np.complex128)
    lib().oracle_l2l(float(kappa), L, _ptr(alpha), float(h), _ptr(v), _ptr(calpha), float(ch),
                     _ptr(Lp), _ptr(Lc))
    return Lc


def l2p(kappa, L, alpha, h, u, Lc, x):
    alpha, u, Lc, x = _f64(alpha), _f64(u), _c128(Lc), _f64(x)
    p = np.zeros(x.shape[0], dtype=np.complex128)
    lib().oracle_l2p(float(kappa), L, _ptr(alpha), float(h), _ptr(u), _ptr(Lc), x.shape[0],
                     _ptr(x), _ptr(p))
    return p


class FMM:
    """The oracle FMM: tree, traversal, blank passes at construction; apply(q) -> p."""

    def __init__(self, X, Y=None, kappa=0.0, params: Params | None = None):
        self.params = params or Params()
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.same = Y is None
        self.Y = self.X if self.same else np.ascontiguousarray(Y, dtype=np.float64)
        self.kappa = float(kappa)
        self._p = self.params.c()
        self.h = lib().oracle_fmm_create(_ptr(self.X), self.X.shape[0], _ptr(self.Y),
                                         self.Y.shape[0], 1 if self.same else 0, self.kappa,
                                         ctypes.byref(self._p))
        self.last_seconds = None

    def close(self):
        if self.h:
            lib().oracle_fmm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, q):
        q = np.ascontiguousarray(q, dtype=np.complex128)
        p = np.zeros(self.X.shape[0], dtype=np.complex128)
        self.last_seconds = lib().oracle_fmm_apply(self.h, _ptr(q), _ptr(p))
        return p

    def info(self):
        a = np.zeros(16, dtype=np.int64)
        lib().oracle_fmm_info(self.h, _ptr(a))
        keys = ["levels_x", "levels_y", "lstar", "cells_x", "cells_y", "m2l_pairs", "p2p_pairs",
                "p2p_point_pairs", "exp_x", "exp_y", "unique_offsets", "max_dir_level"]
        return {k: int(a[i]) for i, k in enumerate(keys)}

    def geometry(self):
        o = np.zeros(3)
        D = lib().oracle_fmm_geometry(self.h, _ptr(o))
        return D, o

    def perm(self, tree=0):
        n = lib().oracle_fmm_perm(self.h, tree, None)
        a = np.zeros(n, dtype=np.int64)
        lib().oracle_fmm_perm(self.h, tree, _ptr(a))
        return a

    def cells(self, tree=0):
        n = lib().oracle_fmm_cells(self.h, tree, None, None, None, None, None)
        lev = np.zeros(n, dtype=np.int32)
        ijk = np.zeros((n, 3), dtype=np.int64)
        first = np.zeros(n, dtype=np.int64)
        count = np.zeros(n, dtype=np.int64)
        leaf = np.zeros(n, dtype=np.int32)
        lib().oracle_fmm_cells(self.h, tree, _ptr(lev), _ptr(ijk), _ptr(first), _ptr(count),
                               _ptr(leaf))
        return dict(level=lev, ijk=ijk, first=first, count=count, is_leaf=leaf)

    def m2l(self):
        n = lib().oracle_fmm_m2l(self.h, None, None, None, None, None)
        lev = np.zeros(n, dtype=np.int32)
        t = np.zeros(n, dtype=np.int64)
        s = np.zeros(n, dtype=np.int64)
        d = np.zeros((n, 3), dtype=np.int32)
        u = np.zeros(n, dtype=np.int32)
        lib().oracle_fmm_m2l(self.h, _ptr(lev), _ptr(t), _ptr(s), _ptr(d), _ptr(u))
        return dict(level=lev, t=t, s=s, delta=d, dir=u)

    def p2p(self):
        n = lib().oracle_fmm_p2p(self.h, None, None)
        t = np.zeros(n, dtype=np.int64)
        s = np.zeros(n, dtype=np.int64)
        lib().oracle_fmm_p2p(self.h, _ptr(t), _ptr(s))
        return dict(t=t, s=s)

    def expansions(self, tree=0):
        n = lib().oracle_fmm_expansions(self.h, tree, None, None, None, None)
        L3 = self.params.L ** 3
        cell = np.zeros(n, dtype=np.int64)
        d = np.zeros(n, dtype=np.int32)
        M = np.zeros((n, L3), dtype=np.complex128)
        Lc = np.zeros((n, L3), dtype=np.complex128)
        lib().oracle_fmm_expansions(self.h, tree, _ptr(cell), _ptr(d), _ptr(M), _ptr(Lc))
        return dict(cell=cell, dir=d, M=M, L=Lc)
