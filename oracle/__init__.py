"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the plain FP64 CPU oracle.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It shares no code with the HIP library (``paper_2510_18838_amd``)
and neither imports the other; the library must never fall back to it.

The oracle computes the local weighted polynomial fitting transfer of the
PCMS paper (Section 3.2.1, Eq. 1) in FP64 on the host: see ``pcms_oracle.c``
for the definition it follows and the readings it takes where the paper is
silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpcms_oracle.so")
SRC = os.path.join(HERE, "pcms_oracle.c")

FIXED, KNN, GROW = 0, 1, 2
OK, UNDERDETERMINED, SINGULAR, RADIUS_EXHAUSTED, CAPPED = 0, 1, 2, 3, 0x10
WENDLAND_C2, C4, GAUSSIAN, CONST, IMQ = 0, 1, 2, 3, 4


def build() -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=c11",
           "-D_GNU_SOURCE", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Radius(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("r", ctypes.c_double), ("k", ctypes.c_int),
                ("n_min", ctypes.c_int), ("max_iter", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.orc_neighbors.argtypes = [P, ctypes.c_int64, ctypes.c_int, P, P, ctypes.c_int64,
                                    ctypes.POINTER(_Radius), ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, P, P, P, P, P]
        L.orc_neighbors.restype = ctypes.c_int
        L.orc_transfer.argtypes = [P, ctypes.c_int64, ctypes.c_int, P, P, ctypes.c_int, P,
                                   ctypes.c_int64, ctypes.c_int, ctypes.POINTER(_Radius),
                                   ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, P, P, P, P, P, P]
        L.orc_transfer.restype = ctypes.c_int
        L.orc_weight.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_weight.restype = ctypes.c_double
        L.orc_num_monomials.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_num_monomials.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def radius(mode, r=0.0, k=0, n_min=0, max_iter=40):
    return _Radius(int(mode), float(r), int(k), int(n_min), int(max_iter))


def weight(kind: int, q: float) -> float:
    return lib().orc_weight(int(kind), float(q))


def max_threads() -> int:
    return lib().orc_max_threads()


def num_monomials(dim: int, degree: int) -> int:
    return lib().orc_num_monomials(dim, degree)


def neighbors(src, tgt, mode, r=0.0, k=0, n_min=0, max_iter=40, k_cap=32, inv_scale=None,
              brute=False, nthreads=0):
    """Neighbour lists.  Returns dict(nbr[n_tgt, k_cap] (-1 padded), n_kept, n_found, r2, status)."""
    src, tgt = _f64(src), _f64(tgt)
    n_src, dim = src.shape
    n_tgt = tgt.shape[0]
    g = None if inv_scale is None else _f64(inv_scale)
    nbr = np.full((n_tgt, k_cap), -1, dtype=np.int32)
    n_kept = np.zeros(n_tgt, np.int32)
    n_found = np.zeros(n_tgt, np.int32)
    r2 = np.zeros(n_tgt)
    st = np.zeros(n_tgt, np.uint8)
    rs = radius(mode, r, k, n_min, max_iter)
    rc = lib().orc_neighbors(_p(src), n_src, dim, _p(g), _p(tgt), n_tgt, ctypes.byref(rs),
                             k_cap, int(brute), int(nthreads), _p(nbr), _p(n_kept), _p(n_found),
                             _p(r2), _p(st))
    if rc != 0:
        raise ValueError(f"orc_neighbors rejected its arguments (rc={rc})")
    return dict(nbr=nbr, n_kept=n_kept, n_found=n_found, r2=r2, status=st)


def transfer(src, vals, tgt, degree, mode, r=0.0, k=0, n_min=0, max_iter=40, k_cap=32,
             inv_scale=None, weight_kind=WENDLAND_C2, lam=0.0, brute=False, nthreads=0,
             want_lists=False, want_shape=False):
    """Field transfer.  Returns dict(out[n_fields, n_tgt], status, pivot_ratio[, nbr, n_kept, shape])."""
    src, tgt = _f64(src), _f64(tgt)
    vals = _f64(vals)
    if vals.ndim == 1:
        vals = vals[None, :]
    n_src, dim = src.shape
    n_tgt = tgt.shape[0]
    n_f = vals.shape[0]
    g = None if inv_scale is None else _f64(inv_scale)
    out = np.empty((n_f, n_tgt))
    st = np.zeros(n_tgt, np.uint8)
    piv = np.full(n_tgt, np.nan)
    nbr = np.full((n_tgt, k_cap), -1, np.int32) if (want_lists or want_shape) else None
    nk = np.zeros(n_tgt, np.int32) if (want_lists or want_shape) else None
    shape = np.full((n_tgt, k_cap), np.nan) if want_shape else None
    rs = radius(mode, r, k, n_min, max_iter)
    rc = lib().orc_transfer(_p(src), n_src, dim, _p(g), _p(vals), n_f, _p(tgt), n_tgt, degree,
                            ctypes.byref(rs), k_cap, int(weight_kind), float(lam), int(brute),
                            int(nthreads), _p(out), _p(st), _p(piv), _p(nbr), _p(nk), _p(shape))
    if rc != 0:
        raise ValueError(f"orc_transfer rejected its arguments (rc={rc})")
    res = dict(out=out, status=st, pivot_ratio=piv)
    if nbr is not None:
        res.update(nbr=nbr, n_kept=nk)
    if shape is not None:
        res["shape"] = shape
    return res


def problem_kwargs(prob):
    """Radius/cap keyword arguments of a ``synth.Problem`` for the oracle calls."""
    return dict(mode=prob.mode, r=prob.radius, k=prob.k, n_min=prob.n_min,
                max_iter=prob.max_iter, k_cap=prob.k_cap, inv_scale=prob.inv_scale)
