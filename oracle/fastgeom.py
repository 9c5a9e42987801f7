"""ctypes access to the oracle's plain-C float64 helpers (oracle/c/geom.c).

The C code restates oracle/spheres.py and oracle/bounds.py loop by loop; the
tests check the two against each other.  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "geom.c")
LIB = os.path.join(HERE, "c", "libgeom.so")

_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                               SRC, "-o", LIB + ".tmp", "-lm"])
        os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        L.og_point_covered.argtypes = [dp, dp, dp, ctypes.c_long, ctypes.c_double]
        L.og_point_covered.restype = ctypes.c_int
        L.og_bounds_one.argtypes = [dp, dp, dp, ctypes.c_long, ctypes.c_double, dp, dp, lp, lp]
        L.og_bounds_one.restype = None
        L.og_uncovered_point.argtypes = [dp, ctypes.c_double, dp, dp, ctypes.c_long, ctypes.c_double, dp, dp]
        L.og_uncovered_point.restype = ctypes.c_int
        L.og_nearest_uncovered.argtypes = [dp, ctypes.c_double, dp, dp, ctypes.c_long, dp, ctypes.c_double,
                                           ctypes.c_double, dp, dp]
        L.og_nearest_uncovered.restype = ctypes.c_int
        L.og_min_valid_radius.argtypes = [dp, ctypes.c_int, dp, dp, ctypes.c_long, ctypes.c_double,
                                          ctypes.c_double, dp, dp, dp, lp]
        L.og_min_valid_radius.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def point_covered(x, P, S, tol):
    x, P, S = _c(x), _c(P), _c(S)
    return bool(lib().og_point_covered(_p(x), _p(P), _p(S), len(S), tol))


def bounds_one(q, P, S, tie):
    q, P, S = _c(q), _c(P), _c(S)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    a, b = ctypes.c_long(), ctypes.c_long()
    lib().og_bounds_one(_p(q), _p(P), _p(S), len(S), tie, ctypes.byref(lo), ctypes.byref(hi),
                        ctypes.byref(a), ctypes.byref(b))
    return lo.value, hi.value, a.value, b.value


def uncovered_point(o, r, P, S, tol, hint=None):
    o, P, S = _c(o), _c(P), _c(S)
    x = np.empty(3)
    h = _p(_c(hint)) if hint is not None else None
    hh = _c(hint) if hint is not None else None
    found = lib().og_uncovered_point(_p(o), float(r), _p(P), _p(S), len(S), tol,
                                     _p(hh) if hh is not None else None, _p(x))
    del h
    return x if found else None


def nearest_uncovered(o, r, P, S, q, bound, tol):
    o, P, S, q = _c(o), _c(P), _c(S), _c(q)
    x = np.empty(3)
    d = ctypes.c_double()
    kind = lib().og_nearest_uncovered(_p(o), float(r), _p(P), _p(S), len(S), _p(q), float(bound), tol,
                                      ctypes.byref(d), _p(x))
    if kind == 0:
        return None
    return d.value, x, {1: "T", 2: "D", 3: "U"}[kind]


def min_valid_radius(q, sigma, P, S, tol, tie, W=None):
    q, P, S = _c(q), _c(P), _c(S)
    Wc = _c(W) if W is not None else None
    x = np.empty(3)
    r = ctypes.c_double()
    i = ctypes.c_long(-1)
    kind = lib().og_min_valid_radius(_p(q), int(sigma), _p(P), _p(S), len(S), tol, tie,
                                     _p(Wc) if Wc is not None else None, ctypes.byref(r), _p(x),
                                     ctypes.byref(i))
    if kind < 0:
        return float("nan"), q.copy(), "X", -1
    return r.value, x, {0: "Z", 1: "T", 2: "D", 3: "U"}[kind], i.value
