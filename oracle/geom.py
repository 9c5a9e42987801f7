"""Chooses between the NumPy restatement (spheres.py) and the plain-C loops
(fastgeom.py) of the same sphere geometry.  Both are exact float64; the C
loops only make test-sized greedy runs finish in seconds."""
from __future__ import annotations

from . import fastgeom, spheres
from .common import TOL
from .common import point_covered as _np_point_covered

USE_C = True


def point_covered(x, P, S, tol=TOL):
    if USE_C:
        return fastgeom.point_covered(x, P, S, tol)
    return _np_point_covered(x, P, S, tol)


def uncovered_point(o, r, P, S, tol=TOL, hint=None):
    if USE_C:
        return fastgeom.uncovered_point(o, r, P, S, tol, hint)
    return spheres.uncovered_point(o, r, P, S, tol, hint)


def nearest_uncovered(o, r, P, S, q, bound, tol=TOL):
    if USE_C:
        return fastgeom.nearest_uncovered(o, r, P, S, q, bound, tol)
    return spheres.nearest_uncovered(o, r, P, S, q, bound, tol)
