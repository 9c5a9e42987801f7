"""Tolerances, codes and the one covered predicate used everywhere in the oracle.

Appendix B of the paper: every intersection and containment check is done in
double precision, the tolerance for the uniqueness of points is 1e-9 and all
other tolerances are 1e-6; only points of [-1,1]^d are considered.
"""
from __future__ import annotations

import numpy as np

TOL = 1e-6          # containment / intersection tolerance (Appendix B)
TIE_TOL = 1e-9      # uniqueness tolerance; used as the tie band of argmax/argmin
DOMAIN_LO = -1.0    # Appendix B: the surface lies in [-1,1]^d
DOMAIN_HI = 1.0

# per-query outcome codes
KIND_HI = 1           # value = hi, tangent to the argmin constraint
KIND_LO = 2           # value = lo, tangent to the argmax constraint
KIND_ZERO = 3         # value 0 (query outside every ball)
KIND_RMIN_T = 4       # minimum valid radius, contour point is a radial foot point
KIND_RMIN_D = 5       # minimum valid radius, nearest point of an intersection circle
KIND_RMIN_U = 6       # minimum valid radius, a triple intersection point
KIND_COINCIDENT = 7   # query coincides with an existing sample
KIND_INFEASIBLE = 254
KIND_UNRESOLVED = 255

# bound flags
FLAG_INFEASIBLE = 1    # lo > hi + TOL
FLAG_INSIDE_POS = 2    # lo > TOL: strictly inside a positive ball
FLAG_INSIDE_NEG = 4    # hi < -TOL: strictly inside a negative ball
FLAG_TIE_LO = 8        # another constraint lies within TIE_TOL of lo
FLAG_TIE_HI = 16       # another constraint lies within TIE_TOL of hi
FLAG_HI_OPPOSITE = 32  # hi is bound by an opposite-sign (non-intersection) constraint
FLAG_LO_OPPOSITE = 64  # lo is bound by an opposite-sign constraint


def sign_class(s):
    """+1, -1 or 0: values within TIE_TOL of zero have no sign."""
    s = np.asarray(s, dtype=np.float64)
    return np.where(s > TIE_TOL, 1, np.where(s < -TIE_TOL, -1, 0))


def dist(a, b):
    """Euclidean distance sqrt(dx*dx + dy*dy + dz*dz), broadcasting over rows."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2])


def covered_by(x, P, S, tol=TOL):
    """Boolean mask: which balls hold point x strictly inside.

    Ball of sample (p, s) is the open ball of radius |s|; a point is covered
    when |x - p| < |s| - tol, so touching points count as uncovered
    (Prop. 1 allows spheres to touch).
    """
    return dist(P, x) < np.abs(S) - tol


def point_covered(x, P, S, tol=TOL) -> bool:
    return bool(covered_by(x, P, S, tol).any())


def points_covered(X, P, S, tol=TOL, chunk=2048) -> np.ndarray:
    """For each row of X: is it strictly inside any ball."""
    out = np.zeros(len(X), dtype=bool)
    R = np.abs(S) - tol
    for s0 in range(0, len(X), chunk):
        xs = X[s0:s0 + chunk]
        d = dist(xs[:, None, :], P[None, :, :])
        out[s0:s0 + chunk] = (d < R[None, :]).any(1)
    return out
