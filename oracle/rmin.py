"""Minimum valid radius (proof of Prop. 2; Corollary 1; Sec. 6 pseudocode).

For a point q strictly inside some ball of sign sigma, the smallest valid
magnitude is the distance from q to the contour C_sigma of the union of all
sigma-balls: the sphere of that radius touches C_sigma (so it has an
uncovered point), stays inside the sigma-union (so it intersects no
opposite-sign sphere and covers no new point).  Outside every sigma-ball the
minimum is 0.

The nearest contour point is, per Prop. 2's proof, a radial foot point of a
sigma-sphere (T), the nearest point of an uncovered intersection-circle arc
(D) or an uncovered triple point (U).  This module finds it sphere by sphere:
the distance from q to the uncovered part of each sigma-sphere, best first
by the lower bound |d_i - |s_i||, stopping when the bound exceeds the best
found.  Candidates on opposite-sign spheres are never nearer than the contour
(the sigma-contour is separated from the other sign), so only sigma-spheres
are searched.  Coverage is tested against every ball, as the paper's
point_uncovered does.  The contour is that of the balls shrunk by the
uniqueness tolerance TIE_TOL only (1e-9, Appendix B), not by TOL: the
contact point then lies outside every TOL-shrunk ball with margin
TOL - TIE_TOL, so the new sphere keeps an uncovered neighbourhood there,
and exactly tangent spheres (which the greedy produces all the time) still
leave non-degenerate gaps.  "q is inside a ball" uses d < |s| - TOL.
"""
from __future__ import annotations

import math

import numpy as np

from . import fastgeom, geom
from .common import TIE_TOL, TOL, dist, sign_class
from .geom import nearest_uncovered


def min_valid_radius(q, sigma, P, S, tol=TOL, W=None):
    """(radius, contour point, kind 'T'|'D'|'U'|'Z', sphere index or -1).

    ``W`` optionally holds one uncovered point per sphere (NaN if unknown).
    An uncovered point of a sigma-sphere lies on the contour, so the nearest
    one bounds the answer from above; it only prunes the search.
    """
    q = np.asarray(q, dtype=np.float64)
    if geom.USE_C:
        return fastgeom.min_valid_radius(q, sigma, P, S, tol, TIE_TOL, W)
    sig = sign_class(S)
    R = np.abs(S)
    d = dist(P, q)
    mine = np.nonzero(sig == sigma)[0]
    inside = d[mine] < R[mine] - tol
    if not inside.any():
        return 0.0, q.copy(), "Z", -1
    best = math.inf
    out = None
    if W is not None:
        dw = dist(W[mine], q)
        dw = dw[np.isfinite(dw)]
        if len(dw):
            best = float(dw.min()) * (1.0 + 1e-12) + 1e-15
    # the deepest ball first: its foot point realises the inner bound exactly
    # when uncovered (no contour point lies closer than max_i(|s_i| - d_i))
    depth = R[mine] - d[mine]
    deepest = mine[int(np.argmax(depth))]
    res = nearest_uncovered(P[deepest], R[deepest], P, S, q, best, TIE_TOL)
    if res is not None:
        best = res[0]
        out = (res[0], res[1], res[2], int(deepest))
        if res[2] == "T":
            return out
    lb = np.abs(d[mine] - R[mine])
    for k in np.argsort(lb, kind="stable"):
        i = int(mine[k])
        if lb[k] >= best:
            break
        if i == deepest:
            continue
        res = nearest_uncovered(P[i], R[i], P, S, q, best, TIE_TOL)
        if res is not None and res[0] < best:
            best = res[0]
            out = (res[0], res[1], res[2], i)
    if out is None and W is not None and math.isfinite(best):
        # nothing strictly nearer than the nearest cached uncovered point
        return min_valid_radius(q, sigma, P, S, tol, None)
    if out is None:
        return math.nan, q.copy(), "X", -1
    return out
