"""Uncovered points of one sphere under a set of open balls (Prop. 1 (ii)).

A point x of sphere S = (o, r) is covered by sample (p, s) when
|x - p| < |s| - TOL (the predicate of ``common``).  The covered part of S
from one ball is an open spherical cap {v : v . u > c} in the unit direction
v = (x - o)/r, with u = (p - o)/|p - o| and
c = (r^2 + D^2 - R^2)/(2 r D), D = |p - o|, R = |s| - TOL.

Existence of an uncovered point.  The uncovered set U of S is closed.  If it
is non-empty and not all of S, it has a boundary point, which lies on the
rim of some cap and in no other cap.  So S has an uncovered point iff no ball
meets S, or some cap rim (a circle on S, the intersection circle of Def. 1)
keeps an angle that no other cap covers.  On the rim of cap e, parametrised
as v(t) = c_e u_e + rho_e (cos t e1 + sin t e2), cap f covers the open arc
A cos t + B sin t > C.  Sweeping those open arcs finds the uncovered gaps;
gap end points are the triple points U of Def. 1 and the rim points nearest
to a query are the circle points D of Def. 1.
"""
from __future__ import annotations

import math

import numpy as np

from .common import TOL, dist

TWO_PI = 2.0 * math.pi


def basis(u):
    """Two unit vectors orthogonal to unit vector u and to each other."""
    a = np.array([1.0, 0.0, 0.0]) if abs(u[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(u, a)
    e1 = e1 / math.sqrt(e1 @ e1)
    e2 = np.cross(u, e1)
    return e1, e2


def sphere_caps(o, r, P, S, tol=TOL):
    """Caps cut from sphere (o, r) by the balls of samples (P, S).

    Returns None when some ball holds the whole sphere strictly inside, else
    (U, C, idx): cap axes, cap thresholds and the sample index of every ball
    whose open ball meets the sphere.
    """
    R = np.abs(S) - tol
    v = P - o
    D = dist(P, o)
    live = R > 0.0
    if np.any(live & (D + r < R)):
        return None
    meet = live & (D > 0.0) & (np.abs(D - r) < R)
    idx = np.nonzero(meet)[0]
    Dm = D[idx]
    U = v[idx] / Dm[:, None]
    C = (r * r + Dm * Dm - R[idx] * R[idx]) / (2.0 * r * Dm)
    return U, C, idx


def rim(u, c):
    """Centre-offset, radius and basis of the rim circle of cap (u, c)."""
    rho = math.sqrt(max(0.0, 1.0 - c * c))
    e1, e2 = basis(u)
    return rho, e1, e2


def rim_gaps(e, U, C):
    """Uncovered closed angle intervals on the rim of cap e.

    Every other cap f covers the open arc rho(e1.u_f) cos t + rho(e2.u_f) sin t
    > c_f - c_e (u_e.u_f).  Returns a list of (t0, t1) with 0 <= t0 <= t1 <=
    2 pi; an empty list means the whole rim is covered.
    """
    ue, ce = U[e], C[e]
    rho, e1, e2 = rim(ue, ce)
    others = np.ones(len(C), dtype=bool)
    others[e] = False
    Uf, Cf = U[others], C[others]
    A = rho * (Uf @ e1)
    B = rho * (Uf @ e2)
    K = Cf - ce * (Uf @ ue)
    amp = np.hypot(A, B)
    if np.any(K < -amp):
        return []                              # one cap holds the whole rim
    act = amp > K                               # non-empty open arcs
    if not act.any():
        return [(0.0, TWO_PI)]
    phi = np.arctan2(B[act], A[act])
    beta = np.arccos(np.clip(K[act] / amp[act], -1.0, 1.0))
    start = phi - beta
    end = phi + beta
    shift = np.floor(start / TWO_PI) * TWO_PI
    start = start - shift
    end = end - shift
    pieces = []
    for a, b in zip(start, end):
        if b > TWO_PI:
            pieces.append((a, math.inf))
            pieces.append((-math.inf, b - TWO_PI))
        else:
            pieces.append((a, b))
    pieces.sort()
    gaps = []
    x = 0.0
    for a, b in pieces:
        if x >= TWO_PI:
            break
        if a < x:
            if b > x:
                x = b
        else:
            gaps.append((x, min(a, TWO_PI)))
            x = b
    if x < TWO_PI:
        gaps.append((x, TWO_PI))
    return gaps


def rim_point(o, r, u, c, t):
    rho, e1, e2 = rim(u, c)
    v = c * u + rho * (math.cos(t) * e1 + math.sin(t) * e2)
    return o + r * v


def _direction(o, hint):
    if hint is None:
        return np.array([1.0, 0.0, 0.0])
    g = np.asarray(hint, dtype=np.float64) - o
    n = math.sqrt(g @ g)
    return g / n if n > 0.0 else np.array([1.0, 0.0, 0.0])


def uncovered_point(o, r, P, S, tol=TOL, hint=None):
    """Some point of sphere (o, r) covered by no ball of (P, S), or None.

    Exact up to float64 rounding.  ``hint`` only orders the search (rims
    nearest to the hint direction first); it never changes the answer.
    A sphere of radius 0 is the point o itself.
    """
    o = np.asarray(o, dtype=np.float64)
    if r <= 0.0:
        return None if bool((dist(P, o) < np.abs(S) - tol).any()) else o.copy()
    caps = sphere_caps(o, r, P, S, tol)
    if caps is None:
        return None
    U, C, _ = caps
    vh = _direction(o, hint)
    if len(C) == 0 or np.all(U @ vh <= C):
        return o + r * vh
    # rims ordered by angular distance from the hint direction
    ang = np.abs(np.arccos(np.clip(U @ vh, -1.0, 1.0)) - np.arccos(np.clip(C, -1.0, 1.0)))
    for e in np.argsort(ang, kind="stable"):
        gaps = rim_gaps(int(e), U, C)
        if gaps:
            t0, t1 = max(gaps, key=lambda g: g[1] - g[0])
            x = rim_point(o, r, U[e], C[e], 0.5 * (t0 + t1))
            return off_rim(o, r, x, U, C, int(e))
    return None


NUDGE = 1e-7


def off_rim(o, r, x, U, C, e):
    """Move a rim point a tiny angle away from cap e, keeping it uncovered.

    A point found on the rim of cap e is exactly at the shrunk radius of
    ball e; moving it into the uncovered side gives the witness a margin
    against rounding.  The original point is kept if the move would enter a
    cap."""
    v = (x - o) / r
    t = U[e] - (U[e] @ v) * v
    tn = math.sqrt(t @ t)
    if tn == 0.0:
        return x
    w = v - NUDGE * t / tn
    w = w / math.sqrt(w @ w)
    if np.all(U @ w <= C):
        return o + r * w
    return x


def _closest_angle_in(gap, tstar):
    """Angle of the closed interval ``gap`` nearest (cyclically) to tstar."""
    t0, t1 = gap
    ts = tstar % TWO_PI
    if t0 <= ts <= t1:
        return ts, True
    d0 = min(abs(ts - t0), TWO_PI - abs(ts - t0))
    d1 = min(abs(ts - t1), TWO_PI - abs(ts - t1))
    return (t0, False) if d0 <= d1 else (t1, False)


def nearest_uncovered(o, r, P, S, q, bound=math.inf, tol=TOL):
    """Nearest point to q of the uncovered part of sphere (o, r).

    Returns (distance, point, kind) with kind 'T' (radial foot point), 'D'
    (nearest point of a rim) or 'U' (end point of an uncovered rim arc, a
    triple point), or None if nothing uncovered is closer than ``bound``.
    The minimum over a closed uncovered set is either an interior critical
    point of the distance on the sphere (the radial foot point) or lies on a
    rim, where it is the rim's nearest point or an arc end point.
    """
    o = np.asarray(o, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    g = q - o
    gn = math.sqrt(g @ g)
    if r <= 0.0:
        if bool((dist(P, o) < np.abs(S) - tol).any()):
            return None
        return (gn, o.copy(), "T") if gn < bound else None
    caps = sphere_caps(o, r, P, S, tol)
    if caps is None:
        return None
    U, C, _ = caps
    if gn > 0.0:
        v0 = g / gn
        d0 = abs(gn - r)
        if d0 >= bound:
            return None
        if len(C) == 0 or np.all(U @ v0 <= C):
            return d0, o + r * v0, "T"
    else:
        if r >= bound:
            return None
        x = uncovered_point(o, r, P, S, tol)
        return None if x is None else (r, x, "T")
    # rim lower bounds: |x - q|^2 = r^2 + gn^2 - 2 r v.g, max of v.g on rim e
    ug = U @ g
    perp = np.sqrt(np.maximum(gn * gn - ug * ug, 0.0))
    rho = np.sqrt(np.maximum(1.0 - C * C, 0.0))
    vg = C * ug + rho * perp
    lb = np.sqrt(np.maximum(r * r + gn * gn - 2.0 * r * vg, 0.0))
    best = None
    bestd = bound
    for e in np.argsort(lb, kind="stable"):
        if lb[e] >= bestd:
            break
        gaps = rim_gaps(int(e), U, C)
        if not gaps:
            continue
        _, e1, e2 = rim(U[e], C[e])
        tstar = math.atan2(e2 @ g, e1 @ g)
        for gap in gaps:
            t, inside = _closest_angle_in(gap, tstar)
            x = rim_point(o, r, U[e], C[e], t)
            d = float(dist(x, q))
            if d < bestd:
                bestd = d
                best = (d, x, "D" if inside else "U")
    return best
