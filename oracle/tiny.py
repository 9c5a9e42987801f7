"""Paper-exact candidate scoring for tiny inputs (Def. 1, Sec. 3.3, Prop. 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The production reading of the greedy ("Level P", oracle.greedy) tries only
the two tangency values lo and hi before the minimum-valid-radius fallback.
This module follows the paper's single-point interpolation as defined: every
candidate grow-to point of Def. 1 (tangent points T, uncovered triple points
U, the nearest and farthest points D of not completely covered intersection
circles, and the point itself), both signs of each distance, scored by the
rule of Sec. 3.3 and tried best first until the augmented set passes Prop. 1.

Readings (the paper leaves these open):
  - the largest possible radius of the scoring rule is max(|lo|, |hi|), the
    cone bounds of the query over the current set (no valid value is larger);
  - normals agree when the surface normals implied by the two spheres at the
    grow-to point q point the same way: n = sign(s) (p - q)/|p - q| for the
    new sphere and sign(s_i) (p_i - q)/|p_i - q| for sphere i, and their dot
    product is positive;
  - the point itself (value 0) is a candidate (it is in P but missing from the
    grow-to listing) and is tried last;
  - grow-to points outside the domain [-1,1]^3 (with the containment
    tolerance) are not considered (Appendix B);
  - equal scores (within the uniqueness tolerance) try the negative value
    first, then keep generation order;
  - `circles="complete"` keeps only circles no other ball touches (the
    refinement shortcut of Sec. 4.3); the default keeps every circle that
    is not completely covered, as Def. 1 states.
Validity is Prop. 1 checked on the whole augmented set: no two spheres of
different sign intersect (beyond the tolerance) and every sphere has a point
inside no other open ball (the exact sphere search of oracle.spheres).
Only sizes of a few dozen spheres are practical: the candidate set grows with
the cube of the set size.
"""
from __future__ import annotations

import math

import numpy as np

from . import geom
from .common import DOMAIN_HI, DOMAIN_LO, TIE_TOL, TOL, dist, sign_class

TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------- geometry

def triple_points(c1, r1, c2, r2, c3, r3):
    """Common points of three spheres (0, 1 or 2).

    Subtracting the first sphere's equation from the other two gives two
    planes through x - c1 = a n1 + b n2 + g (n1 x n2); a and b solve the 2x2
    system, g follows from the first sphere.
    """
    n1 = np.asarray(c2, dtype=np.float64) - c1
    n2 = np.asarray(c3, dtype=np.float64) - c1
    b1 = 0.5 * (r1 * r1 - r2 * r2 + n1 @ n1)
    b2 = 0.5 * (r1 * r1 - r3 * r3 + n2 @ n2)
    g11, g12, g22 = n1 @ n1, n1 @ n2, n2 @ n2
    det = g11 * g22 - g12 * g12
    m = np.array([n1[1] * n2[2] - n1[2] * n2[1], n1[2] * n2[0] - n1[0] * n2[2], n1[0] * n2[1] - n1[1] * n2[0]])
    mm = m @ m
    if not (det > 1e-300) or not (mm > 1e-300):
        return []                       # collinear centres: a circle or nothing
    a = (b1 * g22 - b2 * g12) / det
    b = (b2 * g11 - b1 * g12) / det
    y0 = a * n1 + b * n2
    h = r1 * r1 - y0 @ y0
    if h < 0.0:
        return []
    base = np.asarray(c1, dtype=np.float64) + y0
    if h == 0.0:
        return [base]
    g = math.sqrt(h / mm)
    return [base + g * m, base - g * m]


def circle_of(ci, ri, cj, rj):
    """Intersection circle (centre, radius, unit normal) of two spheres, or None."""
    v = np.asarray(cj, dtype=np.float64) - ci
    D = math.sqrt(v @ v)
    if not (D > 0.0) or not (abs(ri - rj) < D < ri + rj):
        return None
    mu = v / D
    h = (D * D + ri * ri - rj * rj) / (2.0 * D)
    rho = math.sqrt(max(ri * ri - h * h, 0.0))
    return np.asarray(ci, dtype=np.float64) + h * mu, rho, mu


def _perp(mu):
    a = np.array([1.0, 0.0, 0.0]) if abs(mu[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(mu, a)
    e1 /= math.sqrt(e1 @ e1)
    return e1, np.cross(mu, e1)


def circle_extreme_points(p, zeta, rho, mu):
    """Nearest and farthest point of the circle to p (Def. 1, set D).

    With v = p - zeta and w its component along the normal, the in-plane
    direction (v - w)/|v - w| gives the nearest point, its opposite the
    farthest.  On the axis every circle point is equally far; a fixed
    in-plane direction is taken."""
    v = np.asarray(p, dtype=np.float64) - zeta
    u = v - (v @ mu) * mu
    un = math.sqrt(u @ u)
    u = u / un if un > 0.0 else _perp(mu)[0]
    return zeta + rho * u, zeta - rho * u


def circle_cover_arcs(zeta, rho, mu, P, S, skip, tol=TOL):
    """Open arcs of the circle covered by the balls (P, S) other than `skip`.

    Returns None if one ball holds the whole circle, else a list of (centre
    angle, half-width).  A point x(t) = zeta + rho (cos t e1 + sin t e2) is
    inside ball k when |x(t) - p_k|^2 < (|s_k| - tol)^2, i.e. when
    A cos t + B sin t > K with A = -2 rho (zeta - p_k).e1,
    B = -2 rho (zeta - p_k).e2, K = |zeta - p_k|^2 + rho^2 - (|s_k| - tol)^2.
    """
    e1, e2 = _perp(mu)
    arcs = []
    for k in range(len(S)):
        if k in skip:
            continue
        R = abs(S[k]) - tol
        if not (R > 0.0):
            continue
        z = zeta - P[k]
        A = -2.0 * rho * (z @ e1)
        B = -2.0 * rho * (z @ e2)
        K = z @ z + rho * rho - R * R
        amp = math.hypot(A, B)
        if K < -amp:
            return None
        if amp > K:
            arcs.append((math.atan2(B, A), math.acos(max(-1.0, min(1.0, K / amp)))))
    return arcs


def _angdist(x, y):
    return abs((x - y + math.pi) % TWO_PI - math.pi)


def arcs_cover_circle(arcs):
    """Do these open arcs (centre, half-width) cover the whole circle?

    If some point is left uncovered, walking forward from it one reaches the
    start of an arc that no other arc covers (a start is never inside its own
    open arc); conversely an uncovered start is an uncovered point.  So the
    circle is covered iff every arc start lies strictly inside another arc.
    """
    if arcs is None:
        return True
    if not arcs:
        return False
    for j, (cj, wj) in enumerate(arcs):
        a = cj - wj
        if not any(k != j and _angdist(a, ck) < wk for k, (ck, wk) in enumerate(arcs)):
            return False
    return True


def point_uncovered(q, P, S, tol=TOL):
    """q lies in no open ball (shrunk by tol) of the set (Prop. 1 (ii))."""
    return not geom.point_covered(q, P, S, tol)


def in_domain(q):
    return bool(np.all(q >= DOMAIN_LO - TOL) and np.all(q <= DOMAIN_HI + TOL))


# ---------------------------------------------------------- candidate set

def grow_to_points(p, P, S, tol=TOL, circles="partial"):
    """Candidate grow-to points of Def. 1 for query p over the set (P, S).

    Returns a list of (q, i, is_tangent): each point once per sphere it lies
    on, as in the paper's listing.  T: both tangent points of every sphere;
    U: uncovered common points of three spheres; D: nearest and farthest
    points of every intersection circle that is not completely covered (with
    circles="complete": of every circle no other ball touches), when they
    are uncovered.
    """
    p = np.asarray(p, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    n = len(S)
    R = np.abs(S)
    live = R > TIE_TOL
    # spheres that share a point: |r_i - r_j| <= D_ij <= r_i + r_j (a common
    # point of three spheres is a common point of each pair)
    Dm = dist(P[:, None, :], P[None, :, :])
    meet = (Dm <= R[:, None] + R[None, :]) & (Dm >= np.abs(R[:, None] - R[None, :])) & live[:, None] & live[None, :]
    out = []
    for i in range(n):
        d = math.sqrt((p - P[i]) @ (p - P[i]))
        if d > 0.0:
            u = (p - P[i]) / d
            for c in (-1.0, 1.0):
                out.append((P[i] + c * u * R[i], i, True))
    for i in range(n):
        if not live[i]:
            continue
        for j in range(i + 1, n):
            if not meet[i, j]:
                continue
            for k in range(j + 1, n):
                if not (meet[i, k] and meet[j, k]):
                    continue
                for q in triple_points(P[i], R[i], P[j], R[j], P[k], R[k]):
                    if point_uncovered(q, P, S, tol):
                        out += [(q, i, False), (q, j, False), (q, k, False)]
            circ = circle_of(P[i], R[i], P[j], R[j])
            if circ is None:
                continue
            zeta, rho, mu = circ
            arcs = circle_cover_arcs(zeta, rho, mu, P, S, {i, j}, tol)
            if circles == "complete":
                if arcs is None or len(arcs):
                    continue
            elif arcs_cover_circle(arcs):
                continue
            for q in circle_extreme_points(p, zeta, rho, mu):
                if point_uncovered(q, P, S, tol):
                    out += [(q, i, False), (q, j, False)]
    return out


def normals_agree(p, s, pi, si, q):
    """The surface normals implied at q by the new sphere (p, s) and by sphere
    (pi, si) point the same way (positive dot product)."""
    a = np.asarray(p, dtype=np.float64) - q
    b = np.asarray(pi, dtype=np.float64) - q
    na, nb = math.sqrt(a @ a), math.sqrt(b @ b)
    if not (na > 0.0) or not (nb > 0.0) or s == 0.0 or si == 0.0:
        return False
    return math.copysign(1.0, s) * math.copysign(1.0, si) * (a @ b) > 0.0


def score_for_radius(p, s, pi, si, q, is_tangent, max_radius):
    """Sec. 3.3 scoring rule: a type score (tangency with agreeing normals 3M,
    other points with agreeing normals 2M, other points M, tangency with
    disagreeing normals 0) plus the magnitude weighted 2 for negative
    values."""
    agree = normals_agree(p, s, pi, si, q)
    if is_tangent:
        type_score = 3.0 * max_radius if agree else 0.0
    else:
        type_score = (2.0 if agree else 1.0) * max_radius
    sign_score = 1.0 if s > 0.0 else 2.0
    return sign_score * abs(s) + type_score


def cone_extremes(p, P, S):
    d = dist(P, p)
    return float((S - d).max()), float((S + d).min())


def ranked_values(p, P, S, tol=TOL, circles="partial"):
    """(score, value, sphere, grow-to point, is_tangent), best first; the
    point itself (value 0) last."""
    p = np.asarray(p, dtype=np.float64)
    lo, hi = cone_extremes(p, P, S)
    M = max(abs(lo), abs(hi))
    radii = []
    for q, i, tang in grow_to_points(p, P, S, tol, circles):
        if not in_domain(q):
            continue
        r = math.sqrt((q - p) @ (q - p))
        for sgn in (-1.0, 1.0):
            s = sgn * r
            radii.append((score_for_radius(p, s, P[i], S[i], q, tang, M), s, i, q, tang))
    radii.sort(key=lambda t: -t[0])
    # equal scores (within the uniqueness tolerance): negative values first
    out = []
    k = 0
    while k < len(radii):
        g = k
        while g < len(radii) and radii[k][0] - radii[g][0] <= TIE_TOL:
            g += 1
        group = radii[k:g]
        out += [t for t in group if t[1] < 0.0] + [t for t in group if not t[1] < 0.0]
        k = g
    out.append((-math.inf, 0.0, -1, p.copy(), False))
    return out


# ---------------------------------------------------------------- validity

def is_sdf_valid(P, S, tol=TOL, first=None):
    """Prop. 1 on the whole set: (i) no two spheres of different sign
    intersect by more than tol; (ii) every sphere has a point in no other
    open ball (shrunk by tol).  `first` lists spheres to examine first (an
    evaluation order only; every sphere is examined before True)."""
    P = np.asarray(P, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    n = len(S)
    sig = sign_class(S)
    R = np.abs(S)
    for x in range(n):
        d = dist(P, P[x])
        opp = sig[x] * sig < 0
        if np.any(opp & (R[x] + R > d + tol)):
            return False
    order = list(first or []) + [x for x in range(n) if x not in set(first or [])]
    for x in order:
        if geom.uncovered_point(P[x], R[x], P, S, tol) is None:
            return False
    return True


def interpolate_sdf_to(p, P, S, tol=TOL, circles="partial", cone_prefilter=True):
    """Sec. 3.3 single-point interpolation: the best-scoring candidate value
    whose augmented set passes Prop. 1.  Returns (value, sphere, grow-to
    point, is_tangent, rank of the winner in the ranked list).

    With `cone_prefilter` a candidate outside [lo - tol, hi + tol] is
    rejected without the full check: beyond hi + tol the new sphere either
    intersects the opposite-sign sphere b (Prop. 1 (i)), or its ball holds
    all of sphere b, or sphere b's ball holds all of the new sphere (Prop. 1
    (ii)), and symmetrically below lo - tol; so the full check would reject
    it too.  It changes the running time only."""
    p = np.asarray(p, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    Pn = np.vstack([P, p[None, :]])
    n = len(S)
    lo, hi = cone_extremes(p, P, S)
    for rank, (_, s, i, q, tang) in enumerate(ranked_values(p, P, S, tol, circles)):
        if cone_prefilter and not (lo - tol <= s <= hi + tol):
            continue
        Sn = np.append(S, s)
        # spheres meeting the new open ball are the ones that can fail: look
        # at them (and the new sphere) first
        near = [n] + [int(x) for x in np.nonzero(dist(P, p) < abs(s) + np.abs(S))[0]]
        if is_sdf_valid(Pn, Sn, tol, first=near):
            return s, i, q, tang, rank
    return math.nan, -1, p.copy(), False, -1


def interpolate_sequence(P, S, Q, order, tol=TOL, circles="partial"):
    """Values of queries Q assigned one at a time in `order`, each one
    consistent with the inputs and the earlier values (Sec. 4)."""
    P = np.asarray(P, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    vals = np.full(len(Q), np.nan)
    CP, CS = P.copy(), S.copy()
    for j in order:
        s, _, _, _, _ = interpolate_sdf_to(Q[j], CP, CS, tol, circles)
        vals[j] = s
        if math.isfinite(s):
            CP = np.vstack([CP, np.asarray(Q[j], dtype=np.float64)[None, :]])
            CS = np.append(CS, s)
    return vals
