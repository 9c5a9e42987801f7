"""Analytic signed distance functions used to synthesise seeded input data.

These are ground-truth shape definitions (negative inside, positive outside,
as in Eq. 1 of the paper).  They describe the *input* surfaces only; nothing
here implements any step of the interpolation method.
"""
from __future__ import annotations

import numpy as np


def sphere_sdf(x: np.ndarray, centre, radius: float) -> np.ndarray:
    """Exact SDF of a ball: |x - c| - R."""
    c = np.asarray(centre, dtype=np.float64)
    return np.sqrt(((x - c) ** 2).sum(-1)) - radius


def box_sdf(x: np.ndarray, centre, half) -> np.ndarray:
    """Exact SDF of an axis-aligned box with half-extents ``half``."""
    q = np.abs(x - np.asarray(centre, dtype=np.float64)) - np.asarray(half, dtype=np.float64)
    outside = np.sqrt((np.maximum(q, 0.0) ** 2).sum(-1))
    inside = np.minimum(q.max(-1), 0.0)
    return outside + inside


def capsule_sdf(x: np.ndarray, a, b, radius: float) -> np.ndarray:
    """Exact SDF of a capsule (segment a-b swept by a ball of ``radius``)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    ab = b - a
    t = np.clip(((x - a) @ ab) / (ab @ ab), 0.0, 1.0)
    closest = a + t[..., None] * ab
    return np.sqrt(((x - closest) ** 2).sum(-1)) - radius


def _ball_union_exposed_distance(x: np.ndarray, centres: np.ndarray, radii: np.ndarray) -> np.ndarray:
    """Distance from each point of ``x`` to the boundary of a union of balls.

    The boundary of a finite union of balls is made of exposed sphere patches,
    exposed arcs of pairwise intersection circles, and exposed triple points.
    The distance to it is the smallest distance to an exposed feature point:
    the radial foot point on a sphere, the nearest point of an intersection
    circle, or a triple point.  A feature point is exposed when no *other* ball
    holds it strictly inside.  Used only to give the points inside the union
    their exact (true-distance) negative values.
    """
    k = len(radii)
    best = np.full(len(x), np.inf)
    rel = 1e-12

    def exposed(y, skip):
        ok = np.ones(len(y), dtype=bool)
        for j in range(k):
            if j in skip:
                continue
            ok &= np.sqrt(((y - centres[j]) ** 2).sum(-1)) >= radii[j] * (1.0 - rel)
        return ok

    # radial foot points
    for i in range(k):
        v = x - centres[i]
        n = np.sqrt((v ** 2).sum(-1))
        n = np.where(n == 0.0, 1.0, n)
        y = centres[i] + radii[i] * v / n[:, None]
        dist = np.sqrt(((x - y) ** 2).sum(-1))
        best = np.where(exposed(y, {i}), np.minimum(best, dist), best)
    # pairwise circles
    for i in range(k):
        for j in range(i + 1, k):
            dvec = centres[j] - centres[i]
            dd = np.sqrt(dvec @ dvec)
            if dd >= radii[i] + radii[j] or dd <= abs(radii[i] - radii[j]) or dd == 0.0:
                continue
            mu = dvec / dd
            h = (dd * dd + radii[i] ** 2 - radii[j] ** 2) / (2.0 * dd)
            zeta = centres[i] + h * mu
            rho = np.sqrt(max(radii[i] ** 2 - h * h, 0.0))
            v = x - zeta
            w = v - (v @ mu)[:, None] * mu
            wn = np.sqrt((w ** 2).sum(-1))
            # points on the axis are equidistant from the whole circle
            fallback = np.cross(mu, [1.0, 0.0, 0.0] if abs(mu[0]) < 0.9 else [0.0, 1.0, 0.0])
            fallback = fallback / np.sqrt(fallback @ fallback)
            dirn = np.where(wn[:, None] > 0.0, w / np.where(wn == 0.0, 1.0, wn)[:, None], fallback)
            y = zeta + rho * dirn
            dist = np.sqrt(((x - y) ** 2).sum(-1))
            best = np.where(exposed(y, {i, j}), np.minimum(best, dist), best)
    # triple points (two per triple when they exist)
    for i in range(k):
        for j in range(i + 1, k):
            for l in range(j + 1, k):
                pts = _three_sphere_points(centres[i], radii[i], centres[j], radii[j], centres[l], radii[l])
                for y0 in pts:
                    y = np.broadcast_to(y0, x.shape)
                    dist = np.sqrt(((x - y0) ** 2).sum(-1))
                    best = np.where(exposed(y, {i, j, l}), np.minimum(best, dist), best)
    return best


def _three_sphere_points(c1, r1, c2, r2, c3, r3):
    """Intersection points of three spheres (0 or 2 points; tangency gives 1)."""
    ex = c2 - c1
    d = np.sqrt(ex @ ex)
    if d == 0.0:
        return []
    ex = ex / d
    i = ex @ (c3 - c1)
    ey = c3 - c1 - i * ex
    eyn = np.sqrt(ey @ ey)
    if eyn == 0.0:
        return []
    ey = ey / eyn
    ez = np.cross(ex, ey)
    j = ey @ (c3 - c1)
    x = (r1 * r1 - r2 * r2 + d * d) / (2.0 * d)
    y = (r1 * r1 - r3 * r3 + i * i + j * j - 2.0 * i * x) / (2.0 * j)
    z2 = r1 * r1 - x * x - y * y
    if z2 < 0.0:
        return []
    z = np.sqrt(z2)
    base = c1 + x * ex + y * ey
    if z == 0.0:
        return [base]
    return [base + z * ez, base - z * ez]


def ball_union_sdf(x: np.ndarray, centres, radii, chunk: int = 65536) -> np.ndarray:
    """Exact SDF of a union of balls.

    Outside the union the distance is the smallest distance to any ball.
    Inside it is minus the true distance to the union's boundary (not the
    min of the individual SDFs, which underestimates depth where balls
    overlap).
    """
    centres = np.asarray(centres, dtype=np.float64)
    radii = np.asarray(radii, dtype=np.float64)
    out = np.empty(len(x))
    for s in range(0, len(x), chunk):
        xc = x[s:s + chunk]
        dmin = np.full(len(xc), np.inf)
        for c, r in zip(centres, radii):
            dmin = np.minimum(dmin, np.sqrt(((xc - c) ** 2).sum(-1)) - r)
        val = dmin.copy()
        inside = dmin < 0.0
        if inside.any():
            val[inside] = -_ball_union_exposed_distance(xc[inside], centres, radii)
        out[s:s + chunk] = val
    return out
