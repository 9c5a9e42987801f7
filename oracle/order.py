"""Refinement order (Sec. 4.2, "Refinement order").

Each cell's covered area ratio is estimated from 8^d regularly spaced points
in the cell, each tested for containment in the input balls.  A flood fill
starts at the cell with the lowest ratio; popping a cell subdivides it (its
2^d children get their values in ascending order of their own covered
ratio) and pushes its face neighbours, lowest ratio first.  Readings: the
regular points are the (k + 0.5)/8 sub-grid of the cell; ratios use the
input balls only, so the order is fixed before any value is assigned; every
cell of the grid takes part (whole-grid refinement); ties in a ratio go to
the smaller linear index x + N*y + N*N*z, ties among children to the
smaller child index bx + 2*by + 4*bz.
"""
from __future__ import annotations

import heapq
import math

import numpy as np

from .common import TOL, dist

SUB = 8


def _subpoints(lo_corner, size):
    t = (np.arange(SUB, dtype=np.float64) + 0.5) / SUB
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    rel = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    return lo_corner + size * rel


def covered_counts(res, P, S, tol=TOL):
    """Number of the 512 sub-points of each cell of a res^3 grid on [0,1]^3
    that lie strictly inside some input ball."""
    size = 1.0 / res
    half_diag = 0.5 * size * math.sqrt(3.0)
    R = np.abs(S) - tol
    counts = np.empty(res ** 3, dtype=np.int64)
    idx = np.arange(res ** 3)
    cx = idx % res
    cy = (idx // res) % res
    cz = idx // (res * res)
    for c in range(res ** 3):
        corner = np.array([cx[c], cy[c], cz[c]], dtype=np.float64) * size
        centre = corner + 0.5 * size
        dc = dist(P, centre)
        # a ball farther than R + half_diag from the centre misses the cell;
        # a ball with R > dc + half_diag holds the whole cell
        if np.any(R > dc + half_diag):
            counts[c] = SUB ** 3
            continue
        near = R > dc - half_diag
        if not near.any():
            counts[c] = 0
            continue
        pts = _subpoints(corner, size)
        d = dist(pts[:, None, :], P[near][None, :, :])
        counts[c] = int((d < R[near][None, :]).any(1).sum())
    return counts


def flood_fill(counts, res):
    """Best-first flood fill over the res^3 cells keyed by (count, index)."""
    start = int(np.lexsort((np.arange(res ** 3), counts))[0])
    seen = np.zeros(res ** 3, dtype=bool)
    queued = np.zeros(res ** 3, dtype=bool)
    heap = [(int(counts[start]), start)]
    queued[start] = True
    out = []
    while heap:
        _, c = heapq.heappop(heap)
        if seen[c]:
            continue
        seen[c] = True
        out.append(c)
        x, y, z = c % res, (c // res) % res, c // (res * res)
        for dx, dy, dz in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
            X, Y, Z = x + dx, y + dy, z + dz
            if 0 <= X < res and 0 <= Y < res and 0 <= Z < res:
                nb = X + res * Y + res * res * Z
                if not queued[nb]:
                    queued[nb] = True
                    heapq.heappush(heap, (int(counts[nb]), nb))
    return np.array(out, dtype=np.int64)


def refinement_order(P, S, res, tol=TOL):
    """Order of the (2 res)^3 refinement queries (child cell centres)."""
    parent = covered_counts(res, P, S, tol)
    child = covered_counts(2 * res, P, S, tol)
    cells = flood_fill(parent, res)
    fine = 2 * res
    out = np.empty(fine ** 3, dtype=np.int64)
    k = 0
    for c in cells:
        x, y, z = c % res, (c // res) % res, c // (res * res)
        kids = []
        for b in range(8):
            bx, by, bz = b & 1, (b >> 1) & 1, (b >> 2) & 1
            q = (2 * x + bx) + fine * (2 * y + by) + fine * fine * (2 * z + bz)
            kids.append((int(child[q]), b, q))
        kids.sort()
        for _, _, q in kids:
            out[k] = q
            k += 1
    return out, parent, child


def scattered_order(P, S, res, Q, tol=TOL):
    """Scattered queries: bucketed by the input cell holding them, buckets in
    flood-fill order, queries of one bucket by index."""
    parent = covered_counts(res, P, S, tol)
    cells = flood_fill(parent, res)
    cell_of = np.clip(np.floor(np.asarray(Q) * res).astype(np.int64), 0, res - 1)
    lin = cell_of[:, 0] + res * cell_of[:, 1] + res * res * cell_of[:, 2]
    rank = np.empty(res ** 3, dtype=np.int64)
    rank[cells] = np.arange(res ** 3)
    return np.lexsort((np.arange(len(Q)), rank[lin])), parent
