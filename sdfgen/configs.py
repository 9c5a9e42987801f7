"""Seeded synthetic workloads.

Every input sample sits at a cell centre ((i + 0.5)/N) of a regular grid on
the unit cube, as in the paper's grid-based refinement (Sec. 4.1).  Arrays
are float64, points are (count, 3) with x varying fastest: the linear index of
grid cell (x, y, z) is x + N*y + N*N*z.

Workloads (the names used across tests and the benchmark):
  sphere16     exact sphere SDF, 16^3 samples, 32^3 refinement queries
  balls64      exact SDF of a union of 8 balls, 64^3 samples, 128^3 queries
  csg96        CSG pseudo-SDF over 16 primitives, 96^3 samples, 400k scattered
  batch64      64 independent sphere/box unions on uneven grids
  balls48      8-ball union, 48^3 samples, 256k uniform queries
Smaller variants (fewer grid cells, same recipe) serve the CPU tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import shapes


def grid_centres(n: int) -> np.ndarray:
    """Cell centres of an n^3 grid on [0,1]^3, x fastest."""
    t = (np.arange(n, dtype=np.float64) + 0.5) / n
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


@dataclass
class Workload:
    name: str
    points: np.ndarray          # (n, 3) sample positions
    values: np.ndarray          # (n,)  sample SDF values
    queries: np.ndarray         # (m, 3) query positions
    grid: int = 0               # input grid resolution (0 = scattered samples)
    query_grid: int = 0         # query grid resolution (0 = scattered queries)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.values)

    @property
    def m(self) -> int:
        return len(self.queries)


def sphere(grid: int = 16, centre=(0.5, 0.5, 0.5), radius: float = 0.3) -> Workload:
    """Exact SDF of one sphere, refined 2x (queries at the fine cell centres)."""
    p = grid_centres(grid)
    q = grid_centres(2 * grid)
    return Workload(f"sphere{grid}", p, shapes.sphere_sdf(p, centre, radius), q, grid, 2 * grid,
                    {"centre": centre, "radius": radius})


def ball_union_params(seed: int, count: int = 8):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.2, 0.8, size=(count, 3))
    radii = rng.uniform(0.05, 0.2, size=count)
    return centres, radii


def ball_union(grid: int = 64, seed: int = 1002, refine: bool = True,
               query_count: int = 0, query_seed: int = 0) -> Workload:
    """Exact SDF of a union of 8 seeded balls on a grid.

    With ``refine`` the queries are the (2*grid)^3 fine cell centres; otherwise
    ``query_count`` uniform points in [0,1]^3 drawn with ``query_seed``.
    """
    centres, radii = ball_union_params(seed)
    p = grid_centres(grid)
    s = shapes.ball_union_sdf(p, centres, radii)
    if refine:
        q = grid_centres(2 * grid)
        qg = 2 * grid
    else:
        q = np.random.default_rng(query_seed).uniform(0.0, 1.0, size=(query_count, 3))
        qg = 0
    return Workload(f"balls{grid}", p, s, q, grid, qg, {"centres": centres, "radii": radii, "seed": seed})


def csg_primitives(seed: int = 1003):
    """16 primitives in 8 pairs; each pair combined by min, max or max(a, -b)."""
    rng = np.random.default_rng(seed)
    prims = []
    for k in range(16):
        kind = int(rng.integers(0, 3))  # 0 sphere, 1 box, 2 capsule
        if k % 2 == 1:
            centre = prims[k - 1]["centre"] + rng.uniform(-0.1, 0.1, size=3)
        else:
            centre = rng.uniform(0.2, 0.8, size=3)
        if kind == 0:
            prims.append({"kind": "sphere", "centre": centre, "radius": rng.uniform(0.05, 0.25)})
        elif kind == 1:
            prims.append({"kind": "box", "centre": centre, "half": rng.uniform(0.05, 0.25, size=3)})
        else:
            r = rng.uniform(0.05, 0.25)
            half_len = rng.uniform(0.05, 0.25)
            d = rng.normal(size=3)
            d /= np.sqrt(d @ d)
            prims.append({"kind": "capsule", "centre": centre, "radius": r,
                          "a": centre - half_len * d, "b": centre + half_len * d})
    ops = [int(rng.integers(0, 3)) for _ in range(8)]  # 0 min, 1 max, 2 max(a, -b)
    return prims, ops


def _prim_sdf(x, prim):
    if prim["kind"] == "sphere":
        return shapes.sphere_sdf(x, prim["centre"], prim["radius"])
    if prim["kind"] == "box":
        return shapes.box_sdf(x, prim["centre"], prim["half"])
    return shapes.capsule_sdf(x, prim["a"], prim["b"], prim["radius"])


def csg_field(x, prims, ops):
    """Pseudo-SDF of the CSG tree: pairwise min/max/difference, then min."""
    out = np.full(len(x), np.inf)
    for k in range(8):
        a = _prim_sdf(x, prims[2 * k])
        b = _prim_sdf(x, prims[2 * k + 1])
        if ops[k] == 0:
            f = np.minimum(a, b)
        elif ops[k] == 1:
            f = np.maximum(a, b)
        else:
            f = np.maximum(a, -b)
        out = np.minimum(out, f)
    return out


def csg(grid: int = 96, seed: int = 1003, uniform_queries: int = 200000, near_queries: int = 200000,
        uniform_seed: int = 3001, near_seed: int = 3002) -> Workload:
    """CSG pseudo-SDF samples plus scattered extension queries.

    Half the queries are uniform in the unit cube; the other half are drawn
    near the zero level set: points with |f| < 0.002 found by rejection, then
    jittered by N(0, 0.01^2 I) and kept only inside the unit cube.
    """
    prims, ops = csg_primitives(seed)
    p = grid_centres(grid)
    s = csg_field(p, prims, ops)
    qu = np.random.default_rng(uniform_seed).uniform(0.0, 1.0, size=(uniform_queries, 3))
    rng = np.random.default_rng(near_seed)
    near = []
    have = 0
    while have < near_queries:
        cand = rng.uniform(0.0, 1.0, size=(max(4 * near_queries, 65536), 3))
        cand = cand[np.abs(csg_field(cand, prims, ops)) < 0.002]
        cand = cand + rng.normal(0.0, 0.01, size=cand.shape)
        cand = cand[np.all((cand >= 0.0) & (cand <= 1.0), axis=1)]
        near.append(cand)
        have += len(cand)
    qn = np.concatenate(near)[:near_queries]
    q = np.concatenate([qu, qn]) if near_queries else qu
    return Workload(f"csg{grid}", p, s, q, grid, 0, {"prims": prims, "ops": ops})


BATCH_GRIDS = (16, 24, 32, 48, 64, 96)


def batch_instance(i: int, grids=BATCH_GRIDS) -> Workload:
    """One instance of the batched workload: 1-3 disjoint spheres/boxes.

    The primitives keep a clearance of at least 2/N between each other, so the
    min of their SDFs is the exact SDF of the union (the union of disjoint
    solids has the disjoint boundaries as its boundary).
    """
    rng = np.random.default_rng(4000 + i)
    n = int(rng.choice(grids))
    count = int(rng.integers(1, 4))
    prims = []
    tries = 0
    while len(prims) < count and tries < 1000:
        tries += 1
        centre = rng.uniform(0.25, 0.75, size=3)
        if rng.integers(0, 2) == 0:
            prim = {"kind": "sphere", "centre": centre, "radius": rng.uniform(0.08, 0.2)}
            extent = prim["radius"]
        else:
            prim = {"kind": "box", "centre": centre, "half": rng.uniform(0.05, 0.15, size=3)}
            extent = float(np.sqrt(prim["half"] @ prim["half"]))
        ok = True
        for other in prims:
            oext = other["radius"] if other["kind"] == "sphere" else float(np.sqrt(other["half"] @ other["half"]))
            gap = np.sqrt(((other["centre"] - centre) ** 2).sum()) - extent - oext
            if gap < 2.0 / n:
                ok = False
                break
        if ok:
            prims.append(prim)
    p = grid_centres(n)
    s = np.full(len(p), np.inf)
    for prim in prims:
        s = np.minimum(s, _prim_sdf(p, prim))
    return Workload(f"batch{i}", p, s, grid_centres(2 * n), n, 2 * n, {"prims": prims})


def batch(count: int = 64, grids=BATCH_GRIDS) -> list:
    return [batch_instance(i, grids) for i in range(count)]


def by_name(name: str) -> Workload:
    """The five named workloads at full size."""
    if name == "sphere16":
        return sphere(16)
    if name == "balls64":
        return ball_union(64, 1002)
    if name == "csg96":
        return csg(96)
    if name == "balls48":
        return ball_union(48, 1005, refine=False, query_count=262144, query_seed=5001)
    raise KeyError(name)
