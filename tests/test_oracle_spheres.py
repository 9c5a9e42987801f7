"""Pins of the exact uncovered-point search (Prop. 1 (ii); Def. 1 U and D)."""
import math

import numpy as np
import pytest

from oracle import fastgeom, spheres
from oracle.common import TOL, dist


def fib_dirs(n):
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * i / n)
    th = math.pi * (1 + 5 ** 0.5) * i
    return np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)


DIRS = fib_dirs(40000)


def brute_margin(o, r, P, S):
    """max over Fibonacci points of the smallest uncovered margin; > 0 means
    some sampled point is uncovered."""
    X = o + r * DIRS
    best = -np.inf
    for s0 in range(0, len(X), 4000):
        d = dist(X[s0:s0 + 4000, None, :], P[None, :, :])
        marg = (d - (np.abs(S) - TOL)[None, :]).min(1)
        best = max(best, float(marg.max()))
    return best


@pytest.mark.parametrize("impl", ["numpy", "c"])
def test_matches_dense_sampling(impl):
    rng = np.random.default_rng(7)
    agree = 0
    for trial in range(60):
        o = rng.uniform(-0.2, 0.2, 3)
        r = rng.uniform(0.1, 0.3)
        k = int(rng.integers(1, 9))
        P = o + rng.normal(size=(k, 3)) * 0.25
        S = rng.uniform(0.05, 0.35, k)
        if impl == "numpy":
            x = spheres.uncovered_point(o, r, P, S, TOL)
        else:
            x = fastgeom.uncovered_point(o, r, P, S, TOL)
        m = brute_margin(o, r, P, S)
        if abs(m) < 2e-3:
            continue  # too close to call by sampling
        agree += 1
        assert (x is not None) == (m > 0), (trial, m)
        if x is not None:
            assert abs(dist(x, o) - r) < 1e-9
            assert not np.any(dist(P, x) < np.abs(S) - TOL)
    assert agree > 40


def test_concentric_bigger_ball_covers():
    o = np.zeros(3)
    assert spheres.uncovered_point(o, 0.2, np.zeros((1, 3)), np.array([0.3])) is None
    assert fastgeom.uncovered_point(o, 0.2, np.zeros((1, 3)), np.array([0.3]), TOL) is None


def test_touching_is_uncovered():
    # two balls touching at one point cover nothing of each other's sphere
    o = np.zeros(3)
    P = np.array([[0.5, 0, 0]])
    S = np.array([0.3])
    assert spheres.uncovered_point(o, 0.2, P, S) is not None


def test_six_neighbours_cover_then_five_do_not():
    # a sphere of radius 1 with six balls on the axes at distance 1 and radius
    # 0.9: each cap is cos > 0.595, the six caps cover the sphere (every unit
    # vector has a coordinate of size >= 1/sqrt(3) = 0.577 ... too small), so
    # use radius 1.0: cap cos > 0.5 covers (max |coord| >= 0.577 > 0.5)
    o = np.zeros(3)
    axes = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    S = np.full(6, 1.0)
    for impl in (spheres.uncovered_point, lambda *a: fastgeom.uncovered_point(*a, TOL)):
        assert impl(o, 1.0, axes, S) is None
        x = impl(o, 1.0, axes[:5], S[:5])
        assert x is not None and x[2] < -0.5


def test_lens_rim_point():
    # sphere covered everywhere except a thin band: two big caps leave the
    # equator of the z axis uncovered only if they do not overlap
    o = np.zeros(3)
    P = np.array([[0, 0, 1.0], [0, 0, -1.0]])
    S = np.array([1.0, 1.0])   # caps: z > 0.5 and z < -0.5
    x = spheres.uncovered_point(o, 1.0, P, S)
    assert x is not None and abs(x[2]) <= 0.5 + 1e-9
    S2 = np.array([1.5, 1.5])  # caps reach past the equator: covered
    assert spheres.uncovered_point(o, 1.0, P, S2) is None


def test_nearest_uncovered_against_sampling():
    rng = np.random.default_rng(11)
    checked = 0
    for trial in range(40):
        o = np.zeros(3)
        r = 0.3
        k = int(rng.integers(1, 6))
        P = rng.normal(size=(k, 3)) * 0.3
        S = rng.uniform(0.05, 0.3, k)
        q = rng.normal(size=3) * 0.2
        res = spheres.nearest_uncovered(o, r, P, S, q, math.inf, 0.0)
        resc = fastgeom.nearest_uncovered(o, r, P, S, q, math.inf, 0.0)
        X = o + r * DIRS
        unc = ~(dist(X[:, None, :], P[None, :, :]) < np.abs(S)[None, :]).any(1)
        if not unc.any():
            assert res is None and resc is None
            continue
        dmin = dist(X[unc], q).min()
        assert res is not None and resc is not None
        # sampling can only find farther points; the exact answer is at most
        # the sampled one and close to it
        assert res[0] <= dmin + 1e-12 and dmin - res[0] < 0.01
        assert abs(res[0] - resc[0]) < 1e-12
        checked += 1
    assert checked > 20
