"""Pins of the minimum valid radius (Prop. 2 proof; Corollary 1; Sec. 6)."""
import math

import numpy as np
import pytest

from oracle import geom, rmin
from oracle.common import TOL, dist
from sdfgen import configs, shapes


@pytest.fixture(params=[True, False], ids=["c", "numpy"])
def impl(request):
    old = geom.USE_C
    geom.USE_C = request.param
    yield request.param
    geom.USE_C = old


def test_one_ball(impl):
    P = np.array([[0.0, 0.0, 0.0]])
    S = np.array([0.4])
    r, x, k, i = rmin.min_valid_radius(np.array([0.1, 0.0, 0.0]), 1, P, S)
    assert abs(r - 0.3) < 1e-15 and k == "T" and i == 0
    assert abs(dist(x, [0.4, 0, 0])) < 1e-15


def test_outside_every_ball_is_zero(impl):
    P = np.array([[0.0, 0.0, 0.0]])
    r, *_ = rmin.min_valid_radius(np.array([0.5, 0, 0]), 1, P, np.array([0.4]))
    assert r == 0.0


def test_two_ball_lens_closed_form(impl):
    # q on the axis between two equal overlapping balls: the nearest contour
    # point is on the intersection circle, at distance sqrt(rho^2 + dz^2)
    R, h = 0.3, 0.2
    P = np.array([[0, 0, -h], [0, 0, h]])
    S = np.array([R, R])
    q = np.array([0.0, 0.0, 0.05])
    r, x, k, _ = rmin.min_valid_radius(q, 1, P, S)
    # both radial foot points ((0,0,-0.1) and (0,0,0.1)) lie inside the other
    # ball, so the nearest contour point is on an intersection circle.  The
    # contour geometry shrinks the covering ball by the uniqueness tolerance
    # 1e-9: the circle of sphere (0,0,c) radius R with ball (0,0,-c) radius
    # R - 1e-9 lies in the plane z0 = c ((R - 1e-9)^2 - R^2) / (4 c^2) ... for
    # either sphere; the nearer of the two circles is the answer.
    Rs = R - 1e-9
    want = math.inf
    for c in (h, -h):
        z0 = (Rs * Rs - R * R) / (4.0 * c)      # plane of sphere(c, R) with ball(-c, Rs)
        rho2 = R * R - (z0 - c) ** 2
        want = min(want, math.sqrt(rho2 + (0.05 - z0) ** 2))
    assert abs(r - want) < 1e-12 and k == "D"
    assert abs(x[2]) < 1e-8


def test_matches_exact_union_of_balls_interior():
    # the generator computes the union's interior distance by its own feature
    # enumeration; the oracle's r_min against the 8 generating balls must agree
    c, rr = configs.ball_union_params(1002)
    P = c.copy()
    S = rr.copy()
    rng = np.random.default_rng(5)
    X = rng.uniform(0.2, 0.8, (4000, 3))
    phi = shapes.ball_union_sdf(X, c, rr)
    inside = X[phi < -1e-3][:60]
    assert len(inside) > 20
    for x in inside:
        r, *_ = rmin.min_valid_radius(x, 1, P, S)
        # the contour is that of the balls shrunk by 1e-9 (uniqueness tolerance):
        # it moves by 1e-9 on spheres and by 1e-9 / sin(crossing angle) on circles
        assert abs(r + shapes.ball_union_sdf(x[None], c, rr)[0]) < 5e-8


def test_monte_carlo_upper_bound():
    rng = np.random.default_rng(9)
    P = rng.uniform(-0.2, 0.2, (6, 3))
    S = rng.uniform(0.15, 0.3, 6)
    q = P[0] + 0.01
    r, x, k, i = rmin.min_valid_radius(q, 1, P, S)
    # any sampled contour point is at least r away, and some come close
    dirs = rng.normal(size=(20000, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    best = math.inf
    for c in range(6):
        X = P[c] + S[c] * dirs
        unc = ~(dist(X[:, None, :], P[None, :, :]) < S[None, :]).any(1)
        if unc.any():
            best = min(best, dist(X[unc], q).min())
    assert r <= best + 1e-12 and best - r < 0.02


def test_c_radius_search_equals_numpy_definition():
    # the C search skips spheres whose part outside the deepest ball is beyond
    # the bound; the NumPy restatement tries every sphere best first: the two
    # must agree on random ball unions (both signs) and scattered points
    from oracle import fastgeom, spheres  # noqa: F401
    from oracle import rmin as RM
    from oracle import geom as G
    rng = np.random.default_rng(31)
    checked = 0
    for trial in range(40):
        k = int(rng.integers(6, 14))
        P = rng.uniform(0.2, 0.8, (k, 3))
        S = rng.uniform(0.08, 0.25, k) * (1 if trial % 2 == 0 else -1)
        sigma = 1 if trial % 2 == 0 else -1
        for q in rng.uniform(0.2, 0.8, (6, 3)):
            old = G.USE_C
            try:
                G.USE_C = True
                a = RM.min_valid_radius(q, sigma, P, S)
                G.USE_C = False
                b = RM.min_valid_radius(q, sigma, P, S)
            finally:
                G.USE_C = old
            assert (a[3] == -1) == (b[3] == -1)
            if a[3] >= 0:
                assert abs(a[0] - b[0]) <= 1e-12, (trial, a, b)
                checked += 1
    assert checked > 60
