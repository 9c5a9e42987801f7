"""Pins of the oracle's cone bounds (Sec. 4.3 bounds; Appendix B tolerances)."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import bounds as B
from oracle import fastgeom
from oracle.common import FLAG_INSIDE_NEG, FLAG_INSIDE_POS, TIE_TOL
from sdfgen import configs, shapes


def test_constant_values_reduce_to_nearest_neighbour():
    # with s_c = k for every sample: hi = k + NN distance, lo = k - NN distance,
    # and both extremes are attained by the nearest sample (a textbook k-d tree query)
    rng = np.random.default_rng(1)
    P = rng.uniform(0, 1, (300, 3))
    S = np.full(300, 0.125)
    Q = rng.uniform(0, 1, (200, 3))
    lo, hi, a, b, _ = B.cone_bounds(P, S, Q)
    dnn, inn = cKDTree(P).query(Q)
    np.testing.assert_allclose(hi, 0.125 + dnn, atol=1e-14)
    np.testing.assert_allclose(lo, 0.125 - dnn, atol=1e-14)
    np.testing.assert_array_equal(a, inn)
    np.testing.assert_array_equal(b, inn)


def test_single_sample_closed_form():
    P = np.array([[0.2, 0.3, 0.4]])
    S = np.array([-0.05])
    Q = np.array([[0.5, 0.3, 0.4], [0.2, 0.3, 0.42]])
    lo, hi, a, b, f = B.cone_bounds(P, S, Q)
    np.testing.assert_allclose(lo, [-0.05 - 0.3, -0.05 - 0.02], atol=1e-15)
    np.testing.assert_allclose(hi, [-0.05 + 0.3, -0.05 + 0.02], atol=1e-15)
    assert f[1] & FLAG_INSIDE_NEG and not f[0] & FLAG_INSIDE_NEG


@pytest.mark.parametrize("shape", ["sphere", "box", "balls"])
def test_exact_sdf_lies_between_bounds(shape):
    # an exact SDF is 1-Lipschitz, so lo(q) <= phi(q) <= hi(q) everywhere
    P = configs.grid_centres(8)
    Q = np.random.default_rng(2).uniform(0, 1, (400, 3))
    if shape == "sphere":
        f = lambda x: shapes.sphere_sdf(x, (0.45, 0.5, 0.55), 0.27)
    elif shape == "box":
        f = lambda x: shapes.box_sdf(x, (0.5, 0.5, 0.5), (0.2, 0.15, 0.25))
    else:
        c, r = configs.ball_union_params(1002)
        f = lambda x: shapes.ball_union_sdf(x, c, r)
    lo, hi, *_ = B.cone_bounds(P, f(P), Q)
    phi = f(Q)
    assert np.all(lo <= phi + 1e-12) and np.all(phi <= hi + 1e-12)


def test_samples_on_the_ray_pin_the_value():
    # sphere SDF, samples on the ray from the centre through q on both sides of
    # q (all outside): the cones meet exactly at phi(q)
    c = np.array([0.5, 0.5, 0.5])
    u = np.array([1.0, 2.0, 2.0]) / 3.0
    q = c + 0.4 * u
    P = np.stack([c + 0.35 * u, c + 0.47 * u])
    S = shapes.sphere_sdf(P, c, 0.3)
    lo, hi, *_ = B.cone_bounds(P, S, q[None])
    assert abs(lo[0] - 0.1) < 1e-15 and abs(hi[0] - 0.1) < 1e-15


def test_ties_take_the_smallest_index():
    P = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 0, 0]])
    S = np.array([0.2, 0.2, 0.2])
    lo, hi, a, b, f = B.cone_bounds(P, S, np.array([[0.5, 0.0, 0.0]]))
    assert a[0] == 0 and b[0] == 0


def test_flags_inside():
    P = np.array([[0.0, 0, 0]])
    S = np.array([0.5])
    _, _, _, _, f = B.cone_bounds(P, S, np.array([[0.1, 0, 0], [0.7, 0, 0]]))
    assert f[0] & FLAG_INSIDE_POS and not f[1] & FLAG_INSIDE_POS


def test_c_loops_match_numpy():
    rng = np.random.default_rng(3)
    P = rng.uniform(0, 1, (500, 3))
    S = rng.uniform(-0.2, 0.2, 500)
    for q in rng.uniform(0, 1, (50, 3)):
        l, h, a, b, _ = B.bounds_one(q, P, S)
        l2, h2, a2, b2 = fastgeom.bounds_one(q, P, S, TIE_TOL)
        assert l == l2 and h == h2 and a == a2 and b == b2
