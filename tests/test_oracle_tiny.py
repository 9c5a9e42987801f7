"""Pins of the paper-exact tier (Def. 1 candidates, Sec. 3.3 scoring and
single-point interpolation, Prop. 1 validity) and its comparison with the
Level-P reading of the greedy."""
import math

import numpy as np
import pytest

from oracle import bounds as B
from oracle import greedy as G
from oracle import order as O
from oracle import tiny as T
from oracle.common import TOL, dist
from sdfgen import configs


def fibonacci_sphere(k):
    i = np.arange(k) + 0.5
    z = 1.0 - 2.0 * i / k
    r = np.sqrt(1.0 - z * z)
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def brute_valid(P, S, k=20000, known=None):
    """Prop. 1 by dense sampling: (i) on all pairs, (ii) some sampled point of
    every sphere lies in no other open ball.  `known` maps a sphere index to
    one of its points that is tested as well (a sphere touching the others
    only at a point has no uncovered patch for sampling to hit)."""
    P = np.asarray(P, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    R = np.abs(S)
    for x in range(len(S)):
        d = dist(P, P[x])
        opp = np.sign(S[x]) * np.sign(S) < 0
        if np.any(opp & (R[x] + R > d + TOL)):
            return False
    U = fibonacci_sphere(k)
    for x in range(len(S)):
        pts = P[x] + R[x] * U
        if known and x in known:
            pts = np.vstack([pts, known[x]])
        others = np.arange(len(S)) != x
        cov = (dist(pts[:, None, :], P[None, others, :]) < R[None, others] - TOL).any(1)
        if cov.all():
            return False
    return True


def test_triple_points_closed_form():
    # unit spheres at the origin, e_x and e_y meet at (1/2, 1/2, +-1/sqrt 2)
    pts = T.triple_points(np.zeros(3), 1.0, np.array([1.0, 0, 0]), 1.0, np.array([0, 1.0, 0]), 1.0)
    got = sorted(p[2] for p in pts)
    assert len(pts) == 2
    np.testing.assert_allclose(got, [-math.sqrt(0.5), math.sqrt(0.5)], atol=1e-15)
    for p in pts:
        np.testing.assert_allclose(p[:2], [0.5, 0.5], atol=1e-15)
    # too far apart: none; collinear centres: none (a circle or nothing)
    assert T.triple_points(np.zeros(3), 0.4, np.array([1.0, 0, 0]), 0.4, np.array([0, 1.0, 0]), 0.4) == []
    assert T.triple_points(np.zeros(3), 1.0, np.array([1.0, 0, 0]), 1.0, np.array([2.0, 0, 0]), 1.0) == []


def test_triple_points_lie_on_three_spheres():
    rng = np.random.default_rng(3)
    hits = 0
    for _ in range(200):
        C = rng.uniform(0, 1, (3, 3))
        R = rng.uniform(0.3, 0.8, 3)
        for p in T.triple_points(C[0], R[0], C[1], R[1], C[2], R[2]):
            np.testing.assert_allclose(dist(C, p), R, atol=1e-12)
            hits += 1
    assert hits > 50


def test_circle_extreme_points_against_sampling():
    rng = np.random.default_rng(4)
    t = np.linspace(0, 2 * math.pi, 200001)
    for _ in range(20):
        ci, cj = rng.uniform(0, 1, (2, 3))
        ri, rj = rng.uniform(0.4, 0.7, 2)
        circ = T.circle_of(ci, ri, cj, rj)
        if circ is None:
            continue
        zeta, rho, mu = circ
        p = rng.uniform(-1, 1, 3)
        near, far = T.circle_extreme_points(p, zeta, rho, mu)
        e1, e2 = T._perp(mu)
        X = zeta + rho * (np.cos(t)[:, None] * e1 + np.sin(t)[:, None] * e2)
        np.testing.assert_allclose(dist(X, ci), ri, atol=1e-12)
        np.testing.assert_allclose(dist(X, cj), rj, atol=1e-12)
        d = dist(X, p)
        assert dist(near, p) <= d.min() + 1e-9 and dist(far, p) >= d.max() - 1e-9


def test_circle_coverage_against_sampling():
    rng = np.random.default_rng(5)
    t = np.linspace(0, 2 * math.pi, 20000, endpoint=False)
    agree = 0
    for _ in range(300):
        P = rng.uniform(0.3, 0.7, (6, 3))
        S = rng.uniform(0.1, 0.3, 6)
        circ = T.circle_of(P[0], S[0], P[1], S[1])
        if circ is None:
            continue
        zeta, rho, mu = circ
        arcs = T.circle_cover_arcs(zeta, rho, mu, P, S, {0, 1})
        e1, e2 = T._perp(mu)
        X = zeta + rho * (np.cos(t)[:, None] * e1 + np.sin(t)[:, None] * e2)
        margin = (np.abs(S[2:]) - TOL)[None, :] - dist(X[:, None, :], P[None, 2:, :])
        best = margin.max(1)                      # > 0: covered
        if abs(best.min()) < 1e-4:                # the least covered point is nearly on an arc end: skip
            continue
        assert T.arcs_cover_circle(arcs) == bool((best > 0).all())
        agree += 1
    assert agree > 150


def test_is_sdf_valid_matches_dense_sampling():
    rng = np.random.default_rng(6)
    seen = {True: 0, False: 0}
    for _ in range(150):
        k = int(rng.integers(3, 7))
        P = rng.uniform(0.2, 0.8, (k, 3))
        S = rng.uniform(0.05, 0.25, k) * rng.choice([-1.0, 1.0], k)
        want = brute_valid(P, S)
        got = T.is_sdf_valid(P, S)
        # dense sampling may miss a tiny uncovered patch; it never invents one
        assert got or not want
        if got == want:
            seen[got] += 1
    assert seen[True] > 10 and seen[False] > 10


@pytest.mark.parametrize("d_over_s", [0.5, 2.0, 2.9, 3.1, 5.0])
def test_one_sample_closed_form(d_over_s):
    # T only: hi = s + d (score 3M + d + s) against lo = s - d (3M + 2 (d - s)
    # when negative): hi iff d < 3 s
    s = 0.1
    P = np.array([[0.2, 0.2, 0.2]])
    q = P[0] + np.array([d_over_s * s, 0.0, 0.0])
    v, i, _, tang, rank = T.interpolate_sdf_to(q, P, np.array([s]))
    d = d_over_s * s
    assert tang and i == 0 and rank == 0
    assert abs(v - (s + d if d < 3 * s else s - d)) < 1e-15


def test_normals_agree_on_tangent_points():
    # the agreeing tangency values are the cone values s_i - d and s_i + d
    P = np.array([[0.0, 0.0, 0.0]])
    for si in (0.3, -0.3):
        p = np.array([0.5, 0.0, 0.0])
        d = 0.5
        for c, s_agree in ((1.0, si - math.copysign(1.0, si) * d), (-1.0, si + math.copysign(1.0, si) * d)):
            q = P[0] + c * np.array([1.0, 0, 0]) * abs(si)
            assert abs(abs(s_agree) - dist(q, p)) < 1e-15
            assert T.normals_agree(p, s_agree, P[0], si, q)
            assert not T.normals_agree(p, -s_agree, P[0], si, q)


# Five positive balls (a constructed case): the query lies in ball 1; both
# tangency values fail Prop. 1 and the best valid candidate is a triple point
# of spheres 2, 3 and 4 (Def. 1 U), where Level P takes the much smaller
# minimum valid radius.
CASE_U = (np.array([[0.46, 0.4, 0.42], [0.5, 0.69, 0.58], [0.59, 0.49, 0.46], [0.67, 0.48, 0.35],
                    [0.61, 0.38, 0.46]]), np.array([0.15, 0.18, 0.08, 0.16, 0.10]), np.array([0.55, 0.54, 0.51]))
# Four positive balls: the winner is the nearest or farthest point of the
# circle of spheres 0 and 1 (Def. 1 D).
CASE_D = (np.array([[0.68, 0.39, 0.35], [0.56, 0.36, 0.41], [0.47, 0.41, 0.56], [0.36, 0.56, 0.35]]),
          np.array([0.15, 0.2, 0.17, 0.19]), np.array([0.52, 0.36, 0.45]))


@pytest.mark.parametrize("case,on", [(CASE_U, [2, 3, 4]), (CASE_D, [0, 1])], ids=["U", "D"])
def test_intersection_candidate_wins_when_lo_and_hi_fail(case, on):
    P, S, q = case
    assert brute_valid(P, S)
    lo, hi, _, _, _ = B.bounds_one(q, P, S)
    assert lo > TOL                                   # inside a positive ball: the value is positive
    Pn = np.vstack([P, q])
    for s in (lo, hi):
        assert not T.is_sdf_valid(Pn, np.append(S, s))
        assert not brute_valid(Pn, np.append(S, s))
    v, i, x, tang, rank = T.interpolate_sdf_to(q, P, S)
    assert not tang and rank > 0
    np.testing.assert_array_equal(np.nonzero(np.abs(dist(P, x) - S) < 1e-12)[0], on)
    assert not (dist(P, x) < S - TOL).any()           # the grow-to point is uncovered
    assert abs(v - dist(x, q)) < 1e-15 and lo - TOL <= v <= hi + TOL
    # x lies on the new sphere and on the spheres `on`: it is their uncovered point
    assert brute_valid(Pn, np.append(S, v), known={c: x for c in on + [len(S)]})
    # Level P falls back to the minimum valid radius, a smaller valid value
    W, _ = G.input_witnesses(P, S)
    r = G.greedy_interpolate(P, S, q[None], [0], W)
    assert r.kind[0] in (4, 5, 6) and r.values[0] < v
    assert T.is_sdf_valid(Pn, np.append(S, r.values[0]))


def test_cone_prefilter_changes_nothing():
    w = configs.ball_union(3, 1002)
    rng = np.random.default_rng(8)
    for q in rng.uniform(0.1, 0.9, (4, 3)):
        a = T.interpolate_sdf_to(q, w.points, w.values, cone_prefilter=True)
        b = T.interpolate_sdf_to(q, w.points, w.values, cone_prefilter=False)
        assert a[0] == b[0] and a[1] == b[1]


def level_p_vs_exact(w, steps):
    """Replays Level P's first `steps` decisions; at each step the paper-exact
    winner is computed from the same current set.  Returns (Level P kinds,
    disagreeing steps, invalid Level P steps)."""
    order, _, _ = O.refinement_order(w.points, w.values, w.grid)
    W, _ = G.input_witnesses(w.points, w.values)
    r = G.greedy_interpolate(w.points, w.values, w.queries, order, W, stop=steps)
    CP, CS = w.points.copy(), w.values.copy()
    dis, bad = [], []
    for k, j in enumerate(order[:steps]):
        v = T.interpolate_sdf_to(w.queries[j], CP, CS)[0]
        Pn = np.vstack([CP, w.queries[j]])
        if not T.is_sdf_valid(Pn, np.append(CS, r.values[j]), first=[len(CS)]):
            bad.append(k)
        if not abs(v - r.values[j]) <= 1e-9:
            dis.append(k)
        CP, CS = Pn, np.append(CS, r.values[j])
    return r.kind[order[:steps]], dis, bad


@pytest.mark.slow
@pytest.mark.parametrize("make,steps", [(lambda: configs.sphere(3), 40), (lambda: configs.ball_union(3, 1002), 40)],
                         ids=["sphere3", "balls3"])
def test_level_p_against_paper_exact(make, steps):
    """Reports (does not gate) how often Level P and the paper-exact rule
    choose different values, and requires every Level P value to pass the
    paper's own validity test."""
    w = make()
    kinds, dis, bad = level_p_vs_exact(w, steps)
    fallback = np.nonzero(np.isin(kinds, [4, 5, 6]))[0]
    print(f"{w.name}: {len(dis)} of {steps} steps differ from the paper-exact choice "
          f"({len(fallback)} minimum-valid-radius fallbacks); steps {dis}", flush=True)
    assert bad == []
    # every tangency (lo/hi) decision of Level P is also the paper-exact one here
    assert set(dis) <= set(fallback.tolist())
