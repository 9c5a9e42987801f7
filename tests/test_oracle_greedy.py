"""Pins of the greedy interpolation oracle (Sec. 3.3, Sec. 4, Prop. 1, Prop. 2)."""
import numpy as np
import pytest

from oracle import bounds as B
from oracle import certify as C
from oracle import geom
from oracle import greedy as G
from oracle import order as O
from oracle.common import (KIND_HI, KIND_INFEASIBLE, KIND_LO, KIND_UNRESOLVED, TOL, dist)
from sdfgen import configs


def run(w):
    W, ok = G.input_witnesses(w.points, w.values)
    assert ok.all()
    order, _, _ = O.refinement_order(w.points, w.values, w.grid)
    return G.greedy_interpolate(w.points, w.values, w.queries, order, W), order


@pytest.mark.parametrize("d_over_s", [0.5, 2.0, 2.9, 3.1, 5.0])
def test_one_sample_one_query_closed_form(d_over_s):
    # lo = s - d, hi = s + d; the score prefers hi (weight 1) over lo (weight 2
    # when negative) iff s + d > 2 (d - s), i.e. d < 3 s; with a single sample
    # both tangent points are uncovered, so the preferred one is valid
    s = 0.1
    P = np.array([[0.2, 0.2, 0.2]])
    S = np.array([s])
    q = P[0] + np.array([d_over_s * s, 0.0, 0.0])
    W, ok = G.input_witnesses(P, S)
    r = G.greedy_interpolate(P, S, q[None], [0], W)
    d = d_over_s * s
    want = s + d if d < 3 * s else s - d
    assert abs(r.values[0] - want) < 1e-15
    assert r.kind[0] == (KIND_HI if d < 3 * s else KIND_LO)


def test_score_tie_prefers_negative():
    s = 0.1
    P = np.array([[0.2, 0.2, 0.2]])
    q = P[0] + np.array([0.3, 0.0, 0.0])   # d = 3 s exactly: scores 0.4 and 2*0.2
    r = G.greedy_interpolate(P, np.array([s]), q[None], [0], G.input_witnesses(P, np.array([s]))[0])
    assert r.values[0] < 0


@pytest.mark.parametrize("make", [lambda: configs.sphere(5), lambda: configs.sphere(6),
                                  lambda: configs.ball_union(5)], ids=["sphere5", "sphere6", "balls5"])
def test_greedy_output_is_valid(make):
    w = make()
    r, order = run(w)
    assert not np.any(r.kind == KIND_INFEASIBLE) and not np.any(r.kind == KIND_UNRESOLVED)
    P = np.vstack([w.points, w.queries])
    S = np.concatenate([w.values, r.values])
    W = np.vstack([r.sample_witness, r.witness])
    cert = C.certify(P, S, W)
    assert cert["violations"] == 0, cert
    # every value lies within the bounds of the input samples (later values
    # only tighten them) and the sign is forced inside a ball (Sec. 4.3)
    lo, hi, _, _, flags = B.cone_bounds(w.points, w.values, w.queries)
    assert np.all(r.values >= lo - TOL) and np.all(r.values <= hi + TOL)
    assert np.all(r.values[lo > TOL] > 0) and np.all(r.values[hi < -TOL] < 0)


def test_c_and_numpy_paths_agree():
    w = configs.sphere(4)
    old = geom.USE_C
    try:
        geom.USE_C = True
        a, _ = run(w)
        geom.USE_C = False
        b, _ = run(w)
    finally:
        geom.USE_C = old
    np.testing.assert_array_equal(a.kind, b.kind)
    np.testing.assert_allclose(a.values, b.values, atol=1e-12)
    np.testing.assert_array_equal(a.active, b.active)


def test_failure_mode_opposite_sign_intersection():
    # growing past the tangent point of an opposite-sign sphere (Fig.
    # growing-spheres, top): the cone hi stops exactly at contact
    P = np.array([[0.0, 0.0, 0.0]])
    S = np.array([-0.2])
    q = np.array([0.5, 0.0, 0.0])
    lo, hi, a, b, _ = B.bounds_one(q, P, S)
    assert abs(hi - 0.3) < 1e-15      # |s| + |s_c| = d: touching, not intersecting


def test_failure_mode_new_sphere_fully_covered():
    # (Fig. growing-spheres, middle) the lo candidate inside ball 0 touches it
    # at w, but w lies inside ball 1: the new sphere has no uncovered point
    P = np.array([[0.0, 0.0, 0.0], [0.25, 0.0, 0.0]])
    S = np.array([0.3, 0.2])
    q = np.array([0.05, 0.0, 0.0])
    W, ok = G.input_witnesses(P, S)
    lo, hi, a, b, d = B.bounds_one(q, P, S)
    assert a == 0
    w = P[0] + S[0] * (q - P[0]) / d[0]
    ok, _, _ = G.candidate_valid(q, lo, w, P, S, W)
    assert not ok


def test_failure_mode_existing_sphere_fully_covered():
    # (Fig. growing-spheres, bottom) a big new ball swallowing a small sphere
    # everywhere but at its tangency, where a third ball covers it
    P = np.array([[0.0, 0.0, 0.0], [0.3, 0.0, 0.0], [0.45, 0.0, 0.0]])
    S = np.array([0.05, 0.2, 0.12])
    W, ok = G.input_witnesses(P, S)
    q = np.array([-0.1, 0.0, 0.0])
    s = 0.1 + 0.05                      # internally tangent to ball 0 at (0.05, 0, 0)
    w = np.array([0.05, 0.0, 0.0])      # inside ball 1 (|0.05 - 0.3| = 0.25 > 0.2? no)
    ok_new, _, _ = G.candidate_valid(q, s, w, P, S, W)
    # ball 0's whole sphere lies in the new open ball except its tangent point,
    # which ball 1 does not reach: valid
    assert ok_new
    S2 = np.array([0.05, 0.26, 0.12])   # now ball 1 covers the tangent point
    W2, ok2 = G.input_witnesses(P, S2)
    assert ok2.all()
    ok_new2, _, _ = G.candidate_valid(q, s, w, P, S2, W2)
    assert not ok_new2


def test_input_with_covered_sphere_has_no_witness():
    P = np.array([[0.0, 0.0, 0.0], [0.05, 0.0, 0.0]])
    S = np.array([0.3, 0.1])              # sphere 1 lies inside ball 0
    W, ok = G.input_witnesses(P, S)
    assert ok[0] and not ok[1]


def test_order_is_permutation_and_deterministic():
    w = configs.sphere(4)
    o1, pc, cc = O.refinement_order(w.points, w.values, w.grid)
    o2, _, _ = O.refinement_order(w.points, w.values, w.grid)
    assert sorted(o1.tolist()) == list(range(w.m))
    np.testing.assert_array_equal(o1, o2)


def test_covered_counts_match_brute_force():
    w = configs.sphere(4)
    counts = O.covered_counts(4, w.points, w.values)
    R = np.abs(w.values) - TOL
    for c in range(64):
        x, y, z = c % 4, (c // 4) % 4, c // 16
        pts = O._subpoints(np.array([x, y, z]) / 4.0, 0.25)
        d = dist(pts[:, None, :], w.points[None, :, :])
        assert counts[c] == int((d < R[None, :]).any(1).sum())


def test_flood_fill_hand_grid():
    # 2x2x2 grid: start at the lowest count, then its face neighbours by count
    counts = np.array([5, 1, 7, 3, 2, 6, 4, 0])
    cells = O.flood_fill(counts, 2)
    # start 7 (count 0); neighbours of 7 = 6, 5, 3 -> pop 3 (count 3);
    # neighbours of 3: 2, 1 -> heap {6:4, 5:6, 2:7, 1:1} -> pop 1, then 0 or ...
    assert cells[0] == 7 and cells[1] == 3 and cells[2] == 1
    assert sorted(cells.tolist()) == list(range(8))


def test_children_sorted_by_child_ratio():
    w = configs.sphere(4)
    order, parent, child = O.refinement_order(w.points, w.values, w.grid)
    for k in range(0, w.m, 8):
        kids = child[order[k:k + 8]]
        assert np.all(np.diff(kids) >= 0)
