"""Pins of pseudo-SDF repair (Sec. 6, Corollary 1), the certificate and the adjoint."""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import certify as C
from oracle import greedy as G
from oracle import repair as R
from oracle.common import KIND_RMIN_D, KIND_RMIN_U, dist
from sdfgen import configs


def test_repair_of_exact_sdf_is_identity():
    w = configs.sphere(5)
    out, removed, qv, kind, _ = R.repair(w.points, w.values, np.zeros((0, 3)))
    assert not removed.any()
    np.testing.assert_array_equal(out, w.values)


@pytest.fixture(scope="module")
def csg10():
    w = configs.csg(10, uniform_queries=40, near_queries=40)
    return w, R.repair(w.points, w.values, w.queries)


def test_repair_keeps_signs_and_grows(csg10):
    w, (out, removed, qv, kind, _) = csg10
    assert removed.any()
    assert np.all(np.sign(out) == np.sign(w.values))
    assert np.all(np.abs(out) >= np.abs(w.values) - 1e-12)
    assert not np.any(kind == 255)


def test_repaired_set_is_valid(csg10):
    w, (out, removed, qv, kind, _) = csg10
    P = np.vstack([w.points, w.queries])
    S = np.concatenate([out, qv])
    W, ok = G.input_witnesses(P, S)
    assert ok.all()
    assert C.certify(P, S, W)["violations"] == 0


def test_repair_is_order_independent(csg10):
    w, (out, removed, qv, kind, _) = csg10
    perm = np.random.default_rng(0).permutation(len(w.queries))
    out2, removed2, qv2, _, _ = R.repair(w.points, w.values, w.queries[perm])
    np.testing.assert_array_equal(out, out2)
    np.testing.assert_array_equal(qv[perm], qv2)


def test_certificate_detects_planted_violations():
    w = configs.sphere(4)
    W, ok = G.input_witnesses(w.points, w.values)
    assert C.certify(w.points, w.values, W)["violations"] == 0
    S = w.values.copy()
    i = int(np.argmax(S))
    S[i] += 0.2                             # too big: swallows neighbours, breaks the cone
    cert = C.certify(w.points, S, W)
    assert cert["pair_same"] > 0 and cert["witness_off_sphere"] >= 1
    W2 = W.copy()
    W2[0] = w.points[0]                     # witness moved off its sphere
    assert C.certify(w.points, w.values, W2)["witness_off_sphere"] == 1


def _forward(P, S, Q, order):
    W, ok = G.input_witnesses(P, S)
    return G.greedy_interpolate(P, S, Q, order, W)


def test_adjoint_matches_finite_differences():
    rng = np.random.default_rng(4)
    w = configs.sphere(3)
    Q = rng.uniform(0.1, 0.9, (12, 3))
    order = np.arange(len(Q))
    base = _forward(w.points, w.values, Q, order)
    gs, gp, multi = A.adjoint(w.points, w.values, Q, base.values, base.kind, base.active, order)
    single = ~np.isin(base.kind, [KIND_RMIN_D, KIND_RMIN_U])
    h = 1e-6
    checked = 0
    for i in range(w.n):
        for comp in range(4):
            Sp, Sm = w.values.copy(), w.values.copy()
            Pp, Pm = w.points.copy(), w.points.copy()
            if comp == 3:
                Sp[i] += h
                Sm[i] -= h
                an = gs[i]
            else:
                Pp[i, comp] += h
                Pm[i, comp] -= h
                an = gp[i, comp]
            rp = _forward(Pp, Sp, Q, order)
            rm = _forward(Pm, Sm, Q, order)
            same = (np.array_equal(rp.kind, base.kind) and np.array_equal(rm.kind, base.kind)
                    and np.array_equal(rp.active, base.active) and np.array_equal(rm.active, base.active))
            if not same or not single.all():
                continue
            fd = (rp.values.sum() - rm.values.sum()) / (2 * h)
            assert abs(fd - an) <= 1e-6 + 1e-5 * abs(fd), (i, comp, fd, an)
            checked += 1
    assert checked > 20


def test_adjoint_subtree_counts():
    # d(sum)/d(s_i) counts the queries whose chain of active parents reaches i
    # when every link is a cone link (derivative 1 w.r.t. the parent value)
    w = configs.sphere(3)
    Q = np.random.default_rng(6).uniform(0.1, 0.9, (20, 3))
    order = np.arange(len(Q))
    r = _forward(w.points, w.values, Q, order)
    gs, _, _ = A.adjoint(w.points, w.values, Q, r.values, r.kind, r.active, order)
    if not np.all(np.isin(r.kind, [1, 2, 7])):
        pytest.skip("fallback values present")
    counts = np.zeros(w.n)
    for j in range(len(Q)):
        t = r.active[j]
        while t >= w.n:
            t = r.active[t - w.n]
        counts[t] += 1
    np.testing.assert_allclose(gs, counts)
