"""Pins of oracle parts checked by hand-derived cases: the order of scattered
queries (Sec. 4.2 order, bucketed by input cell), the bound flags (Sec. 4.3
sign forcing and bound families), and every branch of the adjoint
(HI, LO, COINCIDENT, RMIN_T links) by central finite differences."""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import bounds as B
from oracle import greedy as G
from oracle import order as O
from oracle.common import (FLAG_HI_OPPOSITE, FLAG_INFEASIBLE, FLAG_INSIDE_NEG, FLAG_INSIDE_POS,
                           FLAG_LO_OPPOSITE, FLAG_TIE_HI, FLAG_TIE_LO, KIND_COINCIDENT, KIND_HI, KIND_LO,
                           KIND_RMIN_T, KIND_ZERO)
from sdfgen import configs

# A 2x2x2 input grid (cell centres 0.25 / 0.75).  A ball at a cell centre
# covers the sub-points (k + 0.5)/16 of its own cell whose offsets from the
# centre, (a, b, c)/32 with odd a, b, c in {1, 3, 5, 7}, satisfy
# (a^2 + b^2 + c^2)/1024 < (r - 1e-6)^2 and none of the next cell (r < 0.25):
#   r = 0.001 -> 0;  r = 0.06 (> sqrt 3/32) -> the 8 with a = b = c = 1;
#   r = 0.11 (> sqrt 11/32, < sqrt 19/32) -> those 8 and the 24 with one 3.
HAND_R = np.array([0.11, 0.001, 0.06, 0.11, 0.06, 0.001, 0.11, 0.06])
HAND_COUNTS = [32, 0, 8, 32, 8, 0, 32, 8]
# Flood fill by (count, index): start at cell 1; push 0, 3, 5; pop 5 (count 0),
# push 4, 7; pop 4 (8), push 6; pop 7 (8); pop 0 (32), push 2; pop 2 (8);
# pop 3, then 6.
HAND_CELLS = [1, 5, 4, 7, 0, 2, 3, 6]


def hand_grid():
    t = np.array([0.25, 0.75])
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1), HAND_R.copy()


def test_covered_counts_and_flood_fill_hand_grid():
    P, S = hand_grid()
    np.testing.assert_array_equal(O.covered_counts(2, P, S), HAND_COUNTS)
    np.testing.assert_array_equal(O.flood_fill(np.array(HAND_COUNTS), 2), HAND_CELLS)


def test_scattered_order_hand_grid():
    P, S = hand_grid()
    Q = np.array([[0.1, 0.1, 0.1],     # cell 0 (rank 4)
                  [0.9, 0.1, 0.1],     # cell 1 (rank 0)
                  [0.6, 0.2, 0.7],     # cell 5 (rank 1)
                  [0.3, 0.3, 0.3],     # cell 0 (rank 4)
                  [0.2, 0.8, 0.2],     # cell 2 (rank 5)
                  [0.99, 0.99, 0.99],  # cell 7 (rank 3)
                  [1.0, 0.0, 0.6]])    # on the box face x = 1: the last cell along x, cell 5 (rank 1)
    order, parent = O.scattered_order(P, S, 2, Q)
    np.testing.assert_array_equal(parent, HAND_COUNTS)
    # by cell rank, then by query index
    np.testing.assert_array_equal(order, [1, 2, 6, 5, 0, 3, 4])


def test_flags_hand_cases():
    # each flag from a configuration whose bounds are worked out by hand
    P = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    # q at 0.3 from a positive ball of radius 0.5: lo = 0.2 > tol (inside +);
    # hi = min(0.5 + 0.3, -0.1 + 0.7) = 0.6 from the negative sample
    # (opposite sign to hi): HI_OPPOSITE
    lo, hi, a, b, f = B.cone_bounds(P, np.array([0.5, -0.1]), np.array([[0.3, 0.0, 0.0]]))
    assert abs(lo[0] - 0.2) < 1e-15 and abs(hi[0] - 0.6) < 1e-15 and b[0] == 1
    assert f[0] == FLAG_INSIDE_POS | FLAG_HI_OPPOSITE
    # mirrored: inside a negative ball, lo bound by the positive sample
    lo, hi, a, b, f = B.cone_bounds(P, np.array([-0.5, 0.1]), np.array([[0.3, 0.0, 0.0]]))
    assert abs(lo[0] + 0.6) < 1e-15 and abs(hi[0] + 0.2) < 1e-15 and a[0] == 1
    assert f[0] == FLAG_INSIDE_NEG | FLAG_LO_OPPOSITE
    # intersecting opposite-sign balls: the positive ball of radius 0.6 at 0
    # and the negative one of radius 0.6 at 1 overlap; at x = 0.5:
    # lo = 0.6 - 0.5 = 0.1, hi = -0.6 + 0.5 = -0.1
    lo, hi, a, b, f = B.cone_bounds(P, np.array([0.6, -0.6]), np.array([[0.5, 0.0, 0.0]]))
    assert f[0] & FLAG_INFEASIBLE and f[0] & FLAG_INSIDE_POS and f[0] & FLAG_INSIDE_NEG
    # equidistant equal samples: both extremes tie
    lo, hi, a, b, f = B.cone_bounds(P, np.array([0.1, 0.1]), np.array([[0.5, 0.3, 0.0]]))
    assert f[0] & FLAG_TIE_LO and f[0] & FLAG_TIE_HI and a[0] == 0 and b[0] == 0
    # outside every (positive) ball: lo = 0.2 - 0.640... < 0 is set by a
    # positive sample (LO_OPPOSITE), hi = 0.1 + 0.640... > 0 by a positive one
    lo, hi, a, b, f = B.cone_bounds(P, np.array([0.1, 0.2]), np.array([[0.5, 0.4, 0.0]]))
    assert a[0] == 1 and b[0] == 0 and lo[0] < 0.0 < hi[0]
    assert f[0] == FLAG_LO_OPPOSITE
    # a point on a sample: both extremes are that sample's value, no sign clash
    lo, hi, a, b, f = B.cone_bounds(P, np.array([0.3, 0.25]), np.array([[0.0, 0.0, 0.0]]))
    assert lo[0] == hi[0] == 0.3 and a[0] == b[0] == 0
    assert f[0] == FLAG_INSIDE_POS


def adjoint_instance():
    """Nine-ball union samples (27) and 14 queries, two of them placed on
    samples: the greedy yields HI, LO, COINCIDENT, RMIN_T and an RMIN_D value,
    and the RMIN_T value's parent is an earlier query."""
    w = configs.ball_union(3, 1013)
    Q = np.random.default_rng(11).uniform(0.1, 0.9, (14, 3))
    Q[3] = w.points[5]
    Q[9] = w.points[13]
    return w.points, w.values, Q, np.arange(len(Q))


def forward(P, S, Q, order):
    W, _ = G.input_witnesses(P, S)
    return G.greedy_interpolate(P, S, Q, order, W)


def test_adjoint_branches_match_finite_differences():
    P, S, Q, order = adjoint_instance()
    n = len(S)
    base = forward(P, S, Q, order)
    single = {KIND_HI, KIND_LO, KIND_COINCIDENT, KIND_RMIN_T, KIND_ZERO}
    # weight 1 on values whose chain of parents has single-parent links only
    clean = np.zeros(len(Q), dtype=bool)
    for j in order:
        t = int(base.active[j])
        clean[j] = int(base.kind[j]) in single and (t < n or clean[t - n])
    for k in (KIND_HI, KIND_LO, KIND_COINCIDENT, KIND_RMIN_T):
        assert np.any(clean & (base.kind == k)), k
    rmin_t = int(np.nonzero(base.kind == KIND_RMIN_T)[0][0])
    assert base.active[rmin_t] >= n                       # its parent is a query
    wts = clean.astype(np.float64)
    gs, gp, _ = A.adjoint(P, S, Q, base.values, base.kind, base.active, order, wts)
    h = 1e-6
    checked = 0
    hit = set()
    for i in range(n):
        for comp in range(4):
            Sp, Sm, Pp, Pm = S.copy(), S.copy(), P.copy(), P.copy()
            if comp == 3:
                Sp[i] += h
                Sm[i] -= h
                an = gs[i]
            else:
                Pp[i, comp] += h
                Pm[i, comp] -= h
                an = gp[i, comp]
            rp, rm = forward(Pp, Sp, Q, order), forward(Pm, Sm, Q, order)
            if not (np.array_equal(rp.kind, base.kind) and np.array_equal(rm.kind, base.kind)
                    and np.array_equal(rp.active, base.active) and np.array_equal(rm.active, base.active)):
                continue
            fd = (wts @ rp.values - wts @ rm.values) / (2 * h)
            assert abs(fd - an) <= 1e-6 + 1e-5 * abs(fd), (i, comp, fd, an)
            checked += 1
            if abs(fd) > 0.1:
                # which branches carry this sample's derivative
                for j in np.nonzero(clean)[0]:
                    t = int(base.active[j])
                    while t >= n:
                        t = int(base.active[t - n])
                    if t == i:
                        hit.add(int(base.kind[j]))
    assert checked >= 80
    assert {KIND_HI, KIND_LO, KIND_COINCIDENT, KIND_RMIN_T} <= hit, hit
