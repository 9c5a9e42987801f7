"""Error paths and edge cases of the C ABI on the GPU: inputs that break the
entry points' contracts (NaN, outside the domain box, off the stated grid,
an order that is not a permutation), inputs that violate Prop. 1 (forced
INFEASIBLE values, the input check), and the certificate's float32 screen at
coordinates far from the unit cube."""
import numpy as np
import pytest
import torch

from oracle import bounds as OB
from oracle import certify as OC
from oracle import greedy as OG
from oracle.common import KIND_INFEASIBLE, TOL
from paper_2605_01919_amd import sdfi
from sdfgen import configs

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def status_of(fn, *a, **k):
    try:
        fn(*a, **k)
    except sdfi.SdfiError as e:
        msg = str(e)
        return int(msg.split("status ")[1].split(":")[0]), msg
    return 0, ""


def test_certify_band_follows_the_coordinates():
    # sphere4 shifted by +100 on every axis: float32 coordinates there carry
    # rounding errors of ~4e-6, above a fixed 4e-6 band; violations planted
    # 3e-7 past tol (and non-violations 3e-7 short of it) must still be
    # counted exactly as in float64
    print("certify shifted by 100", flush=True)
    w = configs.sphere(4)
    W, ok = OG.input_witnesses(w.points, w.values)
    assert ok.all()
    P = w.points + 100.0
    Wt = W + 100.0
    S = w.values.copy()
    rng = np.random.default_rng(9)
    for x in rng.choice(len(S), 6, replace=False):
        d = np.sqrt(((P - P[x]) ** 2).sum(1))
        y = int(np.argsort(d)[1])            # nearest other sample
        sign = 1.0 if rng.random() < 0.5 else -1.0
        S[y] = S[x] + sign * (d[y] + TOL + (3e-7 if rng.random() < 0.5 else -3e-7))
    # witnesses moved 3e-7 inside / outside a neighbour's shrunk ball
    for x in rng.choice(len(S), 4, replace=False):
        d = np.sqrt(((P - P[x]) ** 2).sum(1))
        y = int(np.argsort(d)[1])
        u = (Wt[x] - P[y]) / np.linalg.norm(Wt[x] - P[y])
        Wt[x] = P[y] + u * (abs(S[y]) - TOL + (-3e-7 if rng.random() < 0.5 else 3e-7))
    want = OC.certify(P, S, Wt)
    got = sdfi.certify(dev(np.c_[P, S]), dev(Wt))
    print("oracle", want, "gpu", got, flush=True)
    assert got["pair"] == want["pair_opposite"] + want["pair_same"] > 0
    # the library counts spheres whose witness fails either test, each once
    assert got["witness"] == want["spheres_without_witness"] > 0


def test_greedy_rejects_nan_inputs():
    w = configs.sphere(3)
    S = np.c_[w.points, w.values]
    S[5, 3] = np.nan
    st, msg = status_of(sdfi.greedy, dev(S), dev(w.queries), grid=w.grid)
    assert st == 1 and "NaN" in msg
    Q = w.queries.copy()
    Q[7, 1] = np.inf
    st, msg = status_of(sdfi.greedy, dev(np.c_[w.points, w.values]), dev(Q), grid=w.grid)
    assert st == 1 and "NaN" in msg
    st, msg = status_of(sdfi.repair, dev(S))
    assert st == 1
    st, msg = status_of(sdfi.min_valid_radius, dev(S), dev(w.queries))
    assert st == 1


def test_greedy_rejects_an_order_that_is_not_a_permutation():
    w = configs.sphere(3)
    s, q = dev(np.c_[w.points, w.values]), dev(w.queries)
    bad = np.arange(w.m)
    bad[4] = bad[9]                          # a repeat (and a missing entry)
    st, msg = status_of(sdfi.greedy, s, q, order=dev(bad, torch.int64))
    assert st == 1 and "permutation" in msg
    bad = np.arange(w.m)
    bad[0] = w.m                             # out of range
    st, msg = status_of(sdfi.greedy, s, q, order=dev(bad, torch.int64))
    assert st == 1 and "permutation" in msg
    # the valid permutation runs
    perm = np.random.default_rng(1).permutation(w.m)
    out = sdfi.greedy(s, q, order=dev(perm, torch.int64))
    assert torch.equal(out["order"].cpu(), torch.tensor(perm))


def test_domain_errors():
    w = configs.sphere(3)
    Q = w.queries.copy()
    Q[3] = [1.5, 0.5, 0.5]                   # a query outside [-1, 1]^3
    st, msg = status_of(sdfi.greedy, dev(np.c_[w.points, w.values]), dev(Q),
                        order=dev(np.arange(w.m), torch.int64))
    assert st == 5 and "domain" in msg
    S = np.c_[w.points, w.values]
    S[0, 0] = -1.5                           # a sample point outside the box
    st, msg = status_of(sdfi.repair, dev(S))
    assert st == 5
    st, msg = status_of(sdfi.min_valid_radius, dev(np.c_[w.points, w.values]), dev(Q))
    assert st == 5
    # spheres may reach past the box (the far corner sample's does here)
    assert np.any(w.points.max(1) + np.abs(w.values) > 1.0)
    assert status_of(sdfi.repair, dev(np.c_[w.points, w.values]))[0] == 0
    # the refinement order needs the samples on the grid's cell centres
    off = w.points.copy()
    off[4, 1] += 0.2                          # moved into the next cell
    st, msg = status_of(sdfi.refinement_order, dev(np.c_[off, w.values]), w.grid)
    assert st == 5 and "cells" in msg
    st, msg = status_of(sdfi.greedy, dev(np.c_[off, w.values]), dev(w.queries), grid=w.grid)
    assert st == 5
    Qs = w.queries[::-1].copy()               # refinement queries out of their cells
    st, msg = status_of(sdfi.greedy, dev(np.c_[w.points, w.values]), dev(Qs), grid=w.grid)
    assert st == 5


def opposite_pair():
    # a positive ball of radius 0.3 at x = 0.3 and a negative one of radius 0.3
    # at x = 0.7 intersect (0.4 < 0.6): between them lo = 0.1 > hi = -0.1
    P = np.array([[0.3, 0.5, 0.5], [0.7, 0.5, 0.5], [0.5, 0.9, 0.9]])
    S = np.array([0.3, -0.3, 0.05])
    Q = np.array([[0.5, 0.5, 0.5], [0.5, 0.2, 0.9]])
    return P, S, Q


def test_infeasible_queries_and_the_input_check():
    P, S, Q = opposite_pair()
    order = dev(np.arange(len(Q)), torch.int64)
    out = sdfi.greedy(dev(np.c_[P, S]), dev(Q), order=order)
    kind = out["kind"].cpu().numpy()
    vals = out["values"].cpu().numpy()
    W, _ = OG.input_witnesses(P, S)
    r = OG.greedy_interpolate(P, S, Q, np.arange(len(Q)), W)
    assert kind[0] == KIND_INFEASIBLE == r.kind[0] and np.isnan(vals[0]) and np.isnan(r.values[0])
    assert kind[1] == r.kind[1] and abs(vals[1] - r.values[1]) <= 1e-9
    assert out["report"]["n_infeasible"] == 1
    st, msg = status_of(sdfi.greedy, dev(np.c_[P, S]), dev(Q), order=order, input_check=True)
    assert st == 4 and "cone" in msg
    # a fully covered input sphere fails the other half of the check
    P2 = np.array([[0.2, 0.2, 0.2], [0.22, 0.2, 0.2], [0.6, 0.6, 0.6]])
    S2 = np.array([0.15, 0.05, 0.1])
    st, msg = status_of(sdfi.greedy, dev(np.c_[P2, S2]), dev(Q[:1]), order=order[:1], input_check=True)
    assert st == 4 and "uncovered" in msg
    # a valid input passes the check and gives the same values as without it
    w = configs.sphere(3)
    a = sdfi.greedy(dev(np.c_[w.points, w.values]), dev(w.queries), grid=w.grid, input_check=True)
    b = sdfi.greedy(dev(np.c_[w.points, w.values]), dev(w.queries), grid=w.grid)
    assert torch.equal(a["values"], b["values"])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_bounds_with_nan_inputs(precision):
    w = configs.ball_union(6, 1002)
    S = np.c_[w.points, w.values]
    S[17, 3] = np.nan                        # this sample takes part in no extreme
    S[40, 0] = np.nan
    Q = w.queries[:3000].copy()
    Q[5, 2] = np.nan                         # this query gets (-inf, +inf, -1, -1)
    lo, hi, a, b, f = [t.cpu().numpy() for t in sdfi.bounds(dev(S), dev(Q), precision)]
    assert lo[5] == -np.inf and hi[5] == np.inf and a[5] == -1 and b[5] == -1
    keep = np.ones(w.n, dtype=bool)
    keep[[17, 40]] = False
    idx = np.nonzero(keep)[0]
    ok = np.arange(len(Q)) != 5
    olo, ohi, oa, ob, of = OB.cone_bounds(w.points[keep], w.values[keep], Q[ok])
    np.testing.assert_allclose(lo[ok], olo, rtol=0, atol=1e-12)
    np.testing.assert_allclose(hi[ok], ohi, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(a[ok], idx[oa])
    np.testing.assert_array_equal(b[ok], idx[ob])
