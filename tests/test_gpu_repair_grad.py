"""GPU parity of the minimum valid radius, the pseudo-SDF repair and the
backward pass against the oracle (Prop. 2 proof, Corollary 1, Sec. 6)."""
import numpy as np
import pytest
import torch

from oracle import adjoint as OA
from oracle import certify as OC
from oracle import greedy as OG
from oracle import repair as OR
from oracle import rmin as OM
from oracle.common import TOL, dist
from paper_2605_01919_amd import sdfi
from sdfgen import configs

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def test_min_valid_radius_matches_oracle():
    w = configs.csg(10, uniform_queries=150, near_queries=50)
    print("rmin csg10", flush=True)
    val, kind, wit = sdfi.min_valid_radius(dev(np.c_[w.points, w.values]), dev(w.queries))
    val, kind = val.cpu().numpy(), kind.cpu().numpy()
    # the oracle computes each point on its own (Corollary 1: order-free)
    Wn, ok = OG.input_witnesses(w.points, w.values)
    R = np.abs(w.values)
    for j, q in enumerate(w.queries):
        d = dist(w.points, q)
        inside = d < R - TOL
        if not inside.any():
            assert kind[j] == 3 and val[j] == 0.0
            continue
        sig = int(np.sign(w.values[inside][np.argmax(R[inside] - d[inside])]))
        r, x, k, _ = OM.min_valid_radius(q, sig, w.points, w.values, TOL, Wn)
        assert abs(val[j] - sig * r) <= 1e-9, (j, val[j], sig * r)


def test_repair_matches_oracle():
    w = configs.csg(10, uniform_queries=60, near_queries=60)
    print("repair csg10", flush=True)
    rv, removed, qv, kind, rep = sdfi.repair(dev(np.c_[w.points, w.values]), dev(w.queries))
    out, orem, oqv, okind, _ = OR.repair(w.points, w.values, w.queries)
    np.testing.assert_array_equal(removed.cpu().numpy().astype(bool), orem)
    np.testing.assert_allclose(rv.cpu().numpy(), out, rtol=0, atol=1e-9)
    np.testing.assert_allclose(qv.cpu().numpy(), oqv, rtol=0, atol=1e-9)
    k = kind.cpu().numpy()
    assert np.array_equal(np.isin(k, [4, 5, 6]), np.isin(okind, [4, 5, 6]))
    assert rep["n_removed"] == int(orem.sum())


def test_repair_exact_sdf_is_identity():
    w = configs.sphere(8)
    rv, removed, _, kind, rep = sdfi.repair(dev(np.c_[w.points, w.values]))
    assert rep["n_removed"] == 0 and torch.equal(rv, dev(w.values))


def test_backward_matches_oracle_adjoint():
    w = configs.sphere(5)
    samples = dev(np.c_[w.points, w.values])
    g = sdfi.greedy(samples, dev(w.queries), grid=w.grid)
    vals, kind, act = g["values"], g["kind"], g["active"]
    gs, gp = sdfi.greedy_backward(torch.ones(w.m, dtype=torch.float64, device="cuda"), samples, dev(w.queries),
                                  vals, act, kind)
    ogs, ogp, _ = OA.adjoint(w.points, w.values, w.queries, vals.cpu().numpy(), kind.cpu().numpy(),
                             act.cpu().numpy(), g["order"].cpu().numpy())
    np.testing.assert_allclose(gs.cpu().numpy(), ogs, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gp.cpu().numpy(), ogp, rtol=1e-12, atol=1e-12)


def test_autograd_function_matches_finite_differences():
    # the 5^3 sphere's greedy takes only hi/lo values (single active parents)
    rng = np.random.default_rng(5002)
    w = configs.sphere(5)
    pts = dev(w.points).requires_grad_(True)
    vals = dev(w.values).requires_grad_(True)
    Q = dev(w.queries)
    out, kind, act = sdfi.GreedyInterpolate.apply(pts, vals, Q, w.grid)
    out.sum().backward()
    base_kind, base_act = kind.clone(), act.clone()
    h = 1e-6
    checked = 0
    single = not np.isin(kind.cpu().numpy(), [5, 6]).any()
    for i in rng.choice(w.n, 10, replace=False):
        for comp in range(4):
            vals_p, vals_m = w.values.copy(), w.values.copy()
            P_p, P_m = w.points.copy(), w.points.copy()
            if comp == 3:
                vals_p[i] += h
                vals_m[i] -= h
                an = vals.grad[i].item()
            else:
                P_p[i, comp] += h
                P_m[i, comp] -= h
                an = pts.grad[i, comp].item()
            fp = sdfi.greedy(dev(np.c_[P_p, vals_p]), Q, grid=w.grid)
            fm = sdfi.greedy(dev(np.c_[P_m, vals_m]), Q, grid=w.grid)
            if not (torch.equal(fp["kind"], base_kind) and torch.equal(fm["kind"], base_kind)
                    and torch.equal(fp["active"], base_act) and torch.equal(fm["active"], base_act)):
                continue
            if not single:
                continue
            fd = (fp["values"].sum().item() - fm["values"].sum().item()) / (2 * h)
            assert abs(fd - an) <= 1e-6 + 1e-5 * abs(fd), (i, comp, fd, an)
            checked += 1
    print("checked", checked, flush=True)
    assert checked >= 10
