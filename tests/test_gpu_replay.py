"""Replay parity of full-size greedy runs: the GPU's decisions at seeded
steps re-decided by the oracle from the GPU's own earlier values (the
sequential definition of Sec. 3.3 / Sec. 4 step by step), the order of
scattered queries, the backward pass on minimum-valid-radius parents, and
the rarely taken search paths, proven taken by device counters."""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest
import torch

from oracle import adjoint as OA
from oracle import greedy as OG
from oracle import order as OO
from oracle.common import KIND_COINCIDENT, KIND_HI, KIND_LO, KIND_RMIN_T, KIND_ZERO
from paper_2605_01919_amd import sdfi
from sdfgen import configs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
REPLAY = os.path.join(HERE, "replay_oracle.py")


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def replay(P, S, Q, g, steps, procs=14, timeout=1500):
    """Oracle decisions of the given steps of run g (see replay_oracle.py),
    computed in a CPU-only child process."""
    with tempfile.TemporaryDirectory() as td:
        inp, out = os.path.join(td, "in.npz"), os.path.join(td, "out.npz")
        np.savez(inp, P=P, S=S, Q=Q, order=g["order"].cpu().numpy(), values=g["values"].cpu().numpy(),
                 kind=g["kind"].cpu().numpy(), SW=g["sample_witness"].cpu().numpy(),
                 QW=g["witness"].cpu().numpy(), steps=np.asarray(steps, dtype=np.int64))
        subprocess.run([sys.executable, "-u", REPLAY, inp, out, str(procs)], check=True, timeout=timeout)
        z = np.load(out)
        return {k: z[k] for k in z.files}


def assert_replay_matches(g, r, n):
    order = g["order"].cpu().numpy()
    vals = g["values"].cpu().numpy()
    kind = g["kind"].cpu().numpy().astype(np.int64)
    act = g["active"].cpu().numpy()
    j = order[r["steps"]]
    assert np.all(r["bad"] == 0), "a final witness failed the oracle's check"
    # a contact point that is both a circle's nearest point and an arc end
    # carries either label: D and U compare as one class
    kg = np.where(kind[j] == 6, 5, kind[j])
    ko = np.where(r["kind"] == 6, 5, r["kind"])
    mism = np.nonzero(kg != ko)[0]
    assert len(mism) == 0, [(int(r["steps"][i]), int(kind[j[i]]), float(vals[j[i]]), int(r["kind"][i]),
                             float(r["values"][i])) for i in mism[:5]]
    both_nan = np.isnan(vals[j]) & np.isnan(r["values"])
    diff = np.where(both_nan, 0.0, np.abs(vals[j] - r["values"]))
    assert np.all(diff <= 1e-5), float(np.nanmax(diff))
    single = np.isin(ko, [KIND_HI, KIND_LO, KIND_COINCIDENT])
    np.testing.assert_array_equal(act[j][single], r["active"][single])
    return diff


def test_scattered_order_matches_oracle():
    w = configs.ball_union(16, 1002)
    Q = np.random.default_rng(7).uniform(0.0, 1.0, (5000, 3))
    Q[:3] = [[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.5, 0.5, 0.5]]   # box corners and a cell face
    got = sdfi.refinement_order(dev(np.c_[w.points, w.values]), w.grid, dev(Q)).cpu().numpy()
    want, _ = OO.scattered_order(w.points, w.values, w.grid, Q)
    np.testing.assert_array_equal(got, want)


def test_replay_sphere16_full_run():
    """The whole sphere16 workload (4096 samples, 32768 queries) on the GPU;
    150 seeded steps re-decided by the oracle (its deep minimum-radius steps
    take up to minutes each on one core)."""
    w = configs.sphere(16)
    print("greedy sphere16 full", flush=True)
    g = sdfi.greedy(dev(np.c_[w.points, w.values]), dev(w.queries), grid=w.grid, certify=True, sample_witness=True)
    rep = g["report"]
    assert rep["n_violations_pairwise"] == 0 and rep["n_violations_witness"] == 0, rep
    assert rep["n_unresolved"] == 0 and rep["n_search_capped"] == 0, rep
    steps = np.sort(np.random.default_rng(2016).choice(w.m, 150, replace=False))
    print("replaying 150 steps on the CPU", flush=True)
    r = replay(w.points, w.values, w.queries, g, steps)
    diff = assert_replay_matches(g, r, w.n)
    kinds = np.unique(r["kind"], return_counts=True)
    print("replayed kinds", dict(zip(kinds[0].tolist(), kinds[1].tolist())), "max |dv|", float(diff.max()), flush=True)
    assert len(kinds[0]) >= 3


def test_replay_balls16_subset():
    """The eight-ball recipe (seed 1002) with scattered queries, at a size the
    oracle can follow step by step: the 16^3 samples with a seeded 1024-query
    subset (seed 2002) of the 32^3 refinement queries, in their bucketed
    order; 64 seeded steps replayed."""
    w = configs.ball_union(16, 1002)
    idx = np.sort(np.random.default_rng(2002).choice(w.m, 1024, replace=False))
    Q = w.queries[idx]
    s = dev(np.c_[w.points, w.values])
    order = sdfi.refinement_order(s, w.grid, dev(Q))
    want, _ = OO.scattered_order(w.points, w.values, w.grid, Q)
    np.testing.assert_array_equal(order.cpu().numpy(), want)
    print("greedy balls16 samples + 1024 scattered queries", flush=True)
    g = sdfi.greedy(s, dev(Q), order=order, certify=True, sample_witness=True)
    rep = g["report"]
    assert rep["n_violations_pairwise"] == 0 and rep["n_violations_witness"] == 0, rep
    assert rep["n_unresolved"] == 0 and rep["n_search_capped"] == 0, rep
    steps = np.sort(np.random.default_rng(2003).choice(len(Q), 64, replace=False))
    print("replaying 64 steps on the CPU", flush=True)
    r = replay(w.points, w.values, Q, g, steps)
    assert_replay_matches(g, r, w.n)


def test_backward_with_minimum_radius_parents():
    """HI, LO, COINCIDENT and RMIN_T links (the RMIN_T parent an earlier
    query): the GPU forward equals the oracle's, and the GPU adjoint equals
    the oracle adjoint with weights on the values whose parent chains hold
    single-parent links only."""
    w = configs.ball_union(3, 1013)
    Q = np.random.default_rng(11).uniform(0.1, 0.9, (14, 3))
    Q[3] = w.points[5]
    Q[9] = w.points[13]
    order = np.arange(len(Q))
    s, q = dev(np.c_[w.points, w.values]), dev(Q)
    g = sdfi.greedy(s, q, order=dev(order, torch.int64))
    W, _ = OG.input_witnesses(w.points, w.values)
    r = OG.greedy_interpolate(w.points, w.values, Q, order, W)
    kind = g["kind"].cpu().numpy()
    act = g["active"].cpu().numpy()
    vals = g["values"].cpu().numpy()
    np.testing.assert_array_equal(np.where(kind == 6, 5, kind), np.where(r.kind == 6, 5, r.kind))
    np.testing.assert_allclose(vals, r.values, rtol=0, atol=1e-9)
    assert np.any(kind == KIND_RMIN_T) and np.any(kind == KIND_COINCIDENT)
    single = {KIND_HI, KIND_LO, KIND_COINCIDENT, KIND_RMIN_T, KIND_ZERO}
    n = w.n
    clean = np.zeros(len(Q), dtype=bool)
    for j in order:
        t = int(r.active[j])
        clean[j] = int(r.kind[j]) in single and (t < n or clean[t - n])
    np.testing.assert_array_equal(act[clean], r.active[clean])
    wts = clean.astype(np.float64)
    gs, gp = sdfi.greedy_backward(dev(wts), s, q, g["values"], g["active"], g["kind"])
    ogs, ogp, _ = OA.adjoint(w.points, w.values, Q, vals, kind, act, order, wts)
    np.testing.assert_allclose(gs.cpu().numpy(), ogs, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gp.cpu().numpy(), ogp, rtol=1e-12, atol=1e-12)
    # an RMIN_T link carries a nonzero derivative
    t = int(act[np.nonzero(kind == KIND_RMIN_T)[0][0]])
    while t >= n:
        t = int(act[t - n])
    assert abs(gs.cpu().numpy()[t]) > 0.1


def test_rare_search_paths_match_oracle():
    """A 5^3 box instance whose minimum-radius searches take the second,
    wider pass, run once as is and once with every refined search forced onto
    the exhaustive rim walk (the searches' last resort): device counters show
    both paths, and every one of the 1000 steps of each run is replayed."""
    x = configs.batch_instance(4, grids=(5,))
    s, q = dev(np.c_[x.points, x.values]), dev(x.queries)
    runs = {}
    for exhaustive in (False, True):
        sdfi.timing(True)
        g = sdfi.greedy(s, q, grid=x.grid, certify=True, sample_witness=True, exhaustive=exhaustive)
        walks = sdfi.counter_read("ln_fallback")
        passes, calls = sdfi.counter_read("rmin_passes"), sdfi.counter_read("rmin_calls")
        sdfi.timing(False)
        print("exhaustive", exhaustive, "walks", walks, "second passes", passes - calls, flush=True)
        assert passes > calls
        assert (walks > 0) == exhaustive
        rep = g["report"]
        assert rep["n_violations_pairwise"] == 0 and rep["n_violations_witness"] == 0, rep
        runs[exhaustive] = g
    # the profile changes nothing
    g2 = sdfi.greedy(s, q, grid=x.grid)
    assert torch.equal(torch.nan_to_num(runs[False]["values"], nan=7.0), torch.nan_to_num(g2["values"], nan=7.0))
    # both search paths give the same kinds and values up to rounding
    a, b = runs[False], runs[True]
    assert torch.equal(a["kind"], b["kind"]) and torch.equal(a["order"], b["order"])
    assert torch.allclose(a["values"], b["values"], rtol=0, atol=1e-9, equal_nan=True)
    for g in (a, b):
        r = replay(x.points, x.values, x.queries, g, np.arange(x.m))
        assert_replay_matches(g, r, x.n)
