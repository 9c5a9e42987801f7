"""Replay of a greedy run's decisions with the oracle (CPU only).

    python tests/replay_oracle.py IN.npz OUT.npz [processes]

IN holds a finished run (see save_greedy_run.py): samples P (n, 3), S (n,),
queries Q (m, 3), the acceptance order, values, kinds and active ids, the
final witnesses of the
samples (n, 3) and of the queries (m, 3), and `steps`, the positions k in the
order to replay.  Step k is decided again by the oracle's greedy step against
the constraint set the run had built before it: the samples plus the queries
accepted at positions < k with the run's values.  A witness that is uncovered
in the final set is uncovered in every earlier set (fewer balls), so the
final witnesses serve every step; those the step can consult (within the
largest candidate radius of the query) are checked first against that set,
and a failed check is reported.  OUT gets, per replayed step, the oracle's
value, kind and active id (sample i, or n + j for query j) and the number of
bad witnesses.  When IN holds the run's active ids, the decisions are also
compared with the run's (exit status 1 on any difference).

Runs in a process of its own, started by the GPU tests, so that its worker
processes never share a process with GPU state.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import greedy as OG  # noqa: E402
from oracle.bounds import bounds_one  # noqa: E402
from oracle.common import KIND_INFEASIBLE, KIND_UNRESOLVED, TOL, dist  # noqa: E402

_D = {}


def _prefix(k):
    """Constraint rows before step k: samples, then accepted queries in order."""
    d = _D
    acc = d["acc_upto"][k]
    qs = d["accepted"][:acc]
    P = np.vstack([d["P"], d["Q"][qs]])
    S = np.concatenate([d["S"], d["values"][qs]])
    W = np.vstack([d["SW"], d["QW"][qs]])
    return P, S, W, qs


def _bad_witnesses(q, radius, P, S, W):
    """Witnesses within `radius` of q that are off their sphere or covered."""
    near = np.nonzero(dist(W, q) < radius)[0]
    bad = 0
    R = np.abs(S)
    for c in near:
        if not abs(float(dist(W[c], P[c])) - R[c]) <= TOL:
            bad += 1
            continue
        cov = dist(P, W[c]) < R - TOL - 1e-9
        cov[c] = False
        bad += int(cov.any())
    return bad


def _one(k):
    d = _D
    j = int(d["order"][k])
    q = d["Q"][j]
    P, S, W, qs = _prefix(k)
    lo, hi, _, _, _ = bounds_one(q, P, S)
    radius = max(abs(lo), abs(hi)) + TOL if np.isfinite(lo) and np.isfinite(hi) else np.inf
    bad = _bad_witnesses(q, radius, P, S, W)
    v, kind, t, _, _ = OG.greedy_step(q, P, S, W)
    n = len(d["S"])
    act = -1 if t < 0 else (t if t < n else n + int(qs[t - n]))
    return k, float(v), int(kind), int(act), bad


def main():
    inp, out = sys.argv[1], sys.argv[2]
    procs = int(sys.argv[3]) if len(sys.argv) > 3 else 8
    z = np.load(inp)
    for key in ("P", "S", "Q", "order", "values", "kind", "SW", "QW", "steps"):
        _D[key] = z[key]
    ok = ~np.isin(_D["kind"][_D["order"]], [KIND_INFEASIBLE, KIND_UNRESOLVED])
    _D["accepted"] = _D["order"][ok]
    _D["acc_upto"] = np.concatenate([[0], np.cumsum(ok)])
    # a seeded shuffle spreads the costly late steps over the workers
    steps = [int(k) for k in np.asarray(_D["steps"])[np.random.default_rng(5).permutation(len(_D["steps"]))]]
    res = []
    with mp.get_context("fork").Pool(procs) as pool:
        for i, r in enumerate(pool.imap_unordered(_one, steps, chunksize=1)):
            res.append(r)
            if (i + 1) % 10 == 0:
                print(f"replayed {i + 1}/{len(steps)}", flush=True)
    res.sort()
    arr = np.array(res, dtype=np.float64).reshape(-1, 5)
    r = {"steps": arr[:, 0].astype(np.int64), "values": arr[:, 1], "kind": arr[:, 2].astype(np.int64),
         "active": arr[:, 3].astype(np.int64), "bad": arr[:, 4].astype(np.int64)}
    np.savez(out, **r)
    if "active" in z.files:
        sys.exit(0 if report(z, r) else 1)


def report(z, r):
    """Compares the replayed decisions with the run's and prints a summary:
    kinds equal (a circle's nearest point and an arc end count as one
    class), values within 1e-5, the same parent for single-parent kinds, no
    failed witness check."""
    j = z["order"][r["steps"]]
    kg = z["kind"][j].astype(np.int64)
    kg = np.where(kg == 6, 5, kg)
    ko = np.where(r["kind"] == 6, 5, r["kind"])
    vals = z["values"][j]
    nan2 = np.isnan(vals) & np.isnan(r["values"])
    diff = np.where(nan2, 0.0, np.abs(vals - r["values"]))
    single = np.isin(ko, [1, 2, 7])
    act_ok = np.array_equal(z["active"][j][single], r["active"][single])
    kinds = {int(k): int(c) for k, c in zip(*np.unique(r["kind"], return_counts=True))}
    ok = bool(np.array_equal(kg, ko) and np.all(diff <= 1e-5) and act_ok and np.all(r["bad"] == 0))
    print(f"replayed {len(j)} steps (first {int(r['steps'].min())}, last {int(r['steps'].max())}); oracle kinds "
          f"{kinds}; kinds equal {bool(np.array_equal(kg, ko))}; max |value difference| {float(np.nanmax(diff)):.3e}; "
          f"parents equal {act_ok}; failed witness checks {int(r['bad'].sum())}; match {ok}", flush=True)
    return ok


if __name__ == "__main__":
    main()
