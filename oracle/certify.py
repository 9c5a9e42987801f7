"""Certificate of Prop. 1 for a final set of samples.

(i)  every pair satisfies the cone |s_x - s_y| <= d_xy + TOL; for opposite
     signs this is "no intersection" and for equal signs "neither sphere lies
     strictly inside the other ball";
(ii) every sphere's witness lies on it (within TOL) and in no other ball,
     which shows it has an uncovered point.
Together they prove Prop. 1 for the set, up to the tolerance.  Counts are
kept per family.
"""
from __future__ import annotations

import numpy as np

from .common import TOL, dist, sign_class

# rounding allowance when re-testing a witness placed on a cap rim
WITNESS_SLACK = 1e-9


def certify(P, S, W, tol=TOL, chunk=1024):
    P = np.asarray(P, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    N = len(S)
    sig = sign_class(S)
    R = np.abs(S)
    out = {"pair_opposite": 0, "pair_same": 0, "witness_off_sphere": 0, "witness_covered": 0,
           "witness_missing": int(np.isnan(W).any(1).sum()), "pairs_checked": 0,
           "spheres_without_witness": 0}
    for s0 in range(0, N, chunk):
        rows = slice(s0, min(N, s0 + chunk))
        d = dist(P[rows, None, :], P[None, :, :])
        bad = np.abs(S[rows, None] - S[None, :]) > d + tol
        # each unordered pair once
        ii = np.arange(s0, rows.stop)[:, None]
        jj = np.arange(N)[None, :]
        bad &= jj > ii
        opp = (sig[rows, None] * sig[None, :]) < 0
        out["pair_opposite"] += int((bad & opp).sum())
        out["pair_same"] += int((bad & ~opp).sum())
        out["pairs_checked"] += int((jj > ii).sum())
        # witnesses
        dw = dist(W[rows, None, :], P[None, :, :])
        cov = dw < (R[None, :] - tol - WITNESS_SLACK)
        cov[np.arange(rows.stop - s0), np.arange(s0, rows.stop)] = False
        out["witness_covered"] += int(cov.any(1).sum())
        off = np.abs(dist(W[rows], P[rows]) - R[rows]) > tol
        out["witness_off_sphere"] += int(off.sum())
        # spheres whose witness fails either way (or is missing), each once
        out["spheres_without_witness"] += int((cov.any(1) | ~(np.abs(dist(W[rows], P[rows]) - R[rows]) <= tol)).sum())
    out["violations"] = (out["pair_opposite"] + out["pair_same"] + out["witness_off_sphere"]
                         + out["witness_covered"] + out["witness_missing"])
    return out
