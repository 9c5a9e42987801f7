"""Greedy sequential interpolation (Sec. 3.3 "interpolate_sdf_to", Sec. 4).

Queries are assigned one at a time in the refinement order; each value must
keep the set {inputs} + {values accepted so far} valid in the sense of
Prop. 1:
  (i)  no two spheres of different sign intersect (touching allowed);
  (ii) every sphere keeps a point that lies in no other open ball.

Candidate set (reading "Level P").  The paper scores every grow-to point of
Def. 1 and returns the best-scoring valid one.  The tangency candidates whose
normals agree with the tangent sphere carry the highest type score; solving
the agreement condition gives exactly the cone values s_c - d_c and s_c + d_c,
and among those only lo (tangent to the argmax) and hi (tangent to the
argmin) pass the pairwise bounds of Sec. 4.3.  So the two candidates are hi
and lo, ranked by the paper's score: sign_score * |s| with sign_score 1 for
s > 0 and 2 otherwise (the type score is common to both and cancels).  Equal
scores (within the uniqueness tolerance) go to the negative value, then hi.
If neither is valid the paper's fallback applies (Sec. 4.3 last paragraph):
the minimum valid radius, which is 0 when q lies in no ball.

Validity of a candidate (s, tangent constraint t, tangent point w), exactly
Prop. 1 on the augmented set:
  - w lies in the domain [-1,1]^3 (Appendix B);
  - (i) and the pairwise half of (ii) hold because lo <= s <= hi;
  - the new sphere has an uncovered point: w itself if no ball covers it,
    otherwise an exact search over the new sphere's cap rims (Sec. 4.3:
    the growing sphere is valid if it hits an uncovered point, otherwise new
    uncovered intersection points are looked for);
  - every existing sphere keeps an uncovered point: each sphere caches one
    uncovered point (its witness); only spheres whose witness falls inside the
    new open ball can lose all of them, and for those an exact search on the
    sphere with the new ball added decides (Sec. 4.3: an existing sphere whose
    uncovered points lie outside the growing sphere stays valid).
The exact searches make decisions independent of which witness is cached.
"""
from __future__ import annotations

import math

import numpy as np

from . import fastgeom
from . import geom
from .bounds import bounds_one
from .common import (DOMAIN_HI, DOMAIN_LO, KIND_COINCIDENT, KIND_HI, KIND_INFEASIBLE, KIND_LO,
                     KIND_RMIN_D, KIND_RMIN_T, KIND_RMIN_U, KIND_UNRESOLVED, KIND_ZERO, TIE_TOL, TOL,
                     dist, sign_class)
from .geom import point_covered, uncovered_point
from .rmin import min_valid_radius

RMIN_KIND = {"T": KIND_RMIN_T, "D": KIND_RMIN_D, "U": KIND_RMIN_U}


def input_witnesses(P, S, tol=TOL):
    """One uncovered point per input sphere, or NaN when it is fully covered.

    The search is exact; the hint (the point of the sphere facing the sample
    e minimising sign(s_i) s_e + d_ie, i.e. the neighbour lying towards the
    surface) only orders it.
    """
    P = np.asarray(P, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    n = len(S)
    W = np.full((n, 3), np.nan)
    ok = np.zeros(n, dtype=bool)
    sig = sign_class(S)
    for i in range(n):
        d = dist(P, P[i])
        key = (sig[i] if sig[i] != 0 else 1) * S + d
        key[i] = np.inf
        e = int(np.argmin(key))
        hint = P[e] if d[e] > 0 else None
        x = uncovered_point(P[i], abs(S[i]), P, S, tol, hint)
        if x is not None:
            W[i] = x
            ok[i] = True
    return W, ok


def _in_domain(w):
    return bool(np.all(w >= DOMAIN_LO - TOL) and np.all(w <= DOMAIN_HI + TOL))


def candidates(q, lo, hi, a, b, d, P, S):
    """hi and lo with their tangent constraints and tangent points, best first."""
    out = []
    for s, t, kind in ((hi, b, KIND_HI), (lo, a, KIND_LO)):
        u = (q - P[t]) / d[t]
        w = P[t] - S[t] * u if kind == KIND_HI else P[t] + S[t] * u
        score = (1.0 if s > 0.0 else 2.0) * abs(s)
        out.append((score, s, t, kind, w))
    h, l = out
    if abs(h[0] - l[0]) <= TIE_TOL:
        # tie: negative value first, then hi
        if l[1] < 0.0 <= h[1]:
            return [l, h]
        return [h, l]
    return [h, l] if h[0] > l[0] else [l, h]


def candidate_valid(q, s, w, P, S, W, tol=TOL):
    """Prop. 1 on (P, S) + (q, s).  Returns (ok, new witness, {c: new W_c})."""
    if not _in_domain(w):
        return False, None, None
    r = abs(s)
    if point_covered(w, P, S, tol):
        nw = uncovered_point(q, r, P, S, tol, hint=w)
        if nw is None:
            return False, None, None
    else:
        nw = np.array(w, dtype=np.float64)
    updates = {}
    rn = r - tol
    if rn > 0.0:
        threatened = np.nonzero(dist(W, q) < rn)[0]
        if len(threatened):
            Pn = np.vstack([P, q[None, :]])
            Sn = np.append(S, s)
            for c in threatened:
                x = uncovered_point(P[c], abs(S[c]), Pn, Sn, tol, hint=W[c])
                if x is None:
                    return False, None, None
                updates[int(c)] = x
    return True, nw, updates


def greedy_step(q, P, S, W, tol=TOL):
    """Value of one query against the current constraint set.

    Returns (value, kind, active constraint, witness, witness updates).
    """
    q = np.asarray(q, dtype=np.float64)
    if geom.USE_C:
        lo, hi, a, b = fastgeom.bounds_one(q, P, S, TIE_TOL)
        d = {a: float(dist(P[a], q)), b: float(dist(P[b], q))}
    else:
        lo, hi, a, b, d = bounds_one(q, P, S)
    if lo > hi + tol:
        return math.nan, KIND_INFEASIBLE, -1, q.copy(), {}
    for c in (a, b):
        if d[c] <= TIE_TOL:
            return float(S[c]), KIND_COINCIDENT, int(c), W[c].copy(), {}
    for _, s, t, kind, w in candidates(q, lo, hi, a, b, d, P, S):
        ok, nw, upd = candidate_valid(q, s, w, P, S, W, tol)
        if ok:
            return float(s), kind, int(t), nw, upd
    if lo <= tol and hi >= -tol:
        return 0.0, KIND_ZERO, -1, q.copy(), {}
    sigma = 1 if lo > tol else -1
    r, x, k, i = min_valid_radius(q, sigma, P, S, tol, W)
    if not math.isfinite(r):
        return math.nan, KIND_UNRESOLVED, -1, q.copy(), {}
    # Corollary 1: the minimal sphere covers no contour point.  A cached witness
    # is only uncovered w.r.t. the tolerance-shrunk balls and may sit just
    # inside the union, so witnesses inside the new ball are searched again.
    return sigma * r, RMIN_KIND[k], int(i), x, refresh_witnesses(q, sigma * r, P, S, W, tol)


def refresh_witnesses(q, s, P, S, W, tol=TOL):
    """New uncovered points for the spheres whose witness lies in the new ball."""
    updates = {}
    rn = abs(s) - tol
    if rn <= 0.0:
        return updates
    threatened = np.nonzero(dist(W, q) < rn)[0]
    if len(threatened):
        Pn = np.vstack([P, q[None, :]])
        Sn = np.append(S, s)
        for c in threatened:
            x = uncovered_point(P[c], abs(S[c]), Pn, Sn, tol, hint=W[c])
            if x is not None:
                updates[int(c)] = x
    return updates


class GreedyResult:
    def __init__(self, m):
        self.values = np.full(m, np.nan)
        self.kind = np.zeros(m, dtype=np.uint8)
        self.active = np.full(m, -1, dtype=np.int64)
        self.witness = np.full((m, 3), np.nan)
        self.order = None
        self.sample_witness = None


def greedy_interpolate(P, S, Q, order, W_in=None, tol=TOL, progress=None, stop=None):
    """Assign values to queries Q in ``order``.

    ``active`` holds the constraint each value is tangent to: ids below n are
    input samples, id n + j is query j.
    """
    P = np.asarray(P, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    n, m = len(S), len(Q)
    if W_in is None:
        W_in, _ = input_witnesses(P, S, tol)
    cap = n + m
    CP = np.empty((cap, 3))
    CS = np.empty(cap)
    CW = np.empty((cap, 3))
    CP[:n], CS[:n], CW[:n] = P, S, W_in
    N = n
    src = np.full(cap, -1, dtype=np.int64)   # query index held at each list position
    res = GreedyResult(m)
    res.order = np.asarray(order, dtype=np.int64)
    for k, j in enumerate(res.order):
        if stop is not None and k >= stop:
            break
        v, kind, t, w, upd = greedy_step(Q[j], CP[:N], CS[:N], CW[:N], tol)
        res.values[j], res.kind[j], res.witness[j] = v, kind, w
        res.active[j] = t if t < n else n + src[t]
        if kind in (KIND_INFEASIBLE, KIND_UNRESOLVED):
            continue
        for c, x in upd.items():
            CW[c] = x
        CP[N], CS[N], CW[N] = Q[j], v, w
        src[N] = j
        N += 1
        if progress is not None and k % progress == 0:
            print(f"  greedy {k}/{m}", flush=True)
    res.sample_witness = CW[:n].copy()
    # witnesses of query spheres as last updated
    for pos in range(n, N):
        res.witness[src[pos]] = CW[pos]
    return res
