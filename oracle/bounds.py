"""Pairwise consistency bounds of a query (Sec. 4.3, "Further performance improvements").

For a new point q and existing samples (p_c, s_c) with d_c = |q - p_c|, the
paper bounds the admissible value before any candidate is examined: a value
must not intersect an opposite-sign sphere and must not fully contain, or be
fully contained by, any one same-sign sphere.  In signed form both families
reduce to the 1-Lipschitz cone |s - s_c| <= d_c:
  opposite signs:  |s| + |s_c| <= d_c  <=>  |s - s_c| <= d_c
  same sign:       ||s| - |s_c|| <= d_c <=>  |s - s_c| <= d_c
so every admissible value lies in [lo, hi] with
  lo = max_c (s_c - d_c),   hi = min_c (s_c + d_c).
The argmax / argmin is the smallest constraint index within TIE_TOL of the
extreme (Appendix B's uniqueness tolerance used as the tie band).
"""
from __future__ import annotations

import numpy as np

from .common import (FLAG_HI_OPPOSITE, FLAG_INFEASIBLE, FLAG_INSIDE_NEG, FLAG_INSIDE_POS,
                     FLAG_LO_OPPOSITE, FLAG_TIE_HI, FLAG_TIE_LO, TIE_TOL, TOL, dist, sign_class)


def flags_of(lo, hi, lo_vals_tied, hi_vals_tied, s_a, s_b):
    f = np.zeros(np.shape(lo), dtype=np.uint32)
    f |= np.where(lo > hi + TOL, FLAG_INFEASIBLE, 0).astype(np.uint32)
    f |= np.where(lo > TOL, FLAG_INSIDE_POS, 0).astype(np.uint32)
    f |= np.where(hi < -TOL, FLAG_INSIDE_NEG, 0).astype(np.uint32)
    f |= np.where(lo_vals_tied, FLAG_TIE_LO, 0).astype(np.uint32)
    f |= np.where(hi_vals_tied, FLAG_TIE_HI, 0).astype(np.uint32)
    f |= np.where(sign_class(hi) * sign_class(s_b) < 0, FLAG_HI_OPPOSITE, 0).astype(np.uint32)
    f |= np.where(sign_class(lo) * sign_class(s_a) < 0, FLAG_LO_OPPOSITE, 0).astype(np.uint32)
    return f


def cone_bounds(P, S, Q, chunk: int = 256):
    """lo, hi, argmax, argmin, flags of every query against all samples."""
    P = np.asarray(P, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    m = len(Q)
    lo = np.empty(m)
    hi = np.empty(m)
    am = np.empty(m, dtype=np.int64)
    bm = np.empty(m, dtype=np.int64)
    tlo = np.empty(m, dtype=bool)
    thi = np.empty(m, dtype=bool)
    for s0 in range(0, m, chunk):
        d = dist(Q[s0:s0 + chunk, None, :], P[None, :, :])
        lower = S[None, :] - d
        upper = S[None, :] + d
        l = lower.max(1)
        h = upper.min(1)
        inl = lower >= (l - TIE_TOL)[:, None]
        inh = upper <= (h + TIE_TOL)[:, None]
        lo[s0:s0 + chunk] = l
        hi[s0:s0 + chunk] = h
        am[s0:s0 + chunk] = inl.argmax(1)
        bm[s0:s0 + chunk] = inh.argmax(1)
        tlo[s0:s0 + chunk] = inl.sum(1) > 1
        thi[s0:s0 + chunk] = inh.sum(1) > 1
    flags = flags_of(lo, hi, tlo, thi, S[am], S[bm])
    return lo, hi, am, bm, flags


def bounds_one(q, P, S):
    """Bounds of a single query; the same definition, one row."""
    d = dist(P, q)
    lower = S - d
    upper = S + d
    l = lower.max()
    h = upper.min()
    a = int(np.argmax(lower >= l - TIE_TOL))
    b = int(np.argmax(upper <= h + TIE_TOL))
    return float(l), float(h), a, b, d
