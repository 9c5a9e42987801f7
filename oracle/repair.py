"""Pseudo-SDF repair (Sec. 6, "Application: pseudo-SDF repair").

1. Find every fully covered sphere: a sphere with no point outside all other
   open balls (Prop. 1 (ii) violated).  Reading: coverage is judged against
   all input samples and the whole set F is removed at once.
2. The remaining samples form the base set.
3. Each removed point gets the minimum valid radius against the base set,
   with its original sign (the paper keeps the zero level set; pseudo-SDFs
   underestimate distance, so only radii above the original are expected).
   A removed point that lies in no base ball of its sign keeps its value and
   is reported unresolved.
4. Extension queries get the minimum valid radius with the sign forced by
   containment (Sec. 4.3), or 0 outside every ball.
Corollary 1 makes all of these values jointly valid and independent of the
order in which they are computed.
"""
from __future__ import annotations

import numpy as np

from .common import (KIND_RMIN_D, KIND_RMIN_T, KIND_RMIN_U, KIND_UNRESOLVED, KIND_ZERO, TOL, dist,
                     sign_class)
from .geom import uncovered_point
from .rmin import min_valid_radius

KIND_KEPT = 0
RMIN_KIND = {"T": KIND_RMIN_T, "D": KIND_RMIN_D, "U": KIND_RMIN_U, "Z": KIND_ZERO}


def fully_covered(P, S, tol=TOL, which=None):
    """Boolean mask of spheres that have no uncovered point (with witnesses)."""
    P = np.asarray(P, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    idx = np.arange(len(S)) if which is None else np.asarray(which)
    cov = np.zeros(len(idx), dtype=bool)
    W = np.full((len(idx), 3), np.nan)
    for k, i in enumerate(idx):
        x = uncovered_point(P[i], abs(S[i]), P, S, tol)
        if x is None:
            cov[k] = True
        else:
            W[k] = x
    return cov, W


def repair(P, S, Q, tol=TOL):
    """Returns (repaired values of the n samples, removed mask, query values,
    kinds of the n + m outputs, base witnesses)."""
    P = np.asarray(P, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64).reshape(-1, 3)
    n = len(S)
    removed, Wall = fully_covered(P, S, tol)
    keep = ~removed
    BP, BS = P[keep], S[keep]
    BW = Wall[keep]
    out = S.copy()
    kind = np.zeros(n + len(Q), dtype=np.uint8)
    sig = sign_class(S)
    for i in np.nonzero(removed)[0]:
        if sig[i] == 0:
            kind[i] = KIND_UNRESOLVED
            continue
        r, x, k, _ = min_valid_radius(P[i], int(sig[i]), BP, BS, tol, BW)
        if k in ("Z", "X") or not np.isfinite(r):
            kind[i] = KIND_UNRESOLVED
            continue
        out[i] = sig[i] * r
        kind[i] = RMIN_KIND[k]
    qv = np.zeros(len(Q))
    R = np.abs(BS)
    for j, q in enumerate(Q):
        d = dist(BP, q)
        inside = d < R - tol
        if not inside.any():
            qv[j] = 0.0
            kind[n + j] = KIND_ZERO
            continue
        sigma = int(sign_class(BS[inside][np.argmax(R[inside] - d[inside])]))
        r, x, k, _ = min_valid_radius(q, sigma, BP, BS, tol, BW)
        if not np.isfinite(r):
            kind[n + j] = KIND_UNRESOLVED
            qv[j] = np.nan
            continue
        qv[j] = sigma * r
        kind[n + j] = RMIN_KIND[k]
    return out, removed, qv, kind, BW
