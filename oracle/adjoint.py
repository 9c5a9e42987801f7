"""Reverse sweep of d(sum of interpolated values)/d(input samples).

Each greedy value has one active parent constraint t (the sphere it is
tangent to), so for fixed decisions:
  HI:          v = s_t + |q - p_t|
  LO:          v = s_t - |q - p_t|
  COINCIDENT:  v = s_t
  RMIN_T:      v = sigma * | |q - p_t| - |s_t| |  (radial foot point on sphere t)
  ZERO:        v = 0
RMIN_D / RMIN_U values depend on two or three spheres; they are reported as
multi-parent and contribute nothing here (their closed-form derivative is not
part of this sweep).  A parent that is itself an earlier query passes the
accumulated adjoint on: walking queries in reverse acceptance order,
g_j = 1 + sum over children of g_child * dv_child/ds_j.
Query positions are fixed inputs; gradients flow to the samples' values and
positions only.
"""
from __future__ import annotations

import numpy as np

from .common import (KIND_COINCIDENT, KIND_HI, KIND_LO, KIND_RMIN_T, dist, sign_class)


def adjoint(P, S, Q, values, kind, active, order, grad_values=None):
    """Gradient of sum_j grad_values[j] * values[j] (all weights 1 by default)
    with respect to the sample values and positions, decisions held fixed.
    Returns (grad_s, grad_p, number of multi-parent values met)."""
    P = np.asarray(P, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    n = len(S)
    g = np.ones(len(Q)) if grad_values is None else np.array(grad_values, dtype=np.float64)
    grad_s = np.zeros(n)
    grad_p = np.zeros((n, 3))
    multi = 0
    for j in np.asarray(order)[::-1]:
        k = int(kind[j])
        t = int(active[j])
        if k not in (KIND_HI, KIND_LO, KIND_COINCIDENT, KIND_RMIN_T) or t < 0:
            if k in (5, 6):
                multi += 1
            continue
        if t < n:
            pt, st = P[t], S[t]
        else:
            pt, st = Q[t - n], values[t - n]
        q = Q[j]
        d = float(dist(q, pt))
        unit = (pt - q) / d if d > 0.0 else np.zeros(3)   # d|q - p_t| / dp_t
        if k == KIND_HI:
            ds, dp = 1.0, unit
        elif k == KIND_LO:
            ds, dp = 1.0, -unit
        elif k == KIND_COINCIDENT:
            ds, dp = 1.0, np.zeros(3)
        else:
            sigma = float(np.sign(values[j])) if values[j] != 0.0 else 0.0
            e = d - abs(st)
            se = 1.0 if e > 0.0 else -1.0
            ds = sigma * se * (-float(sign_class(st)))
            dp = sigma * se * unit
        if t < n:
            grad_s[t] += g[j] * ds
            grad_p[t] += g[j] * dp
        else:
            g[t - n] += g[j] * ds
    return grad_s, grad_p, multi
