"""Aperture filters q(x), x = theta / theta_ap, in FP64.

The paper applies a filter Q to the tangential shear (Eq. map_gammat) and
evaluates it from the great-circle distance to the aperture centre
(Sect. 3.1 step 3). The workloads use the first two filters:

* POLY: q(x) = (6/pi) x^2 (1 - x^2), the compensated polynomial filter of
  Schneider (1996), which the paper cites for the aperture mass;
* TANH: q(x) = tanh(x/x_c) / (x/x_c) / (1 + exp(a - b x) + exp(-c + d x))
  with (x_c, a, b, c, d) = (0.15, 6, 150, 47, 50), an NFW-like filter with a
  steep inner switch and a small jump at x = 1;
* TABLE: a filter given by its values at n >= 2 uniform nodes x_k = k/(n-1)
  on [0, 1] (the last one the left limit at x = 1), interpolated by the
  Catmull-Rom cubic: on [x_k, x_k+1] the cubic through q_k-1, q_k, q_k+1,
  q_k+2 in the cardinal-spline form, with ghost nodes q_-1 = 2 q_0 - q_1 and
  q_n = 2 q_n-1 - q_n-2 continuing the end segments as straight lines. The
  paper's filters are closed forms; this form lets a caller supply any
  tabulated filter (Sect. 3.1 step 3 only needs Q at each distance).

All vanish for x >= 1 (outside the aperture). The physical filter is
Q(theta) = q(theta/theta_ap) / theta_ap^2; the 1/theta_ap^2 factor is applied
by the normalisation step, not here.

Pins: tests/test_oracle_filters.py checks special values computed by hand
(q_poly(1/sqrt 2) = 3/(2 pi), q_tanh(0) = 1/(1+e^6+e^-47)), the
compensation identity of the polynomial filter's U counterpart, and
continuity of the tanh expression against mpmath at 50 digits, and for
the table form: node interpolation, exact straight lines everywhere and
quadratics on interior intervals, third-order convergence to a smooth
filter, and one interval against the Hermite cubic solved as a linear system.
"""
from __future__ import annotations

import math

import numpy as np

POLY = 0
TANH = 1
TABLE = 2

TANH_DEFAULT = (0.15, 6.0, 150.0, 47.0, 50.0)


def q_poly(x):
    x = np.asarray(x, dtype=np.float64)
    v = (6.0 / math.pi) * x * x * (1.0 - x * x)
    return np.where((x >= 0) & (x < 1.0), v, 0.0)


def q_tanh(x, params=TANH_DEFAULT):
    xc, a, b, c, d = params
    x = np.asarray(x, dtype=np.float64)
    t = x / xc
    with np.errstate(invalid="ignore", divide="ignore"):
        ratio = np.where(t > 0, np.tanh(t) / np.where(t > 0, t, 1.0), 1.0)
    v = ratio / (1.0 + np.exp(a - b * x) + np.exp(-c + d * x))
    return np.where((x >= 0) & (x < 1.0), v, 0.0)


def q_table(x, samples):
    """Catmull-Rom interpolant of `samples` at uniform nodes on [0, 1]:
    q(x) = 1/2 [1, f, f^2, f^3] M [q_k-1, q_k, q_k+1, q_k+2] on node
    interval k with local coordinate f, M the cardinal-spline basis of
    tension 1/2 (rows (0, 2, 0, 0), (-1, 0, 1, 0), (2, -5, 4, -1),
    (-1, 3, -3, 1)); zero outside [0, 1)."""
    q = np.asarray(samples, dtype=np.float64)
    n = q.size
    if n < 2:
        raise ValueError("a table filter needs at least two samples")
    ext = np.concatenate([[2.0 * q[0] - q[1]], q, [2.0 * q[-1] - q[-2]]])  # ghost nodes
    x = np.asarray(x, dtype=np.float64)
    u = np.clip(x, 0.0, 1.0) * (n - 1)
    k = np.minimum(np.floor(u).astype(np.int64), n - 2)
    f = u - k
    pm, p0, p1, p2 = ext[k], ext[k + 1], ext[k + 2], ext[k + 3]
    v = 0.5 * (2.0 * p0 + f * (p1 - pm) + f * f * (2.0 * pm - 5.0 * p0 + 4.0 * p1 - p2)
               + f * f * f * (-pm + 3.0 * p0 - 3.0 * p1 + p2))
    return np.where((x >= 0) & (x < 1.0), v, 0.0)


def q_of(kind: int, params=None):
    if kind == POLY:
        return q_poly
    if kind == TANH:
        p = TANH_DEFAULT if params is None else tuple(params)
        return lambda x: q_tanh(x, p)
    if kind == TABLE:
        samples = np.asarray(params, dtype=np.float64)
        return lambda x: q_table(x, samples)
    raise ValueError(f"unknown filter kind {kind}")
