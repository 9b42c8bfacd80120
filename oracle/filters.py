"""Aperture filters q(x), x = theta / theta_ap, in FP64.

The paper applies a filter Q to the tangential shear (Eq. map_gammat) and
evaluates it from the great-circle distance to the aperture centre
(Sect. 3.1 step 3). The workloads use two filters:

* POLY: q(x) = (6/pi) x^2 (1 - x^2), the compensated polynomial filter of
  Schneider (1996), which the paper cites for the aperture mass;
* TANH: q(x) = tanh(x/x_c) / (x/x_c) / (1 + exp(a - b x) + exp(-c + d x))
  with (x_c, a, b, c, d) = (0.15, 6, 150, 47, 50), an NFW-like filter with a
  steep inner switch and a small jump at x = 1.

Both vanish for x >= 1 (outside the aperture). The physical filter is
Q(theta) = q(theta/theta_ap) / theta_ap^2; the 1/theta_ap^2 factor is applied
by the normalisation step, not here.

Pins: tests/test_oracle_filters.py checks special values computed by hand
(q_poly(1/sqrt 2) = 3/(2 pi), q_tanh(0) = 1/(1+e^6+e^-47)), the
compensation identity of the polynomial filter's U counterpart, and
continuity of the tanh expression against mpmath at 50 digits.
"""
from __future__ import annotations

import math

import numpy as np

POLY = 0
TANH = 1

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


def q_of(kind: int, params=None):
    if kind == POLY:
        return q_poly
    if kind == TANH:
        p = TANH_DEFAULT if params is None else tuple(params)
        return lambda x: q_tanh(x, p)
    raise ValueError(f"unknown filter kind {kind}")
