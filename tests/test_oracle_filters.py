"""Pins of the oracle's filters (oracle/filters.py)."""
import math

import mpmath as mp
import numpy as np
from scipy import integrate

from oracle import filters as F


def _u_schneider(x):
    """The compensated polynomial U filter of Schneider (1996) in units of
    theta_ap = 1: U(x) = (9/pi) (1 - x^2) (1/3 - x^2)."""
    return (9.0 / math.pi) * (1 - x * x) * (1.0 / 3.0 - x * x)


def test_poly_is_Q_of_compensated_U():
    """The paper relates Q to U by Q(t) = (2/t^2) int_0^t t' U(t') dt' - U(t)
    (Sect. 2, the equation after Eq. gammat; the -U term sits outside the
    integral). Integrating Schneider's U numerically must give q_poly."""
    val, _ = integrate.quad(lambda t: t * _u_schneider(t), 0, 1, epsabs=1e-13)
    assert abs(val) < 1e-14  # compensation condition
    for x in np.linspace(0.02, 0.98, 25):
        I, _ = integrate.quad(lambda t: t * _u_schneider(t), 0, x, epsabs=1e-14, epsrel=1e-13)
        Q = 2.0 / (x * x) * I - _u_schneider(x)
        assert abs(Q - F.q_poly(x)) < 1e-13


def test_poly_support_and_peak():
    assert F.q_poly(1.0) == 0.0 and F.q_poly(1.5) == 0.0 and F.q_poly(0.0) == 0.0
    x = np.linspace(0, 1, 100001)[:-1]
    q = F.q_poly(x)
    # maximum of x^2 (1 - x^2) is 1/4 at x = 1/sqrt 2
    assert abs(q.max() - 6.0 / math.pi / 4.0) < 1e-9
    assert abs(x[q.argmax()] - 1 / math.sqrt(2)) < 1e-4


def test_tanh_limits_and_mp():
    q0 = F.q_tanh(0.0)
    assert abs(q0 - 1.0 / (1.0 + math.exp(6.0) + math.exp(-47.0))) < 1e-17
    assert abs(F.q_tanh(1e-12) - q0) < 1e-12  # slope of the switch is ~150 q0
    assert F.q_tanh(1.0) == 0.0
    mp.mp.dps = 40
    for x in [1e-6, 0.01, 0.04, 0.0400001, 0.1, 0.5, 0.9, 0.999999]:
        t = mp.mpf(x) / mp.mpf("0.15")
        ref = mp.tanh(t) / t / (1 + mp.exp(6 - 150 * mp.mpf(x)) + mp.exp(-47 + 50 * mp.mpf(x)))
        assert abs(F.q_tanh(x) - float(ref)) <= 1e-15 * max(1e-3, float(ref))
    # the two landmarks quoted for this filter: the inner switch and the edge value
    assert abs(F.q_tanh(0.04) - 0.488) < 1e-3
    assert abs(F.q_tanh(1 - 1e-12) - 0.00711) < 1e-4


def test_table_interpolates_nodes_and_reproduces_low_degree():
    """Catmull-Rom facts that any slip in the basis (a wrong tangent factor,
    a shifted node index, a missing ghost node) breaks: the interpolant
    passes through every node; a straight line is reproduced everywhere
    (the ghost nodes continue it); a quadratic is reproduced exactly on
    the interior intervals, where the central-difference tangents are the
    exact derivative."""
    n = 17
    xk = np.linspace(0, 1, n)
    rng = np.random.default_rng(0)
    s = rng.normal(size=n)
    assert np.max(np.abs(F.q_table(xk[:-1], s) - s[:-1])) < 1e-15
    assert F.q_table(1.0, s) == 0.0 and F.q_table(-0.1, s) == 0.0
    x = np.linspace(0, 1, 10001)[:-1]
    line = lambda t: 0.3 - 1.7 * t
    assert np.max(np.abs(F.q_table(x, line(xk)) - line(x))) < 1e-14
    quad = lambda t: 0.2 + 0.5 * t - 2.0 * t * t
    inner = (x >= 1.0 / (n - 1)) & (x < 1.0 - 1.0 / (n - 1))
    assert np.max(np.abs(F.q_table(x[inner], quad(xk)) - quad(x[inner]))) < 1e-14
    # the end intervals use one-sided tangents: a quadratic is not exact there
    assert np.max(np.abs(F.q_table(x[~inner], quad(xk)) - quad(x[~inner]))) > 1e-4


def test_table_converges_to_smooth_filter():
    """Dense samples of the polynomial filter reproduce it with the
    third-order error of the Catmull-Rom spline: halving the node spacing
    divides the interior error by about eight."""
    x = np.linspace(0.05, 0.95, 20001)
    errs = []
    for n in (65, 129, 257, 4097):
        xk = np.linspace(0, 1, n)
        errs.append(np.max(np.abs(F.q_table(x, F.q_poly(xk)) - F.q_poly(x))))
    assert 6.0 < errs[0] / errs[1] < 10.0 and 6.0 < errs[1] / errs[2] < 10.0
    assert errs[3] < 1e-9 * F.q_poly(1 / math.sqrt(2))


def test_table_one_interval_against_hermite_solve():
    """On an interior interval the Catmull-Rom cubic is the cubic with the
    node values at both ends and central-difference slopes there; checked
    against that cubic solved as a 4x4 linear system in the monomial basis,
    a route independent of the basis-matrix form of the oracle."""
    n = 9
    xk = np.linspace(0, 1, n)
    rng = np.random.default_rng(3)
    s = rng.normal(size=n)
    k = 4
    h = 1.0 / (n - 1)
    m0 = (s[k + 1] - s[k - 1]) / (2 * h)
    m1 = (s[k + 2] - s[k]) / (2 * h)
    # the cubic with these end values and slopes, solved as a linear system
    a = np.array([[1, xk[k], xk[k] ** 2, xk[k] ** 3], [1, xk[k + 1], xk[k + 1] ** 2, xk[k + 1] ** 3],
                  [0, 1, 2 * xk[k], 3 * xk[k] ** 2], [0, 1, 2 * xk[k + 1], 3 * xk[k + 1] ** 2]])
    c = np.linalg.solve(a, np.array([s[k], s[k + 1], m0, m1]))
    x = np.linspace(xk[k], xk[k + 1], 101)[:-1]
    ref = c[0] + c[1] * x + c[2] * x * x + c[3] * x ** 3
    assert np.max(np.abs(F.q_table(x, s) - ref)) < 1e-12
