"""Pins for the oracle's closure laws (Section 2.1 eqs. Sw, sc_van, Krw, Krw1; Gardner law).

Each pin checks the oracle against something other than its own formula:
  * C must be the derivative of theta (Section 2: C = d theta / dp), checked by a
    Richardson-extrapolated central difference of the oracle's theta;
  * the closed-form Mualem conductivity (eq. Krw) must equal the Mualem integral
    (eq. Krw1) evaluated by adaptive quadrature in 30-digit arithmetic;
  * special values: saturated branch, p -> -inf limits, m = 1 - 1/n.
"""
import mpmath
import numpy as np
import pytest

from oracle import constitutive as cl

P_GRID = -np.concatenate([np.logspace(-6, 1.3, 40)])


def _richardson_derivative(f, p, d=1e-3):
    d1 = (f(p + d) - f(p - d)) / (2 * d)
    d2 = (f(p + d / 2) - f(p - d / 2)) / d
    return (4 * d2 - d1) / 3


def test_gardner_capacity_is_theta_derivative():
    Ks, a, tr, ts = 1.3, 1.0, 0.05, 0.5
    p = -np.linspace(0.05, 12.0, 57)
    th = lambda q: cl.gardner(q, Ks, a, tr, ts)[1]
    C = cl.gardner(p, Ks, a, tr, ts)[2]
    # step 1e-2: Richardson error O(d^4) ~ 1e-10, rounding of theta ~ 1e-17/d
    dnum = _richardson_derivative(th, p, d=1e-2)
    np.testing.assert_allclose(C, dnum, rtol=1e-8, atol=0)


@pytest.mark.parametrize("alpha,n", [(1.0, 2.0), (3.0, 1.45), (0.4, 1.1), (4.0, 3.6)])
def test_vg_capacity_is_theta_derivative(alpha, n):
    p = -np.logspace(-2, 1, 31)
    th = lambda q: cl.van_genuchten(q, 1.0, alpha, n, 0.05, 0.5)[1]
    C = cl.van_genuchten(p, 1.0, alpha, n, 0.05, 0.5)[2]
    d = 3e-3 * np.abs(p)
    dnum = _richardson_derivative(th, p, d=d)
    np.testing.assert_allclose(C, dnum, rtol=1e-8, atol=0)


def test_saturated_branch():
    p = np.array([0.0, 0.3, 5.0])
    K, th, C = cl.gardner(p, 2.0, 1.0, 0.05, 0.5)
    assert np.all(K == 2.0) and np.all(th == 0.5) and np.all(C == 0.0)
    K, th, C = cl.van_genuchten(p, 2.0, 3.0, 1.45, 0.05, 0.5)
    assert np.all(K == 2.0) and np.all(th == 0.5) and np.all(C == 0.0)


def test_dry_limits():
    K, th, C = cl.gardner(np.array([-800.0]), 1.0, 1.0, 0.05, 0.5)
    assert K[0] == 0.0 and th[0] == 0.05 and C[0] == 0.0
    K, th, C = cl.van_genuchten(np.array([-1e6]), 1.0, 2.0, 2.0, 0.05, 0.5)
    assert K[0] < 1e-12 and abs(th[0] - 0.05) < 1e-6


def _mualem_integral(S, alpha, n):
    """K_rw from eq. Krw1 with the inverse retention curve |p|(S) = (S^(-1/m) - 1)^(1/n) / alpha."""
    mpmath.mp.dps = 30
    m = 1 - mpmath.mpf(1) / n
    inv_p = lambda s: alpha / (s ** (-1 / m) - 1) ** (mpmath.mpf(1) / n)
    num = mpmath.quad(inv_p, [0, S])
    den = mpmath.quad(inv_p, [0, mpmath.mpf(1) / 2, 1])
    return float(mpmath.sqrt(S) * (num / den) ** 2)


@pytest.mark.parametrize("alpha,n", [(1.0, 2.0), (3.0, 1.45), (2.0, 1.6)])
def test_mualem_closed_form_matches_integral(alpha, n):
    for p in (-0.05, -0.4, -2.0, -7.0):
        S = float(cl.vg_saturation(np.array([p]), alpha, n)[0])
        K = float(cl.van_genuchten(np.array([p]), 1.0, alpha, n, 0.05, 0.5)[0][0])
        ref = _mualem_integral(mpmath.mpf(S), alpha, n)
        assert abs(K - ref) <= 1e-9 * max(ref, 1e-300), (p, K, ref)


def test_vg_stable_near_saturation():
    # close to p = 0- the rewrite must stay accurate where 1 - S^(1/m) cancels
    alpha, n = 3.0, 1.45
    p = -1e-9
    mpmath.mp.dps = 50
    m = 1 - mpmath.mpf(1) / n
    u = (mpmath.mpf(alpha) * mpmath.mpf(-p)) ** n
    S = (1 + u) ** (-m)
    # the literal eq. Krw in 50-digit arithmetic, where 1 - S^(1/m) does not cancel
    ref = float(mpmath.sqrt(S) * (1 - (1 - S ** (1 / m)) ** m) ** 2)
    K = float(cl.van_genuchten(np.array([p]), 1.0, alpha, n, 0.05, 0.5)[0][0])
    assert abs(K - ref) <= 1e-13 * ref
