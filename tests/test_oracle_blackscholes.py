"""Pins for the binary64 BlackScholes oracle (map(BSComputation), Section 5.2).

The closed form is pinned by things it does not contain: numerical
integration of the discounted payoff over the lognormal distribution of the
price at expiry (an independent method), put-call parity, homogeneity in
(price, strike), the limits of tiny and huge prices and of vanishing
volatility, and monotonicity in the price.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle

CASES = [  # (s, strike, rate, volatility, years)
    (42.0, 40.0, 0.10, 0.20, 0.5),
    (20.0, 20.0, 0.02, 0.30, 1.0),
    (5.0, 20.0, 0.02, 0.30, 1.0),      # deep out of the money call
    (30.0, 20.0, 0.02, 0.30, 1.0),
    (100.0, 80.0, 0.00, 0.45, 2.5),
    (12.5, 13.0, -0.01, 0.15, 0.1),    # negative rate, short expiry
    (7.0, 3.0, 0.05, 0.80, 10.0),      # long expiry, high volatility
]


def quad_prices(s, k, r, v, t):
    """e^{-rT} E[payoff] with S_T = s exp((r - v^2/2) T + v sqrt(T) Z), Z ~ N(0, 1),
    integrated numerically on both sides of the strike."""
    m, sd = (r - 0.5 * v * v) * t, v * math.sqrt(t)
    z0 = (math.log(k / s) - m) / sd                  # S_T = k at z0
    phi = lambda z: math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)
    st = lambda z: s * math.exp(m + sd * z)
    disc = math.exp(-r * t)
    c, _ = integrate.quad(lambda z: (st(z) - k) * phi(z), z0, z0 + 40, epsabs=1e-13, epsrel=1e-13, limit=400)
    p, _ = integrate.quad(lambda z: (k - st(z)) * phi(z), z0 - 40, z0, epsabs=1e-13, epsrel=1e-13, limit=400)
    return disc * c, disc * p


@pytest.mark.parametrize("case", CASES)
def test_matches_numerical_integration_of_the_payoff(case):
    s, k, r, v, t = case
    got = oracle.blackscholes(np.array([s]), k, r, v, t)[0]
    c, p = quad_prices(s, k, r, v, t)
    scale = s + k
    assert abs(got[0] - c) <= 1e-10 * scale, (got[0], c)
    assert abs(got[1] - p) <= 1e-10 * scale, (got[1], p)


def test_matches_numerical_integration_all_cases():
    for case in CASES:
        test_matches_numerical_integration_of_the_payoff(case)


def test_put_call_parity_and_homogeneity():
    rng = np.random.default_rng(11)
    s = rng.uniform(1.0, 60.0, 5000)
    k, r, v, t = 20.0, 0.02, 0.3, 1.0
    cp = oracle.blackscholes(s, k, r, v, t)
    fwd = s - k * math.exp(-r * t)
    assert np.all(np.abs((cp[:, 0] - cp[:, 1]) - fwd) <= 1e-12 * (s + k))
    # price(l s, l K) = l price(s, K)
    cp3 = oracle.blackscholes(3.0 * s, 3.0 * k, r, v, t)
    assert np.allclose(cp3, 3.0 * cp, rtol=1e-12, atol=1e-12 * k)


def test_limits():
    k, r, v, t = 20.0, 0.02, 0.3, 1.0
    disc = k * math.exp(-r * t)
    tiny = oracle.blackscholes(np.array([1e-6]), k, r, v, t)[0]
    assert tiny[0] < 1e-30 and abs(tiny[1] - (disc - 1e-6)) <= 1e-12 * k
    huge = oracle.blackscholes(np.array([1e5]), k, r, v, t)[0]
    assert abs(huge[0] - (1e5 - disc)) <= 1e-9 * 1e5 and huge[1] < 1e-30
    # vanishing volatility: intrinsic value of the forward
    s = np.array([10.0, 15.0, 25.0, 30.0])
    cp = oracle.blackscholes(s, k, r, 1e-6, t)
    assert np.allclose(cp[:, 0], np.maximum(s - disc, 0.0), atol=1e-9)
    assert np.allclose(cp[:, 1], np.maximum(disc - s, 0.0), atol=1e-9)


def test_at_the_forward_call_equals_put():
    k, r, v, t = 20.0, 0.05, 0.25, 2.0
    s = k * math.exp(-r * t)
    c, p = oracle.blackscholes(np.array([s]), k, r, v, t)[0]
    assert abs(c - p) <= 1e-13 * k
    # and equals s (2 N(v sqrt(T) / 2) - 1), N from erf
    assert abs(c - s * math.erf(v * math.sqrt(t) / 2 / math.sqrt(2))) <= 1e-13 * k


def test_monotone_in_price():
    s = np.linspace(1.0, 60.0, 2000)
    cp = oracle.blackscholes(s, 20.0, 0.02, 0.3, 1.0)
    assert np.all(np.diff(cp[:, 0]) > 0) and np.all(np.diff(cp[:, 1]) < 0)


def test_storage_types_widen_exactly():
    rng = np.random.default_rng(12)
    s16 = rng.uniform(5, 30, 300).astype(np.float16)
    s32 = rng.uniform(5, 30, 300).astype(np.float32)
    for s in (s16, s32):
        assert np.array_equal(oracle.blackscholes(s, 20.0, 0.02, 0.3, 1.0),
                              oracle.blackscholes(s.astype(np.float64), 20.0, 0.02, 0.3, 1.0))
    assert oracle.blackscholes(np.zeros(0, np.float32), 20.0, 0.02, 0.3, 1.0).shape == (0, 2)


@pytest.mark.parametrize("bad", [dict(strike=0.0), dict(volatility=0.0), dict(years=-1.0), dict(rate=math.inf)])
def test_rejects_bad_parameters(bad):
    args = dict(strike=20.0, rate=0.02, volatility=0.3, years=1.0)
    args.update(bad)
    with pytest.raises(RuntimeError):
        oracle.blackscholes(np.ones(3, np.float32), **args)
