"""Pins for the oracle's Alpert log-singular rule (no GPU)."""
import numpy as np
import pytest

from oracle import alpert


def _periodic_log_integral(rule, N, m, t0):
    """int_0^{2 pi} log(4 sin^2((t - t0)/2)) cos(m t) dt by the corrected
    trapezoid rule with the singular point at the node t0."""
    chi, u, a = rule
    h = 2 * np.pi / N

    def f(t):
        return np.log(4 * np.sin((t - t0) / 2) ** 2) * np.cos(m * t)

    i = np.arange(a, N - a + 1)
    return h * np.sum(f(t0 + i * h)) + h * np.sum(u * (f(t0 + chi * h) + f(t0 - chi * h)))


def test_rule_shape():
    chi, u, a = alpert.load_rule()
    assert len(chi) == 15 and a == 10
    assert np.all(chi > 0) and np.all(chi < a) and np.all(np.diff(chi) > 0)
    assert np.all(u > 0)


@pytest.mark.parametrize("m,t0", [(1, 0.0), (3, 0.37), (7, 2.2), (12, -1.3)])
def test_closed_form_log_integral(m, t0):
    # int_0^{2pi} log(4 sin^2(t/2)) cos(m t) dt = -2 pi / m  (m >= 1), shifted by t0
    rule = alpert.load_rule()
    exact = -2 * np.pi * np.cos(m * t0) / m
    assert abs(_periodic_log_integral(rule, 160, m, t0) - exact) < 5e-15


def test_observed_high_order():
    # error falls by well over 2^12 per doubling of N in the pre-asymptotic range
    rule = alpert.load_rule()
    m, t0 = 14, 0.5
    exact = -2 * np.pi * np.cos(m * t0) / m
    e1 = abs(_periodic_log_integral(rule, 40, m, t0) - exact)
    e2 = abs(_periodic_log_integral(rule, 80, m, t0) - exact)
    assert e1 > 1e-9 and e2 < e1 / 4096


def test_moment_equations():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    chi, u, a = alpert.load_rule()
    for p in range(15):
        lhs = sum(mp.mpf(w) * mp.mpf(c) ** p for c, w in zip(chi, u))
        rhs = -mp.zeta(-p, a)
        assert abs(lhs - rhs) <= 1e-13 * max(1, abs(rhs))
        lhs = sum(mp.mpf(w) * mp.mpf(c) ** p * mp.log(mp.mpf(c)) for c, w in zip(chi, u))
        rhs = mp.zeta(-p, a, 1)
        assert abs(lhs - rhs) <= 1e-13 * max(1, abs(rhs))
