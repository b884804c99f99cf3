"""Pins for the oracle's Hankel kernels (no GPU)."""
import numpy as np
import pytest
from scipy import special as sps

from oracle import special


def test_series_wronskian():
    # A&S 9.1.16: J1 Y0 - J0 Y1 = 2/(pi x); the series branch gives J0, J1, Y0
    # and g1m = (i pi x/2) H1 - 1, from which Y1 = -(2/(pi x)) (Re g1m + 1)
    x = np.geomspace(1e-6, special.X_SERIES, 200)
    j0, j1, y0, g1m = special._series_small(x)
    y1 = -(2.0 / (np.pi * x)) * (g1m.real + 1.0)
    w = j1 * y0 - j0 * y1
    assert np.max(np.abs(w * (np.pi * x / 2) - 1.0)) < 5e-15
    # the imaginary part of g1m is (pi x/2) J1
    assert np.max(np.abs(g1m.imag - np.pi * x / 2 * j1)) < 1e-16


def test_series_against_mpmath():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    for x in (1e-7, 3e-4, 0.05, 0.7, 1.3, 2.0):
        h0, g1m, x2h0 = special.hankel_pieces(np.array([x]))
        eh0 = complex(mp.hankel1(0, mp.mpf(x)))
        eg = complex((1j * mp.pi * mp.mpf(x) / 2) * mp.hankel1(1, mp.mpf(x)) - 1)
        assert abs(h0[0] - eh0) <= 1e-15 * abs(eh0)
        assert abs(g1m[0] - eg) <= 2e-15 * abs(eg)


def test_continuity_at_switch():
    xs = special.X_SERIES
    lo = special.hankel_pieces(np.array([xs * (1 - 1e-14)]))
    _, _, _, gser = special._series_small(np.array([xs]))
    gdir = (1j * np.pi * xs / 2) * sps.hankel1(1, xs) - 1
    assert abs(gser[0] - gdir) < 1e-15
    assert abs(lo[1][0] - gdir) < 1e-13


def _G(k, t, s):
    return 0.25j * sps.hankel1(0, k * np.hypot(t[0] - s[0], t[1] - s[1]))


def test_kernels_match_finite_differences_of_G():
    k = 7.3
    t = np.array([0.31, -0.2])
    s = np.array([-0.45, 0.37])
    n = np.array([0.6, -0.8])
    npr = np.array([-0.28, -0.96])
    h = 1e-5
    dv = t - s
    S, D, Ds, T = special.kernels(k, np.array(dv @ dv), np.array(n @ dv), np.array(npr @ dv), np.array(n @ npr))
    # D = dG/dn' (source normal), D* = dG/dn (target normal), T = d2G/dn dn'
    Dfd = (_G(k, t, s + h * npr) - _G(k, t, s - h * npr)) / (2 * h)
    Dsfd = (_G(k, t + h * n, s) - _G(k, t - h * n, s)) / (2 * h)
    Tfd = (_G(k, t + h * n, s + h * npr) - _G(k, t + h * n, s - h * npr)
           - _G(k, t - h * n, s + h * npr) + _G(k, t - h * n, s - h * npr)) / (4 * h * h)
    assert abs(S - _G(k, t, s)) < 1e-15
    assert abs(D - Dfd) < 1e-8
    assert abs(Ds - Dsfd) < 1e-8
    assert abs(T - Tfd) < 1e-5


def test_reciprocity():
    # D*(t, s; n) equals D(s, t) with the target normal used as source normal
    k = 5.0
    t, s = np.array([0.1, 0.2]), np.array([-0.7, 0.5])
    n = np.array([0.0, 1.0])
    dv = t - s
    _, _, Ds, _ = special.kernels(k, np.array(dv @ dv), np.array(n @ dv), np.array(0.0), np.array(0.0))
    _, D2, _, _ = special.kernels(k, np.array(dv @ dv), np.array(0.0), np.array(n @ -dv), np.array(0.0))
    assert abs(Ds - D2) < 1e-15


def test_difference_kernels_equal_plain_differences():
    r2 = np.array([0.3, 1.7, 4.0])
    nd = np.array([0.1, -0.3, 0.5])
    npd = np.array([-0.2, 0.4, 0.3])
    nn = np.array([0.9, 0.7, -0.2])
    a = special.kernels(11.0, r2, nd, npd, nn)
    b = special.kernels(13.0, r2, nd, npd, nn)
    d = special.kernels_diff(11.0, 13.0, r2, nd, npd, nn)
    for x, y, z in zip(a, b, d):
        assert np.max(np.abs((x - y) - z)) < 1e-13


def test_difference_kernel_small_separation_limit():
    # at tiny r the difference of the single-layer kernels tends to
    # -(1/(2 pi)) log(ka/kb); the 1/r^2 parts of T cancel exactly
    ka, kb = 10.0, 16.0
    r2 = np.array([1e-20])
    S, D, Ds, T = special.kernels_diff(ka, kb, r2, np.array(0.0), np.array(0.0), np.array(1.0))
    assert abs(S.real - (-np.log(ka / kb) / (2 * np.pi))) < 1e-12
    # T - T' -> (1/(2 pi r^2)) (g1a - g1b) ~ -(ka^2 - kb^2) log(r)/(4 pi)
    assert np.isfinite(T).all() and abs(T) < 1e3
