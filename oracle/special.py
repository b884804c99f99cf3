"""Hankel-function kernels for the oracle (test infrastructure only).

The free-space Green's function is G = (i/4) H0^(1)(k r) (Sec. 2, eq. (11)).
For arguments above ``X_SERIES`` the Hankel values come from
``scipy.special.hankel1``.  Below it, the pieces that enter the *difference*
kernels of the self blocks (where the 1/r^2 singularities of the two layers
cancel) are summed from the Abramowitz & Stegun ascending series
(A&S 9.1.10, 9.1.11, 9.1.13), so that they keep full relative accuracy.

Quantities (x = k r):
  h0(x)    = H0^(1)(x)
  g1(x)    = (i pi x / 2) H1^(1)(x)           (-> 1 as x -> 0)
  g1m(x)   = g1(x) - 1                          (O(x^2 log x))
  x2h0(x)  = x^2 H0^(1)(x)

Pins (tests/test_oracle_special.py): Wronskian J1 Y0 - J0 Y1 = 2/(pi x)
(A&S 9.1.16), mpmath spot values of g1m, continuity across X_SERIES.
"""
from __future__ import annotations

import numpy as np
from scipy import special as sps

EULER_GAMMA = 0.57721566490153286060651209008240243
X_SERIES = 2.0
_NTERMS = 30


def _series_small(x: np.ndarray):
    """Ascending series for J0, J1, Y0 and g1m at 0 < x <= X_SERIES."""
    x = np.asarray(x, dtype=float)
    z = x / 2.0
    z2 = -z * z
    lg = np.log(z)
    # J0 = sum (-z^2)^m/(m!)^2 ; J1 = z sum (-z^2)^m/(m!(m+1)!)
    j0 = np.zeros_like(x)
    j1 = np.zeros_like(x)
    y0s = np.zeros_like(x)      # sum_{m>=1} (-1)^{m+1} H_m z^{2m}/(m!)^2
    g1s = np.zeros_like(x)      # sum_{m>=0} (psi(m+1)+psi(m+2)) (-z^2)^m/(m!(m+1)!)
    t0 = np.ones_like(x)        # (-z^2)^m/(m!)^2
    t1 = np.ones_like(x)        # (-z^2)^m/(m!(m+1)!)
    harm = 0.0
    for m in range(_NTERMS):
        if m > 0:
            t0 = t0 * z2 / (m * m)
            t1 = t1 * z2 / (m * (m + 1))
            harm += 1.0 / m
        psi1 = -EULER_GAMMA + harm                  # psi(m+1)
        psi2 = -EULER_GAMMA + harm + 1.0 / (m + 1)  # psi(m+2)
        j0 = j0 + t0
        j1 = j1 + t1
        if m > 0:
            y0s = y0s - harm * t0                   # (-1)^{m+1} H_m z^{2m}/(m!)^2
        g1s = g1s + (psi1 + psi2) * t1
    j1 = z * j1
    y0 = (2.0 / np.pi) * ((lg + EULER_GAMMA) * j0 + y0s)
    # (pi x/2) Y1 = -1 + x log(z) J1 - z^2 * g1s  (A&S 9.1.11, n = 1)
    g1m = (1j * np.pi * x / 2.0) * j1 - x * lg * j1 + z * z * g1s
    return j0, j1, y0, g1m


def h0(x):
    x = np.asarray(x, dtype=float)
    return sps.hankel1(0, x)


def hankel_pieces(x):
    """Return (h0, g1m, x2h0) for x > 0 (any shape)."""
    x = np.asarray(x, dtype=float)
    H0 = sps.hankel1(0, x)
    H1 = sps.hankel1(1, x)
    g1m = (1j * np.pi * x / 2.0) * H1 - 1.0
    small = x <= X_SERIES
    if np.any(small):
        j0, j1, y0, gm = _series_small(x[small])
        H0 = H0.copy()
        H0[small] = j0 + 1j * y0
        g1m = g1m.copy()
        g1m[small] = gm
    return H0, g1m, x * x * H0


def kernels(k, r2, nd, npd, nn):
    """The four layer-potential kernels at wavenumber k for a target with unit
    normal n and a source with unit normal n', separation dv = t - s:

      S  = (i/4) H0(k r)                          single layer
      D  = dG/dn'  = (n'.dv / (2 pi r^2)) g1      double layer
      D* = dG/dn   = -(n.dv / (2 pi r^2)) g1      adjoint double layer
      T  = d2G/dn dn'
         = [ (n.n') g1/(2 pi) + (n.dv)(n'.dv)/r^2 ((i/4) x^2 H0 - g1/pi) ] / r^2

    derived from dH0/dx = -H1 and H1' = H0 - H1/x (Sec. 2.2, eq. (19)-(20)).
    Arguments: r2 = |dv|^2, nd = n.dv, npd = n'.dv, nn = n.n'.
    """
    r = np.sqrt(r2)
    H0, g1m, x2h0 = hankel_pieces(k * r)
    g1 = 1.0 + g1m
    S = 0.25j * H0
    D = npd / (2 * np.pi * r2) * g1
    Ds = -nd / (2 * np.pi * r2) * g1
    T = (nn * g1 / (2 * np.pi) + nd * npd / r2 * (0.25j * x2h0 - g1 / np.pi)) / r2
    return S, D, Ds, T


def kernels_diff(ka, kb, r2, nd, npd, nn):
    """K^{ka} - K^{kb} for the four kernels, with the k-independent leading
    singular terms cancelled analytically (only g1m and H0 differences enter)."""
    r = np.sqrt(r2)
    Ha, ga, xa = hankel_pieces(ka * r)
    Hb, gb, xb = hankel_pieces(kb * r)
    dg = ga - gb
    S = 0.25j * (Ha - Hb)
    D = npd / (2 * np.pi * r2) * dg
    Ds = -nd / (2 * np.pi * r2) * dg
    T = (nn * dg / (2 * np.pi) + nd * npd / r2 * (0.25j * (xa - xb) - dg / np.pi)) / r2
    return S, D, Ds, T
