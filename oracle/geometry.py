"""Discretisation geometry for the oracle (test infrastructure only).

Unit cell -d/2 <= x < d/2 (Sec. 2).  Interface normals point down, into the
layer below (Sec. 2.1); wall normals are (1, 0) and radiation-line normals are
(0, 1) (Sec. 2.3-2.4).

* Smooth interface: periodic trapezoid rule in s, s_j = 2 pi (j - 1/2)/N,
  z_j = Z(s_j), w_j = (2 pi/N) |Z'(s_j)|, with Z(s) = (x(s), y0 + f(x(s))),
  x(s) = -d/2 + d s/(2 pi) (Sec. 2.5, eq. (62) and the text after it).
* Cornered interface: one straight segment per vertex pair, Kress grading
  w(s) = 2 pi v^q/(v^q + v(2 pi - s)^q) (Sec. 2.5), midpoint nodes.
* Walls: M_w Gauss-Legendre nodes on L_i = {x = -d/2} between the layer's
  bottom and top boundary (Sec. 2.5, eq. (61)).
* Radiation lines: M_ud midpoint (trapezoid) nodes on U and D (Sec. 2.5).
* Proxies: P points on a circle of radius R about the layer centre, at angle
  2 pi p/P, outward normals (Sec. 2.1, eq. (15)).

Self-interface separations near the Alpert auxiliary nodes are computed from
trigonometric difference identities (sin A - sin B = 2 cos((A+B)/2)
sin((A-B)/2), and the Taylor remainder f(x+h) - f(x) - h f'(x) mode by mode)
so that |dv|^2, n.dv and n'.dv keep full relative accuracy when the two points
are very close.  Pinned in tests/test_oracle_geometry.py against mpmath.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class Curve:
    kind: str
    N: int
    d: float
    y0: float
    x: np.ndarray
    y: np.ndarray
    nx: np.ndarray
    ny: np.ndarray
    w: np.ndarray
    # smooth (fourier) data
    cos_coef: Optional[np.ndarray] = None
    sin_coef: Optional[np.ndarray] = None
    # cornered data
    seg_start: Optional[np.ndarray] = None   # first node index of each segment
    seg_n: Optional[np.ndarray] = None
    seg_of: Optional[np.ndarray] = None      # segment index of each node
    vx: Optional[np.ndarray] = None
    vy: Optional[np.ndarray] = None
    q: float = 6.0

    # ---- smooth profile f(x) and its derivatives -------------------------
    def _omega(self):
        return 2 * np.pi * np.arange(1, len(self.cos_coef) + 1) / self.d

    def f(self, x):
        x = np.asarray(x, dtype=float)[..., None]
        om = self._omega()
        return (self.cos_coef * np.cos(om * x) + self.sin_coef * np.sin(om * x)).sum(-1)

    def fp(self, x):
        x = np.asarray(x, dtype=float)[..., None]
        om = self._omega()
        return (om * (-self.cos_coef * np.sin(om * x) + self.sin_coef * np.cos(om * x))).sum(-1)

    def fdiff(self, x, h):
        """f(x + h) - f(x), via product formulas (no cancellation)."""
        x = np.asarray(x, dtype=float)[..., None]
        h = np.asarray(h, dtype=float)[..., None]
        om = self._omega()
        sh = np.sin(om * h / 2)
        mid = om * (x + h / 2)
        return (-2 * self.cos_coef * np.sin(mid) * sh + 2 * self.sin_coef * np.cos(mid) * sh).sum(-1)

    def fremainder(self, x, h):
        """f(x + h) - f(x) - h f'(x), mode by mode without cancellation."""
        x = np.asarray(x, dtype=float)[..., None]
        h = np.asarray(h, dtype=float)[..., None]
        om = self._omega()
        u = om * h
        cm1 = -2 * np.sin(u / 2) ** 2                     # cos u - 1
        smu = _sin_minus_id(u)                            # sin u - u
        c, s = np.cos(om * x), np.sin(om * x)
        return (self.cos_coef * (c * cm1 - s * smu) + self.sin_coef * (s * cm1 + c * smu)).sum(-1)


def _sin_minus_id(u):
    """sin(u) - u with full relative accuracy (series for |u| < 0.5)."""
    u = np.asarray(u, dtype=float)
    out = np.sin(u) - u
    small = np.abs(u) < 0.5
    if np.any(small):
        us = u[small]
        acc = np.zeros_like(us)
        term = -us ** 3 / 6.0
        n = 3
        for _ in range(12):
            acc = acc + term
            term = -term * us * us / ((n + 1) * (n + 2))
            n += 2
        out = out.copy()
        out[small] = acc
    return out


def kress_w(s, q):
    """Kress grading w(s) and w'(s) on [0, 2 pi] (Sec. 2.5)."""
    s = np.asarray(s, dtype=float)

    def v(t):
        return (1.0 / q - 0.5) * ((np.pi - t) / np.pi) ** 3 + (t - np.pi) / (q * np.pi) + 0.5

    def vp(t):
        return -(3.0 / np.pi) * (1.0 / q - 0.5) * ((np.pi - t) / np.pi) ** 2 + 1.0 / (q * np.pi)

    A = v(s) ** q
    B = v(2 * np.pi - s) ** q
    Ap = q * v(s) ** (q - 1) * vp(s)
    Bp = -q * v(2 * np.pi - s) ** (q - 1) * vp(2 * np.pi - s)
    w = 2 * np.pi * A / (A + B)
    wp = 2 * np.pi * (Ap * B - A * Bp) / (A + B) ** 2
    return w, wp


def kress_wc(s, q):
    """2 pi - w(s), formed as 2 pi v(2 pi - s)^q/(v^q + v(2 pi - s)^q) so that it
    keeps full relative accuracy near s = 2 pi, where w(s) rounds to 2 pi."""
    s = np.asarray(s, dtype=float)

    def v(t):
        return (1.0 / q - 0.5) * ((np.pi - t) / np.pi) ** 3 + (t - np.pi) / (q * np.pi) + 0.5

    A = v(s) ** q
    B = v(2 * np.pi - s) ** q
    return 2 * np.pi * B / (A + B)


def make_curve(iface, d: float) -> Curve:
    if iface.kind == "fourier":
        N = int(iface.n_nodes)
        x = -d / 2 + d * (np.arange(N) + 0.5) / N
        c = Curve("fourier", N, d, float(iface.y0), x, x, x, x, x,
                  cos_coef=np.asarray(iface.cos_coef, float), sin_coef=np.asarray(iface.sin_coef, float))
        fp = c.fp(x)
        nu = np.sqrt(1 + fp * fp)
        c.y = iface.y0 + c.f(x)
        c.nx = fp / nu
        c.ny = -1.0 / nu
        c.w = (d / N) * nu
        return c
    # cornered: straight graded segments
    vx = np.asarray(iface.vx, float)
    vy = np.asarray(iface.vy, float)
    segn = np.asarray(iface.seg_nodes, dtype=int)
    xs, ys, nxs, nys, ws, seg_of = [], [], [], [], [], []
    for c_ in range(len(segn)):
        n = segn[c_]
        s = 2 * np.pi * (np.arange(n) + 0.5) / n
        wv, wpv = kress_w(s, iface.q)
        wc = kress_wc(s, iface.q)
        dx, dy = vx[c_ + 1] - vx[c_], vy[c_ + 1] - vy[c_]
        L = np.hypot(dx, dy)
        # each node is placed from its nearer corner, so that its (tiny)
        # distance to that corner is not lost to rounding
        first = s < np.pi
        xs.append(np.where(first, vx[c_] + wv / (2 * np.pi) * dx, vx[c_ + 1] - wc / (2 * np.pi) * dx))
        ys.append(np.where(first, vy[c_] + wv / (2 * np.pi) * dy, vy[c_ + 1] - wc / (2 * np.pi) * dy))
        nxs.append(np.full(n, dy / L))
        nys.append(np.full(n, -dx / L))
        ws.append(L / n * wpv)
        seg_of.append(np.full(n, c_))
    starts = np.concatenate([[0], np.cumsum(segn)[:-1]])
    X, Y = np.concatenate(xs), np.concatenate(ys)
    # graded nodes of adjacent segments (also across x = +-d/2) must stay
    # distinct in float64; with a very strong grading they round onto the corner
    for l in (-1, 0, 1):
        r2 = (X[:, None] - X[None, :] - l * d) ** 2 + (Y[:, None] - Y[None, :]) ** 2
        if l == 0:
            np.fill_diagonal(r2, 1.0)
        if np.any(r2 == 0.0):
            raise ValueError("graded nodes coincide in float64: lower q or the segment node counts")
    return Curve("polygon", int(segn.sum()), d, float(iface.y0), X, Y,
                 np.concatenate(nxs), np.concatenate(nys), np.concatenate(ws),
                 seg_start=starts, seg_n=segn, seg_of=np.concatenate(seg_of), vx=vx, vy=vy, q=iface.q)


def curve_height_at(curve: Curve, x: float) -> float:
    """Interface height at abscissa x (used for the wall end points)."""
    if curve.kind == "fourier":
        return float(curve.y0 + curve.f(np.array([x]))[0])
    return float(np.interp(x, curve.vx, curve.vy))


@dataclass
class Geometry:
    d: float
    curves: list
    walls: list          # per layer: (x, y) arrays of the M_w wall nodes on L_i
    xU: np.ndarray
    xD: np.ndarray
    yU: float
    yD: float
    centres: np.ndarray  # (I+1, 2) proxy circle centres
    R: float
    P: int


def gauss_legendre(M: int, a: float, b: float):
    t, _ = np.polynomial.legendre.leggauss(M)
    return a + (b - a) * (t + 1) / 2


def make_geometry(stack) -> Geometry:
    d = stack.d
    curves = [make_curve(s, d) for s in stack.interfaces]
    I = len(curves)
    walls = []
    for i in range(I + 1):            # layer i+1 (0-based i)
        top = stack.y_U if i == 0 else curve_height_at(curves[i - 1], -d / 2)
        bot = stack.y_D if i == I else curve_height_at(curves[i], -d / 2)
        y = gauss_legendre(stack.M_w, bot, top)
        walls.append((np.full(stack.M_w, -d / 2), y))
    xud = -d / 2 + d * (np.arange(stack.M_ud) + 0.5) / stack.M_ud
    y0s = [s.y0 for s in stack.interfaces]
    tops = [stack.y_U] + y0s
    bots = y0s + [stack.y_D]
    centres = np.array([[0.0, 0.5 * (t + b)] for t, b in zip(tops, bots)])
    return Geometry(d, curves, walls, xud, xud.copy(), stack.y_U, stack.y_D, centres, stack.R, stack.P)


def proxies(geom: Geometry, layer: int):
    """Proxy points and outward normals of layer ``layer`` (0-based)."""
    th = 2 * np.pi * np.arange(1, geom.P + 1) / geom.P
    cx, cy = geom.centres[layer]
    return cx + geom.R * np.cos(th), cy + geom.R * np.sin(th), np.cos(th), np.sin(th)
