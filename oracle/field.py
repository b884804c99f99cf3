"""Field evaluation from a solved stack (test infrastructure only).

Sec. 3.3, last paragraph: once the densities and proxy strengths are known,
the scattered field in layer j is its representation eq. (16)-(18): the
near-field single- and double-layer potentials of the interfaces bounding
the layer,
each summed over the three copies l = -1, 0, 1 with phase alpha^l (eq. (14)),
plus the layer's proxy expansion sum_p c_p phi_p with the combined-field
basis phi_p = dG/dn_p + i k G (eq. (15)), all at the layer's wavenumber.
Above the line U and below the line D the scattered field is the truncated
Rayleigh-Bloch expansion (eq. (7)-(8)) with the computed Bragg amplitudes.
The discrete potentials use the same plain quadrature as the Nystrom
off-diagonal entries (weights w_j), which is accurate for targets a few node
spacings away from every interface.

Targets outside the unit cell are mapped into it by quasi-periodicity,
u(x + m d, y) = alpha^m u(x, y) (eq. (6)).

The proxy strengths come from the layer least-squares solutions of the
solve: [c_1; a^U] = -X_1 eta_1, c_j = -X_j [eta_{j-1}; eta_j],
[c_{I+1}; a^D] = -X_{I+1} eta_I (Sec. 3.2-3.3).
"""
from __future__ import annotations

import numpy as np

from . import special
from .geometry import curve_height_at, make_geometry, proxies
from .solve import solve_stack


def proxy_strengths(stack, res) -> list:
    """c_j (P complex) for layers j = 0..I (0-based), from a solve kept with
    its blocks (solve_stack(..., keep_blocks=True))."""
    X, eta, P, I = res.blocks["X"], res.eta, stack.P, stack.I
    out = [-(X[0] @ eta[0])[:P]]
    for j in range(1, I):
        out.append(-(X[j] @ np.concatenate([eta[j - 1], eta[j]]))[:P])
    out.append(-(X[I] @ eta[I - 1])[:P])
    return out


def layer_index(stack, geom, x: float, y: float) -> int:
    """-1 above U, 0..I for the layers top to bottom, I+1 below D; x in the
    unit cell."""
    if y >= stack.y_U:
        return -1
    if y <= stack.y_D:
        return stack.I + 1
    for i, c in enumerate(geom.curves):
        if y > curve_height_at(c, x):
            return i
    return stack.I


def _layer_potential(c, k, alpha, tx, ty, tau, sigma):
    """sum_l alpha^l sum_j w_j [D(t, z_j + l d) tau_j + S(t, z_j + l d) sigma_j]."""
    tot = 0j
    for l in (-1, 0, 1):
        dx = tx - (c.x + l * c.d)
        dy = ty - c.y
        r2 = dx * dx + dy * dy
        npd = c.nx * dx + c.ny * dy
        S, D, _, _ = special.kernels(k, r2, np.zeros_like(r2), npd, np.zeros_like(r2))
        tot += alpha ** l * np.sum(c.w * (D * tau + S * sigma))
    return tot


def layer_field(stack, geom, res, c, j: int, xc: float, yc: float) -> complex:
    """Representation eq. (16)-(18) of layer j (0-based) at (xc, yc), wherever
    the point is: the layer potentials of the interfaces above (j-1) and below
    (j) over three copies, plus the layer's proxy expansion."""
    I = stack.I
    k = float(stack.k[j])
    alpha = np.exp(1j * stack.d * stack.k[0] * np.cos(res.theta))
    v = 0j
    for i in (j - 1, j):
        if 0 <= i < I:
            cv = geom.curves[i]
            v += _layer_potential(cv, k, alpha, xc, yc, res.eta[i][:cv.N], res.eta[i][cv.N:])
    px, py, pnx, pny = proxies(geom, j)
    dx, dy = xc - px, yc - py
    r2 = dx * dx + dy * dy
    S, D, _, _ = special.kernels(k, r2, np.zeros_like(r2), pnx * dx + pny * dy, np.zeros_like(r2))
    return v + np.sum(c[j] * (D + 1j * k * S))


def rb_field(stack, res, upper: bool, xc: float, yc: float) -> complex:
    """Truncated Rayleigh-Bloch expansion eq. (7) above U or eq. (8) below D."""
    kappa = stack.k[0] * np.cos(res.theta) + 2 * np.pi * res.orders / stack.d
    if upper:
        return complex(np.sum(res.aU * np.exp(1j * (kappa * xc + res.kU * (yc - stack.y_U)))))
    return complex(np.sum(res.aD * np.exp(1j * (kappa * xc - res.kD * (yc - stack.y_D)))))


def field(stack, theta: float, x, y, res=None):
    """Scattered field u at the targets (x[k], y[k]); returns (u, layer)."""
    if res is None:
        res = solve_stack(stack, theta=theta, keep_blocks=True)
    geom = make_geometry(stack)
    d, I = stack.d, stack.I
    alpha = np.exp(1j * d * stack.k[0] * np.cos(theta))
    c = proxy_strengths(stack, res)
    x = np.atleast_1d(np.asarray(x, float))
    y = np.atleast_1d(np.asarray(y, float))
    u = np.zeros(x.size, dtype=complex)
    lay = np.zeros(x.size, dtype=int)
    for t in range(x.size):
        m = np.floor((x[t] + d / 2) / d)
        xc = x[t] - m * d
        j = layer_index(stack, geom, xc, y[t])
        lay[t] = j
        if j == -1 or j == I + 1:
            v = rb_field(stack, res, j == -1, xc, y[t])
        else:
            v = layer_field(stack, geom, res, c, j, xc, y[t])
        u[t] = alpha ** m * v
    return u, lay


def incident(stack, theta: float, x, y):
    """exp(i k_1 (cos theta x + sin theta y)) (eq. (1))."""
    k1 = float(stack.k[0])
    return np.exp(1j * k1 * (np.cos(theta) * np.asarray(x) + np.sin(theta) * np.asarray(y)))
