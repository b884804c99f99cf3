"""Closed-form scattering by flat multilayers (test infrastructure only).

When every interface is the flat line y = y_i the problem is one-dimensional
(Sec. 1: planar layers reduce to 1-D).  With kappa0 = k_1 cos(theta) and
q_j = sqrt(k_j^2 - kappa0^2) (Re, Im >= 0), the exact solution is, up to the
common factor e^{i kappa0 x},

  layer 1      e^{-i q_1 y} + a^U e^{i q_1 (y - y_U)}
  layer j      A_j e^{-i q_j (y - y_{j-1})} + B_j e^{i q_j (y - y_j)}
  layer I+1    a^D e^{-i q_{I+1} (y - y_D)}

(each exponential referenced where it is bounded), and continuity of u and
du/dy at every y_i gives a 2I x 2I dense linear system.  Only the zeroth
Rayleigh-Bloch order is non-zero.  This is independent of the integral
equation machinery and pins the whole oracle on flat stacks.
"""
from __future__ import annotations

import numpy as np


def _solve(k, y_if, theta, y_U, y_D):
    k = np.asarray(k, float)
    I = len(y_if)
    kappa0 = k[0] * np.cos(theta)
    q = np.sqrt((k * k - kappa0 * kappa0).astype(complex))
    # unknowns: [aU, A_2, B_2, ..., A_I, B_I, aD]  (layers 2..I interior)
    nunk = 2 * I
    M = np.zeros((nunk, nunk), dtype=complex)
    rhs = np.zeros(nunk, dtype=complex)

    def layer_terms(j, y):
        """(value coeffs, derivative coeffs, value const, deriv const) of layer j at y."""
        v = np.zeros(nunk, dtype=complex)
        dv = np.zeros(nunk, dtype=complex)
        c = 0j
        dc = 0j
        if j == 0:
            e = np.exp(1j * q[0] * (y - y_U))
            v[0] = e
            dv[0] = 1j * q[0] * e
            c = np.exp(-1j * q[0] * y)
            dc = -1j * q[0] * c
        elif j == I:
            e = np.exp(-1j * q[I] * (y - y_D))
            v[nunk - 1] = e
            dv[nunk - 1] = -1j * q[I] * e
        else:
            ia, ib = 1 + 2 * (j - 1), 2 + 2 * (j - 1)
            ea = np.exp(-1j * q[j] * (y - y_if[j - 1]))
            eb = np.exp(1j * q[j] * (y - y_if[j]))
            v[ia], v[ib] = ea, eb
            dv[ia], dv[ib] = -1j * q[j] * ea, 1j * q[j] * eb
        return v, dv, c, dc

    for i in range(I):
        y = y_if[i]
        va, dva, ca, dca = layer_terms(i, y)
        vb, dvb, cb, dcb = layer_terms(i + 1, y)
        M[2 * i] = va - vb
        rhs[2 * i] = cb - ca
        M[2 * i + 1] = dva - dvb
        rhs[2 * i + 1] = dcb - dca
    sol = np.linalg.solve(M, rhs)
    return sol[0], sol[-1], q, sol


def flat_stack_total_field(k, y_if, theta, y_U, y_D, x, y):
    """Total field (incident included in layer 1) of the flat stack at the
    points (x, y), from the closed-form layer amplitudes above."""
    k = np.asarray(k, float)
    I = len(y_if)
    aU, aD, q, sol = _solve(k, y_if, theta, y_U, y_D)
    kappa0 = k[0] * np.cos(theta)
    x = np.atleast_1d(np.asarray(x, float))
    y = np.atleast_1d(np.asarray(y, float))
    out = np.zeros(x.size, dtype=complex)
    for t in range(x.size):
        yy = y[t]
        j = 0
        while j < I and yy < y_if[j]:
            j += 1
        if j == 0:
            v = np.exp(-1j * q[0] * yy) + aU * np.exp(1j * q[0] * (yy - y_U))
        elif j == I:
            v = aD * np.exp(-1j * q[I] * (yy - y_D))
        else:
            A, B = sol[1 + 2 * (j - 1)], sol[2 + 2 * (j - 1)]
            v = A * np.exp(-1j * q[j] * (yy - y_if[j - 1])) + B * np.exp(1j * q[j] * (yy - y_if[j]))
        out[t] = v * np.exp(1j * kappa0 * x[t])
    return out


def flat_stack_amplitudes(k, y_if, theta, y_U, y_D):
    """(a^U, a^D, q): the zeroth-order Bragg amplitudes and the vertical
    wavenumbers q_j of the flat stack."""
    aU, aD, q, _ = _solve(k, y_if, theta, y_U, y_D)
    return aU, aD, q
