"""Pins for the oracle's singular self blocks and its cornered interfaces
(no GPU).

* A row of the self block A_ii (all three copies, jump terms removed) applied
  to a smooth density is compared with the integral of the difference kernel
  against that density, computed by adaptive quadrature split at the target
  (scipy.integrate.quad).  For the smooth curve the density is a narrow
  Gaussian about the target, given per copy, so that targets next to the cell
  edge exercise the Alpert window that wraps into the neighbouring copies
  and no truncation of the three-copy sum enters.  For a cornered interface
  the segment-local block is applied to a smooth density on one graded
  segment (Kress exponent q = 8, where the graded rule converges fast
  enough to reach 1e-11).
* Whole solves on cornered stacks: a planar stack carried on graded
  segments must reproduce the Fresnel closed form, with the O(n^-q)
  convergence the grading promises (q = 6); a cornered stack conserves flux;
  a cornered stack with equal wavenumbers scatters nothing.
"""
import warnings

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads
from oracle import alpert, fills, fresnel, geometry, special

RULE = alpert.load_rule()
KM = (9.0, 12.5)


def _quad_split(fun, lo, mid, hi):
    tot = 0.0
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        for a, b in ((lo, mid), (mid, hi)):
            if b <= a:
                continue
            re = integrate.quad(lambda t: fun(t).real, a, b, limit=400, epsabs=1e-15, epsrel=1e-14)[0]
            im = integrate.quad(lambda t: fun(t).imag, a, b, limit=400, epsabs=1e-15, epsrel=1e-14)[0]
            tot += re + 1j * im
    return tot


def _kern(r2, nd, npd, nn):
    S, D, Ds, T = special.kernels_diff(KM[0], KM[1], np.array([r2]), np.array([nd]), np.array([npd]),
                                       np.array([nn]))
    return D[0], S[0], T[0], Ds[0]


BLOCKS = ((0, 0), (0, 1), (1, 0), (1, 1))   # (D, S; T, D*) in units of N


def test_smooth_self_rows_match_adaptive_quadrature():
    N, d, sig = 128, 1.0, 0.12
    iface = workloads.Interface("fourier", 0.0, n_nodes=N, cos_coef=np.array([0.03, -0.02, 0.01]),
                                sin_coef=np.array([0.05, 0.0, -0.015]))
    c = geometry.make_curve(iface, d)
    P = fills.self_pieces(c, KM[0], KM[1], RULE)
    P[1, :N, :N] += np.eye(N)
    P[1, N:, N:] -= np.eye(N)
    f = lambda x: c.f(np.array([x]))[0]
    fp = lambda x: c.fp(np.array([x]))[0]
    worst = 0.0
    for m in (0, 2, 64, 125, 127):                 # 0, 2, 125, 127 wrap into l = -1 / +1
        xm, ym, nxm, nym = c.x[m], c.y[m], c.nx[m], c.ny[m]
        dens = lambda x: np.exp(-((x - xm) / sig) ** 2) * np.exp(3j * x)
        tau = [dens(c.x + l * d) for l in (-1, 0, 1)]
        for which, (br, bc) in enumerate(BLOCKS):
            got = sum((P[li][br * N:(br + 1) * N, bc * N:(bc + 1) * N] @ tau[li])[m] for li in range(3))

            def integrand(x):
                fpx = fp(x)
                nu = np.sqrt(1 + fpx * fpx)
                dx, dy = xm - x, ym - f(x)
                k4 = _kern(dx * dx + dy * dy, nxm * dx + nym * dy, (fpx * dx - dy) / nu, (nxm * fpx - nym) / nu)
                return k4[which] * dens(x) * nu

            ref = _quad_split(integrand, xm - 1.0, xm, xm + 1.0)
            worst = max(worst, abs(got - ref) / max(abs(ref), 1e-2))
    assert worst < 1e-13


def test_polygon_segment_rows_match_adaptive_quadrature():
    d = 1.0
    vx, vy = np.array([-d / 2, 0.1, d / 2]), np.array([-0.08, 0.08, -0.08])
    iface = workloads.Interface("polygon", 0.0, vx=vx, vy=vy, seg_nodes=np.array([120, 140], np.int32), q=8.0)
    c = geometry.make_curve(iface, d)
    N = c.N
    P = fills.self_pieces(c, KM[0], KM[1], RULE)[1]
    P[:N, :N] += np.eye(N)
    P[N:, N:] -= np.eye(N)
    A, B = np.array([vx[0], vy[0]]), np.array([vx[1], vy[1]])
    L = np.hypot(*(B - A))
    t = (B - A) / L
    nrm = np.array([t[1], -t[0]])
    g = lambda u: np.exp(2j * u) * (1 + 0.3 * u)
    cols = np.arange(c.seg_start[0], c.seg_start[0] + c.seg_n[0])
    tau = np.zeros(N, complex)
    tau[cols] = g(np.hypot(c.x[cols] - A[0], c.y[cols] - A[1]))
    worst = 0.0
    for m in (0, 3, 30, 60, 116, 118):
        zm = np.array([c.x[m], c.y[m]])
        um = np.hypot(*(zm - A))
        for which, (br, bc) in enumerate(BLOCKS):
            got = P[br * N + m, bc * N + cols] @ tau[cols]
            if which in (0, 3):
                # double-layer kernels vanish on a straight segment
                assert abs(got) < 1e-14
                continue

            def integrand(u):
                dv = zm - (A + u * t)
                return _kern(dv @ dv, nrm @ dv, nrm @ dv, 1.0)[which] * g(u)

            ref = _quad_split(integrand, 0.0, um, L)
            worst = max(worst, abs(got - ref))
    assert worst < 2e-11


def _flat_err(nper):
    s = workloads.small_polygon_stack(flat=True, nper=nper)
    r = oracle.solve_stack(s)
    aU, aD, _ = fresnel.flat_stack_amplitudes(s.k, [0.0, -0.5], s.thetas[0], s.y_U, s.y_D)
    i0 = list(r.orders).index(0)
    others = max(np.max(np.abs(np.delete(r.aU, i0))), np.max(np.abs(np.delete(r.aD, i0))))
    return max(abs(r.aU[i0] - aU), abs(r.aD[i0] - aD), others)


def test_flat_graded_segments_match_fresnel_at_grading_order():
    e40, e80 = _flat_err(40), _flat_err(80)
    assert e80 < 3e-10
    # Kress grading with q = 6: the error falls like n^-6 (Sec. 2.5)
    assert np.log2(e40 / e80) > 5.0


def test_cornered_stack_conserves_flux():
    r = oracle.solve_stack(workloads.small_polygon_stack(nper=80))
    assert abs(r.flux_err) < 1e-9


def test_cornered_stack_with_equal_wavenumbers_is_transparent():
    s = workloads.small_polygon_stack(nper=80, k=(9.0, 9.0, 9.0))
    r = oracle.solve_stack(s)
    i0 = list(r.orders).index(0)
    assert np.max(np.abs(r.aU)) < 1e-9
    ref = np.exp(1j * s.k[0] * np.sin(s.thetas[0]) * s.y_D)
    assert abs(r.aD[i0] - ref) < 1e-9
    assert np.max(np.abs(np.delete(r.aD, i0))) < 1e-9
