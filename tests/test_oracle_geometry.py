"""Pins for the oracle's quadrature geometry (no GPU)."""
import numpy as np
import pytest
from scipy import integrate

import workloads
from oracle import geometry


def _curve():
    s = workloads.config2(I=2)
    return geometry.make_curve(s.interfaces[0], s.d), s.d


def test_fourier_weights_integrate_arclength():
    c, d = _curve()
    L, _ = integrate.quad(lambda x: np.sqrt(1 + c.fp(np.array([x]))[0] ** 2), -d / 2, d / 2,
                          limit=200, epsabs=1e-14, epsrel=1e-14)
    assert abs(c.w.sum() - L) < 1e-12 * L


def test_normals_unit_down_and_orthogonal():
    c, d = _curve()
    assert np.allclose(c.nx ** 2 + c.ny ** 2, 1.0, atol=1e-15)
    assert np.all(c.ny < 0)
    # tangent (1, f') is orthogonal to the normal
    assert np.max(np.abs(c.nx * 1.0 + c.ny * c.fp(c.x))) < 1e-14


def test_difference_identities_against_mpmath():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    c, d = _curve()
    om = [2 * mp.pi * (m + 1) / d for m in range(len(c.cos_coef))]

    def f(x):
        return mp.fsum(mp.mpf(a) * mp.cos(w * x) + mp.mpf(b) * mp.sin(w * x)
                       for a, b, w in zip(c.cos_coef, c.sin_coef, om))

    def fp(x):
        return mp.fsum(w * (-mp.mpf(a) * mp.sin(w * x) + mp.mpf(b) * mp.cos(w * x))
                       for a, b, w in zip(c.cos_coef, c.sin_coef, om))

    for x0, h in ((0.3, 1e-9), (-2.9, 3e-6), (1.1, 0.04), (2.0, -1e-7), (0.0, 0.7)):
        X, H = mp.mpf(x0), mp.mpf(h)
        ed = f(X + H) - f(X)
        er = ed - H * fp(X)
        gd = c.fdiff(np.array([x0]), np.array([h]))[0]
        gr = c.fremainder(np.array([x0]), np.array([h]))[0]
        assert abs(gd - float(ed)) <= 1e-15 * abs(float(ed)) + 1e-300
        assert abs(gr - float(er)) <= 1e-13 * abs(float(er)) + 1e-300


def test_kress_grading_endpoints():
    for q in (4.0, 6.0, 8.0):
        w, wp = geometry.kress_w(np.array([0.0, np.pi, 2 * np.pi]), q)
        assert abs(w[0]) < 1e-15 and abs(w[1] - np.pi) < 1e-14 and abs(w[2] - 2 * np.pi) < 1e-14
        # w' vanishes at the end points and w is increasing in between
        assert abs(wp[0]) < 1e-14 and abs(wp[2]) < 1e-14
        s = np.linspace(1e-3, 2 * np.pi - 1e-3, 500)
        ws, wps = geometry.kress_w(s, q)
        assert np.all(np.diff(ws) >= 0) and np.all(wps > 0)
        # w' integrates to 2 pi
        val, _ = integrate.quad(lambda t: geometry.kress_w(np.array([t]), q)[1][0], 0, 2 * np.pi)
        assert abs(val - 2 * np.pi) < 1e-10


def test_polygon_segments_arclength():
    s = workloads.config3(I=20, n_angles=1)
    for iface in s.interfaces:
        if iface.kind != "polygon":
            continue
        c = geometry.make_curve(iface, s.d)
        L = np.sum(np.hypot(np.diff(iface.vx), np.diff(iface.vy)))
        assert abs(c.w.sum() - L) < 1e-8 * L
        assert np.allclose(c.nx ** 2 + c.ny ** 2, 1.0)


def test_unknown_count_matches_printed_matrix_sizes():
    # Sec. 4.2: Table 1 structure at I = 1000 gives a 468260 x 287922 matrix
    # (triangles every 8th interface from the 4th, rectangles every 15th from
    # the 4th and winning ties; sine N = 70, triangle 100 x 2, rectangle 100 x 5;
    # P = 60, M_w = 120, M = 60, K = 20).
    I, P, Mw, M, K = 1000, 60, 120, 60, 20
    Ns = []
    for i in range(1, I + 1):
        if i >= 4 and (i - 4) % 15 == 0:
            Ns.append(500)
        elif i >= 4 and (i - 4) % 8 == 0:
            Ns.append(200)
        else:
            Ns.append(70)
    n_den = 2 * sum(Ns)
    rows = n_den + 2 * Mw * (I + 1) + 4 * M
    cols = n_den + (I + 1) * P + 2 * (2 * K + 1)
    assert (rows, cols) == (468260, 287922)


def test_batch_workload_is_within_the_library_limits():
    # the 64-stack batch: every interface has 37..512 nodes and every polygon
    # segment at least 37 (the Alpert window plus its stencil)
    import workloads
    stacks = workloads.config4()
    assert len(stacks) == 64
    for st in stacks:
        assert 10 <= st.I <= 200
        for f in st.interfaces:
            assert 37 <= f.N <= 512
            if f.kind == "polygon":
                assert int(np.min(f.seg_nodes)) >= 37 and int(np.sum(f.seg_nodes)) == f.N
    # the resolved variant: omega in [5, 8], I in 10..100, the same draws
    # otherwise, every interface at least 18 k_max (smooth) or 25 k_max
    # (cornered) nodes and still within the limits
    kw = dict(omega_range=(5.0, 8.0), I_range=(10, 100), P=140, M_w=100)
    res = workloads.config4(nodes_per_k=(18.0, 25.0), **kw)
    for st, st0 in zip(res, workloads.config4(**kw)):
        assert 10 <= st.I <= 100 and st.I == st0.I and st.thetas[0] == st0.thetas[0]
        assert np.all(st.k <= 8.0 * 2.5)
        for i, (f, f0) in enumerate(zip(st.interfaces, st0.interfaces)):
            assert f.kind == f0.kind and f.N >= f0.N and 37 <= f.N <= 512
            kmax = max(st.k[i], st.k[i + 1])
            assert f.N >= (18.0 if f.kind == "fourier" else 25.0) * kmax - 1e-9
            if f.kind == "polygon":
                assert int(np.min(f.seg_nodes)) >= 37 and int(np.sum(f.seg_nodes)) == f.N
