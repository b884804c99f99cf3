"""Pins for the oracle's field evaluation (no GPU), Sec. 3.3 last paragraph.

* Flat stack: the representation eq. (16)-(18) plus the incident wave in
  layer 1, and the Rayleigh-Bloch expansions eq. (7)-(8) outside U and D,
  equal the closed-form layered solution at points in every layer.
* Curved stack: (a) the layer-1 representation on the line U, and inside the
  proxy circle above it, equals the Rayleigh-Bloch expansion with the solved
  amplitudes at abscissae other than the collocation nodes (the same for the
  last layer and D); (b) every layer's representation is quasi-periodic
  across its walls, u(d/2, y) = alpha u(-d/2, y) eq. (6), at heights other
  than the wall collocation nodes; (c) targets outside the unit cell follow
  eq. (6)."""
import numpy as np

import oracle
import workloads
from oracle import field, fresnel
from oracle.geometry import make_geometry

RES = dict(N=160, P=140, M_w=100)


def _solved(stack):
    th = float(stack.thetas[0])
    res = oracle.solve_stack(stack, theta=th, keep_blocks=True)
    return th, res


def test_flat_stack_field_matches_closed_form():
    s = workloads.config1_flat(**RES)
    th, res = _solved(s)
    rng = np.random.default_rng(0)
    # points in every layer, 0.3 or more from the interfaces (y = 0, -2), and
    # above U (y_U = 2) and below D (y_D = -4)
    ys = np.concatenate([rng.uniform(0.3, 1.7, 6), rng.uniform(-1.7, -0.3, 6), rng.uniform(-3.7, -2.3, 6),
                         rng.uniform(2.0, 3.0, 3), rng.uniform(-5.0, -4.0, 3)])
    xs = rng.uniform(-s.d / 2, s.d / 2, ys.size)
    u, lay = field.field(s, th, xs, ys, res=res)
    tot = u + np.where(lay <= 0, field.incident(s, th, xs, ys), 0)
    ref = fresnel.flat_stack_total_field(s.k, [0.0, -2.0], th, s.y_U, s.y_D, xs, ys)
    assert set(lay) == {-1, 0, 1, 2, 3}
    assert np.max(np.abs(tot - ref)) < 1e-10 * np.max(np.abs(ref))


def test_curved_stack_representation_meets_rayleigh_bloch_on_U_and_D():
    s = workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9)
    th, res = _solved(s)
    geom = make_geometry(s)
    c = field.proxy_strengths(s, res)
    xs = np.linspace(-s.d / 2, s.d / 2, 13, endpoint=False) + 0.0123
    scale = max(np.max(np.abs(res.aU)), np.max(np.abs(res.aD)))
    for yoff in (0.0, 0.1):
        for x in xs:
            vu = field.layer_field(s, geom, res, c, 0, x, s.y_U + yoff)
            assert abs(vu - field.rb_field(s, res, True, x, s.y_U + yoff)) < 1e-10 * scale
            vd = field.layer_field(s, geom, res, c, s.I, x, s.y_D - yoff)
            assert abs(vd - field.rb_field(s, res, False, x, s.y_D - yoff)) < 1e-10 * scale


def test_curved_stack_layers_are_quasi_periodic_across_their_walls():
    s = workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9)
    th, res = _solved(s)
    geom = make_geometry(s)
    c = field.proxy_strengths(s, res)
    alpha = np.exp(1j * s.d * s.k[0] * np.cos(th))
    worst, scale = 0.0, 0.0
    for j in range(s.I + 1):
        top = s.y_U if j == 0 else s.interfaces[j - 1].y0 - 0.1
        bot = s.y_D if j == s.I else s.interfaces[j].y0 + 0.1
        for y in np.linspace(bot, top, 7)[1:-1] + 0.0071:
            l = field.layer_field(s, geom, res, c, j, -s.d / 2, y)
            r = field.layer_field(s, geom, res, c, j, s.d / 2, y)
            worst = max(worst, abs(r - alpha * l))
            scale = max(scale, abs(l))
    assert worst < 1e-8 * scale


def test_targets_outside_the_cell_follow_quasi_periodicity():
    s = workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9)
    th, res = _solved(s)
    alpha = np.exp(1j * s.d * s.k[0] * np.cos(th))
    x0 = np.array([0.13, -0.21, 0.4])
    y0 = np.array([-0.27, -1.22, 0.31])
    u0, _ = field.field(s, th, x0, y0, res=res)
    u2, _ = field.field(s, th, x0 + 2 * s.d, y0, res=res)
    um, _ = field.field(s, th, x0 - s.d, y0, res=res)
    assert np.allclose(u2, alpha ** 2 * u0, rtol=1e-13, atol=0)
    assert np.allclose(um, u0 / alpha, rtol=1e-13, atol=0)
