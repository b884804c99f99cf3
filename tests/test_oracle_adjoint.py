"""Pins for the oracle's gradient of the zeroth-order reflected efficiency
(no GPU).

* On a flat stack the closed-form layered solution gives dJ/dn exactly:
  the oracle's derivative matches central differences of the closed form.
* On a flat stack a sinusoidal perturbation of any interface scatters into
  the orders +-m only at first order, so the zeroth order moves at second
  order: dJ/dc = 0 there.
* On a curved stack, halving the step changes the central differences by
  O(h^2) only (Richardson consistency of the derivative)."""
import numpy as np

import workloads
from oracle import adjoint, fresnel


def test_flat_stack_index_gradient_matches_closed_form():
    pb = workloads.small_shape_problem(flat=True, I=2, N=64, P=50, M_w=40, thetas=(-0.7,))
    nc = pb.c.size
    th = float(pb.base.thetas[0])
    y_if = [f.y0 for f in pb.base.interfaces]

    def J_closed(n):
        aU, _, _ = fresnel.flat_stack_amplitudes(pb.omega * n, y_if, th, pb.base.y_U, pb.base.y_D)
        return abs(aU) ** 2
    h = 1e-5
    for j in range(pb.n.size):
        e = np.zeros_like(pb.n)
        e[j] = h
        ref = (J_closed(pb.n + e) - J_closed(pb.n - e)) / (2 * h)
        g = adjoint.gradient_fd(pb, which=[nc + j], h=h)[0]
        assert abs(g - ref) < 1e-9 * max(1.0, abs(ref)), (j, g, ref)


def test_flat_stack_shape_gradient_vanishes():
    pb = workloads.small_shape_problem(flat=True, I=2, N=64, P=50, M_w=40, thetas=(-0.7,))
    nc = pb.c.size
    g_c = adjoint.gradient_fd(pb, which=range(nc), h=1e-4)
    g_n = adjoint.gradient_fd(pb, which=[nc + 1], h=1e-5)
    assert np.max(np.abs(g_c)) < 1e-8 * max(1.0, abs(g_n[0])), g_c


def test_curved_stack_central_differences_are_consistent():
    pb = workloads.small_shape_problem(I=2, N=64, P=50, M_w=40, thetas=(-0.7,))
    which = [0, 4, pb.c.size + 1]
    g1 = adjoint.gradient_fd(pb, which=which, h=2e-5)
    g2 = adjoint.gradient_fd(pb, which=which, h=1e-5)
    assert np.max(np.abs(g1 - g2)) < 1e-6 * np.max(np.abs(g2))
