"""Gradient of the summed zeroth-order reflected Bragg efficiency (test
infrastructure only).

The objective over incident angles theta_1..theta_m is
  J = sum_j e^U_0(theta_j),  e^U_0 = k^U_0 |a^U_0|^2 / (k_1 |sin theta|) = |a^U_0|^2
(eq. (86)'s efficiency of the zeroth reflected order; k^U_0 = k_1 |sin theta|
for that order).  Its parameters are those of workloads.ShapeProblem: the
sine amplitudes c of every interface and the layer indices n.

The oracle's gradient is the definition of the derivative taken on the
oracle's own forward map: central differences (J(p + h e_q) - J(p - h e_q))/2h
per parameter q, error O(h^2) from the truncation and O(eps_J/h) from the
forward map's rounding; with h ~ 1e-5 both stay below 1e-8 relative on the
test problems.  It is slow (two forward solves per parameter and angle) and
meant for small problems.
"""
from __future__ import annotations

import numpy as np

from .solve import solve_stack


def efficiency0(res) -> float:
    """|a^U_0|^2 of a solve (the zeroth order's reflected efficiency)."""
    return float(np.abs(res.aU[list(res.orders).index(0)]) ** 2)


def objective(problem, p=None, thetas=None) -> float:
    st = problem.stack(p)
    th = st.thetas if thetas is None else thetas
    return float(sum(efficiency0(solve_stack(st, theta=float(t))) for t in th))


def gradient_fd(problem, which=None, h: float = 1e-5, thetas=None) -> np.ndarray:
    """dJ/dp_q by central differences for the parameter indices `which`
    (default: all), step h."""
    p0 = problem.params()
    which = range(p0.size) if which is None else which
    out = []
    for q in which:
        e = np.zeros_like(p0)
        e[q] = h
        out.append((objective(problem, p0 + e, thetas) - objective(problem, p0 - e, thetas)) / (2 * h))
    return np.array(out)
