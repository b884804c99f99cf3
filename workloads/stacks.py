"""Seeded synthetic stack generators (inputs only).

Geometry conventions shared by every consumer (they are part of the input
description, not of the method):

* period ``d``; the unit cell is ``-d/2 <= x < d/2``;
* interfaces are listed top (Gamma_1) to bottom (Gamma_I);
* a ``fourier`` interface is the graph
  ``y = y0 + sum_m cos_coef[m-1] cos(2 pi m x/d) + sin_coef[m-1] sin(2 pi m x/d)``;
* a ``polygon`` interface is the periodic broken line through the vertices
  ``(vx[c], vy[c])``, ``vx[0] = -d/2``, ``vx[-1] = d/2``, ``vy[0] = vy[-1]``,
  one straight segment per consecutive vertex pair, ``seg_nodes[c]`` nodes on
  segment ``c``, Kress grading exponent ``q``;
* ``k`` has I+1 real layer wavenumbers, top layer first;
* ``y_U`` / ``y_D`` are the heights of the upper / lower radiation lines.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np


@dataclass
class Interface:
    kind: str                      # "fourier" or "polygon"
    y0: float
    n_nodes: int = 0               # fourier: N_i
    cos_coef: np.ndarray = field(default_factory=lambda: np.zeros(0))
    sin_coef: np.ndarray = field(default_factory=lambda: np.zeros(0))
    vx: np.ndarray = field(default_factory=lambda: np.zeros(0))
    vy: np.ndarray = field(default_factory=lambda: np.zeros(0))
    seg_nodes: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int32))
    q: float = 6.0

    @property
    def N(self) -> int:
        if self.kind == "fourier":
            return int(self.n_nodes)
        return int(np.sum(self.seg_nodes))


@dataclass
class Stack:
    name: str
    d: float
    k: np.ndarray                  # (I+1,)
    interfaces: List[Interface]
    y_U: float
    y_D: float
    P: int
    R: float
    M_w: int
    M_ud: int
    K: int
    thetas: np.ndarray             # incident angles in (-pi, 0)
    ls_mu: float = 1e-14           # Tikhonov weight relative to ||Q||_F

    @property
    def I(self) -> int:
        return len(self.interfaces)

    @property
    def n_den(self) -> int:
        return 2 * sum(s.N for s in self.interfaces)

    @property
    def n_tot(self) -> int:
        return self.n_den + (self.I + 1) * self.P + 2 * (2 * self.K + 1)


def _scaled_fourier(rng: np.random.Generator, d: float, n_modes: int, peak: float):
    """Draw cos/sin coefficients ~ N(0,1) (cos first, then sin) and scale the
    profile so that its peak |value| on a 4096-point grid equals ``peak``."""
    a = rng.standard_normal(n_modes)
    b = rng.standard_normal(n_modes)
    x = -d / 2 + d * np.arange(4096) / 4096
    m = np.arange(1, n_modes + 1)[:, None]
    f = (a[:, None] * np.cos(2 * np.pi * m * x / d) + b[:, None] * np.sin(2 * np.pi * m * x / d)).sum(0)
    s = peak / np.max(np.abs(f))
    return a * s, b * s


def config1(N: int = 120, P: int = 60, M_w: int = 60, M_ud: int = 60, K: int = 25,
            amplitude: float = 0.3, k=(10.0, 13.0, 16.0)) -> Stack:
    """Three layers, two interfaces y = 0.3 sin x and y = -2 + 0.3 sin x, d = 2 pi."""
    d = 2 * np.pi
    ifs = [Interface("fourier", y0, n_nodes=N, cos_coef=np.zeros(1),
                     sin_coef=np.array([amplitude])) for y0 in (0.0, -2.0)]
    return Stack("config1", d, np.array(k, dtype=float), ifs, y_U=2.0, y_D=-4.0,
                 P=P, R=d, M_w=M_w, M_ud=M_ud, K=K, thetas=np.array([-np.pi / 6]))


def config1_flat(**kw) -> Stack:
    """Flat twin of config1 (amplitude 0): a 1-D layered problem."""
    s = config1(amplitude=0.0, **kw)
    s.name = "config1_flat"
    return s


def homogeneous(kval: float = 10.0, **kw) -> Stack:
    """config1 geometry with every layer at the same wavenumber."""
    s = config1(k=(kval, kval, kval), **kw)
    s.name = "homogeneous"
    return s


def config2(seed: int = 2, I: int = 50, N: int = 100, P: int = 50, M_w: int = 50,
            M_ud: int = 60, K: int = 25, wood_layer: Optional[int] = 26,
            theta: float = -np.pi / 6) -> Stack:
    """I random smooth interfaces (Fourier modes 1..5, peak 0.3, spacing 1.5),
    k_j = 10 n_j with n_j ~ U[1,2]; layer ``wood_layer`` (1-based) is retuned
    so that kappa_m = k_j exactly for some order m (a Wood anomaly).

    Draw order: for each interface top to bottom, 5 cos then 5 sin N(0,1)
    coefficients; then I+1 uniforms for n_j."""
    d = 2 * np.pi
    rng = np.random.default_rng(seed)
    ifs = []
    for i in range(I):
        a, b = _scaled_fourier(rng, d, 5, 0.3)
        ifs.append(Interface("fourier", -1.5 * i, n_nodes=N, cos_coef=a, sin_coef=b))
    n = rng.uniform(1.0, 2.0, I + 1)
    k = 10.0 * n
    if wood_layer is not None and 1 <= wood_layer <= I + 1:
        kappa0 = k[0] * math.cos(theta)
        g = 2 * np.pi / d
        j = wood_layer - 1
        m = round((k[j] - kappa0) / g)
        kw = kappa0 + m * g
        if kw > 20.0:
            kw -= g
        if kw < 10.0:
            kw += g
        k[j] = kw
    return Stack("config2", d, k, ifs, y_U=1.5, y_D=-1.5 * (I - 1) - 1.5, P=P, R=d,
                 M_w=M_w, M_ud=M_ud, K=K, thetas=np.array([theta]))


def small_stack(seed: int = 0, I: int = 3, N: int = 64, P: int = 40, M_w: int = 40,
                M_ud: int = 40, K: int = 8, d: float = 1.0, omega: float = 8.0,
                spacing: float = 0.5, peak: float = 0.08, theta: float = -np.pi / 5,
                n_modes: int = 3) -> Stack:
    """Small random smooth stack (paper-like scale: d = 1) for quick tests."""
    rng = np.random.default_rng(seed)
    ifs = []
    for i in range(I):
        a, b = _scaled_fourier(rng, d, n_modes, peak)
        ifs.append(Interface("fourier", -spacing * i, n_nodes=N, cos_coef=a, sin_coef=b))
    n = rng.uniform(1.0, 1.5, I + 1)
    n[0] = 1.0
    return Stack("small", d, omega * n, ifs, y_U=spacing, y_D=-spacing * I,
                 P=P, R=1.5 * d, M_w=M_w, M_ud=M_ud, K=K, thetas=np.array([theta]))


def _polygon(kind: str, y0: float, d: float, h: float, nseg: int):
    """Vertices of one period of a cornered profile of height ``h`` about y0."""
    if kind == "triangle":          # valley at x = +-d/2, peak at 0: 2 segments
        vx = np.array([-d / 2, 0.0, d / 2])
        vy = np.array([y0 - h, y0 + h, y0 - h])
    elif kind == "trapezoid":       # flat, up, top, down, flat: 5 segments
        vx = np.array([-d / 2, -d / 4, -d / 8, d / 8, d / 4, d / 2])
        vy = np.array([y0 - h, y0 - h, y0 + h, y0 + h, y0 - h, y0 - h])
    else:                           # triangle on a flat: 4 segments
        vx = np.array([-d / 2, -d / 6, 0.0, d / 6, d / 2])
        vy = np.array([y0 - h, y0 - h, y0 + h, y0 - h, y0 - h])
    return vx, vy


def config3(seed: int = 3, I: int = 1000, n_angles: int = 100, N_smooth: int = 120,
            N_corner: int = 250, P: int = 60, M_w: int = 60, M_ud: int = 60,
            K: int = 25) -> Stack:
    """I interfaces, a seeded 70/30 mix of smooth random-Fourier (N_smooth nodes)
    and cornered (N_corner nodes over 2-5 graded segments) profiles, spacing 1.5,
    k_j = 10 n_j with n_j ~ U[1,2], and ``n_angles`` angles uniform in (-pi/2, 0)."""
    d = 2 * np.pi
    rng = np.random.default_rng(seed)
    corner = rng.permutation(I) < int(round(0.3 * I))
    ifs = []
    kinds = ("triangle", "trapezoid", "tri_on_flat")
    for i in range(I):
        y0 = -1.5 * i
        a, b = _scaled_fourier(rng, d, 5, 0.3)
        kind = kinds[int(rng.integers(0, 3))]
        if not corner[i]:
            ifs.append(Interface("fourier", y0, n_nodes=N_smooth, cos_coef=a, sin_coef=b))
            continue
        vx, vy = _polygon(kind, y0, d, 0.3, 0)
        seglen = np.hypot(np.diff(vx), np.diff(vy))
        nodes = np.maximum(40, np.round(N_corner * seglen / seglen.sum()).astype(np.int32))
        nodes[np.argmax(nodes)] += N_corner - int(nodes.sum())
        ifs.append(Interface("polygon", y0, vx=vx, vy=vy, seg_nodes=nodes.astype(np.int32), q=6.0))
    n = rng.uniform(1.0, 2.0, I + 1)
    thetas = -(np.pi / 2) * (np.arange(n_angles) + 0.5) / n_angles
    return Stack("config3", d, 10.0 * n, ifs, y_U=1.5, y_D=-1.5 * (I - 1) - 1.5, P=P, R=d,
                 M_w=M_w, M_ud=M_ud, K=K, thetas=thetas)


def config4(seed: int = 4, n_stacks: int = 64, I_range=(10, 200), N_range=(60, 250), omega_range=(5.0, 20.0),
            n_range=(1.0, 2.5), P: int = 60, M_w: int = 60, M_ud: int = 60, K: int = 25,
            min_seg: int = 40, nodes_per_k: Optional[Tuple[float, float]] = None) -> List[Stack]:
    """``n_stacks`` independent stacks, each with I ~ U{I_range} interfaces of
    N ~ U{N_range} nodes (drawn per interface), a seeded 70/30 mix of smooth
    random-Fourier and cornered profiles (as config3; a cornered interface
    takes at least ``min_seg`` nodes per segment), spacing 1.5, d = 2 pi,
    k_j = omega n_j with omega ~ U[omega_range] per stack and
    n_j ~ U[n_range], and one incident angle ~ U(-pi/2, 0) per stack.

    ``nodes_per_k = (c_smooth, c_corner)`` raises an interface's drawn N to
    at least c k_max, k_max the larger wavenumber of the two layers it
    separates (the resolved variant; N stays uneven through the draw).

    Draw order per stack: I, omega, theta; then per interface N, the smooth /
    cornered choice, 5 cos and 5 sin N(0,1) coefficients and a shape index;
    then the I+1 layer indices."""
    d = 2 * np.pi
    rng = np.random.default_rng(seed)
    kinds = ("triangle", "trapezoid", "tri_on_flat")
    out = []
    for _ in range(n_stacks):
        I = int(rng.integers(I_range[0], I_range[1] + 1))
        omega = float(rng.uniform(*omega_range))
        theta = -float(rng.uniform(0.0, np.pi / 2))
        theta = min(max(theta, -np.pi / 2 + 1e-3), -1e-3)
        drawn = []
        for i in range(I):
            N = int(rng.integers(N_range[0], N_range[1] + 1))
            cornered = rng.uniform() < 0.3
            a, b = _scaled_fourier(rng, d, 5, 0.3)
            kind = kinds[int(rng.integers(0, 3))]
            drawn.append((N, cornered, a, b, kind))
        n = rng.uniform(n_range[0], n_range[1], I + 1)
        ifs = []
        for i, (N, cornered, a, b, kind) in enumerate(drawn):
            y0 = -1.5 * i
            if nodes_per_k is not None:
                kmax = omega * max(n[i], n[i + 1])
                N = max(N, int(math.ceil(nodes_per_k[1 if cornered else 0] * kmax)))
            if not cornered:
                ifs.append(Interface("fourier", y0, n_nodes=N, cos_coef=a, sin_coef=b))
                continue
            vx, vy = _polygon(kind, y0, d, 0.3, 0)
            seglen = np.hypot(np.diff(vx), np.diff(vy))
            N = max(N, min_seg * len(seglen))
            extra = N - min_seg * len(seglen)  # shared in proportion to segment length
            nodes = min_seg + np.floor(extra * seglen / seglen.sum()).astype(np.int32)
            nodes[np.argmax(seglen)] += N - int(nodes.sum())
            ifs.append(Interface("polygon", y0, vx=vx, vy=vy, seg_nodes=nodes.astype(np.int32), q=6.0))
        out.append(Stack("config4", d, omega * n, ifs, y_U=1.5, y_D=-1.5 * (I - 1) - 1.5, P=P, R=d,
                         M_w=M_w, M_ud=M_ud, K=K, thetas=np.array([theta])))
    return out


@dataclass
class ShapeProblem:
    """A stack parametrised for differentiation: interface i is the graph
    y = y0_i + sum_{m=1..M} c[i, m-1] sin(2 pi m x/d + psi[i, m-1]) with the
    phases psi fixed, and layer j has wavenumber k_j = omega n[j].  The
    parameters are the amplitudes c (I x M) and the indices n (I+1)."""
    c: np.ndarray
    psi: np.ndarray
    n: np.ndarray
    omega: float
    base: Stack                    # sizes, lines, proxies; its shapes and k are replaced

    @property
    def n_params(self) -> int:
        return self.c.size + self.n.size

    def params(self) -> np.ndarray:
        """Flat parameter vector: c row by row, then n."""
        return np.concatenate([self.c.ravel(), self.n])

    def stack(self, p: Optional[np.ndarray] = None) -> Stack:
        """The stack at parameter vector p (default: the problem's own)."""
        p = self.params() if p is None else np.asarray(p, float)
        c = p[:self.c.size].reshape(self.c.shape)
        n = p[self.c.size:]
        ifs = []
        for i, f in enumerate(self.base.interfaces):
            ifs.append(Interface("fourier", f.y0, n_nodes=f.n_nodes, cos_coef=c[i] * np.sin(self.psi[i]),
                                 sin_coef=c[i] * np.cos(self.psi[i])))
        b = self.base
        return Stack(b.name, b.d, self.omega * n, ifs, y_U=b.y_U, y_D=b.y_D, P=b.P, R=b.R, M_w=b.M_w,
                     M_ud=b.M_ud, K=b.K, thetas=b.thetas, ls_mu=b.ls_mu)


def config5(seed: int = 5, I: int = 100, N: int = 100, P: int = 50, M_w: int = 50, M_ud: int = 60, K: int = 25,
            omega: float = 10.0, n_modes: int = 5, n_angles: int = 10, spacing: float = 1.5,
            peak: float = 0.3) -> ShapeProblem:
    """The differentiation workload: I smooth interfaces, interface i the
    graph sum_{m=1..5} c_{i,m} sin(m x + psi_{i,m}) (d = 2 pi) about
    y0 = -spacing i, with c_{i,m} ~ N(0,1) scaled so that the profile's peak
    is ``peak`` and psi ~ U[0, 2 pi) fixed; n_j ~ U[1,2], k_j = omega n_j;
    ``n_angles`` angles theta_j = -(pi/3)(j - 1/2)/n_angles.

    Draw order: per interface 5 amplitudes then 5 phases; then I+1 indices."""
    d = 2 * np.pi
    rng = np.random.default_rng(seed)
    c = np.zeros((I, n_modes))
    psi = np.zeros((I, n_modes))
    xs = np.linspace(-d / 2, d / 2, 4096, endpoint=False)
    m = np.arange(1, n_modes + 1)
    for i in range(I):
        ci = rng.standard_normal(n_modes)
        pi_ = rng.uniform(0.0, 2 * np.pi, n_modes)
        prof = (ci[None, :] * np.sin(2 * np.pi * m[None, :] * xs[:, None] / d + pi_[None, :])).sum(1)
        c[i] = ci * peak / np.max(np.abs(prof))
        psi[i] = pi_
    n = rng.uniform(1.0, 2.0, I + 1)
    thetas = -(np.pi / 3) * (np.arange(n_angles) + 0.5) / n_angles
    ifs = [Interface("fourier", -spacing * i, n_nodes=N) for i in range(I)]
    base = Stack("config5", d, omega * n, ifs, y_U=spacing, y_D=-spacing * (I - 1) - spacing, P=P, R=d,
                 M_w=M_w, M_ud=M_ud, K=K, thetas=thetas)
    return ShapeProblem(c, psi, n, omega, base)


def small_shape_problem(seed: int = 12, I: int = 3, N: int = 64, P: int = 40, M_w: int = 40, M_ud: int = 40,
                        K: int = 8, omega: float = 8.0, peak: float = 0.06, n_modes: int = 3,
                        thetas=(-0.6, -1.1), flat: bool = False) -> ShapeProblem:
    """Paper-scale (d = 1) version of config5 for tests: spacing 0.5,
    n_0 = 1 in the top layer, n_j ~ U[1, 1.5] below; ``flat`` zeroes the
    amplitudes (the phases are still drawn)."""
    d = 1.0
    rng = np.random.default_rng(seed)
    c = np.zeros((I, n_modes))
    psi = np.zeros((I, n_modes))
    xs = np.linspace(-d / 2, d / 2, 4096, endpoint=False)
    m = np.arange(1, n_modes + 1)
    for i in range(I):
        ci = rng.standard_normal(n_modes)
        pi_ = rng.uniform(0.0, 2 * np.pi, n_modes)
        prof = (ci[None, :] * np.sin(2 * np.pi * m[None, :] * xs[:, None] / d + pi_[None, :])).sum(1)
        c[i] = 0.0 if flat else ci * peak / np.max(np.abs(prof))
        psi[i] = pi_
    n = rng.uniform(1.0, 1.5, I + 1)
    n[0] = 1.0
    ifs = [Interface("fourier", -0.5 * i, n_nodes=N) for i in range(I)]
    base = Stack("small_shape", d, omega * n, ifs, y_U=0.5, y_D=-0.5 * I, P=P, R=1.5 * d, M_w=M_w,
                 M_ud=M_ud, K=K, thetas=np.asarray(thetas, dtype=float))
    return ShapeProblem(c, psi, n, omega, base)


def small_polygon_stack(flat: bool = False, nper: int = 60, q: float = 6.0, k=(8.0, 10.0, 11.0),
                        P: int = 60, M_w: int = 40, M_ud: int = 40, K: int = 8,
                        height: float = 0.08, theta: float = -np.pi / 5) -> Stack:
    """Two cornered interfaces at d = 1: a triangle (2 segments, peak at x = 0)
    over a triangle-on-a-flat (4 segments), ``nper`` graded nodes per segment.
    ``flat=True`` puts every vertex at the interface's mean height, which gives
    a planar stack carried on graded segments."""
    d = 1.0
    ifs = []
    h = 0.0 if flat else height
    for i, y0 in enumerate((0.0, -0.5)):
        if i == 0:
            vx = np.array([-d / 2, 0.0, d / 2])
            vy = np.array([y0 - h, y0 + h, y0 - h])
        else:
            vx = np.array([-d / 2, -d / 6, 0.0, d / 6, d / 2])
            vy = np.array([y0 - h, y0 - h, y0 + h, y0 - h, y0 - h])
        ns = np.full(len(vx) - 1, nper, dtype=np.int32)
        ifs.append(Interface("polygon", y0, vx=vx, vy=vy, seg_nodes=ns, q=q))
    return Stack("small_polygon", d, np.array(k, dtype=float), ifs, y_U=0.5, y_D=-1.0, P=P, R=1.5 * d,
                 M_w=M_w, M_ud=M_ud, K=K, thetas=np.array([theta]))


def small_mixed_stack(seed: int = 7, I: int = 4, N_smooth: int = 72, seg_scale: int = 60,
                      P: int = 60, M_w: int = 40, M_ud: int = 40, K: int = 8, d: float = 1.0,
                      omega: float = 8.0, spacing: float = 0.5, peak: float = 0.08,
                      q: float = 6.0, theta: float = -np.pi / 5, min_seg: int = 40) -> Stack:
    """Paper-scale (d = 1) stack alternating smooth random-Fourier interfaces
    (N_smooth nodes) and cornered ones (triangle, trapezoid, triangle on a
    flat; about ``seg_scale`` graded nodes per unit of d along each segment,
    at least ``min_seg`` per segment): uneven node counts across the interfaces.

    Draw order: per interface, 3 cos then 3 sin N(0,1) coefficients, one
    shape index; then I+1 uniforms for the layer indices."""
    rng = np.random.default_rng(seed)
    kinds = ("triangle", "trapezoid", "tri_on_flat")
    ifs = []
    for i in range(I):
        y0 = -spacing * i
        a, b = _scaled_fourier(rng, d, 3, peak)
        kind = kinds[int(rng.integers(0, 3))]
        if i % 2 == 0:
            ifs.append(Interface("fourier", y0, n_nodes=N_smooth, cos_coef=a, sin_coef=b))
            continue
        vx, vy = _polygon(kind, y0, d, peak, 0)
        seglen = np.hypot(np.diff(vx), np.diff(vy))
        nodes = np.maximum(min_seg, np.round(seg_scale * seglen / d).astype(np.int32))
        ifs.append(Interface("polygon", y0, vx=vx, vy=vy, seg_nodes=nodes.astype(np.int32), q=q))
    n = rng.uniform(1.0, 1.5, I + 1)
    n[0] = 1.0
    return Stack("small_mixed", d, omega * n, ifs, y_U=spacing, y_D=-spacing * I,
                 P=P, R=1.5 * d, M_w=M_w, M_ud=M_ud, K=K, thetas=np.array([theta]))


def kappa_grid_thetas(stack: Stack, n_angles: int = 100, n_alpha: int = 20, span: float = 0.6) -> np.ndarray:
    """Incident angles whose kappa_0 = k_1 cos(theta) lie on a uniform grid of
    spacing 2 pi/(n_alpha d) centred on 0: the grid holds exactly n_alpha
    distinct Bloch phases alpha, each shared by every n_alpha-th angle.  The
    grid must fit in (-span k_1, span k_1).  Its offset (a multiple of
    spacing/64) keeps every order kappa_0 + 2 pi n/d furthest from the
    grazing points +-k_1 and +-k_{I+1}."""
    d = stack.d
    g = 2 * np.pi / (n_alpha * d)
    if (n_angles - 1) * g > 2 * span * stack.k[0]:
        raise ValueError("grid does not fit inside (-span k_1, span k_1)")
    base = -0.5 * (n_angles - 1) * g + g * np.arange(n_angles)
    period = 2 * np.pi / d
    best, off_best = -1.0, 0.0
    for t in range(64):
        off = g * t / 64
        worst = np.inf
        for kk in (stack.k[0], stack.k[-1]):
            for sgn in (1.0, -1.0):
                r = np.mod(base + off - sgn * kk, period)
                worst = min(worst, float(np.min(np.minimum(r, period - r))))
        if worst > best:
            best, off_best = worst, off
    return -np.arccos((base + off_best) / stack.k[0])
