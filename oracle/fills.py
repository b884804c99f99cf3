"""Matrix blocks of the discretised coupled system (test infrastructure only).

Each function returns either an alpha-independent *piece* or a block already
combined with the Bloch phase alpha.  Pieces follow the sweep splitting of
Sec. 3.4: every operator with neighbour sums is sum_{l=-1..1} alpha^l P_l
(eq. (19)-(20)); wall blocks are alpha^{-2} C_R - alpha C_L (eq. (42)-(44))
and alpha^{-1} Q_R - Q_L (eq. (45), (61)).

Layer-potential blocks map [tau; sigma] on the source curve to
[values; normal derivatives] at the targets:  [[D, S], [T, D*]] with the
source quadrature weights folded in (Sec. 2.5, Nystrom).

Self blocks A_ii (eq. (37)) use the difference kernels of layers i and i+1,
plain trapezoid entries outside the Alpert window |J - m| >= a of the
extended three-copy index J = j + l N, and Alpert's auxiliary-node correction
inside it, with 16-point Lagrange interpolation of the density from the
nodes; stencil nodes that fall in the neighbouring copies carry alpha^{+-1}
(Sec. 2.5 and its Remark on the quasi-periodic wrap).  The jump terms give
-I on the (tau, tau) block and +I on the (sigma, sigma) block.  Cornered
interfaces apply the correction per graded segment (see
_self_pieces_polygon).
"""
from __future__ import annotations

import numpy as np

from . import special
from .geometry import Curve, Geometry, kress_w, kress_wc, proxies

STENCIL = 16


# --------------------------------------------------------------------------
# geometry helpers
# --------------------------------------------------------------------------
def _pair_geom(tx, ty, tnx, tny, sx, sy, snx, sny):
    """Separation invariants for targets (rows) x sources (cols)."""
    dx = tx[:, None] - sx[None, :]
    dy = ty[:, None] - sy[None, :]
    r2 = dx * dx + dy * dy
    nd = tnx[:, None] * dx + tny[:, None] * dy
    npd = snx[None, :] * dx + sny[None, :] * dy
    nn = tnx[:, None] * snx[None, :] + tny[:, None] * sny[None, :]
    return r2, nd, npd, nn


def _self_geom_fourier(c: Curve, m, dxs):
    """Invariants for target node m and a source on the same smooth curve at
    abscissa x_m + dxs (any shape broadcast with m).  Returns r2, nd, npd, nn
    and the source speed factor nu_s = sqrt(1 + f'(x_s)^2)."""
    xm = c.x[m]
    xs = xm + dxs
    fm = c.fp(xm)
    fs = c.fp(xs)
    num = np.sqrt(1 + fm * fm)
    nus = np.sqrt(1 + fs * fs)
    df = c.fdiff(xm, dxs)
    r2 = dxs * dxs + df * df
    nd = c.fremainder(xm, dxs) / num
    npd = -c.fremainder(xs, -dxs) / nus
    nn = (fm * fs + 1) / (num * nus)
    return r2, nd, npd, nn, nus


def _lp_block(S, D, Ds, T, w):
    """[[D, S], [T, D*]] with source weights w on the columns."""
    return np.block([[D * w, S * w], [T * w, Ds * w]])


# --------------------------------------------------------------------------
# A blocks
# --------------------------------------------------------------------------
def self_pieces(c: Curve, ka: float, kb: float, rule) -> np.ndarray:
    """Pieces P_l (l = -1, 0, 1) of A_ii, each 2N x 2N (identity in P_0)."""
    if c.kind != "fourier":
        return _self_pieces_polygon(c, ka, kb, rule)
    N, d = c.N, c.d
    chi, u, a = rule
    out = np.zeros((3, 2 * N, 2 * N), dtype=complex)
    m = np.arange(N)
    # plain trapezoid part, outside the window |J - m| < a
    for li, l in enumerate((-1, 0, 1)):
        J = np.arange(N) + l * N
        off = J[None, :] - m[:, None]
        mask = np.abs(off) >= a
        dxs = off * (d / N)
        mm = np.broadcast_to(m[:, None], off.shape)
        offs = np.where(mask, dxs, d)          # dummy separation inside the window
        r2, nd, npd, nn, _ = _self_geom_fourier(c, mm, offs)
        S, D, Ds, T = special.kernels_diff(ka, kb, r2, nd, npd, nn)
        blk = _lp_block(S, D, Ds, T, c.w[None, :])
        out[li] += blk * np.tile(mask, (2, 2))
    # Alpert correction: 2 x 15 auxiliary nodes per target
    for sgn in (1.0, -1.0):
        t = m[:, None] + sgn * chi[None, :]                     # N x 15, index units
        dxs = sgn * chi[None, :] * (d / N) + 0 * m[:, None]
        mm = np.broadcast_to(m[:, None], t.shape)
        r2, nd, npd, nn, nus = _self_geom_fourier(c, mm, dxs)
        S, D, Ds, T = special.kernels_diff(ka, kb, r2, nd, npd, nn)
        aw = u[None, :] * (d / N) * nus                          # aux weights
        j0 = np.floor(t).astype(int) - (STENCIL // 2 - 1)
        for q in range(STENCIL):
            Jq = j0 + q
            Lq = np.ones_like(t)
            for r in range(STENCIL):
                if r != q:
                    Lq = Lq * (t - (j0 + r)) / (q - r)
            coef = aw * Lq
            l = np.floor_divide(Jq, N)
            col = Jq - l * N
            for kk in range(len(chi)):
                rows = m
                cols = col[:, kk]
                li = l[:, kk] + 1
                cf = coef[:, kk]
                np.add.at(out, (li, rows, cols), D[:, kk] * cf)
                np.add.at(out, (li, rows, N + cols), S[:, kk] * cf)
                np.add.at(out, (li, N + rows, cols), T[:, kk] * cf)
                np.add.at(out, (li, N + rows, N + cols), Ds[:, kk] * cf)
    out[1, :N, :N] -= np.eye(N)
    out[1, N:, N:] += np.eye(N)
    return out


def _self_pieces_polygon(c: Curve, ka, kb, rule):
    """Pieces of A_ii for a cornered interface (Sec. 2.5).

    Every segment carries its own Kress-graded trapezoid rule in the segment
    parameter s in [0, 2 pi).  Interactions between different segments, and
    all interactions with the neighbouring copies l = +-1, are plain Nystrom
    entries.  Within one segment the rule is treated as periodic in s with no
    Bloch phase (the graded Jacobian vanishes to high order at both segment
    ends, so the integrand continues smoothly across s = 0 ~ 2 pi): entries
    with cyclic segment-local index distance < a are replaced by Alpert's
    auxiliary nodes s_m +- chi_k h.  What is interpolated to the auxiliary
    nodes is the product of the density and the graded Jacobian |Z'(w(s))|
    w'(s), which is smooth and periodic in s, whereas the density alone is not
    continuous across the segment ends; the auxiliary weight is then u_k and
    the interpolation weights multiply the node weights w_j."""
    N, d = c.N, c.d
    chi, u, a = rule
    out = np.zeros((3, 2 * N, 2 * N), dtype=complex)
    seg = c.seg_of
    loc = np.arange(N) - c.seg_start[seg]            # segment-local index
    nseg = c.seg_n[seg]
    for li, l in enumerate((-1, 0, 1)):
        r2, nd, npd, nn = _pair_geom(c.x, c.y, c.nx, c.ny, c.x + l * d, c.y, c.nx, c.ny)
        mask = np.ones((N, N), dtype=bool)
        if l == 0:
            same = seg[:, None] == seg[None, :]
            dist = np.mod(loc[None, :] - loc[:, None], nseg[:, None])
            cyc = np.minimum(dist, nseg[:, None] - dist)
            mask = ~(same & (cyc < a))
        r2 = np.where(mask, r2, 1.0)                 # dummy separation inside the window
        S, D, Ds, T = special.kernels_diff(ka, kb, r2, nd, npd, nn)
        out[li] += _lp_block(S, D, Ds, T, c.w[None, :]) * np.tile(mask, (2, 2))
    # Alpert correction on each straight segment: the separation from node m
    # to the point at parameter s is (w(s_m) - w(s))/(2 pi) times the chord,
    # orthogonal to the (constant) normal
    for sg in range(len(c.seg_n)):
        n = int(c.seg_n[sg])
        s0 = int(c.seg_start[sg])
        L = np.hypot(c.vx[sg + 1] - c.vx[sg], c.vy[sg + 1] - c.vy[sg])
        h = 2 * np.pi / n
        m = np.arange(n)
        sm = h * (m + 0.5)
        wm, _ = kress_w(sm, c.q)
        wcm = kress_wc(sm, c.q)
        for sgn in (1.0, -1.0):
            t = m[:, None] + sgn * chi[None, :]                  # local index units
            sa = np.mod(h * (t + 0.5), 2 * np.pi)
            wa, _ = kress_w(sa, c.q)
            wca = kress_wc(sa, c.q)
            # near the far corner both w round to 2 pi: use the complements
            far = (sm[:, None] >= np.pi) & (sa >= np.pi)
            dw = np.where(far, wca - wcm[:, None], wm[:, None] - wa) / (2 * np.pi) * L
            zero = np.zeros_like(dw)
            S, D, Ds, T = special.kernels_diff(ka, kb, dw * dw, zero, zero, zero + 1.0)
            j0 = np.floor(t).astype(int) - (STENCIL // 2 - 1)
            for q in range(STENCIL):
                Jq = j0 + q
                Lq = np.ones_like(t)
                for r in range(STENCIL):
                    if r != q:
                        Lq = Lq * (t - (j0 + r)) / (q - r)
                cols = s0 + np.mod(Jq, n)
                coef = u[None, :] * Lq * c.w[cols]
                rows = np.broadcast_to(s0 + m[:, None], t.shape)
                for blk_r, blk_c, K in ((0, 0, D), (0, N, S), (N, 0, T), (N, N, Ds)):
                    np.add.at(out, (1, blk_r + rows, blk_c + cols), K * coef)
    out[1, :N, :N] -= np.eye(N)
    out[1, N:, N:] += np.eye(N)
    return out


def pair_pieces(ct: Curve, cs: Curve, k: float) -> np.ndarray:
    """Pieces of [[D~, S~], [T~, D~*]]^k from source curve cs to targets on ct
    (plain Nystrom, three copies), shape (3, 2 Nt, 2 Ns)."""
    out = np.zeros((3, 2 * ct.N, 2 * cs.N), dtype=complex)
    for li, l in enumerate((-1, 0, 1)):
        r2, nd, npd, nn = _pair_geom(ct.x, ct.y, ct.nx, ct.ny, cs.x + l * cs.d, cs.y, cs.nx, cs.ny)
        S, D, Ds, T = special.kernels(k, r2, nd, npd, nn)
        out[li] = _lp_block(S, D, Ds, T, cs.w[None, :])
    return out


# --------------------------------------------------------------------------
# proxy, wall and radiation blocks
# --------------------------------------------------------------------------
def proxy_block(tx, ty, tnx, tny, prox, k: float) -> np.ndarray:
    """[phi_p; d phi_p/dn] at the targets, phi_p = dG/dn_p + i k G (eq. (15))."""
    px, py, pnx, pny = prox
    r2, nd, npd, nn = _pair_geom(tx, ty, tnx, tny, px, py, pnx, pny)
    S, D, Ds, T = special.kernels(k, r2, nd, npd, nn)
    return np.vstack([D + 1j * k * S, T + 1j * k * Ds])


def wall_C_pieces(wall, cs: Curve, k: float) -> np.ndarray:
    """(C_R, C_L): targets x_m + 2d and x_m - d on the left wall, normal (1,0)
    (eq. (42)-(44): alpha^{-1} u(R) - u(L) reduces to two far copies)."""
    wx, wy = wall
    one, zero = np.ones_like(wx), np.zeros_like(wx)
    out = []
    for shift in (2 * cs.d, -cs.d):
        r2, nd, npd, nn = _pair_geom(wx + shift, wy, one, zero, cs.x, cs.y, cs.nx, cs.ny)
        S, D, Ds, T = special.kernels(k, r2, nd, npd, nn)
        out.append(_lp_block(S, D, Ds, T, cs.w[None, :]))
    return np.stack(out)


def wall_Q_pieces(wall, prox, k: float, d: float) -> np.ndarray:
    """(Q_R, Q_L): proxy fields at x_m + d and at x_m, normal (1,0) (eq. (61))."""
    wx, wy = wall
    one, zero = np.ones_like(wx), np.zeros_like(wx)
    return np.stack([proxy_block(wx + shift, wy, one, zero, prox, k) for shift in (d, 0.0)])


def rad_Z_pieces(xs, yline: float, cs: Curve, k: float) -> np.ndarray:
    """Pieces of Z_U or Z_D: layer potentials of one interface at the
    radiation-line nodes with the upward normal (0, 1) (Sec. 2.4)."""
    out = np.zeros((3, 2 * len(xs), 2 * cs.N), dtype=complex)
    one, zero = np.ones_like(xs), np.zeros_like(xs)
    ys = np.full_like(xs, yline)
    for li, l in enumerate((-1, 0, 1)):
        r2, nd, npd, nn = _pair_geom(xs, ys, zero, one, cs.x + l * cs.d, cs.y, cs.nx, cs.ny)
        S, D, Ds, T = special.kernels(k, r2, nd, npd, nn)
        out[li] = _lp_block(S, D, Ds, T, cs.w[None, :])
    return out


def rb_orders(k1: float, theta: float, d: float, K: int):
    """Orders n with kappa_n = k1 cos(theta) + 2 pi n/d nearest 0 (2K+1 of them)."""
    kappa0 = k1 * np.cos(theta)
    n0 = int(np.floor(-kappa0 * d / (2 * np.pi) + 0.5))
    n = np.arange(n0 - K, n0 + K + 1)
    return n, kappa0 + 2 * np.pi * n / d


def vertical_wavenumbers(k: float, kappa: np.ndarray) -> np.ndarray:
    """k_n = sqrt(k^2 - kappa_n^2), branch Re >= 0 and Im >= 0 (Sec. 1);
    |k^2 - kappa^2| <= 1e-14 k^2 is treated as grazing (k_n = 0)."""
    q = k * k - kappa * kappa
    kn = np.sqrt(q.astype(complex))
    kn[np.abs(q) <= 1e-14 * k * k] = 0.0
    return kn


def rad_W(xs, kappa, kn, upper: bool) -> np.ndarray:
    """W_U = -[e^{i kappa x}; i k^U e^{i kappa x}], W_D = -[e; -i k^D e] (eq. (59))."""
    e = np.exp(1j * kappa[None, :] * xs[:, None])
    s = 1.0 if upper else -1.0
    return -np.vstack([e, s * 1j * kn[None, :] * e])


def rhs_f(c1: Curve, k1: float, theta: float) -> np.ndarray:
    """f_1 = [-u_inc; -du_inc/dn] on Gamma_1 (Sec. 2.2, eq. (1))."""
    kx, ky = k1 * np.cos(theta), k1 * np.sin(theta)
    ui = np.exp(1j * (kx * c1.x + ky * c1.y))
    dui = 1j * (kx * c1.nx + ky * c1.ny) * ui
    return np.concatenate([-ui, -dui])


# --------------------------------------------------------------------------
# all alpha-independent pieces of one stack
# --------------------------------------------------------------------------
def stack_pieces(stack, geom: Geometry, rule) -> dict:
    I = len(geom.curves)
    k = np.asarray(stack.k, float)
    cv = geom.curves
    out = {"A_self": [], "A_up": [], "A_dn": [], "B_own": [], "B_below": [],
           "C_own": [], "C_above": [], "Q": []}
    for i in range(I):
        out["A_self"].append(self_pieces(cv[i], k[i], k[i + 1], rule))
    for i in range(I - 1):
        # A_{i,i+1} = -[...]^{k_{i+1}} from Gamma_{i+1} to Gamma_i ; A_{i+1,i} = +[...] back
        out["A_up"].append(-pair_pieces(cv[i], cv[i + 1], k[i + 1]))
        out["A_dn"].append(pair_pieces(cv[i + 1], cv[i], k[i + 1]))
    for i in range(I):
        c = cv[i]
        out["B_own"].append(proxy_block(c.x, c.y, c.nx, c.ny, proxies(geom, i), k[i]))
        out["B_below"].append(-proxy_block(c.x, c.y, c.nx, c.ny, proxies(geom, i + 1), k[i + 1]))
    for j in range(I + 1):               # layer j (0-based): touches Gamma_{j-1}, Gamma_j
        out["Q"].append(wall_Q_pieces(geom.walls[j], proxies(geom, j), k[j], geom.d))
        out["C_own"].append(wall_C_pieces(geom.walls[j], cv[j], k[j]) if j < I else None)
        out["C_above"].append(wall_C_pieces(geom.walls[j], cv[j - 1], k[j]) if j > 0 else None)
    out["Z_U"] = rad_Z_pieces(geom.xU, geom.yU, cv[0], k[0])
    out["Z_D"] = rad_Z_pieces(geom.xD, geom.yD, cv[I - 1], k[I])
    one = np.ones_like(geom.xU)
    out["V_U"] = proxy_block(geom.xU, np.full_like(geom.xU, geom.yU), 0 * one, one, proxies(geom, 0), k[0])
    out["V_D"] = proxy_block(geom.xD, np.full_like(geom.xD, geom.yD), 0 * one, one, proxies(geom, I), k[I])
    return out


def combine3(p, alpha):
    return p[0] / alpha + p[1] + alpha * p[2]


def combine_C(p, alpha):
    return p[0] / alpha ** 2 - alpha * p[1]


def combine_Q(p, alpha):
    return p[0] / alpha - p[1]
