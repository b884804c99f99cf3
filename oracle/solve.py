"""Schur eliminations, block-tridiagonal solve, Bragg amplitudes and flux
(test infrastructure only).

Follows Sec. 3 of the paper:

* rearranged unknowns x_1 = [c_1; a^U], x_j = c_j, x_{I+1} = [c_{I+1}; a^D]
  with the primed end blocks Q'_1 = [[Q_1, 0], [V_U, W_U]],
  C'_{1,1} = [C_{1,1}; Z_U], Q'_{I+1} = [[Q_{I+1}, 0], [V_D, W_D]],
  C'_{I+1,I} = [C_{I+1,I}; Z_D] (Sec. 3.1; the paper prints Z_U in the last
  one, which is read as Z_D: the bottom layer meets the line D);
* per layer X_j = Q_j^+ [C_{j,j-1}, C_{j,j}] computed by a backward-stable
  least-squares solve, never by forming a pseudo-inverse (Sec. 3.2).  The
  least-squares problem is defined here as the Tikhonov-stacked problem
  min ||Q X - C||^2 + mu^2 ||X||^2 with mu = mu_rel ||Q||_F, solved by
  Householder QR of [Q; mu I]; a column-pivoted QR basic solution
  (what a dense backslash does) is also provided.  Both select a small-norm
  quasi-periodic Green's function (Remark after eq. (78)); only the Bragg
  amplitudes, not the densities, are independent of that choice;
* Schur blocks eq. (74)-(78), then the block-tridiagonal system eq. (73)
  solved with a plain sparse direct solver (SuperLU), deliberately not with
  the block sweep the GPU uses;
* x_1 = -X_1 eta_1, x_{I+1} = -X_{I+1} eta_I (Sec. 3.3), a^U / a^D are their
  last 2K+1 entries;
* flux error eq. (86) with the incident vertical flux k_1 |sin theta| (the
  paper prints k_1 cos theta, which is zero at normal incidence; the
  |sin theta| form is what the Fresnel pin in the tests confirms).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import alpert, fills
from .geometry import make_geometry


def ls_tikhonov(Q: np.ndarray, C: np.ndarray, mu_rel: float) -> np.ndarray:
    m, n = Q.shape
    mu = mu_rel * np.linalg.norm(Q)
    A = np.vstack([Q, mu * np.eye(n)])
    Qh, R = np.linalg.qr(A, mode="reduced")
    return sla.solve_triangular(R, Qh[:m].conj().T @ C)


def ls_cpqr(Q: np.ndarray, C: np.ndarray, rtol: Optional[float] = None) -> np.ndarray:
    m, n = Q.shape
    Qh, R, piv = sla.qr(Q, mode="economic", pivoting=True)
    if rtol is None:
        rtol = max(m, n) * np.finfo(float).eps
    r = int(np.sum(np.abs(np.diag(R)) > rtol * abs(R[0, 0])))
    y = sla.solve_triangular(R[:r, :r], Qh[:, :r].conj().T @ C)
    X = np.zeros((n, C.shape[1]), dtype=complex)
    X[piv[:r]] = y
    return X


@dataclass
class SolveResult:
    theta: float
    alpha: complex
    orders: np.ndarray
    aU: np.ndarray
    aD: np.ndarray
    kU: np.ndarray
    kD: np.ndarray
    flux_err: float
    eta: list = field(default_factory=list)
    blocks: Optional[dict] = None


def flux_error(aU, aD, kU, kD, k1, theta) -> float:
    pu = (np.abs(kU.imag) == 0) & (kU.real > 0)
    pd = (np.abs(kD.imag) == 0) & (kD.real > 0)
    out = np.sum(kU.real[pu] * np.abs(aU[pu]) ** 2) + np.sum(kD.real[pd] * np.abs(aD[pd]) ** 2)
    inc = k1 * abs(np.sin(theta))
    return float((out - inc) / inc)


def assemble_blocks(stack, theta: float, pieces: dict, geom) -> dict:
    """All blocks of eq. (67) at one incident angle."""
    I = stack.I
    k = np.asarray(stack.k, float)
    alpha = np.exp(1j * stack.d * k[0] * np.cos(theta))
    n, kappa = fills.rb_orders(k[0], theta, stack.d, stack.K)
    kU = fills.vertical_wavenumbers(k[0], kappa)
    kD = fills.vertical_wavenumbers(k[I], kappa)
    b = {"alpha": alpha, "orders": n, "kappa": kappa, "kU": kU, "kD": kD}
    b["A_self"] = [fills.combine3(p, alpha) for p in pieces["A_self"]]
    b["A_up"] = [fills.combine3(p, alpha) for p in pieces["A_up"]]
    b["A_dn"] = [fills.combine3(p, alpha) for p in pieces["A_dn"]]
    b["B_own"] = pieces["B_own"]
    b["B_below"] = pieces["B_below"]
    b["Q"] = [fills.combine_Q(p, alpha) for p in pieces["Q"]]
    b["C_own"] = [None if p is None else fills.combine_C(p, alpha) for p in pieces["C_own"]]
    b["C_above"] = [None if p is None else fills.combine_C(p, alpha) for p in pieces["C_above"]]
    b["Z_U"] = fills.combine3(pieces["Z_U"], alpha)
    b["Z_D"] = fills.combine3(pieces["Z_D"], alpha)
    b["V_U"] = pieces["V_U"]
    b["V_D"] = pieces["V_D"]
    b["W_U"] = fills.rad_W(geom.xU, kappa, kU, True)
    b["W_D"] = fills.rad_W(geom.xD, kappa, kD, False)
    b["f1"] = fills.rhs_f(geom.curves[0], k[0], theta)
    return b


def layer_ls(stack, b: dict, ls: str = "tikhonov", mu_rel: Optional[float] = None):
    """X_j for j = 1..I+1 (0-based list).  X[0] acts on eta_1, X[I] on eta_I,
    interior X[j] on [eta_j; eta_{j+1}] (0-based interface indices j-1, j)."""
    I = stack.I
    mu_rel = stack.ls_mu if mu_rel is None else mu_rel
    P, nK = stack.P, 2 * stack.K + 1

    def LS(Q, C):
        return ls_tikhonov(Q, C, mu_rel) if ls == "tikhonov" else ls_cpqr(Q, C)

    X = []
    Q1p = np.block([[b["Q"][0], np.zeros((b["Q"][0].shape[0], nK))], [b["V_U"], b["W_U"]]])
    X.append(LS(Q1p, np.vstack([b["C_own"][0], b["Z_U"]])))
    for j in range(1, I):
        X.append(LS(b["Q"][j], np.hstack([b["C_above"][j], b["C_own"][j]])))
    QLp = np.block([[b["Q"][I], np.zeros((b["Q"][I].shape[0], nK))], [b["V_D"], b["W_D"]]])
    X.append(LS(QLp, np.vstack([b["C_above"][I], b["Z_D"]])))
    return X


def schur_blocks(stack, b: dict, X: list):
    """A'_{i,i}, A'_{i,i+1}, A'_{i+1,i} (eq. (74)-(78)), 0-based interfaces."""
    I, P = stack.I, stack.P
    n = [c.shape[0] for c in b["A_self"]]
    diag, up, dn = [], [], []
    for i in range(I):
        # X for the layer above interface i is X[i]; below is X[i+1]
        Xa = X[i][:P] if i == 0 else X[i][:, n[i - 1]:]          # acts on eta_i
        Xb = X[i + 1][:P] if i == I - 1 else X[i + 1][:, :n[i]]  # acts on eta_i
        diag.append(b["A_self"][i] - b["B_own"][i] @ Xa - b["B_below"][i] @ Xb)
    for i in range(I - 1):
        up.append(b["A_up"][i] - b["B_below"][i] @ X[i + 1][:, n[i]:])
        dn.append(b["A_dn"][i] - b["B_own"][i + 1] @ X[i + 1][:, :n[i]])
    return diag, up, dn


def block_tridiag_solve(diag, up, dn, f1):
    I = len(diag)
    rows = [[None] * I for _ in range(I)]
    for i in range(I):
        rows[i][i] = sp.csc_matrix(diag[i])
        if i + 1 < I:
            rows[i][i + 1] = sp.csc_matrix(up[i])
            rows[i + 1][i] = sp.csc_matrix(dn[i])
    A = sp.bmat(rows, format="csc")
    rhs = np.zeros(A.shape[0], dtype=complex)
    rhs[:len(f1)] = f1
    eta = spla.spsolve(A, rhs)
    out, o = [], 0
    for dblk in diag:
        out.append(eta[o:o + dblk.shape[0]])
        o += dblk.shape[0]
    return out


def solve_stack(stack, theta: Optional[float] = None, rule=None, ls: str = "tikhonov",
                mu_rel: Optional[float] = None, pieces: Optional[dict] = None,
                keep_blocks: bool = False) -> SolveResult:
    theta = float(stack.thetas[0]) if theta is None else float(theta)
    rule = alpert.load_rule() if rule is None else rule
    geom = make_geometry(stack)
    if pieces is None:
        pieces = fills.stack_pieces(stack, geom, rule)
    b = assemble_blocks(stack, theta, pieces, geom)
    X = layer_ls(stack, b, ls, mu_rel)
    diag, up, dn = schur_blocks(stack, b, X)
    eta = block_tridiag_solve(diag, up, dn, b["f1"])
    P, I = stack.P, stack.I
    aU = -(X[0] @ eta[0])[P:]
    aD = -(X[I] @ eta[I - 1])[P:]
    fe = flux_error(aU, aD, b["kU"], b["kD"], stack.k[0], theta)
    if keep_blocks:
        b["X"] = X
        b["A_diag"], b["A_upS"], b["A_dnS"] = diag, up, dn
    return SolveResult(theta, b["alpha"], b["orders"], aU, aD, b["kU"], b["kD"], fe, eta,
                       b if keep_blocks else None)


def solve_full_system(stack, theta: Optional[float] = None, rule=None) -> SolveResult:
    """Cross-check for small I: assemble the whole rearranged rectangular
    system eq. (67) and solve it by dense least squares (no Schur
    complements, no block elimination)."""
    theta = float(stack.thetas[0]) if theta is None else float(theta)
    rule = alpert.load_rule() if rule is None else rule
    geom = make_geometry(stack)
    pieces = fills.stack_pieces(stack, geom, rule)
    b = assemble_blocks(stack, theta, pieces, geom)
    I, P, nK = stack.I, stack.P, 2 * stack.K + 1
    n = [blk.shape[0] for blk in b["A_self"]]
    nd = sum(n)
    off = np.concatenate([[0], np.cumsum(n)])
    # unknown columns: eta (nd), then x_1 = [c_1; a^U], c_2..c_I, x_{I+1} = [c_{I+1}; a^D]
    xcol = [nd]
    for j in range(I + 1):
        xcol.append(xcol[-1] + P + (nK if j in (0, I) else 0))
    ncol = xcol[-1]
    mw = b["Q"][0].shape[0]
    mud = b["V_U"].shape[0]
    nrow = nd + (I + 1) * mw + 2 * mud
    M = np.zeros((nrow, ncol), dtype=complex)
    rhs = np.zeros(nrow, dtype=complex)
    for i in range(I):
        r = slice(off[i], off[i + 1])
        M[r, off[i]:off[i + 1]] = b["A_self"][i]
        if i + 1 < I:
            M[r, off[i + 1]:off[i + 2]] = b["A_up"][i]
            M[off[i + 1]:off[i + 2], off[i]:off[i + 1]] = b["A_dn"][i]
        M[r, xcol[i]:xcol[i] + P] = b["B_own"][i]
        M[r, xcol[i + 1]:xcol[i + 1] + P] = b["B_below"][i]
    rhs[:n[0]] = b["f1"]
    row = nd
    for j in range(I + 1):
        r = slice(row, row + mw)
        if j < I:
            M[r, off[j]:off[j + 1]] = b["C_own"][j]
        if j > 0:
            M[r, off[j - 1]:off[j]] = b["C_above"][j]
        M[r, xcol[j]:xcol[j] + P] = b["Q"][j]
        row += mw
    r = slice(row, row + mud)
    M[r, off[0]:off[1]] = b["Z_U"]
    M[r, xcol[0]:xcol[0] + P] = b["V_U"]
    M[r, xcol[0] + P:xcol[1]] = b["W_U"]
    row += mud
    r = slice(row, row + mud)
    M[r, off[I - 1]:off[I]] = b["Z_D"]
    M[r, xcol[I]:xcol[I] + P] = b["V_D"]
    M[r, xcol[I] + P:xcol[I + 1]] = b["W_D"]
    sol = np.linalg.lstsq(M, rhs, rcond=None)[0]
    aU = sol[xcol[0] + P:xcol[1]]
    aD = sol[xcol[I] + P:xcol[I + 1]]
    fe = flux_error(aU, aD, b["kU"], b["kD"], stack.k[0], theta)
    return SolveResult(theta, b["alpha"], b["orders"], aU, aD, b["kU"], b["kD"], fe)
