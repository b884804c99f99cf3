"""Stage-by-stage parity of the solve phase (GPU vs oracle) on one angle:
alpha assembly, per-layer least squares, Schur complements, the sweep."""
import numpy as np
import pytest

import workloads
import oracle
from oracle import alpert, fills, geometry, solve as osolve
from tests.gpu_common import context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return context()


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b)))


def _oracle_blocks(desc):
    geom = geometry.make_geometry(desc)
    pieces = fills.stack_pieces(desc, geom, alpert.load_rule())
    b = osolve.assemble_blocks(desc, desc.thetas[0], pieces, geom)
    X = osolve.layer_ls(desc, b)
    diag, up, dn = osolve.schur_blocks(desc, b, X)
    eta = osolve.block_tridiag_solve(diag, up, dn, b["f1"])
    return b, X, diag, up, dn, eta


@pytest.mark.parametrize("name", ["config1", "small4"])
def test_solve_stages(ctx, name):
    import paper_1410_5003_amd as mlh
    desc = workloads.config1() if name == "config1" else workloads.small_stack(seed=7, I=4, N=48, P=40,
                                                                                M_w=30, M_ud=30, K=8)
    b, X, diag, up, dn, eta = _oracle_blocks(desc)
    st = mlh.Stack(ctx, desc)
    I, P, nK = desc.I, desc.P, 2 * desc.K + 1
    th = desc.thetas[0]
    report = {}
    # phase 1: assembled blocks
    st.solve_partial(th, 1)
    for i in range(I):
        n = b["A_self"][i].shape[0]
        Dg = st.work("Dg", i)
        report["A_self%d" % i] = _rel(Dg[:, :n], b["A_self"][i])
        if i == 0:
            report["f1"] = _rel(Dg[:, n], b["f1"])
        if i + 1 < I:
            report["A_up%d" % i] = _rel(st.work("Up", i), b["A_up"][i])
            report["A_dn%d" % i] = _rel(st.work("Dn", i), b["A_dn"][i])
    mw2, mud2 = 2 * desc.M_w, 2 * desc.M_ud
    for j in range(I + 1):
        S = st.work("S", j)
        R = st.work("RHS", j)
        if j in (0, I):
            Qp = np.block([[b["Q"][j], np.zeros((mw2, nK))], [b["V_U" if j == 0 else "V_D"], b["W_U" if j == 0 else "W_D"]]])
            Cp = np.vstack([b["C_own"][0] if j == 0 else b["C_above"][I], b["Z_U" if j == 0 else "Z_D"]])
            m = mw2 + mud2
        else:
            Qp = b["Q"][j]
            Cp = np.hstack([b["C_above"][j], b["C_own"][j]])
            m = mw2
        report["Q%d" % j] = _rel(S[:m], Qp)
        report["C%d" % j] = _rel(R[:m], Cp)
    # phase 2: least squares.  X itself is not unique to rounding (the
    # Remark after eq. (78)); check that the GPU X satisfies the Tikhonov
    # normal equations (Q^H Q + mu^2 I) X = Q^H C of the same problem.
    st.solve_partial(th, 2)
    Xgpu = []
    for j in range(I + 1):
        R = st.work("RHS", j)
        S1 = st.work("S", j)
        c = X[j].shape[0]
        m = S1.shape[0] - c
        Xg = R[:c]
        Xgpu.append(Xg)
        if j in (0, I):
            Qp = np.block([[b["Q"][j], np.zeros((mw2, nK))], [b["V_U" if j == 0 else "V_D"], b["W_U" if j == 0 else "W_D"]]])
            Cp = np.vstack([b["C_own"][0] if j == 0 else b["C_above"][I], b["Z_U" if j == 0 else "Z_D"]])
        else:
            Qp = b["Q"][j]
            Cp = np.hstack([b["C_above"][j], b["C_own"][j]])
        mu = desc.ls_mu * np.linalg.norm(Qp)
        ne = Qp.conj().T @ (Qp @ Xg - Cp) + mu * mu * Xg
        report["LSnormal%d" % j] = np.linalg.norm(ne) / (np.linalg.norm(Qp) * np.linalg.norm(Cp))
        report["X%d" % j] = _rel(Xg, X[j])
    # phase 3: Schur complements.  Each block must equal eq. (74)-(78)
    # evaluated from the GPU's own least-squares solutions X (X is not unique,
    # so the oracle's X would not do), within rounding of the products
    st.solve_partial(th, 3)
    Xg_all = Xgpu
    diag_ref, up_ref, dn_ref = osolve.schur_blocks(desc, b, Xg_all)
    dg_g, up_g, dn_g, f_g = [], [], [], None
    for i in range(I):
        n = diag[i].shape[0]
        W = st.work("Dg", i)
        dg_g.append(W[:, :n])
        if i == 0:
            f_g = W[:, n]
        report["Adiag%d" % i] = _rel(dg_g[i], diag[i])
        report["SchurD%d" % i] = _schur_err(dg_g[i], diag_ref[i], b["A_self"][i], b, i, Xg_all, desc, "diag")
        if i + 1 < I:
            up_g.append(st.work("Up", i))
            dn_g.append(st.work("Dn", i))
            report["Aup%d" % i] = _rel(up_g[i], up[i])
            report["Adn%d" % i] = _rel(dn_g[i], dn[i])
            report["SchurU%d" % i] = _schur_err(up_g[i], up_ref[i], b["A_up"][i], b, i, Xg_all, desc, "up")
            report["SchurL%d" % i] = _schur_err(dn_g[i], dn_ref[i], b["A_dn"][i], b, i, Xg_all, desc, "dn")
    # phase 4: the block-tridiagonal solve (Sec. 3.3), held to the GPU's own
    # A' and f: normwise backward error, and the forward error against a
    # plain sparse direct solve of the same system scaled by its condition
    st.solve_partial(th, 4)
    eta_g = [st.work("eta", i)[:, 0] for i in range(I)]
    eta_ref = osolve.block_tridiag_solve(dg_g, up_g, dn_g, f_g)
    Ag = _assemble(dg_g, up_g, dn_g)
    x = np.concatenate(eta_g)
    rhs = np.zeros(Ag.shape[0], dtype=complex)
    rhs[:f_g.size] = f_g
    report["eta_backward"] = np.linalg.norm(Ag @ x - rhs) / (np.linalg.norm(Ag, 2) * np.linalg.norm(x))
    cond = np.linalg.cond(Ag)
    report["eta_forward_over_cond"] = _rel(x, np.concatenate(eta_ref)) / cond
    for i in range(I):
        report["eta%d" % i] = _rel(eta_g[i], eta[i])
    print(name, "cond A' %.1e" % cond, {k: "%.1e" % v for k, v in report.items()})
    for k, v in report.items():
        if k[0] in "fQC" or k.startswith("A_"):
            assert v < 1e-12, (k, v)
        if k.startswith("LSnormal"):
            assert v < 1e-13, (k, v)
        if k.startswith("Schur"):
            assert v < 1e-13, (k, v)
        if k == "eta_backward":
            assert v < 1e-13, (k, v)
        if k == "eta_forward_over_cond":
            assert v < 1e-12, (k, v)


def _assemble(diag, up, dn):
    n = [d.shape[0] for d in diag]
    off = np.concatenate([[0], np.cumsum(n)])
    A = np.zeros((off[-1], off[-1]), dtype=complex)
    for i in range(len(diag)):
        A[off[i]:off[i + 1], off[i]:off[i + 1]] = diag[i]
        if i + 1 < len(diag):
            A[off[i]:off[i + 1], off[i + 1]:off[i + 2]] = up[i]
            A[off[i + 1]:off[i + 2], off[i]:off[i + 1]] = dn[i]
    return A


def _schur_err(gpu, ref, A, b, i, X, desc, which):
    """max |A'_gpu - A'_ref| over the scale of the terms it is formed from,
    max |A| + max (|B| |X|)."""
    P, I = desc.P, desc.I
    n = [blk.shape[0] for blk in b["A_self"]]
    if which == "diag":
        Xa = X[i][:P] if i == 0 else X[i][:, n[i - 1]:]
        Xb = X[i + 1][:P] if i == I - 1 else X[i + 1][:, :n[i]]
        prod = np.abs(b["B_own"][i]) @ np.abs(Xa) + np.abs(b["B_below"][i]) @ np.abs(Xb)
    elif which == "up":
        prod = np.abs(b["B_below"][i]) @ np.abs(X[i + 1][:, n[i]:])
    else:
        prod = np.abs(b["B_own"][i + 1]) @ np.abs(X[i + 1][:, :n[i]])
    scale = np.abs(A).max() + prod.max()
    return np.abs(gpu - ref).max() / scale
