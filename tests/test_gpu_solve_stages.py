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
    Qs, Cs = [], []
    for j in range(I + 1):
        R = st.work("RHS", j)
        S1 = st.work("S", j)
        c = X[j].shape[0]
        m = S1.shape[0] - c
        Xg = R[:c]
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
    # phase 3: Schur complements
    st.solve_partial(th, 3)
    for i in range(I):
        n = diag[i].shape[0]
        report["Adiag%d" % i] = _rel(st.work("Dg", i)[:, :n], diag[i])
        if i + 1 < I:
            report["Aup%d" % i] = _rel(st.work("Up", i), up[i])
            report["Adn%d" % i] = _rel(st.work("Dn", i), dn[i])
    # phase 4: sweep
    st.solve_partial(th, 4)
    for i in range(I):
        report["eta%d" % i] = _rel(st.work("eta", i)[:, 0], eta[i])
    print(name, {k: "%.1e" % v for k, v in report.items()})
    for k, v in report.items():
        if k[0] in "fQC" or k.startswith("A_"):
            assert v < 1e-12, (k, v)
        if k.startswith("LSnormal"):
            assert v < 1e-13, (k, v)
