"""Entrywise parity of every alpha-independent fill piece (GPU vs oracle)."""
import numpy as np
import pytest

import workloads
import oracle
from oracle import alpert, fills, geometry
from tests.gpu_common import context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return context()


def _compare_all(ctx, desc, tol=1e-12):
    import paper_1410_5003_amd as mlh
    st = mlh.Stack(ctx, desc)
    geom = geometry.make_geometry(desc)
    P = fills.stack_pieces(desc, geom, alpert.load_rule())
    I = desc.I
    worst = {}

    def cmp(name, idx, pc, ref):
        got = st.piece(name, idx, pc)
        assert got.shape == ref.shape, (name, idx, pc, got.shape, ref.shape)
        err = np.max(np.abs(got - ref)) / max(1.0, np.max(np.abs(ref)))
        worst[name] = max(worst.get(name, 0.0), err)
        assert err < tol, (name, idx, pc, err)

    for i in range(I):
        for p in range(3):
            cmp("A_self", i, p, P["A_self"][i][p])
        cmp("B_own", i, 0, P["B_own"][i])
        cmp("B_below", i, 0, P["B_below"][i])
    for i in range(I - 1):
        for p in range(3):
            cmp("A_up", i, p, P["A_up"][i][p])
            cmp("A_dn", i, p, P["A_dn"][i][p])
    for j in range(I + 1):
        for p in range(2):
            cmp("Q", j, p, P["Q"][j][p])
            if j < I:
                cmp("C_own", j, p, P["C_own"][j][p])
            if j > 0:
                cmp("C_above", j, p, P["C_above"][j][p])
    for p in range(3):
        cmp("Z_U", 0, p, P["Z_U"][p])
        cmp("Z_D", 0, p, P["Z_D"][p])
    cmp("V_U", 0, 0, P["V_U"])
    cmp("V_D", 0, 0, P["V_D"])
    print(desc.name, {k: "%.1e" % v for k, v in worst.items()})
    st.close()


def test_fill_pieces_config1(ctx):
    _compare_all(ctx, workloads.config1())


def test_fill_pieces_small_ragged(ctx):
    # N not a multiple of the 64 x 4 fill tile, paper-scale period d = 1
    _compare_all(ctx, workloads.small_stack(seed=3, I=3, N=45, P=37, M_w=29, M_ud=33, K=8))


def test_fill_pieces_config2_head(ctx):
    _compare_all(ctx, workloads.config2(I=4))


def test_fill_pieces_cornered(ctx):
    # graded segments: per-segment Alpert window, plain entries across corners
    _compare_all(ctx, workloads.small_polygon_stack(nper=40))


def test_fill_pieces_mixed_uneven(ctx):
    _compare_all(ctx, workloads.small_mixed_stack(min_seg=40))


def test_fill_pieces_config3_head(ctx):
    # 120-node smooth and 250-node cornered interfaces at d = 2 pi
    _compare_all(ctx, workloads.config3(I=4, n_angles=1))
