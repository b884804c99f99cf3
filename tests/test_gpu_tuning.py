"""Launch choices of the solve (mlh_tuning): every choice, and the autotuned
one, gives the oracle's Bragg amplitudes; out-of-range choices are rejected.
The choices change launch shapes and the rounding order only."""
import numpy as np
import pytest

import workloads
import oracle
from tests.gpu_common import context, rel_amp_err

pytestmark = pytest.mark.gpu

TOL = 1e-10  # relative, on the Bragg amplitudes (as for the other parity tests)


@pytest.fixture(scope="module")
def ctx():
    return context()


@pytest.fixture(scope="module")
def case():
    # ragged layer sizes; 4 interfaces give cyclic-reduction levels of 2, 1
    # and 1 matrices, so both right-hand-side placements occur
    desc = workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9)
    th = float(desc.thetas[0])
    return desc, th, oracle.solve_stack(desc, theta=th)


VARIANTS = [
    {},
    {"rhs_in_step_pct": 0},
    {"rhs_in_step_pct": 0, "gje_rhs_cols": 8},
    {"rhs_in_step_pct": 1000},
    {"ls_row_blocks": 4},
    {"asm_in_panels": 0},
    {"rhs_in_step_pct": 0, "ls_row_blocks": 4, "gje_rhs_cols": 8, "asm_in_panels": 0},
]


@pytest.mark.parametrize("choice", VARIANTS, ids=lambda c: "-".join("%s=%d" % kv for kv in c.items()) or "default")
def test_every_choice_matches_oracle(ctx, case, choice):
    import paper_1410_5003_amd as mlh
    desc, th, o = case
    st = mlh.Stack(ctx, desc)
    assert st.get_tuning() == {"rhs_in_step_pct": 300, "ls_row_blocks": 3, "gje_rhs_cols": 16, "asm_in_panels": 1}
    st.set_tuning(**choice)
    for k, v in choice.items():
        assert st.get_tuning()[k] == v
    # twice: the second solve replays the captured graph of this choice
    for _ in range(2):
        g = st.solve([th])
        err = rel_amp_err(g.aU[0], g.aD[0], o.aU, o.aD)
        assert err < TOL, (choice, err)
        assert abs(g.flux_err[0]) < 1e-9
    st.close()


def test_out_of_range_choices_are_rejected(ctx, case):
    import paper_1410_5003_amd as mlh
    desc, _, _ = case
    st = mlh.Stack(ctx, desc)
    before = st.get_tuning()
    for bad in ({"ls_row_blocks": 5}, {"gje_rhs_cols": 12}, {"asm_in_panels": 2}, {"rhs_in_step_pct": -1},
                {"rhs_in_step_pct": 1001}):
        with pytest.raises(mlh.MlhError):
            st.set_tuning(**bad)
        assert st.get_tuning() == before
    st.close()


def test_autotune_keeps_a_valid_choice_that_matches_oracle(ctx, case):
    import paper_1410_5003_amd as mlh
    desc, th, o = case
    st = mlh.Stack(ctx, desc)
    t = st.autotune([th], reps=1)
    assert t == st.get_tuning()
    assert t["rhs_in_step_pct"] in (0, 100, 150, 200, 300, 500, 1000)
    assert t["ls_row_blocks"] in (3, 4) and t["gje_rhs_cols"] in (16, 8) and t["asm_in_panels"] in (0, 1)
    g = st.solve([th])
    assert rel_amp_err(g.aU[0], g.aD[0], o.aU, o.aD) < TOL
    st.close()
