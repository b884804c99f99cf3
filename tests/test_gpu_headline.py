"""Parity at the sizes the benchmark runs: Bragg amplitudes of the GPU path
against the oracle at 1e-10 relative, order labels exact, flux error
<= 1e-9 on both sides (Sec. 3.3, eq. (86)).

The two large cases read the oracle's results from tests/golden/ (written by
tests/golden/make_golden.py, which calls only the oracle): the 50-interface
resolved stack (N = 260, P = 120, M_w = 80), and the first 40 interfaces of
the 1000-layer mixed smooth / cornered stack at its resolved sizes with
three angles, two of which share the Bloch phase.  The smaller cases run the
oracle live: a stack whose layer systems fall in both size classes of the
least-squares kernels, and an odd interface count, whose cyclic-reduction
levels have odd active sets."""
import numpy as np
import pytest

import workloads
import oracle
from tests.golden.make_golden import RES3, config3_res40_thetas, load as load_golden
from tests.gpu_common import context, rel_amp_err

pytestmark = pytest.mark.gpu

TOL = 1e-10
FLUX = 1e-9


@pytest.fixture(scope="module")
def ctx():
    return context()


def _compare(g, a, ref, label):
    assert np.array_equal(g.orders[a], ref["orders"]), label
    err = rel_amp_err(g.aU[a], g.aD[a], ref["aU"], ref["aD"])
    print("%s: rel amp err %.2e  flux gpu %.2e oracle %.2e" % (label, err, g.flux_err[a], ref["flux_err"]))
    assert abs(ref["flux_err"]) <= FLUX, label
    assert abs(g.flux_err[a]) <= FLUX, label
    assert err < TOL, (label, err)


@pytest.fixture(scope="module")
def config2_resolved(ctx):
    import paper_1410_5003_amd as mlh
    desc = workloads.config2(N=260, P=120, M_w=80)
    st = mlh.Stack(ctx, desc)
    yield desc, st, load_golden("config2_resolved")
    st.close()


def test_config2_resolved_default_choices(config2_resolved):
    desc, st, gold = config2_resolved
    st.set_tuning(rhs_in_step_pct=300, ls_row_blocks=3, gje_rhs_cols=16, asm_in_panels=1)
    th = np.array([gold[0]["theta"]])
    for rep in range(2):  # the second solve replays the captured graph
        _compare(st.solve(th), 0, gold[0], "config2_resolved default, solve %d" % rep)


@pytest.mark.parametrize("choice", [dict(rhs_in_step_pct=0, gje_rhs_cols=8),
                                    dict(ls_row_blocks=4, asm_in_panels=0)],
                         ids=["replay-8col", "4rowblocks-asm-own-launch"])
def test_config2_resolved_other_choices(config2_resolved, choice):
    desc, st, gold = config2_resolved
    st.set_tuning(rhs_in_step_pct=300, ls_row_blocks=3, gje_rhs_cols=16, asm_in_panels=1)
    st.set_tuning(**choice)
    _compare(st.solve(np.array([gold[0]["theta"]])), 0, gold[0], "config2_resolved %s" % choice)


def test_config2_resolved_autotuned(config2_resolved):
    desc, st, gold = config2_resolved
    th = np.array([gold[0]["theta"]])
    t = st.autotune(th, reps=1)
    print("autotuned", t)
    _compare(st.solve(th), 0, gold[0], "config2_resolved autotuned")


def test_config3_first40_resolved_shared_alpha(ctx):
    import paper_1410_5003_amd as mlh
    desc = workloads.config3(I=40, n_angles=3, **RES3)
    gold = load_golden("config3_res40")
    th = np.array([a["theta"] for a in gold])
    assert np.allclose(th, config3_res40_thetas(desc), rtol=0, atol=1e-15)
    st = mlh.Stack(ctx, desc)
    g = st.solve(th)
    for a in range(len(th)):
        _compare(g, a, gold[a], "config3 first 40 layers, angle %d" % a)
    st.close()


@pytest.mark.parametrize("row_blocks", [3, 4])
def test_both_least_squares_size_classes(ctx, row_blocks):
    # interior layer system [Q; mu I] of 2 M_w + P = 340 rows (<= 384: the
    # small class), end layers 2 M_w + 2 M_ud + P + 2K + 1 = 511 rows (the
    # large class)
    import paper_1410_5003_amd as mlh
    desc = workloads.config1(N=160, P=140, M_w=100)
    o = oracle.solve_stack(desc)
    st = mlh.Stack(ctx, desc)
    st.set_tuning(ls_row_blocks=row_blocks)
    ref = {"orders": o.orders, "aU": o.aU, "aD": o.aD, "flux_err": o.flux_err}
    _compare(st.solve(desc.thetas[:1]), 0, ref, "config1 N=160 P=140 M_w=100, %d row blocks" % row_blocks)
    st.close()


@pytest.mark.parametrize("I", [7, 11])
def test_odd_interface_counts(ctx, I):
    # cyclic reduction levels of 7 -> 4 -> 2 -> 1 and 11 -> 6 -> 3 -> 2 -> 1
    # blocks: odd active sets, a last block without a right neighbour
    import paper_1410_5003_amd as mlh
    desc = workloads.small_stack(seed=20 + I, I=I, N=72, P=50, M_w=40, M_ud=40, K=8)
    o = oracle.solve_stack(desc)
    st = mlh.Stack(ctx, desc)
    ref = {"orders": o.orders, "aU": o.aU, "aD": o.aD, "flux_err": o.flux_err}
    for pct in (300, 0):  # right-hand sides inside the steps, then replayed
        st.set_tuning(rhs_in_step_pct=pct)
        _compare(st.solve(desc.thetas[:1]), 0, ref, "small stack I=%d rhs_in_step_pct=%d" % (I, pct))
    st.close()
