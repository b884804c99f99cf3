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
    {"gemm_slab_k": 16},
    {"rhs_in_step_pct": 0, "ls_row_blocks": 4, "gje_rhs_cols": 8, "asm_in_panels": 0, "gemm_slab_k": 16},
]


@pytest.mark.parametrize("choice", VARIANTS, ids=lambda c: "-".join("%s=%d" % kv for kv in c.items()) or "default")
def test_every_choice_matches_oracle(ctx, case, choice):
    import paper_1410_5003_amd as mlh
    desc, th, o = case
    st = mlh.Stack(ctx, desc)
    assert st.get_tuning() == {"rhs_in_step_pct": 300, "ls_row_blocks": 3, "gje_rhs_cols": 16, "asm_in_panels": 1,
                               "gemm_slab_k": 8}
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
    for bad in ({"ls_row_blocks": 5}, {"gje_rhs_cols": 12}, {"asm_in_panels": 2}, {"gemm_slab_k": 12},
                {"rhs_in_step_pct": -1},
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


def test_batched_shared_alpha_angles_under_non_default_choices(ctx):
    # three angles, two of them sharing alpha (kappa_0 one grid step apart),
    # so one system carries two right-hand sides; every placement choice is
    # off its default: replay after the last step with 8-column tiles, four
    # row blocks, assembly in its own launch
    import paper_1410_5003_amd as mlh
    desc = workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9)
    g = 2 * np.pi / desc.d
    k0 = float(np.cos(desc.thetas[0]) * desc.k[0])
    th = -np.arccos(np.array([k0, k0 - g, 0.5 * k0]) / desc.k[0])
    assert np.all(np.isfinite(th))
    st = mlh.Stack(ctx, desc)
    st.set_tuning(rhs_in_step_pct=0, gje_rhs_cols=8, ls_row_blocks=4, asm_in_panels=0)
    out = st.solve(th)
    for a, t in enumerate(th):
        o = oracle.solve_stack(desc, theta=t)
        assert np.array_equal(out.orders[a], o.orders)
        assert rel_amp_err(out.aU[a], out.aD[a], o.aU, o.aD) < TOL
    st.close()


def test_autotuned_choices_are_reused_by_size_class(ctx, case):
    # an autotune records its choices under (device architecture, size class);
    # a second stack of the same class takes them without timing, a stack of
    # another class (other block orders) finds nothing and keeps its own
    import paper_1410_5003_amd as mlh
    desc, th, o = case
    st = mlh.Stack(ctx, desc)
    t = st.autotune([th], reps=1)
    st.close()
    twin = workloads.small_stack(seed=7, I=4, N=80, P=45, M_w=35, M_ud=40, K=9, theta=th)
    s2 = mlh.Stack(ctx, twin)
    s2.set_tuning(rhs_in_step_pct=0, ls_row_blocks=4, gje_rhs_cols=8, asm_in_panels=0)
    found, got = s2.tune_cached([th])
    assert found and got == t and s2.get_tuning() == t
    g = s2.solve([th])
    ot = oracle.solve_stack(twin, theta=th)
    assert rel_amp_err(g.aU[0], g.aD[0], ot.aU, ot.aD) < TOL
    s2.close()
    other = workloads.config1(N=160, P=140, M_w=100)  # block order 320, 2 interfaces
    s3 = mlh.Stack(ctx, other)
    before = s3.get_tuning()
    found, got = s3.tune_cached([float(other.thetas[0])])
    assert not found and got == before == s3.get_tuning()
    s3.close()


_CACHE_SCRIPT = r"""
import json, sys
sys.path.insert(0, %(root)r)
import workloads
import paper_1410_5003_amd as mlh
ctx = mlh.Context(0)
d = workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9)
st = mlh.Stack(ctx, d)
th = [float(d.thetas[0])]
if sys.argv[1] == "tune":
    print(json.dumps(st.autotune(th, reps=1)))
else:
    print(json.dumps(st.tune_cached(th)))
st.close()
"""


def test_tuning_cache_file_carries_choices_to_the_next_process(tmp_path):
    # with MLH_TUNING_CACHE set, one process's autotune is found by the next
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = tmp_path / "cache_probe.py"
    script.write_text(_CACHE_SCRIPT % {"root": root})
    env = dict(os.environ, MLH_TUNING_CACHE=str(tmp_path / "tuning.txt"))
    run = lambda mode: subprocess.run([sys.executable, str(script), mode], env=env, capture_output=True, text=True,
                                      timeout=240)
    a = run("tune")
    assert a.returncode == 0, a.stderr[-2000:]
    tuned = json.loads(a.stdout.strip().splitlines()[-1])
    lines = (tmp_path / "tuning.txt").read_text().split("\n")
    assert len([l for l in lines if l.strip()]) == 1
    b = run("lookup")
    assert b.returncode == 0, b.stderr[-2000:]
    found, got = json.loads(b.stdout.strip().splitlines()[-1])
    assert found and got == tuned
