"""The captured launch graph is replayed across solves (new angles, same
batch shape) and gives the same amplitudes as direct launches and the oracle."""
import numpy as np
import pytest

import workloads
import oracle
from tests.gpu_common import context, rel_amp_err

pytestmark = pytest.mark.gpu


def test_graph_replay_matches_oracle_for_new_angles():
    import paper_1410_5003_amd as mlh
    ctx = context()
    desc = workloads.config1(N=160, P=140, M_w=100)
    st = mlh.Stack(ctx, desc)
    for th in (-0.4, -1.1, -2.3, -0.4):      # same batch shape: captured once, replayed
        g = st.solve([th])
        o = oracle.solve_stack(desc, theta=th)
        assert rel_amp_err(g.aU[0], g.aD[0], o.aU, o.aD) < 1e-10
    # eager launches (no replay) of the inspection path agree with the replay
    st.solve_partial(-1.1, 4)
    eta = st.work("eta", 0)[:, 0]
    assert np.all(np.isfinite(eta))
    g1 = st.solve([-1.1])
    g2 = st.solve([-1.1])
    assert np.array_equal(g1.aU, g2.aU) and np.array_equal(g1.aD, g2.aD)
    st.close()


def test_profiled_solve_times_its_phases_and_leaves_the_results_alone():
    """The per-kernel profile runs the solve's launches one at a time, each
    bracketed by HIP events, inside a bracket of its own: every phase of a
    4-interface stack has a finite positive time, the phases add up to no
    more than the total, and the graph path's amplitudes are unchanged."""
    import paper_1410_5003_amd as mlh
    ctx = context()
    desc = workloads.small_stack(I=4)
    st = mlh.Stack(ctx, desc)
    th = [-0.4, -1.1]
    g1 = st.solve(th)
    p = st.profile_solve(th)
    for k in ("fill_self_ms", "fill_alpert_ms", "fill_pairs_ms", "ls_panel_ms", "ls_rhs_ms", "schur_ms",
              "bragg_ms", "total_ms"):
        assert np.isfinite(p[k]) and p[k] > 0, k
    parts = sum(v for k, v in p.items() if k.endswith("_ms") and k != "total_ms")
    assert parts <= p["total_ms"]
    q = st.profile_step(-0.4)
    assert np.isfinite(q["total_ms"]) and q["total_ms"] > 0
    g2 = st.solve(th)
    assert np.array_equal(g1.aU, g2.aU) and np.array_equal(g1.aD, g2.aD)
    st.close()
