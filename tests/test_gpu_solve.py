"""End-to-end parity of Bragg amplitudes and flux (GPU vs oracle), through the
C ABI, plus closed-form checks of the GPU path and its error handling."""
import numpy as np
import pytest

import workloads
import oracle
from oracle import fresnel
from tests.gpu_common import context, rel_amp_err

pytestmark = pytest.mark.gpu

TOL = 1e-10  # relative, on the Bragg amplitudes


@pytest.fixture(scope="module")
def ctx():
    return context()


def _gpu(ctx, desc, thetas=None):
    import paper_1410_5003_amd as mlh
    st = mlh.Stack(ctx, desc)
    out = st.solve(desc.thetas if thetas is None else thetas)
    st.close()
    return out


def _check(ctx, desc, resolved=True):
    """Resolved stacks (oracle flux error <= 1e-9): amplitudes agree to 1e-10.
    Under-resolved (literal) stacks: the amplitudes are only determined by
    the method to about its discretisation error, and the least-squares Schur
    solves may pick different (equally valid) quasi-periodic Green's functions
    from rounding-level differences in their inputs (the Remark after
    eq. (78)); there the bar is max(1e-10, |flux error|)."""
    g = _gpu(ctx, desc)
    o = oracle.solve_stack(desc)
    assert np.array_equal(g.orders[0], o.orders)
    err = rel_amp_err(g.aU[0], g.aD[0], o.aU, o.aD)
    tol = TOL if resolved else max(TOL, abs(o.flux_err))
    print(desc.name, "rel err %.2e (tol %.1e)  flux gpu %.2e oracle %.2e" % (err, tol, g.flux_err[0], o.flux_err))
    if resolved:
        assert abs(o.flux_err) < 1e-9
        assert abs(g.flux_err[0]) < 1e-9
    assert err < tol
    assert abs(g.flux_err[0] - o.flux_err) < 1e-9 + 10 * tol
    return g, o


def test_config1_literal(ctx):
    _check(ctx, workloads.config1(), resolved=False)


def test_config1_resolved_twin(ctx):
    _check(ctx, workloads.config1(N=160, P=140, M_w=100))


def test_flat_twin_matches_fresnel(ctx):
    s = workloads.config1_flat(N=160, P=140, M_w=100)
    g = _gpu(ctx, s)
    aU, aD, _ = fresnel.flat_stack_amplitudes(s.k, [0.0, -2.0], s.thetas[0], s.y_U, s.y_D)
    i0 = list(g.orders[0]).index(0)
    assert abs(g.aU[0, i0] - aU) < 1e-11 and abs(g.aD[0, i0] - aD) < 1e-11
    assert np.max(np.abs(np.delete(g.aU[0], i0))) < 1e-10


def test_homogeneous_stack(ctx):
    s = workloads.homogeneous(N=160, P=140, M_w=100)
    g = _gpu(ctx, s)
    i0 = list(g.orders[0]).index(0)
    assert np.max(np.abs(g.aU[0])) < 1e-10
    assert abs(g.aD[0, i0] - np.exp(1j * s.k[0] * np.sin(s.thetas[0]) * s.y_D)) < 1e-10


def test_single_interface_and_ragged_sizes(ctx):
    s = workloads.small_stack(seed=5, I=1, N=41, P=33, M_w=27, M_ud=31, K=7)
    _check(ctx, s)
    s = workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9)
    _check(ctx, s)


def test_multi_angle_batch(ctx):
    s = workloads.config1(N=160, P=140, M_w=100)
    th = np.array([-0.3, -np.pi / 6, -1.2, -2.5])
    g = _gpu(ctx, s, th)
    for a, t in enumerate(th):
        o = oracle.solve_stack(s, theta=t)
        assert rel_amp_err(g.aU[a], g.aD[a], o.aU, o.aD) < TOL


def test_wood_anomaly_top_layer(ctx):
    s = workloads.config1(N=160, P=140, M_w=100)
    th = -np.arccos(1 - 2 * np.pi / (s.d * s.k[0]))
    g = _gpu(ctx, s, [th])
    o = oracle.solve_stack(s, theta=th)
    assert rel_amp_err(g.aU[0], g.aD[0], o.aU, o.aD) < TOL
    assert abs(g.flux_err[0]) < 1e-9


def test_config2_literal(ctx):
    _check(ctx, workloads.config2(), resolved=False)


def test_errors_are_reported(ctx):
    import paper_1410_5003_amd as mlh
    s = workloads.config1()
    st = mlh.Stack(ctx, s)
    with pytest.raises(mlh.MlhError) as e:
        st.solve([0.3])
    assert e.value.status == 1
    st.close()
    bad = workloads.config1(M_ud=40)          # M_ud < 2K+1
    with pytest.raises(mlh.MlhError) as e:
        mlh.Stack(ctx, bad)
    assert e.value.status == 1
    bad = workloads.config1()
    bad.interfaces[1].y0 = 0.1                # lies above Gamma_1
    with pytest.raises(mlh.MlhError) as e:
        mlh.Stack(ctx, bad)
    assert e.value.status == 2
    bad = workloads.config1()
    bad.R = 2.0                               # circle does not enclose the cell
    with pytest.raises(mlh.MlhError) as e:
        mlh.Stack(ctx, bad)
    assert e.value.status == 2
    bad = workloads.config1(N=30)             # fewer nodes than the Alpert stencil
    with pytest.raises(mlh.MlhError) as e:
        mlh.Stack(ctx, bad)
    assert e.value.status == 1
    bad = workloads.config1(N=600)            # more nodes than one block holds
    with pytest.raises(mlh.MlhError) as e:
        mlh.Stack(ctx, bad)
    assert e.value.status == 7


def test_cornered_errors_are_reported(ctx):
    import paper_1410_5003_amd as mlh
    bad = workloads.small_polygon_stack(nper=30)          # segment shorter than the Alpert window
    with pytest.raises(mlh.MlhError) as e:
        mlh.Stack(ctx, bad)
    assert e.value.status == 1
    bad = workloads.small_polygon_stack(nper=70, q=12.0)   # graded nodes collide with the corners
    with pytest.raises(mlh.MlhError) as e:
        mlh.Stack(ctx, bad)
    assert e.value.status == 1
    bad = workloads.small_polygon_stack(nper=60)
    bad.interfaces[0].vx = bad.interfaces[0].vx[::-1].copy()  # not a graph from -d/2 to d/2
    with pytest.raises(mlh.MlhError) as e:
        mlh.Stack(ctx, bad)
    assert e.value.status == 1
    bad = workloads.small_polygon_stack(nper=60)
    bad.interfaces[0].vy = bad.interfaces[0].vy - 0.6        # crosses the interface below
    with pytest.raises(mlh.MlhError) as e:
        mlh.Stack(ctx, bad)
    assert e.value.status == 2


def test_cornered_planar_stack_matches_fresnel(ctx):
    s = workloads.small_polygon_stack(flat=True, nper=72)
    g, o = _check(ctx, s)
    aU, aD, _ = fresnel.flat_stack_amplitudes(s.k, [0.0, -0.5], s.thetas[0], s.y_U, s.y_D)
    i0 = list(g.orders[0]).index(0)
    assert abs(g.aU[0, i0] - aU) < 3e-10 and abs(g.aD[0, i0] - aD) < 3e-10


def test_cornered_stack_resolved(ctx):
    _check(ctx, workloads.small_polygon_stack(nper=72))


def test_mixed_smooth_and_cornered_resolved(ctx):
    # uneven node counts: 72, 144, 72, 288
    _check(ctx, workloads.small_mixed_stack(min_seg=72))


RES3 = dict(N_smooth=260, N_corner=500, P=140, M_w=100)


@pytest.mark.parametrize("replay_cols", [16, 8])
def test_config3_head_resolved_twin(ctx, replay_cols):
    # first interfaces of the 1000-layer mixed smooth / cornered workload,
    # refined until the oracle's flux error is below 1e-9, three angles.  The
    # cornered interfaces give diagonal blocks of order 1000: their
    # right-hand-side replay keeps a 16-column tile in registers by default
    # and a 10-column LDS tile with the narrow launch choice
    import paper_1410_5003_amd as mlh
    s = workloads.config3(I=4, n_angles=3, **RES3)
    st = mlh.Stack(ctx, s)
    st.set_tuning(gje_rhs_cols=replay_cols)
    g = st.solve(s.thetas)
    st.close()
    for a, t in enumerate(s.thetas):
        o = oracle.solve_stack(s, theta=t)
        assert abs(o.flux_err) < 1e-9 and abs(g.flux_err[a]) < 1e-9
        err = rel_amp_err(g.aU[a], g.aD[a], o.aU, o.aD)
        print("config3 resolved head angle %d rel err %.2e" % (a, err))
        assert err < TOL


def test_config3_head_literal(ctx):
    # The first interfaces of the 1000-layer workload at the literal sizes
    # (N = 120 smooth, 250 cornered, P = 60 at k d up to 126: far from
    # resolved), three angles.  There the least-squares Schur solves are rank
    # deficient and the amplitudes are fixed by the method only up to what an
    # equally valid choice in them changes (the Remark closing Sec. 3.2):
    # noise 100 times below the fill parity bar moves them by more than 5e-4
    # (tests/test_oracle_solve.py).  So the path is held stage by stage:
    #   1. every fill piece entrywise to 1e-12 of the oracle's;
    #   2. the amplitudes to 5e-5 of the oracle's solve stages applied to the
    #      GPU's own fill pieces (their rounding spread, up to 2e-5 when the
    #      least-squares rows are rotated by random unitaries, is also pinned
    #      in tests/test_oracle_solve.py);
    #   3. the amplitudes to 5e-4 of the oracle's end-to-end solve.
    import paper_1410_5003_amd as mlh
    from oracle import alpert, fills
    from oracle.geometry import make_geometry
    from tests.gpu_common import gpu_pieces, max_piece_diff
    s = workloads.config3(I=4, n_angles=3)
    st = mlh.Stack(ctx, s)
    g = st.solve(s.thetas)
    rule = alpert.load_rule()
    op = fills.stack_pieces(s, make_geometry(s), rule)
    gp = gpu_pieces(st, s.I)
    st.close()
    dfill = max_piece_diff(gp, op)
    print("config3 literal head: fill pieces max rel diff %.2e" % dfill)
    assert dfill < 1e-12
    for a, t in enumerate(s.thetas):
        o = oracle.solve_stack(s, theta=t, rule=rule, pieces=op)
        og = oracle.solve_stack(s, theta=t, rule=rule, pieces=gp)
        assert np.array_equal(g.orders[a], o.orders)
        e_stage = rel_amp_err(g.aU[a], g.aD[a], og.aU, og.aD)
        e_full = rel_amp_err(g.aU[a], g.aD[a], o.aU, o.aD)
        print("config3 literal head angle %d: vs oracle on GPU pieces %.2e, vs oracle %.2e (flux %.1e)" %
              (a, e_stage, e_full, o.flux_err))
        assert e_stage < 5e-5
        assert e_full < 5e-4


def test_shared_alpha_angles_solved_as_one_system(ctx):
    # angles whose kappa_0 = k_1 cos(theta) differ by multiples of 2 pi/d share
    # alpha and hence every matrix (Sec. 3.4); they are solved as one system
    # with several right-hand sides.  Each angle must still match its own
    # oracle solve and the GPU's solve of that angle alone.
    import paper_1410_5003_amd as mlh
    s = workloads.config1(N=160, P=140, M_w=100)
    g = 2 * np.pi / s.d
    kap = [0.3 - 7 * g, 0.65 - g, 0.3, 0.3 + 3 * g, 0.65 + 4 * g, 0.3 - 2 * g, 0.3 + 8 * g]
    th = -np.arccos(np.array(kap) / s.k[0])
    st = mlh.Stack(ctx, s)
    out = st.solve(th)
    for a, t in enumerate(th):
        o = oracle.solve_stack(s, theta=t)
        assert np.array_equal(out.orders[a], o.orders)
        err = rel_amp_err(out.aU[a], out.aD[a], o.aU, o.aD)
        one = st.solve([t])
        err1 = rel_amp_err(out.aU[a], out.aD[a], one.aU[0], one.aD[0])
        print("kappa0 %+.3f rel err vs oracle %.2e vs single-angle GPU %.2e flux %.1e" %
              (kap[a], err, err1, out.flux_err[a]))
        assert err < TOL and err1 < 1e-11
        assert abs(out.flux_err[a]) < 1e-9
    st.close()


def test_solve_in_several_workspace_batches_matches_one_batch(ctx, monkeypatch):
    # distinct Bloch phases are independent systems; a workspace cap that
    # fits one system at a time splits the call into a batch per system
    # (a fresh stack then holds a workspace for one system only), with the
    # same arithmetic per system
    import paper_1410_5003_amd as mlh
    desc = workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9)  # flux error ~1e-11
    th = np.linspace(-1.3, -0.2, 6)
    st = mlh.Stack(ctx, desc)
    one = st.solve(th)
    bytes_one = st.info()["device_bytes"]
    st.close()
    monkeypatch.setenv("MLH_WORKSPACE_LIMIT_MB", "0.01")
    st = mlh.Stack(ctx, desc)
    many = st.solve(th)
    bytes_many = st.info()["device_bytes"]
    monkeypatch.delenv("MLH_WORKSPACE_LIMIT_MB")
    again = st.solve(th)  # the workspace grows back to one batch
    st.close()
    assert bytes_many < bytes_one
    for a in range(th.size):
        assert np.array_equal(one.orders[a], many.orders[a])
        assert rel_amp_err(many.aU[a], many.aD[a], one.aU[a], one.aD[a]) < 1e-13
        assert rel_amp_err(again.aU[a], again.aD[a], one.aU[a], one.aD[a]) < 1e-13
    o = oracle.solve_stack(desc, theta=float(th[2]))
    assert rel_amp_err(many.aU[2], many.aD[2], o.aU, o.aD) < TOL
