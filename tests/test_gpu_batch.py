"""Batches of independent stacks (mlh_batch_*): every stack of a batch,
solved with the others in shared launches, against its own mlh_solve and
against the oracle (Sec. 3.2-3.3 per stack; Bragg amplitudes and flux error
eq. (86)).  Order labels exact; amplitudes at 1e-10 relative."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_common import context, rel_amp_err

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _stacks():
    """Heterogeneous small stacks: interface counts, node counts (smooth,
    cornered, ragged), proxy and wall counts, Bragg orders, wavenumbers and
    periods all differ between them."""
    return [
        workloads.small_stack(seed=1, I=3, N=64, P=40, M_w=40, M_ud=40, K=8, theta=-0.7),
        workloads.small_mixed_stack(seed=7, I=5, theta=-1.1),
        workloads.small_stack(seed=2, I=2, N=77, P=45, M_w=35, M_ud=40, K=9, theta=-0.4),
        workloads.small_polygon_stack(theta=-0.9),
        workloads.small_stack(seed=3, I=7, N=50, P=36, M_w=32, M_ud=34, K=6, omega=6.0, theta=-1.3),
    ]


@pytest.fixture(scope="module")
def batch():
    import paper_1410_5003_amd as mlh
    ctx = context()
    descs = _stacks()
    sts = [mlh.Stack(ctx, d) for d in descs]
    b = mlh.Batch(ctx, sts)
    th = np.array([float(d.thetas[0]) for d in descs])
    yield descs, sts, b, th
    b.close()
    for s in sts:
        s.close()


def _check_against_single(descs, sts, out, th, label):
    for i, (d, st) in enumerate(zip(descs, sts)):
        one = st.solve(th[i:i + 1])
        assert np.array_equal(out.orders[i], one.orders[0]), (label, i)
        err = rel_amp_err(out.aU[i], out.aD[i], one.aU[0], one.aD[0])
        assert err < TOL, (label, i, err)
        assert abs(out.flux_err[i] - one.flux_err[0]) < 1e-12, (label, i)


def test_batch_matches_each_stack_solved_alone(batch):
    descs, sts, b, th = batch
    out = b.solve(th)
    _check_against_single(descs, sts, out, th, "first solve")
    # the captured graph replayed with other angles (new descriptors only)
    th2 = th * 0.8 - 0.1
    _check_against_single(descs, sts, b.solve(th2), th2, "replay")


def test_batch_refill_recomputes_the_same_pieces(batch):
    descs, sts, b, th = batch
    a = b.solve(th)
    r = b.solve(th, refill=True)
    for i in range(len(descs)):
        assert np.array_equal(a.aU[i], r.aU[i]) and np.array_equal(a.aD[i], r.aD[i])


def test_batch_stack_times_are_device_clock_intervals(batch):
    descs, sts, b, th = batch
    out = b.solve(th)
    assert np.all(np.isfinite(out.stack_ms)) and np.all(out.stack_ms > 0)
    assert np.all(out.stack_ms < 60e3)


def test_batch_against_the_oracle():
    # three resolved stacks (oracle flux error below 1e-9) in one batch
    import paper_1410_5003_amd as mlh
    ctx = context()
    descs = [workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9, theta=-0.6),
             workloads.small_stack(seed=8, I=3, N=70, P=44, M_w=40, M_ud=40, K=8, theta=-1.0),
             workloads.small_stack(seed=9, I=6, N=64, P=42, M_w=38, M_ud=40, K=8, omega=7.0, theta=-0.3)]
    sts = [mlh.Stack(ctx, d) for d in descs]
    b = mlh.Batch(ctx, sts)
    th = np.array([float(d.thetas[0]) for d in descs])
    out = b.solve(th)
    for i, d in enumerate(descs):
        o = oracle.solve_stack(d, theta=float(th[i]))
        assert np.array_equal(out.orders[i], o.orders), i
        err = rel_amp_err(out.aU[i], out.aD[i], o.aU, o.aD)
        print("stack %d: rel amp err %.2e  flux gpu %.2e oracle %.2e" % (i, err, out.flux_err[i], o.flux_err))
        assert abs(o.flux_err) <= 1e-9 and abs(out.flux_err[i]) <= 1e-9, i
        assert err < TOL, (i, err)
    b.close()
    for s in sts:
        s.close()


def test_resolved_batch_stacks_against_stored_oracle_results():
    # three stacks of the resolved 64-stack workload (omega ~ U[5,8], nodes
    # raised to 18 k_max smooth / 25 k_max cornered, P = 140, M_w = 100; the
    # oracle's flux error is below 1e-9 on each) in one batch, against the
    # oracle results that tests/golden/make_golden.py stores
    import paper_1410_5003_amd as mlh
    from tests.golden.make_golden import C4R, C4R_STACKS, load as load_golden
    ctx = context()
    every = workloads.config4(**C4R)
    descs = [every[j] for j in C4R_STACKS]
    sts = [mlh.Stack(ctx, d) for d in descs]
    b = mlh.Batch(ctx, sts)
    th = np.array([float(d.thetas[0]) for d in descs])
    out = b.solve(th)
    for i, j in enumerate(C4R_STACKS):
        gold = load_golden("config4_resolved_s%d" % j)[0]
        assert abs(gold["theta"] - th[i]) < 1e-15
        assert np.array_equal(out.orders[i], gold["orders"]), j
        err = rel_amp_err(out.aU[i], out.aD[i], gold["aU"], gold["aD"])
        print("stack %d (I=%d): rel amp err %.2e  flux gpu %.2e oracle %.2e" % (j, descs[i].I, err, out.flux_err[i],
                                                                             gold["flux_err"]))
        assert abs(gold["flux_err"]) <= 1e-9 and abs(out.flux_err[i]) <= 1e-9, j
        assert err < TOL, (j, err)
    b.close()
    for s in sts:
        s.close()


def test_batch_autotune_keeps_results(batch):
    descs, sts, b, th = batch
    t = b.autotune(th, reps=1)
    assert set(t) == {"rhs_in_step_pct", "ls_row_blocks", "gje_rhs_cols", "asm_in_panels", "gemm_slab_k"}
    _check_against_single(descs, sts, b.solve(th), th, "tuned")
    b.set_tuning(rhs_in_step_pct=300, ls_row_blocks=3, gje_rhs_cols=16, asm_in_panels=1)


def test_batch_rejects_bad_input(batch):
    import ctypes as C
    import paper_1410_5003_amd as mlh
    descs, sts, b, th = batch
    with pytest.raises(mlh.MlhError) as e:  # a stack twice
        mlh.Batch(sts[0].ctx, [sts[0], sts[0]])
    assert e.value.status == 1
    with pytest.raises(mlh.MlhError) as e:  # an angle outside (-pi, 0)
        b.solve(np.where(np.arange(th.size) == 2, 0.1, th))
    assert e.value.status == 1
    hs = (C.c_void_p * 2)(sts[0]._h.value, None)
    h = C.c_void_p()
    assert mlh.lib().mlh_batch_create(sts[0].ctx.handle, 2, hs, C.byref(h)) == 1
