"""The solve's boundary (include/mlh.h): device-resident outputs, the
optional densities and the opt-in accuracy report, through the C ABI."""
import numpy as np
import pytest

import workloads
from tests.gpu_common import context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return context()


@pytest.fixture(scope="module")
def stack(ctx):
    import paper_1410_5003_amd as mlh
    # ragged sizes; three angles, two of which share alpha (one system with
    # two right-hand sides) and a third on its own
    desc = workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9)
    g = 2 * np.pi / desc.d
    k0 = float(np.cos(desc.thetas[0]) * desc.k[0])
    th = -np.arccos(np.array([k0, 0.5 * k0, k0 - g]) / desc.k[0])
    st = mlh.Stack(ctx, desc)
    yield desc, st, th
    st.close()


def test_device_outputs_match_host_outputs_bitwise(stack):
    import torch
    desc, st, th = stack
    host = st.solve(th, eta=True)
    na, nK, nden = th.size, 2 * desc.K + 1, st.info()["n_den"]
    dev = torch.device("cuda", 0)
    aU = torch.zeros((na, nK), dtype=torch.complex128, device=dev)
    aD = torch.zeros_like(aU)
    orders = torch.zeros((na, nK), dtype=torch.int32, device=dev)
    flux = torch.zeros(na, dtype=torch.float64, device=dev)
    eta = torch.zeros((na, nden), dtype=torch.complex128, device=dev)
    st.solve_into(th, aU, aD, orders, flux, eta)
    torch.cuda.current_stream().synchronize()
    assert np.array_equal(aU.cpu().numpy(), host.aU)
    assert np.array_equal(aD.cpu().numpy(), host.aD)
    assert np.array_equal(orders.cpu().numpy(), host.orders)
    assert np.array_equal(flux.cpu().numpy(), host.flux_err)
    assert np.array_equal(eta.cpu().numpy(), host.eta)
    # optional outputs may be left out
    st.solve_into(th, aU, aD)
    torch.cuda.current_stream().synchronize()
    assert np.array_equal(aU.cpu().numpy(), host.aU)


def test_densities_are_the_block_solve_result(stack):
    # eta returned by the solve is the solution of the block-tridiagonal
    # system (Sec. 3.3) that the inspection path leaves in the workspace
    desc, st, th = stack
    out = st.solve(th[:1], eta=True)
    st.solve_partial(float(th[0]), 4)
    n = [2 * f.N for f in desc.interfaces]
    off = np.concatenate([[0], np.cumsum(n)])
    assert out.eta.shape == (1, off[-1])
    for i in range(desc.I):
        ref = st.work("eta", i)[:, 0]
        assert np.max(np.abs(out.eta[0, off[i]:off[i + 1]] - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_densities_of_angles_sharing_alpha_are_their_own(stack):
    # the two angles sharing alpha have separate right-hand sides, so their
    # densities differ.  The densities themselves are not unique: the Schur
    # step picks one of many admissible quasi-periodic Green's functions
    # (Remark after eq. (78)), and on this stack the oracle's own densities
    # move by tens of percent between Tikhonov weights 1e-14 and 1e-13 while
    # the amplitudes move by 1e-12.  So each angle is held to its own
    # single-angle solve through what is unique, the Bragg amplitudes.
    desc, st, th = stack
    out = st.solve(th, eta=True)
    for a in range(th.size):
        one = st.solve(th[a:a + 1], eta=True)
        assert np.array_equal(out.orders[a], one.orders[0])
        scale = max(np.max(np.abs(one.aU)), np.max(np.abs(one.aD)))
        err = max(np.max(np.abs(out.aU[a] - one.aU[0])), np.max(np.abs(out.aD[a] - one.aD[0])))
        assert err < 1e-10 * scale, (a, err / scale)
        assert np.all(np.isfinite(out.eta[a])) and np.max(np.abs(out.eta[a])) > 0
    assert np.max(np.abs(out.eta[0] - out.eta[2])) > 1e-3 * np.max(np.abs(out.eta[0]))


def test_accuracy_report_is_opt_in(stack):
    import paper_1410_5003_amd as mlh
    desc, st, th = stack
    ok = st.solve(th)                       # no tolerance set: no report
    st.set_flux_tolerance(1e-300)           # below any attainable flux error
    with pytest.raises(mlh.MlhError) as e:
        st.solve(th)
    assert e.value.status == 6 and "flux error" in str(e.value)
    st.set_flux_tolerance(10 * np.max(np.abs(ok.flux_err)) + 1e-300)
    st.solve(th)                            # within the tolerance
    with pytest.raises(mlh.MlhError) as e:
        st.set_flux_tolerance(-1.0)
    assert e.value.status == 1
    st.set_flux_tolerance(0.0)
    nK = 2 * desc.K + 1
    aU, aD = np.zeros(nK, dtype=np.complex128), np.zeros(nK, dtype=np.complex128)
    t1 = np.array(th[:1])
    with pytest.raises(mlh.MlhError) as e:  # outputs_on_device must be 0 or 1
        mlh.check(mlh.lib().mlh_solve(st._h, 1, mlh._lib.dptr(t1), 2, aU.ctypes.data, aD.ctypes.data,
                                      None, None, None))
    assert e.value.status == 1 and "outputs_on_device" in str(e.value)
