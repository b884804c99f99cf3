"""The allocation-free solve (mlh_solve_noalloc, include/mlh.h) against
mlh_solve through the C ABI: two calls in a row, the second on a smaller
input, held to the amplitude bar of the parity tests (1e-10 relative, order
labels exact); and the clear rejection of a stack whose workspace exceeds
the fixed area."""
import ctypes as C

import numpy as np
import pytest

import workloads
from tests.gpu_common import context, rel_amp_err

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _solve(st, th, noalloc, on_device=False):
    """One call of mlh_solve or mlh_solve_noalloc with host outputs, or with
    device outputs in torch tensors."""
    import paper_1410_5003_amd as mlh
    th = np.ascontiguousarray(th, dtype=np.float64)
    na, nK, nden = th.size, 2 * st.K + 1, st.info()["n_den"]
    fn = mlh.lib().mlh_solve_noalloc if noalloc else mlh.lib().mlh_solve
    if not on_device:
        aU = np.zeros((na, nK), dtype=np.complex128)
        aD = np.zeros_like(aU)
        orders = np.zeros((na, nK), dtype=np.int32)
        flux = np.zeros(na)
        eta = np.zeros((na, nden), dtype=np.complex128)
        mlh.check(fn(st._h, na, mlh._lib.dptr(th), 0, aU.ctypes.data, aD.ctypes.data, orders.ctypes.data,
                     flux.ctypes.data, eta.ctypes.data))
        return aU, aD, orders, flux, eta
    import torch
    dev = torch.device("cuda", 0)
    t = dict(aU=torch.zeros((na, nK), dtype=torch.complex128, device=dev),
             aD=torch.zeros((na, nK), dtype=torch.complex128, device=dev),
             orders=torch.zeros((na, nK), dtype=torch.int32, device=dev),
             flux=torch.zeros(na, dtype=torch.float64, device=dev),
             eta=torch.zeros((na, nden), dtype=torch.complex128, device=dev))
    mlh.check(fn(st._h, na, mlh._lib.dptr(th), 1, t["aU"].data_ptr(), t["aD"].data_ptr(), t["orders"].data_ptr(),
                 t["flux"].data_ptr(), t["eta"].data_ptr()))
    torch.cuda.current_stream().synchronize()
    return tuple(t[k].cpu().numpy() for k in ("aU", "aD", "orders", "flux", "eta"))


def _same(ref, got, label):
    aU, aD, orders, flux, eta = got
    assert np.array_equal(orders, ref[2]), label
    for a in range(aU.shape[0]):
        err = rel_amp_err(aU[a], aD[a], ref[0][a], ref[1][a])
        assert err < TOL, (label, a, err)
        assert abs(flux[a] - ref[3][a]) <= 1e-12, (label, a)
    # the densities are the block solve's result for the same matrices
    assert np.max(np.abs(eta - ref[4])) <= 1e-10 * np.max(np.abs(ref[4])), label


def test_noalloc_matches_solve_twice_second_smaller():
    import paper_1410_5003_amd as mlh
    ctx = context()
    # first call: ragged sizes, three angles of which two share alpha
    big = workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9)
    g = 2 * np.pi / big.d
    k0 = float(np.cos(big.thetas[0]) * big.k[0])
    th_big = -np.arccos(np.array([k0, 0.5 * k0, k0 - g]) / big.k[0])
    st_big = mlh.Stack(ctx, big)
    ref = _solve(st_big, th_big, noalloc=False)
    _same(ref, _solve(st_big, th_big, noalloc=True), "first call, host outputs")
    # second call: a smaller stack and one angle, device outputs; the area
    # still holds the first call's contents
    small = workloads.small_stack(seed=11, I=2, N=48, P=40, M_w=32, M_ud=34, K=8)
    st_small = mlh.Stack(ctx, small)
    th_small = np.asarray(small.thetas[:1], dtype=float)
    ref_s = _solve(st_small, th_small, noalloc=False)
    _same(ref_s, _solve(st_small, th_small, noalloc=True, on_device=True), "second call, device outputs")
    # and the larger one again, after the smaller
    _same(ref, _solve(st_big, th_big, noalloc=True, on_device=True), "third call, device outputs")
    st_small.close()
    st_big.close()
    ctx.close()


def test_noalloc_rejects_a_stack_beyond_the_area():
    import paper_1410_5003_amd as mlh
    ctx = context()
    # 50 interfaces of 200 unknowns: one system needs ~200 MiB of workspace
    desc = workloads.config2()
    st = mlh.Stack(ctx, desc)
    th = np.asarray(desc.thetas[:1], dtype=float)
    with pytest.raises(mlh.MlhError) as e:
        st.solve(th, noalloc=True)
    assert e.value.status == 7 and "allocation-free" in str(e.value)
    st.close()
    ctx.close()
