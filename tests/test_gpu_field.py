"""Field evaluation on the GPU (mlh_field) against the oracle's field and
the closed-form flat-stack field (Sec. 3.3, last paragraph; eq. (16)-(18),
(7)-(8), (6)).

The densities are not unique (Remark after eq. (78)), the field is: far
from the interfaces the oracle's own fields for Tikhonov weights 1e-14 and
1e-13 agree to ~3e-12, while within a few node spacings of an interface
the uncorrected quadrature of the potentials turns the density differences
into field differences of up to ~1e-1.  Targets are therefore kept at least
eight node spacings from every interface."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import field as ofield
from oracle import fresnel
from oracle.geometry import curve_height_at, make_geometry
from tests.gpu_common import context

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _targets(desc, n, seed, spacings=8.0, cells=1.5):
    """Targets across every region, also outside the unit cell, at least
    `spacings` node spacings from every interface."""
    geom = make_geometry(desc)
    gap = max(float(np.max(np.hypot(np.diff(c.x), np.diff(c.y)))) for c in geom.curves)
    h = gap * spacings
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    while len(xs) < n:
        x = rng.uniform(-cells * desc.d, cells * desc.d)
        y = rng.uniform(desc.y_D - 0.6, desc.y_U + 0.6)
        xc = x - np.floor((x + desc.d / 2) / desc.d) * desc.d
        if min(abs(y - curve_height_at(c, xc)) for c in geom.curves) >= h:
            xs.append(x)
            ys.append(y)
    return np.array(xs), np.array(ys)


@pytest.mark.parametrize("which", ["smooth", "mixed"])
def test_field_matches_the_oracle(which):
    import paper_1410_5003_amd as mlh
    ctx = context()
    desc = (workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9) if which == "smooth"
            else workloads.small_mixed_stack(seed=7, I=4, P=60, M_w=40, M_ud=40, K=8))
    th = float(desc.thetas[0])
    x, y = _targets(desc, 160, seed=3)
    st = mlh.Stack(ctx, desc)
    u, reg = st.field(th, x, y)
    res = oracle.solve_stack(desc, theta=th, keep_blocks=True)
    uo, lo = ofield.field(desc, th, x, y, res=res)
    assert np.array_equal(reg, lo)
    assert set(lo) == set(range(-1, desc.I + 2))
    err = np.max(np.abs(u - uo)) / np.max(np.abs(uo))
    # the field is fixed by the method only up to its discretisation error:
    # the bar is the larger of 1e-10 and the oracle's flux error (the smooth
    # stack is resolved, 2.5e-11; the cornered one is not, 1.7e-8)
    bar = max(TOL, abs(res.flux_err))
    print("%s: field rel err %.2e over %d targets (bar %.1e)" % (which, err, x.size, bar))
    assert err < bar, err
    st.close()


def test_flat_stack_field_is_the_closed_form():
    import paper_1410_5003_amd as mlh
    ctx = context()
    desc = workloads.config1_flat(N=160, P=140, M_w=100)
    th = float(desc.thetas[0])
    x, y = _targets(desc, 120, seed=4)
    st = mlh.Stack(ctx, desc)
    u, reg = st.field(th, x, y)
    tot = u + np.where(reg <= 0, ofield.incident(desc, th, x, y), 0)
    ref = fresnel.flat_stack_total_field(desc.k, [0.0, -2.0], th, desc.y_U, desc.y_D, x, y)
    err = np.max(np.abs(tot - ref)) / np.max(np.abs(ref))
    print("flat: total field rel err %.2e" % err)
    assert err < TOL, err
    st.close()


def test_field_device_outputs_and_edge_cases():
    import torch
    import paper_1410_5003_amd as mlh
    ctx = context()
    desc = workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9)
    th = float(desc.thetas[0])
    x, y = _targets(desc, 300, seed=5)
    st = mlh.Stack(ctx, desc)
    u, reg = st.field(th, x, y)
    dev = torch.device("cuda", 0)
    ud = torch.zeros(x.size, dtype=torch.complex128, device=dev)
    rd = torch.zeros(x.size, dtype=torch.int32, device=dev)
    xs, ys = np.ascontiguousarray(x), np.ascontiguousarray(y)
    mlh.check(mlh.lib().mlh_field(st._h, th, x.size, mlh._lib.dptr(xs), mlh._lib.dptr(ys), 1, ud.data_ptr(),
                                  rd.data_ptr()))
    torch.cuda.current_stream().synchronize()
    assert np.array_equal(ud.cpu().numpy(), u) and np.array_equal(rd.cpu().numpy(), reg)
    # no targets; a non-finite target; an angle outside (-pi, 0)
    e0 = st.field(th, np.zeros(0), np.zeros(0))
    assert e0[0].size == 0
    with pytest.raises(mlh.MlhError) as e:
        st.field(th, np.array([0.0, np.nan]), np.array([0.0, 0.0]))
    assert e.value.status == 1
    with pytest.raises(mlh.MlhError) as e:
        st.field(0.3, x[:3], y[:3])
    assert e.value.status == 1
    st.close()
