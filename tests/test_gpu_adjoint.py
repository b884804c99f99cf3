"""The adjoint gradient (mlh_adjoint) of the summed zeroth-order reflected
efficiency with respect to the layer wavenumbers, against the oracle's
gradient (central differences of the oracle's forward map) and against
central differences of the GPU's own forward solve (step 1e-6 in the layer
index), on smooth and cornered stacks; and its torch.autograd wrapper."""
import numpy as np
import pytest

import workloads
from oracle import adjoint as oadj
from tests.gpu_common import context

pytestmark = pytest.mark.gpu


def _gpu_J(ctx, desc, thetas):
    import paper_1410_5003_amd as mlh
    st = mlh.Stack(ctx, desc)
    out = st.solve(thetas)
    st.close()
    i0 = [list(o).index(0) for o in out.orders]
    return float(sum(abs(out.aU[a, i0[a]]) ** 2 for a in range(len(thetas))))


def test_adjoint_matches_the_oracle_gradient():
    import paper_1410_5003_amd as mlh
    ctx = context()
    pb = workloads.small_shape_problem(I=3, N=64, P=44, M_w=40, thetas=(-0.6, -1.1))
    th = pb.base.thetas
    st = mlh.Stack(ctx, pb.stack())
    J, gk = st.adjoint(th)
    st.close()
    nc = pb.c.size
    Jo = oadj.objective(pb)
    go = oadj.gradient_fd(pb, which=range(nc + 1, nc + pb.n.size), h=1e-5) / pb.omega  # dJ/dk_j, j >= 1
    print("J gpu %.12e oracle %.12e" % (J, Jo))
    print("dJ/dk gpu", gk[1:], "oracle", go)
    assert abs(J - Jo) < 1e-10 * abs(Jo)
    assert np.isnan(gk[0])
    err = np.max(np.abs(gk[1:] - go)) / np.max(np.abs(go))
    print("adjoint vs oracle: rel err %.2e" % err)
    assert err < 1e-6, err


@pytest.mark.parametrize("which", ["smooth", "mixed"])
def test_adjoint_matches_gpu_central_differences(which):
    import paper_1410_5003_amd as mlh
    ctx = context()
    if which == "smooth":
        desc = workloads.small_stack(seed=6, I=4, N=77, P=45, M_w=35, M_ud=40, K=9)
    else:
        desc = workloads.small_mixed_stack(seed=7, I=4, P=60, M_w=40, M_ud=40, K=8)
    th = np.array([-0.55, -0.9, -1.25])
    st = mlh.Stack(ctx, desc)
    J, gk = st.adjoint(th)
    st.close()
    h = 1e-6
    fd = []
    for j in range(1, desc.I + 1):
        dp = workloads.Stack(**{**desc.__dict__, "k": desc.k + h * np.eye(desc.I + 1)[j]})
        dm = workloads.Stack(**{**desc.__dict__, "k": desc.k - h * np.eye(desc.I + 1)[j]})
        fd.append((_gpu_J(ctx, dp, th) - _gpu_J(ctx, dm, th)) / (2 * h))
    fd = np.array(fd)
    err = np.max(np.abs(gk[1:] - fd)) / np.max(np.abs(fd))
    print("%s: adjoint %s  fd %s  rel err %.2e" % (which, gk[1:], fd, err))
    assert err < 1e-5, err


def test_autograd_function_returns_the_adjoint_gradient():
    import torch
    import paper_1410_5003_amd as mlh
    ctx = context()
    pb = workloads.small_shape_problem(I=3, N=64, P=44, M_w=40, thetas=(-0.6, -1.1))
    F = mlh.EfficiencyObjective.function()
    c = torch.tensor(pb.c, dtype=torch.float64, requires_grad=True)
    n = torch.tensor(pb.n, dtype=torch.float64, requires_grad=True)
    J = F.apply(c, n, pb, ctx, pb.base.thetas)
    J.backward()
    st = mlh.Stack(ctx, pb.stack())
    J2, gk, gs = st.adjoint(pb.base.thetas, shape=True)
    st.close()
    assert abs(J.item() - J2) < 1e-14 * abs(J2)
    assert n.grad[0].item() == 0.0
    # the contractions sum tile results with atomics, in no fixed order
    scale = np.max(np.abs(pb.omega * gk[1:]))
    assert np.max(np.abs(n.grad.numpy()[1:] - pb.omega * gk[1:])) < 1e-10 * scale
    gc = _chain_c(pb, gs)
    assert np.max(np.abs(c.grad.numpy().ravel() - gc)) < 1e-10 * np.max(np.abs(gc))


def _chain_c(pb, gs):
    """dJ/dc from dJ/d(cos_coef, sin_coef): cos_coef = c sin psi, sin_coef = c cos psi."""
    M = pb.c.shape[1]
    g = gs.reshape(-1, 2, M)
    return (g[:, 0, :] * np.sin(pb.psi) + g[:, 1, :] * np.cos(pb.psi)).ravel()


def test_shape_adjoint_matches_the_oracle_gradient():
    import paper_1410_5003_amd as mlh
    ctx = context()
    pb = workloads.small_shape_problem(I=3, N=64, P=44, M_w=40, thetas=(-0.6, -1.1))
    st = mlh.Stack(ctx, pb.stack())
    J, gk, gs = st.adjoint(pb.base.thetas, shape=True)
    st.close()
    gc = _chain_c(pb, gs)
    go = oadj.gradient_fd(pb, which=range(pb.c.size), h=1e-5)
    err = np.max(np.abs(gc - go)) / np.max(np.abs(go))
    print("shape adjoint", gc, "\noracle", go, "\nrel err %.2e" % err)
    assert err < 1e-5, err


def test_adjoint_matches_gpu_central_differences_on_the_100_interface_problem():
    # 20 random parameters (12 amplitudes, 8 layer indices) of the
    # 100-interface, 10-angle problem at resolved sizes (N = 260, P = 120,
    # M_w = 80: flux error 2e-9 at most).  The adjoint differentiates the
    # discrete system as a consistent one (da0 = -l^T dE u), which holds to
    # the discretisation error; at the literal N = 100, P = 50 the
    # discretisation error is of order one and the two derivatives part.
    import paper_1410_5003_amd as mlh
    ctx = context()
    pb = workloads.config5(N=260, P=120, M_w=80)
    th = pb.base.thetas
    st = mlh.Stack(ctx, pb.stack())
    out = st.solve(th)
    print("flux error: max %.2e" % np.max(np.abs(out.flux_err)))
    assert np.max(np.abs(out.flux_err)) < 5e-9
    J, gk, gs = st.adjoint(th, shape=True)
    st.close()
    gc = _chain_c(pb, gs)
    gn = pb.omega * gk
    rng = np.random.default_rng(20)
    pick_c = rng.choice(pb.c.size, 12, replace=False)
    pick_n = 1 + rng.choice(pb.n.size - 1, 8, replace=False)
    h = 1e-6
    p0 = pb.params()
    worst = 0.0
    scale = max(np.max(np.abs(gc)), np.max(np.abs(gn[1:])))
    for q in list(pick_c) + [pb.c.size + j for j in pick_n]:
        e = np.zeros_like(p0)
        e[q] = h
        fd = (_gpu_J(ctx, pb.stack(p0 + e), th) - _gpu_J(ctx, pb.stack(p0 - e), th)) / (2 * h)
        ad = gc[q] if q < pb.c.size else gn[q - pb.c.size]
        worst = max(worst, abs(ad - fd))
        print("param %4d adjoint % .10e fd % .10e" % (q, ad, fd))
    print("max abs diff %.2e, scale %.2e" % (worst, scale))
    assert worst < 1e-5 * scale
