"""GPU unit parity: the device Hankel routine and the FP64-MFMA GEMM."""
import numpy as np
import pytest

from oracle import special
from tests.gpu_common import context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return context()


def test_hankel_all_branches(ctx):
    x = np.concatenate([np.geomspace(1e-7, 2.0, 300), np.linspace(2.0, 20.0, 500)[1:],
                        np.linspace(20.0, 80.0, 300), np.geomspace(80.0, 2000.0, 200)])
    out = ctx.hankel(x)
    h0, g1m, _ = special.hankel_pieces(x)
    e0 = np.abs(out[:, 0] - h0) / np.abs(h0)
    e1 = np.abs(out[:, 1] - g1m) / np.abs(g1m)
    assert np.max(e0) < 5e-15, (x[np.argmax(e0)], np.max(e0))
    assert np.max(e1) < 5e-15, (x[np.argmax(e1)], np.max(e1))


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (16, 16, 4), (33, 17, 9), (64, 64, 16),
                                   (200, 201, 50), (241, 111, 67), (5, 300, 200)])
def test_zgemm_matches_numpy(ctx, m, n, k):
    rng = np.random.default_rng(m * 1000 + n * 10 + k)
    A = rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k))
    B = rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n))
    C0 = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    alpha = -0.7 + 0.3j
    got = ctx.zgemm(alpha, A, B, C0)
    want = C0 + alpha * (A @ B)
    assert np.max(np.abs(got - want)) < 1e-13 * max(1.0, k ** 0.5) * 4
