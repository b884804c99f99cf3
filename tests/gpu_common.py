"""Shared helpers for the GPU parity tests."""
import numpy as np
import pytest


def context():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1410_5003_amd as mlh
    return mlh.Context(0)


def rel_amp_err(gU, gD, oU, oD):
    """max over orders (U and D together) of |a_gpu - a_oracle| / max |a_oracle|."""
    scale = max(np.max(np.abs(oU)), np.max(np.abs(oD)))
    return max(np.max(np.abs(gU - oU)), np.max(np.abs(gD - oD))) / scale
