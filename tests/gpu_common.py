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


def gpu_pieces(st, I):
    """Every alpha-independent fill piece of a GPU stack, in the layout of
    ``oracle.fills.stack_pieces`` (inspection calls of the C ABI)."""
    def many(name, idx, npieces):
        return np.stack([st.piece(name, idx, p) for p in range(npieces)])
    out = {"A_self": [many("A_self", i, 3) for i in range(I)],
           "A_up": [many("A_up", i, 3) for i in range(I - 1)],
           "A_dn": [many("A_dn", i, 3) for i in range(I - 1)],
           "B_own": [st.piece("B_own", i) for i in range(I)],
           "B_below": [st.piece("B_below", i) for i in range(I)],
           "C_own": [many("C_own", j, 2) if j < I else None for j in range(I + 1)],
           "C_above": [many("C_above", j, 2) if j > 0 else None for j in range(I + 1)],
           "Q": [many("Q", j, 2) for j in range(I + 1)],
           "Z_U": many("Z_U", 0, 3), "Z_D": many("Z_D", 0, 3),
           "V_U": st.piece("V_U"), "V_D": st.piece("V_D")}
    return out


def max_piece_diff(gp, op):
    """Largest entrywise difference of two piece sets, relative to the
    largest entry of each oracle piece."""
    worst = 0.0
    for key, o in op.items():
        g = gp[key]
        pairs = zip(g, o) if isinstance(o, list) else [(g, o)]
        for a, b in pairs:
            if b is None:
                continue
            worst = max(worst, float(np.abs(np.asarray(a) - b).max() / np.abs(b).max()))
    return worst
