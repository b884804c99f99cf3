"""Write the oracle's Bragg amplitudes for the large parity cases.

The oracle needs about a minute per angle on these stacks, so the GPU tests
read its results from the JSON files written here instead of recomputing
them.  This script calls only ``oracle`` and ``workloads`` (no GPU code):

    python tests/golden/make_golden.py            # every case
    python tests/golden/make_golden.py NAME ...   # some of them

Each file holds, per angle: theta, the order labels, a^U and a^D as
(re, im) pairs and the flux error (Sec. 3.3 and eq. (86)).
"""
import json
import os
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402
from oracle import alpert, fills  # noqa: E402
from oracle.geometry import make_geometry  # noqa: E402

RES3 = dict(N_smooth=260, N_corner=500, P=140, M_w=100)


def config3_res40_thetas(desc):
    """Two angles whose kappa_0 = k_1 cos(theta) differ by 2 pi/d (one Bloch
    phase, hence one system with two right-hand sides) and a third angle with
    its own phase."""
    g = 2 * np.pi / desc.d
    k1 = desc.k[0]
    kap = np.array([0.35 * k1, 0.35 * k1 - g, -0.2 * k1])
    return -np.arccos(kap / k1)


# the resolved 64-stack batch: omega ~ U[5,8], I ~ U{10..100} and every
# interface raised to 18 k_max (smooth) / 25 k_max (cornered) nodes
C4R = dict(omega_range=(5.0, 8.0), I_range=(10, 100), P=140, M_w=100, nodes_per_k=(18.0, 25.0))
C4R_STACKS = (58, 34, 36)  # the three with the fewest interfaces (10, 10, 12)

CASES = {
    # name: (stack generator, angle chooser)
    "config2_resolved": (lambda: workloads.config2(N=260, P=120, M_w=80), lambda d: d.thetas[:1]),
    "config3_res40": (lambda: workloads.config3(I=40, n_angles=3, **RES3), config3_res40_thetas),
}
for _j in C4R_STACKS:
    CASES["config4_resolved_s%d" % _j] = ((lambda j=_j: workloads.config4(**C4R)[j]), lambda d: d.thetas)


def make(name):
    gen, pick = CASES[name]
    desc = gen()
    thetas = np.asarray(pick(desc), dtype=float)
    rule = alpert.load_rule()
    t0 = time.perf_counter()
    pieces = fills.stack_pieces(desc, make_geometry(desc), rule)
    out = []
    for t in thetas:
        o = oracle.solve_stack(desc, theta=float(t), rule=rule, pieces=pieces)
        out.append({"theta": float(t), "orders": [int(v) for v in o.orders],
                    "aU": [[float(z.real), float(z.imag)] for z in o.aU],
                    "aD": [[float(z.real), float(z.imag)] for z in o.aD],
                    "flux_err": float(o.flux_err)})
        print("%s theta %.15f flux %.3e (%.0f s)" % (name, t, o.flux_err, time.perf_counter() - t0), flush=True)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump({"case": name, "written_by": "tests/golden/make_golden.py (oracle only)", "angles": out}, f,
                  indent=1)


def load(name):
    """The stored oracle results of one case: list of dicts with theta,
    orders (int array), aU, aD (complex arrays) and flux_err."""
    with open(os.path.join(HERE, name + ".json")) as f:
        data = json.load(f)
    res = []
    for a in data["angles"]:
        res.append({"theta": a["theta"], "orders": np.array(a["orders"], dtype=np.int32),
                    "aU": np.array([complex(*z) for z in a["aU"]]),
                    "aD": np.array([complex(*z) for z in a["aD"]]),
                    "flux_err": a["flux_err"]})
    return res


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
