"""Self-convergence of the oracle's Bragg amplitudes under refinement.

The paper's stacks carry no printed amplitudes, so beside the closed forms
and invariants the oracle is pinned by the convergence rates its
discretisation must show (Sec. 2.5 and Sec. 4):

* smooth interfaces, N nodes: the periodic trapezoid rule with Alpert's
  order-16 log correction converges at high algebraic order (about 15
  observed here);
* proxy count P: super-algebraic (geometric) convergence of the proxy basis;
* cornered interfaces, n graded nodes per segment: order q of the Kress
  grading (q = 6 here).

Each rate is measured against a reference solve at a much finer
discretisation of the same stack.  A dropped term, a wrong sign or a
mis-indexed correction breaks these rates, even where the flux still
balances.
"""
import numpy as np

import oracle
import workloads


def _rel(o, ref):
    scale = max(np.abs(ref.aU).max(), np.abs(ref.aD).max())
    return max(np.abs(o.aU - ref.aU).max(), np.abs(o.aD - ref.aD).max()) / scale


def _orders(ns, errs):
    return [np.log(errs[i] / errs[i + 1]) / np.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)]


def _smooth(**kw):
    return oracle.solve_stack(workloads.small_stack(seed=3, I=2, M_w=40, M_ud=40, K=8, **kw))


def test_smooth_node_refinement_high_order():
    ref = _smooth(N=160, P=80)
    ns = [40, 48, 56, 64]
    errs = [_rel(_smooth(N=n, P=80), ref) for n in ns]
    orders = _orders(ns, errs)
    print("N", ns, ["%.2e" % e for e in errs], "orders", ["%.1f" % p for p in orders])
    assert all(p > 12 for p in orders), orders
    assert errs[-1] < 1e-12


def test_proxy_refinement_geometric():
    ref = _smooth(N=160, P=80)
    ps = [16, 24, 32, 40]
    errs = [_rel(_smooth(N=160, P=p), ref) for p in ps]
    ratios = [errs[i] / errs[i + 1] for i in range(len(ps) - 1)]
    print("P", ps, ["%.2e" % e for e in errs], "ratios per +8", ["%.0f" % r for r in ratios])
    # geometric decay: a fixed factor per added batch of proxies, not a
    # power of P (a power law would give ratios falling towards 1)
    assert all(r > 50 for r in ratios), ratios
    assert errs[-1] < 1e-11


def test_corner_refinement_order_q():
    ref = oracle.solve_stack(workloads.small_polygon_stack(nper=160))
    ns = [40, 48, 56, 64]
    errs = [_rel(oracle.solve_stack(workloads.small_polygon_stack(nper=n)), ref) for n in ns]
    orders = _orders(ns, errs)
    print("nper", ns, ["%.2e" % e for e in errs], "orders", ["%.2f" % p for p in orders])
    # the Kress grading exponent q = 6 sets the rate
    assert all(5.5 < p < 6.8 for p in orders), orders
