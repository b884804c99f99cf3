#!/usr/bin/env python3
"""Throughput of the multilayer quasi-periodic Helmholtz solve on one MI355X.

One step = one pass of the whole hot path over one batch of incident angles:
the alpha-independent fills (Nystrom self/neighbour blocks with the Alpert
correction, proxy, wall and radiation blocks), alpha assembly, the per-layer
Tikhonov least-squares Schur eliminations, the Schur-complement GEMMs, the
block-tridiagonal solve, the back substitution and the Bragg/flux
extraction.  Inputs (interface geometry, wavenumbers) are resident on the
device before timing starts; the Bragg amplitudes are copied back each step.

Default workload: the 1000-interface stack, 70 % random smooth interfaces
(Fourier modes 1..5, peak 0.3) and 30 % cornered ones (triangle, trapezoid,
triangle on a flat; Kress-graded segments, q = 6), spacing 1.5, d = 2 pi,
k_j = 10 n_j with n_j ~ U[1,2], discretised at N = 260 (smooth) / 500
(cornered) nodes, P = 140, M_w = 100, M_ud = 60, K = 25 (804242 unknowns per
angle); one step is a sweep of 100 incident angles uniform in (-pi/2, 0),
each with its own Bloch phase, in one graph-captured launch sequence
(Sec. 3.4: the alpha-independent pieces are filled once per step).

Other workloads (--workload): the same stack on a kappa_0 grid of 20 Bloch
phases (angles that share a phase share one factorisation), the literal
sizes, the 50-interface stack, the 64-stack batch (mlh_batch_solve), the
adjoint gradient of the 100-interface problem (mlh_adjoint) and the field at
a million targets (mlh_field).
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "multilayer solves/s (unknowns/s) at flux err ≤1e-9; adjoint grads/s; % FP64 peak"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6

RES3 = dict(N_smooth=260, N_corner=500, P=140, M_w=100)
WORKLOADS = {
    # name: (generator name, kwargs, description, angles of one step)
    #   angles: "first" = the generator's single angle, "all" = its angle list,
    #   "kgrid" = a kappa_0 grid holding 20 distinct alpha, 5 angles each
    "config2_resolved": ("config2", dict(N=260, P=120, M_w=80),
                         "I=50 random Fourier interfaces, N=260, P=120, M_w=80, M_ud=60, K=25", "first"),
    "config2": ("config2", dict(), "I=50 random Fourier interfaces, N=100, P=50, M_w=50, M_ud=60, K=25", "first"),
    "config1_resolved": ("config1", dict(N=160, P=140, M_w=100),
                         "I=2 sine interfaces, N=160, P=140, M_w=100, M_ud=60, K=25", "first"),
    "config1": ("config1", dict(), "I=2 sine interfaces, N=120, P=60, M_w=60, M_ud=60, K=25", "first"),
    "config3_resolved": ("config3", RES3,
                         "I=1000, 70% random Fourier (N=260) / 30% cornered (N=500, Kress q=6), P=140, M_w=100, "
                         "M_ud=60, K=25; sweep of 100 angles uniform in (-pi/2, 0)", "all"),
    "config3_kgrid_resolved": ("config3", RES3,
                               "I=1000 stack of config3_resolved; sweep of 100 angles on a kappa_0 grid of "
                               "spacing 2 pi/(20 d) (20 distinct alpha, 5 angles each)", "kgrid"),
    "config3": ("config3", dict(),
                "I=1000, 70% random Fourier (N=120) / 30% cornered (N=250), P=60, M_w=60, M_ud=60, K=25; "
                "sweep of 100 angles uniform in (-pi/2, 0)", "all"),
    # a batch of independent stacks: solved by mlh_batch_solve, one angle each
    "config4": ("config4", dict(),
                "64 independent stacks, I ~ U{10..200}, N ~ U{60..250} per interface, 70% random Fourier / 30% "
                "cornered, k = omega n with omega ~ U[5,20], n ~ U[1,2.5], P=60, M_w=60, M_ud=60, K=25; one "
                "random angle per stack", "batch"),
    # resolved twin: omega ~ U[5,8] (k <= 20), I ~ U{10..100} (the device
    # memory of all 64 stacks at once), every interface raised to 18 k_max
    # (smooth) / 25 k_max (cornered) nodes, k_max the larger adjacent wavenumber
    "config4_resolved": ("config4", dict(omega_range=(5.0, 8.0), I_range=(10, 100), P=140, M_w=100,
                                         nodes_per_k=(18.0, 25.0)),
                         "64 independent stacks, I ~ U{10..100}, N ~ U{60..250} per interface raised to 18 k_max "
                         "(smooth) / 25 k_max (cornered), 70% random Fourier / 30% cornered, k = omega n with "
                         "omega ~ U[5,8], n ~ U[1,2.5], P=140, M_w=100, M_ud=60, K=25; one random angle per stack",
                         "batch"),
    # the scattered field at a million targets of the 50-interface resolved stack (mlh_field)
    "field": ("config2", dict(N=260, P=120, M_w=80),
              "I=50 random Fourier interfaces, N=260, P=120, M_w=80, M_ud=60, K=25, one angle; scattered field "
              "at 1e6 seeded targets uniform in the cell from y_D - 1 to y_U + 1", "field"),
    # the adjoint gradient of a ShapeProblem (mlh_adjoint)
    "config5_resolved": ("config5", dict(N=260, P=120, M_w=80),
                         "I=100 smooth interfaces, 5 sine amplitudes each (500) and 101 layer indices, omega=10, "
                         "N=260, P=120, M_w=80, M_ud=60, K=25; J = summed zeroth-order reflected efficiency over 10 "
                         "angles in (-pi/3, 0)", "adjoint"),
    "config5": ("config5", dict(),
                "I=100 smooth interfaces, 5 sine amplitudes each and 101 layer indices, omega=10, N=100, P=50, "
                "M_w=50, M_ud=60, K=25 (literal sizes, under-resolved); J over 10 angles in (-pi/3, 0)",
                "adjoint"),
}


def make_desc(name, I=None):
    import workloads
    gen, kw, _, _ = WORKLOADS[name]
    kw = dict(kw)
    if I is not None:
        kw["I"] = I
    return getattr(workloads, gen)(**kw)


def step_thetas(name, desc):
    import numpy as np
    import workloads
    mode = WORKLOADS[name][3]
    if mode == "first":
        return np.asarray(desc.thetas[:1], dtype=float)
    if mode == "all":
        return np.asarray(desc.thetas, dtype=float)
    return workloads.kappa_grid_thetas(desc, n_angles=100, n_alpha=20)


def distinct_alpha(desc, thetas, tol=1e-12):
    """Number of distinct Bloch phases among the angles (same rule as the library)."""
    import math
    fr = []
    for t in thetas:
        x = desc.d * desc.k[0] * math.cos(t) / (2 * math.pi)
        f = x - math.floor(x)
        if not any(min(abs(f - g), 1 - abs(f - g)) < tol for g in fr):
            fr.append(f)
    return len(fr)


def algorithmic_work(desc):
    """Real float64 flops (complex multiply-add = 8) of each kernel group for
    one Bloch phase, and the bytes the fill kernels must write (16 per
    complex entry)."""
    I, P, K, Mw, Mud = desc.I, desc.P, desc.K, desc.M_w, desc.M_ud
    n = [2 * f.N for f in desc.interfaces]
    nK = 2 * K + 1
    nb = 16
    w = {}
    # block Thomas sweep in Gauss-Jordan form: interface i applies the inverse
    # of its diagonal block to [A'_{i,i+1} | f_i] (n_{i+1} + 1 columns)
    gu = gp = gr = 0.0
    for i in range(I):
        rhs = (n[i + 1] if i + 1 < I else 0) + 1
        for k in range(0, n[i], nb):
            b = min(nb, n[i] - k)
            rest = n[i] - k - b
            gu += 8.0 * n[i] * rest * b + 8.0 * b * b * rest
            L = n[i] - k
            gp += 4.0 * L * b * b + 4.0 * (L - b) * b * b
            gr += 8.0 * n[i] * rhs * b + 8.0 * b * b * rhs
    w["gje_update"] = gu
    w["gje_panel"] = gp
    w["gje_rhs"] = gr
    w["sweep_gemm"] = sum(8.0 * n[i] * (n[i] + 1) * n[i - 1] for i in range(1, I))
    w["schur"] = sum(8.0 * P * 2 * n[i] * n[i] for i in range(I)) + \
        sum(8.0 * P * 2 * n[i] * n[i + 1] for i in range(I - 1))
    qr = ap = 0.0
    for j in range(I + 1):
        end = j in (0, I)
        m = 2 * Mw + (2 * Mud if end else 0)
        c = P + (nK if end else 0)
        M = m + c
        ncol = n[0] if j == 0 else (n[I - 1] if j == I else n[j - 1] + n[j])
        qr += 8.0 * M * c * c - 8.0 * c ** 3 / 3.0
        ap += ncol * (16.0 * M * c - 4.0 * c * c)
    w["ls_qr"] = qr
    w["ls_rhs"] = ap
    w["backsub"] = sum(8.0 * n[i] * n[i + 1] for i in range(I - 1))
    # fill: complex entries written (three copies for A and Z, two for C and Q)
    ent_self = sum(3 * n[i] * n[i] for i in range(I))
    ent_pair = sum(3 * 2 * n[i] * n[i + 1] for i in range(I - 1)) + sum(2 * n[i] * P for i in range(I)) + \
        sum(2 * 2 * Mw * (n[j] if j < I else 0) + 2 * 2 * Mw * (n[j - 1] if j > 0 else 0) + 2 * 2 * Mw * P
            for j in range(I + 1)) + 3 * 2 * Mud * (n[0] + n[I - 1]) + 2 * 2 * Mud * P
    w["fill_self_bytes"] = 16.0 * ent_self
    w["fill_pairs_bytes"] = 16.0 * ent_pair
    return w


# HBM bytes moved per dispatch (KiB read, KiB written), from one rocprofv3
# --pmc FETCH_SIZE pass and one WRITE_SIZE pass over the named workload's
# `bench.py --workload W --steps 1 --warmup 0 --no-cpu-baseline --autotune off`
# (default launch choices), each scaled by what the same counter reads for a
# plain 256 MiB device copy (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000) and
# averaged over every dispatch of the run.  An entry counts only while its
# kernel source is the one the counters were taken on (SHA-1 prefix).
MEASURED_TRAFFIC = {
    # the 1000-interface, 100-angle sweep (counters on zgemm_kernel dispatches only; taken on source
    # 8a7b2ec360d9, whose kernel compiles to the same instructions as this source's zgemm_kernel<8>,
    # the default slab depth)
    ("config3_resolved", "zgemm_kernel"): ("kernels_linalg.hip", "ee13a24040af", 105633771.4, 7694270.4),
}


def measured_traffic(workload, kernel):
    import hashlib
    e = MEASURED_TRAFFIC.get((workload, kernel))
    if e is None:
        return None
    src, sha, rd, wr = e
    path = os.path.join(ROOT, "paper_1410_5003_amd", "csrc", src)
    if hashlib.sha1(open(path, "rb").read()).hexdigest()[:12] != sha:
        return None
    return (rd + wr) * 1024.0


# Kernel groups of the timed path: (kernel name as the profiler reports it,
# profile time keys, launch-count keys, work keys, bound).  Work keys name
# either counts the library returns with the profile (flops of the
# descriptors each launch processed) or entries of algorithmic_work().
GROUPS = [
    ("zgemm_kernel", ("schur_ms", "sweep_gemm_ms"), ("n_schur_gemm", "n_sweep_gemm"),
     ("schur_flops", "sweep_gemm_flops"), "mfma"),
    ("gje_step_kernel", ("gje_step_ms",), ("n_gje_step",), ("gje_step_flops",), "mfma"),
    ("gje_rhs_kernel (with gje_premul_kernel)", ("gje_rhs_ms",), ("n_gje_rhs",), ("gje_rhs_flops",), "mfma"),
    ("gje_panel_kernel + gje_update_kernel", ("gje_panel_ms", "gje_update_ms"), ("n_gje_panel",),
     ("gje_panel_update_flops",), "mfma"),
    ("hq_panel_kernel", ("ls_panel_ms",), (), ("@ls_qr",), "alu"),
    ("hq_rhs_kernel", ("ls_rhs_ms",), (), ("@ls_rhs",), "mfma"),
    ("gemv_step_kernel", ("backsub_ms",), ("n_backsub",), ("@backsub",), "alu"),
    ("self_kernel", ("fill_self_ms",), (), ("@fill_self_bytes",), "hbm"),
    ("fill_kernel", ("fill_pairs_ms",), (), ("@fill_pairs_bytes",), "hbm"),
]


def roofline(desc, prof, n_sys=1, workload=None):
    """Roofline of the kernel with the largest device time in the profile."""
    alg = algorithmic_work(desc)

    def work(keys):
        tot = 0.0
        for k in keys:
            if k.startswith("@"):
                v = alg[k[1:]]
                tot += v if k.startswith("@fill") else v * n_sys
            else:
                tot += prof[k]
        return tot

    def t_ms(g):
        return sum(prof[k] for k in g[1])

    name, tkeys, nkeys, wkeys, bound = max(GROUPS, key=t_ms)
    t = t_ms((name, tkeys)) * 1e-3
    launches = int(sum(prof[k] for k in nkeys)) if nkeys else 1
    w = work(wkeys)
    if bound == "hbm":
        ach, peak, unit = w / t / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        ach, peak, unit = w / t / 1e12, FP64_PEAK_TFS, "TFLOP/s"
    traffic = measured_traffic(workload, name.split(" ")[0])
    return {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak, "traffic": traffic,
            "kernel": name, "launches_per_step": launches, "avg_launch_ms": t * 1e3 / launches,
            "work_per_launch": w / launches}


def phase_fractions(desc, prof, n_sys):
    """FP64 fraction of the least-squares, Schur and block-solve phase in the
    method's own flops (a block Thomas sweep, not cyclic reduction's extra
    work), and the HBM fraction of the fills in bytes written."""
    w = algorithmic_work(desc)
    flops = n_sys * (w["ls_qr"] + w["ls_rhs"] + w["schur"] + w["gje_panel"] + w["gje_update"] + w["gje_rhs"] +
                     w["sweep_gemm"] + w["backsub"])
    t = 1e-3 * sum(prof[k] for k in ("ls_panel_ms", "ls_update_ms", "ls_rhs_ms", "schur_ms", "sweep_gemm_ms",
                                     "gje_step_ms", "gje_panel_ms", "gje_update_ms", "gje_rhs_ms", "backsub_ms"))
    fb = w["fill_self_bytes"] + w["fill_pairs_bytes"]
    tf = 1e-3 * (prof["fill_self_ms"] + prof["fill_alpert_ms"] + prof["fill_pairs_ms"])
    return {"schur_blocklu_fp64": {"method_flops": flops, "device_s": t, "achieved_tflops": flops / t / 1e12,
                                   "peak_tflops": FP64_PEAK_TFS, "frac": flops / t / 1e12 / FP64_PEAK_TFS},
            "fill_hbm": {"bytes_written": fb, "device_s": tf, "achieved_gbs": fb / tf / 1e9,
                         "peak_gbs": HBM_PEAK_GBS, "frac": fb / tf / 1e9 / HBM_PEAK_GBS}}


def available_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(name, sample_I, threads):
    """Time the oracle on the first `sample_I` interfaces of the workload, one
    angle, with `threads` BLAS/OpenMP threads (separate process); the caller
    scales linearly in the number of layers."""
    code = (
        "import os,sys,time;sys.path.insert(0,%r);"
        "import bench,oracle;d=bench.make_desc(%r,I=%d);"
        "t=time.perf_counter();r=oracle.solve_stack(d,theta=float(bench.step_thetas(%r,d)[0]));"
        "print(time.perf_counter()-t)"
    ) % (ROOT, name, sample_I, name)
    n = str(threads)
    env = dict(os.environ, OPENBLAS_NUM_THREADS=n, OMP_NUM_THREADS=n, MKL_NUM_THREADS=n)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    if out.returncode != 0:
        raise RuntimeError(out.stderr)
    return float(out.stdout.strip().splitlines()[-1])


def tuning_angles(desc, thetas, systems=2, tol=1e-12):
    """The angles of the sweep's first `systems` distinct Bloch phases."""
    import math
    import numpy as np
    fr, keep = [], []
    for t in thetas:
        x = desc.d * desc.k[0] * math.cos(t) / (2 * math.pi)
        f = x - math.floor(x)
        hit = [g for g in fr if min(abs(f - g), 1 - abs(f - g)) < tol]
        if not hit and len(fr) >= systems:
            continue
        if not hit:
            fr.append(f)
        keep.append(t)
    return np.asarray(keep, dtype=float)


def pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x, dtype=float), q))


def bench_batch(args):
    """Many independent stacks: one step = refill of every stack's pieces and
    one batched solve of all of them (one angle each), in shared launches."""
    import numpy as np
    import torch
    import workloads
    import paper_1410_5003_amd as mlh
    gen, kw, desc_txt, _ = WORKLOADS[args.workload]
    descs = getattr(workloads, gen)(**kw)
    ctx = mlh.Context(0)
    sts = [mlh.Stack(ctx, d) for d in descs]
    b = mlh.Batch(ctx, sts)
    th = np.array([float(d.thetas[0]) for d in descs])
    n_tot = sum(s.info()["n_tot"] for s in sts)
    steps = args.steps if args.steps is not None else 10
    warmup = args.warmup if args.warmup is not None else 2
    print("workload %s: %d stacks, %d interfaces, %d unknowns" % (args.workload, len(descs), sum(d.I for d in descs),
                                                                  n_tot),
          file=sys.stderr, flush=True)
    autotuned = args.autotune in ("auto", "on")
    if autotuned:
        ta = time.perf_counter()
        if not (args.autotune == "auto" and b.tune_cached()[0]):
            b.autotune(th, reps=1)
        print("autotune %s in %.2f s" % (b.get_tuning(), time.perf_counter() - ta), file=sys.stderr, flush=True)
    out = None
    for _ in range(warmup):
        out = b.solve(th, refill=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = b.solve(th, refill=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    lat = out.stack_ms
    flux = np.abs(out.flux_err)
    tuning = b.get_tuning()
    # the batch's workspace and pieces are released before the plain solves
    b.close()
    for s in sts:
        s.close()
    # the same stacks one at a time (refill + one-angle solve each, each
    # timed to its own completion after an untimed solve that captures its
    # graph); each is created on its own and destroyed after, since every
    # stack keeps a solve workspace of its own
    plain = []
    for i, d in enumerate(descs):
        st = mlh.Stack(ctx, d)
        st.solve(th[i:i + 1])
        torch.cuda.synchronize()
        tp = time.perf_counter()
        st.refill()
        st.solve(th[i:i + 1])
        plain.append((time.perf_counter() - tp) * 1e3)
        st.close()
    plain_total = float(np.sum(plain))
    line = {
        "metric": METRIC, "value": len(descs) / (ms * 1e-3), "unit": "solves/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (complex128)", "data": "synthetic (seeded stacks)",
        "config": {"workload": args.workload, "description": desc_txt, "stacks": len(descs),
                   "interfaces": int(sum(d.I for d in descs)), "unknowns": int(n_tot)},
        "unknowns_per_s": n_tot / (ms * 1e-3), "flux_err_median": float(np.median(flux)),
        "flux_err_max": float(flux.max()), "stacks_flux_le_1e-9": int(np.sum(flux <= 1e-9)),
        "interfaces_of_worst_stack": int(descs[int(np.argmax(flux))].I),
        "latency_ms": {"batched_p50": pct(lat, 50), "batched_p99": pct(lat, 99), "plain_p50": pct(plain, 50),
                       "plain_p99": pct(plain, 99), "plain_total": plain_total},
        "speedup_vs_plain": plain_total / ms,
        "tuning": dict(tuning, autotuned=autotuned),
    }
    print("batched %.2f ms per step (%d stacks); plain %.2f ms; latency p50 %.2f p99 %.2f ms" %
          (ms, len(descs), plain_total, pct(lat, 50), pct(lat, 99)), file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


def bench_field(args):
    """One step = mlh_field at a million targets: the solve for the angle,
    the proxy strengths, then the layer representations (or Rayleigh-Bloch
    sums) at every target.  Beside it the plain solve of the same angle, so
    that the evaluation's own rate can be read off."""
    import numpy as np
    import torch
    import paper_1410_5003_amd as mlh
    desc = make_desc(args.workload)
    theta = float(desc.thetas[0])
    rng = np.random.default_rng(7)
    n_pts = 1_000_000
    x = rng.uniform(-desc.d / 2, desc.d / 2, n_pts)
    y = rng.uniform(desc.y_D - 1.0, desc.y_U + 1.0, n_pts)
    ctx = mlh.Context(0)
    st = mlh.Stack(ctx, desc)
    steps = args.steps if args.steps is not None else 5
    warmup = args.warmup if args.warmup is not None else 1
    for _ in range(warmup):
        u, reg = st.field(theta, x, y)
        st.solve([theta])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        u, reg = st.field(theta, x, y)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        st.solve([theta])
    torch.cuda.synchronize()
    solve_ms = (time.perf_counter() - t0) * 1e3 / steps
    # kernel evaluations: a target in layer j sums S and D over the three
    # copies of each bounding interface (6 N each) and the layer's P proxies
    N = [f.N for f in desc.interfaces]
    evals = 0
    for j in range(desc.I + 1):
        cnt = int(np.sum(reg == j))
        evals += cnt * (6 * ((N[j - 1] if j > 0 else 0) + (N[j] if j < desc.I else 0)) + desc.P)
    st.close()
    eval_ms = max(ms - solve_ms, 1e-9)
    line = {
        "metric": METRIC, "value": n_pts / (ms * 1e-3), "unit": "targets/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (complex128)", "data": "synthetic (seeded stacks and targets)",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload][2], "interfaces": desc.I,
                   "targets": n_pts},
        "solve_ms": solve_ms, "evaluation_ms": eval_ms, "targets_per_s_evaluation": n_pts / (eval_ms * 1e-3),
        "kernel_evals_per_s": evals / (eval_ms * 1e-3),
        "targets_above_U": int(np.sum(reg == -1)), "targets_below_D": int(np.sum(reg == desc.I + 1)),
    }
    print("field %.1f ms per call (solve %.1f ms, evaluation %.1f ms); %.3g targets/s, %.3g kernel evaluations/s" %
          (ms, solve_ms, eval_ms, line["value"], line["kernel_evals_per_s"]), file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


def bench_adjoint(args):
    """One step = the gradient of J (summed zeroth-order reflected
    efficiency over the problem's angles) in every shape amplitude and
    layer index below the top: refill, forward solve, transposed solve,
    least-squares adjoint, derivative fills and contractions (mlh_adjoint).
    Beside it: the same gradient by central differences of the GPU forward
    solve, timed on a few parameters and scaled to all of them."""
    import numpy as np
    import torch
    import workloads
    import paper_1410_5003_amd as mlh
    gen, kw, desc_txt, _ = WORKLOADS[args.workload]
    pb = getattr(workloads, gen)(**kw)
    desc = pb.stack()
    th = np.asarray(desc.thetas, dtype=float)
    ctx = mlh.Context(0)
    st = mlh.Stack(ctx, desc)
    info = st.info()
    n_par = pb.c.size + pb.n.size - 1
    steps = args.steps if args.steps is not None else 5
    warmup = args.warmup if args.warmup is not None else 1
    print("workload %s: I=%d n_tot=%d angles %d parameters %d" % (args.workload, desc.I, info["n_tot"], th.size,
                                                                 n_par), file=sys.stderr, flush=True)
    for _ in range(warmup):
        st.refill()
        st.adjoint(th, shape=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms = []
    for _ in range(steps):
        ts = time.perf_counter()
        st.refill()
        J, gk, gs = st.adjoint(th, shape=True)
        step_ms.append((time.perf_counter() - ts) * 1e3)  # mlh_adjoint returns its results on the host
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    out = st.solve(th)
    flux = np.abs(out.flux_err)
    st.close()
    # central differences of the forward solve (stack built and solved per
    # evaluation, as a caller without the adjoint would; the release of each
    # stack's device memory is left out of the time)
    nfd = 8
    p0 = pb.params()
    fd_s = 0.0
    for q in range(nfd):
        for sgn in (1.0, -1.0):
            e = np.zeros_like(p0)
            e[q] = sgn * 1e-6
            desc_q = pb.stack(p0 + e)
            torch.cuda.synchronize()
            tf = time.perf_counter()
            s2 = mlh.Stack(ctx, desc_q)
            s2.solve(th)
            torch.cuda.synchronize()
            fd_s += time.perf_counter() - tf
            s2.close()
    fd_per_param = fd_s / nfd
    fd_total = fd_per_param * n_par
    line = {
        "metric": METRIC, "value": 1e3 / ms, "unit": "grads/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (complex128)", "data": "synthetic (seeded stacks)",
        "config": {"workload": args.workload, "description": desc_txt, "interfaces": desc.I,
                   "unknowns": info["n_tot"], "angles": int(th.size), "parameters": int(n_par)},
        "step_ms": [round(v, 1) for v in step_ms], "J": J, "flux_err_max": float(flux.max()),
        "fd_by_gpu": {"s_per_gradient": fd_total, "s_per_parameter": fd_per_param, "sampled_parameters": nfd},
        "speedup_vs_fd": fd_total / (ms * 1e-3),
    }
    print("adjoint %.1f ms per gradient; central differences %.1f s (%.3f s per parameter)" %
          (ms, fd_total, fd_per_param), file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="config3_resolved", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-layers", type=int, default=None,
                    help="interfaces of the workload the oracle solves for the CPU baseline "
                         "(default: 8 for sweeps, 6 otherwise)")
    ap.add_argument("--plain-sample", type=int, default=4,
                    help="sweeps: angles timed one by one (refill + one-angle solve each)")
    ap.add_argument("--autotune", choices=("auto", "on", "off"), default="auto",
                    help="time the solve under candidate launch choices before the warmup and keep the "
                         "fastest (sweeps are tuned on the angles of their first two Bloch phases, which "
                         "run the launch shapes of one batch of the sweep); auto takes the choices the "
                         "library has recorded for this size class instead, if any (MLH_TUNING_CACHE), "
                         "on always times them")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (calibrates the HBM "
                         "byte counters of a profiler against a known size) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        x = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU (there is no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if WORKLOADS[args.workload][3] == "batch":
        return bench_batch(args)
    if WORKLOADS[args.workload][3] == "adjoint":
        return bench_adjoint(args)
    if WORKLOADS[args.workload][3] == "field":
        return bench_field(args)
    import numpy as np
    import torch
    import paper_1410_5003_amd as mlh

    desc = make_desc(args.workload)
    thetas = step_thetas(args.workload, desc)
    sweep = len(thetas) > 1
    # a sweep of 100 distinct Bloch phases is about a minute per step
    n_sys0 = distinct_alpha(desc, thetas)
    steps = args.steps if args.steps is not None else (1 if n_sys0 > 40 else (5 if sweep else 20))
    warmup = args.warmup if args.warmup is not None else (1 if sweep else 3)
    sample_layers = args.cpu_sample_layers or (8 if sweep else 6)
    ctx = mlh.Context(0)
    st = mlh.Stack(ctx, desc)
    info = st.info()
    n_sys = distinct_alpha(desc, thetas)
    print("workload %s: I=%d n_tot=%d device MB %.1f angles %d distinct alpha %d" %
          (args.workload, desc.I, info["n_tot"], info["device_bytes"] / 2 ** 20, len(thetas), n_sys),
          file=sys.stderr, flush=True)
    autotuned = args.autotune in ("auto", "on")
    cached = False
    if autotuned:  # outside the timed region
        ta = time.perf_counter()
        st.refill()
        tune_th = tuning_angles(desc, thetas) if sweep else thetas
        # choices recorded for this size class (MLH_TUNING_CACHE) are taken as they are
        cached = args.autotune == "auto" and st.tune_cached(tune_th)[0]
        if not cached:
            st.autotune(tune_th, reps=1 if sweep else 3)
        print("autotune %s on %d angles in %.2f s%s" % (st.get_tuning(), len(tune_th), time.perf_counter() - ta,
                                                        " (recorded choices)" if cached else ""),
              file=sys.stderr, flush=True)
    tuning = dict(st.get_tuning(), autotuned=autotuned, from_cache=bool(cached))
    out = None
    for _ in range(warmup):
        st.refill()
        out = st.solve(thetas)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st.refill()
        out = st.solve(thetas)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    solves_per_s = len(thetas) / (ms * 1e-3)
    flux = np.abs(out.flux_err)
    print("step %.3f ms  flux err max %.2e median %.2e" % (ms, flux.max(), np.median(flux)),
          file=sys.stderr, flush=True)

    # per-kernel device times (HIP events on the library's stream, around
    # the launches of the timed path run one at a time)
    if sweep:
        prof = st.profile_solve(thetas)
    else:
        profs = [st.profile_step(thetas[0]) for _ in range(3)]
        prof = {k: float(np.mean([p[k] for p in profs])) for k in profs[0]}
    print("profile " + json.dumps({k: round(v, 4) for k, v in prof.items()}), file=sys.stderr, flush=True)
    roof = roofline(desc, prof, n_sys, args.workload)
    phases = phase_fractions(desc, prof, n_sys)
    line = {
        "metric": METRIC, "value": solves_per_s, "unit": "solves/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (complex128)", "data": "synthetic (seeded stacks)",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload][2],
                   "interfaces": desc.I, "unknowns": info["n_tot"], "angles_per_step": len(thetas),
                   "distinct_alpha": n_sys},
        "unknowns_per_s": solves_per_s * info["n_tot"], "flux_err": float(out.flux_err[0]),
        "flux_err_max": float(flux.max()),
        "phase_ms": {k: round(v, 4) for k, v in prof.items() if k.endswith("_ms")},
        "roofline": roof,
        "schur_blocklu_fp64": phases["schur_blocklu_fp64"],
        "fill_hbm": phases["fill_hbm"],
        "tuning": tuning,
    }
    if sweep and args.plain_sample > 0:
        # the same angles solved one at a time, each with its own refill
        npl = min(args.plain_sample, len(thetas))
        idx = np.linspace(0, len(thetas) - 1, npl).round().astype(int)
        st.refill()
        st.solve(thetas[idx[:1]])
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for a in idx:
            st.refill()
            st.solve(thetas[a:a + 1])
        torch.cuda.synchronize()
        plain = (time.perf_counter() - tp0) / npl
        batched = ms * 1e-3 / len(thetas)
        line["sweep"] = {"plain_s_per_angle": plain, "batched_s_per_angle": batched,
                         "speedup_vs_plain": plain / batched, "plain_sample_angles": int(npl)}
        print("sweep: plain %.3f s/angle, batched %.3f s/angle, speed-up %.2fx" % (plain, batched, plain / batched),
              file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        cores = available_cores()
        t1 = cpu_baseline(args.workload, sample_layers, 1)
        tn = cpu_baseline(args.workload, sample_layers, cores)
        scale = desc.I / sample_layers
        line["cpu_baseline"] = {"value": 1.0 / (tn * scale), "unit": "solves/s", "cores": cores, "kind": "oracle",
                                "sample": "oracle solve of the first %d of %d interfaces of the same stack, one "
                                          "angle: %.2f s on %d threads (%.2f s on 1 thread, %.4f solves/s); scaled "
                                          "linearly in the number of layers" % (sample_layers, desc.I, tn, cores,
                                                                                t1, 1.0 / (t1 * scale)),
                                "value_1_core": 1.0 / (t1 * scale)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
