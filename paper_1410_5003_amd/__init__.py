"""MI355X-native robust periodic multilayer Helmholtz solver.

Python front end of libmlh.so (include/mlh.h): a hand-written gfx950 HIP
implementation of the Cho & Barnett periodizing integral-equation scheme
(arXiv:1410.5003) -- dense complex float64 Nystrom/proxy/wall/radiation fills,
per-layer least-squares Schur eliminations and the block-tridiagonal LU sweep.
PyTorch only supplies the HIP stream the library enqueues its work on.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np

from ._lib import (ABI_VERSION, MLH_IFACE_FOURIER, MLH_IFACE_POLYGON, PIECES, MlhError, check,
                   dptr, iptr, lib, mlh_interface, mlh_profile, mlh_stack_desc, mlh_tuning)

__all__ = ["Context", "Stack", "Batch", "SolveOutput", "BatchOutput", "MlhError", "lib"]


def _current_stream_handle():
    try:
        import torch
    except ImportError:  # no torch: the null stream
        return None
    if not torch.cuda.is_available():
        raise MlhError(4, "no HIP device visible")
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A device plus the HIP stream work is enqueued on (torch's current stream
    by default)."""

    def __init__(self, device: int = 0, stream=None):
        self._h = C.c_void_p()
        if stream is None:
            stream = _current_stream_handle()
        check(lib().mlh_ctx_create(device, stream, C.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().mlh_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hankel(self, x) -> np.ndarray:
        """(H0(x), (i pi x/2) H1(x) - 1) from the device routine, shape (n, 2) complex."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros(4 * x.size)
        check(lib().mlh_debug_hankel(self._h, x.size, dptr(x), dptr(out)))
        return out.view(np.complex128).reshape(-1, 2)

    def zgemm(self, alpha: complex, A: np.ndarray, B: np.ndarray, Cm: np.ndarray) -> np.ndarray:
        """C + alpha A B computed by the library's FP64-MFMA kernel."""
        m, k = A.shape
        k2, n = B.shape
        assert k == k2 and Cm.shape == (m, n)
        a = np.asfortranarray(A, dtype=np.complex128)
        b = np.asfortranarray(B, dtype=np.complex128)
        c = np.asfortranarray(Cm, dtype=np.complex128).copy(order="F")
        al = np.array([alpha.real, alpha.imag])
        check(lib().mlh_debug_zgemm(self._h, m, n, k, dptr(al), dptr(a), dptr(b), dptr(c)))
        return c


@dataclass
class SolveOutput:
    aU: np.ndarray       # (n_angles, 2K+1) complex
    aD: np.ndarray
    orders: np.ndarray   # (n_angles, 2K+1) int
    flux_err: np.ndarray  # (n_angles,)
    eta: Optional[np.ndarray] = None  # (n_angles, N_den) complex densities, if asked for


class Stack:
    """A prepared multilayer structure on the device.

    ``desc`` is any object with the attributes of ``workloads.Stack``:
    d, k, interfaces (kind, y0, n_nodes, cos_coef, sin_coef, vx, vy,
    seg_nodes, q), y_U, y_D, P, R, M_w, M_ud, K and optionally ls_mu."""

    def __init__(self, ctx: Context, desc):
        self.ctx = ctx
        self._keep = []
        ifs = (mlh_interface * len(desc.interfaces))()
        for i, f in enumerate(desc.interfaces):
            e = ifs[i]
            e.y0 = float(f.y0)
            if f.kind == "fourier":
                ca = np.ascontiguousarray(f.cos_coef, dtype=np.float64)
                sa = np.ascontiguousarray(f.sin_coef, dtype=np.float64)
                assert ca.size == sa.size
                self._keep += [ca, sa]
                e.kind = MLH_IFACE_FOURIER
                e.n_modes = ca.size
                e.cos_coef = dptr(ca)
                e.sin_coef = dptr(sa)
                e.n_nodes = int(f.n_nodes)
            else:
                vx = np.ascontiguousarray(f.vx, dtype=np.float64)
                vy = np.ascontiguousarray(f.vy, dtype=np.float64)
                sn = np.ascontiguousarray(f.seg_nodes, dtype=np.int32)
                self._keep += [vx, vy, sn]
                e.kind = MLH_IFACE_POLYGON
                e.n_vert = vx.size
                e.vx, e.vy, e.seg_nodes = dptr(vx), dptr(vy), iptr(sn)
                e.q = float(f.q)
        k = np.ascontiguousarray(desc.k, dtype=np.float64)
        self._keep += [ifs, k]
        d = mlh_stack_desc()
        d.abi_version = ABI_VERSION
        d.I = len(desc.interfaces)
        d.iface = C.cast(ifs, C.POINTER(mlh_interface))
        d.k = dptr(k)
        d.d, d.y_U, d.y_D = float(desc.d), float(desc.y_U), float(desc.y_D)
        d.P, d.R = int(desc.P), float(desc.R)
        d.M_w, d.M_ud, d.K = int(desc.M_w), int(desc.M_ud), int(desc.K)
        d.ls_mu = float(getattr(desc, "ls_mu", 0.0))
        self.K = int(desc.K)
        self._k = np.array(k)
        self._n_shape = sum(2 * len(f.cos_coef) for f in desc.interfaces if f.kind == "fourier")
        self._h = C.c_void_p()
        check(lib().mlh_stack_create(ctx.handle, C.byref(d), C.byref(self._h)))
        self._keep = []

    def close(self):
        if self._h:
            lib().mlh_stack_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def refill(self):
        check(lib().mlh_stack_refill(self._h))

    def info(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().mlh_stack_info(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return {"n_den": a.value, "n_tot": b.value, "device_bytes": c.value}

    def solve(self, thetas, eta: bool = False, noalloc: bool = False) -> SolveOutput:
        """Bragg amplitudes, order labels and flux errors of the angles
        ``thetas`` in host arrays (and the densities if ``eta``).  With
        ``noalloc`` the call goes to mlh_solve_noalloc, whose workspace is the
        library's fixed per-device area."""
        th = np.ascontiguousarray(np.atleast_1d(thetas), dtype=np.float64)
        na, nK = th.size, 2 * self.K + 1
        aU = np.zeros((na, nK), dtype=np.complex128)
        aD = np.zeros((na, nK), dtype=np.complex128)
        orders = np.zeros((na, nK), dtype=np.int32)
        flux = np.zeros(na)
        dens = np.zeros((na, self.info()["n_den"]), dtype=np.complex128) if eta else None
        fn = lib().mlh_solve_noalloc if noalloc else lib().mlh_solve
        check(fn(self._h, na, dptr(th), 0, aU.ctypes.data, aD.ctypes.data, orders.ctypes.data,
                 flux.ctypes.data, dens.ctypes.data if eta else None))
        return SolveOutput(aU, aD, orders, flux, dens)

    def solve_into(self, thetas, aU, aD, orders=None, flux_err=None, eta=None):
        """Solve with device-resident outputs: ``aU``, ``aD`` (complex128,
        (n_angles, 2K+1)), ``orders`` (int32), ``flux_err`` (float64,
        (n_angles,)) and ``eta`` (complex128, (n_angles, N_den)) are
        contiguous torch tensors on the context's device; None skips an
        optional output.  Returns once the work is enqueued on the context's
        stream."""
        th = np.ascontiguousarray(np.atleast_1d(thetas), dtype=np.float64)
        na, nK = th.size, 2 * self.K + 1

        def ptr(t, dtype, shape):
            if t is None:
                return None
            if not (t.is_cuda and t.is_contiguous() and t.dtype == dtype and tuple(t.shape) == shape):
                raise ValueError("output tensor must be a contiguous %s device tensor of shape %s" % (dtype, shape))
            return t.data_ptr()

        import torch
        check(lib().mlh_solve(self._h, na, dptr(th), 1, ptr(aU, torch.complex128, (na, nK)),
                              ptr(aD, torch.complex128, (na, nK)), ptr(orders, torch.int32, (na, nK)),
                              ptr(flux_err, torch.float64, (na,)),
                              ptr(eta, torch.complex128, (na, self.info()["n_den"]))))

    def field(self, theta: float, x, y):
        """Scattered field at the targets (x, y) after solving for ``theta``
        (mlh_field): returns (u complex, region int32: -1 above U, 0..I the
        layers, I+1 below D)."""
        xs = np.ascontiguousarray(np.ravel(x), dtype=np.float64)
        ys = np.ascontiguousarray(np.ravel(y), dtype=np.float64)
        assert xs.size == ys.size
        u = np.zeros(xs.size, dtype=np.complex128)
        reg = np.zeros(xs.size, dtype=np.int32)
        check(lib().mlh_field(self._h, float(theta), xs.size, dptr(xs), dptr(ys), 0, u.ctypes.data,
                              reg.ctypes.data))
        return u, reg

    def adjoint(self, thetas, shape: bool = False):
        """J = sum of the zeroth-order reflected efficiencies at ``thetas``,
        dJ/dk_j (entry 0, the incident medium, is NaN) and, with ``shape``,
        dJ/d(cos_coef, sin_coef) of the Fourier interfaces, interface by
        interface (mlh_adjoint)."""
        th = np.ascontiguousarray(np.atleast_1d(thetas), dtype=np.float64)
        g = np.zeros(len(self._k))
        gs = np.zeros(self._n_shape) if shape else None
        J = C.c_double()
        check(lib().mlh_adjoint(self._h, th.size, dptr(th), C.byref(J), dptr(g),
                                gs.ctypes.data if shape else None))
        return (J.value, g, gs) if shape else (J.value, g)

    def set_flux_tolerance(self, tol: float):
        """Report MLH_E_ACCURACY from solves whose |flux error| exceeds tol
        (0 turns the check off)."""
        check(lib().mlh_stack_set_flux_tolerance(self._h, float(tol)))

    def profile_step(self, theta: float) -> dict:
        """Per-kernel device times (ms) of one refill + one-angle solve."""
        p = mlh_profile()
        check(lib().mlh_profile_step(self._h, float(theta), C.byref(p)))
        return {name: getattr(p, name) for name, _ in p._fields_}

    def profile_solve(self, thetas) -> dict:
        """Per-kernel device times (ms) of one refill + a solve of all ``thetas``."""
        th = np.ascontiguousarray(np.atleast_1d(thetas), dtype=np.float64)
        p = mlh_profile()
        check(lib().mlh_profile_solve(self._h, th.size, dptr(th), C.byref(p)))
        return {name: getattr(p, name) for name, _ in p._fields_}

    def get_tuning(self) -> dict:
        """The stack's launch choices (see ``mlh_tuning`` in mlh.h)."""
        t = mlh_tuning()
        check(lib().mlh_stack_get_tuning(self._h, C.byref(t)))
        return {name: getattr(t, name) for name, _ in t._fields_}

    def set_tuning(self, **choices):
        """Replace some of the launch choices; the others stay."""
        cur = self.get_tuning()
        unknown = set(choices) - set(cur)
        if unknown:
            raise KeyError("unknown launch choices: %s" % sorted(unknown))
        cur.update(choices)
        t = mlh_tuning(**{k: int(v) for k, v in cur.items()})
        check(lib().mlh_stack_set_tuning(self._h, C.byref(t)))

    def autotune(self, thetas, reps: int = 2) -> dict:
        """Time solves of ``thetas`` under candidate launch choices, keep and
        return the fastest (also recorded in the launch-choice cache)."""
        th = np.ascontiguousarray(np.atleast_1d(thetas), dtype=np.float64)
        t = mlh_tuning()
        check(lib().mlh_stack_autotune(self._h, th.size, dptr(th), int(reps), C.byref(t)))
        return {name: getattr(t, name) for name, _ in t._fields_}

    def tune_cached(self, thetas):
        """Take the launch choices recorded for this stack's size class and
        these angles, if any: returns (found, choices)."""
        th = np.ascontiguousarray(np.atleast_1d(thetas), dtype=np.float64)
        t, found = mlh_tuning(), C.c_int32()
        check(lib().mlh_stack_tune_cached(self._h, th.size, dptr(th), C.byref(t), C.byref(found)))
        return bool(found.value), {name: getattr(t, name) for name, _ in t._fields_}

    def solve_partial(self, theta: float, stop_phase: int):
        """Inspection: run one angle up to a phase (1 assembly, 2 least squares,
        3 Schur, 4 sweep) and keep its workspace for ``work``."""
        check(lib().mlh_debug_solve_partial(self._h, float(theta), int(stop_phase)))

    WORK = {"Dg": 0, "Up": 1, "Dn": 2, "S": 3, "RHS": 4, "UG": 5, "eta": 6}

    def work(self, name: str, index: int) -> np.ndarray:
        which = self.WORK[name]
        r, c = C.c_int32(), C.c_int32()
        check(lib().mlh_debug_get_work(self._h, which, index, None, C.byref(r), C.byref(c)))
        out = np.zeros((c.value, r.value), dtype=np.complex128)
        check(lib().mlh_debug_get_work(self._h, which, index, dptr(out), C.byref(r), C.byref(c)))
        return out.T

    def piece(self, name: str, index: int = 0, piece: int = 0) -> np.ndarray:
        which = PIECES[name]
        r, c = C.c_int32(), C.c_int32()
        check(lib().mlh_debug_get_piece(self._h, which, index, piece, None, C.byref(r), C.byref(c)))
        out = np.zeros((c.value, r.value), dtype=np.complex128)  # column-major storage
        check(lib().mlh_debug_get_piece(self._h, which, index, piece, dptr(out),
                                        C.byref(r), C.byref(c)))
        return out.T


@dataclass
class BatchOutput:
    aU: list              # per stack: (2K_s+1,) complex
    aD: list
    orders: list          # per stack: (2K_s+1,) int
    flux_err: np.ndarray  # (n_stacks,)
    stack_ms: np.ndarray  # (n_stacks,) device time from the solve's start to each stack's results


class Batch:
    """Independent stacks solved together, one incident angle each, with the
    per-layer work of all of them sharing every launch (mlh_batch_*)."""

    def __init__(self, ctx: Context, stacks):
        self.ctx = ctx
        self.stacks = list(stacks)  # the stacks must outlive the batch
        self._nK = [2 * s.K + 1 for s in self.stacks]
        hs = (C.c_void_p * len(self.stacks))(*[s._h.value for s in self.stacks])
        self._h = C.c_void_p()
        check(lib().mlh_batch_create(ctx.handle, len(self.stacks), hs, C.byref(self._h)))

    def close(self):
        if self._h:
            lib().mlh_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, thetas, refill: bool = False) -> BatchOutput:
        th = np.ascontiguousarray(thetas, dtype=np.float64)
        assert th.size == len(self.stacks)
        tot = sum(self._nK)
        aU = np.zeros(tot, dtype=np.complex128)
        aD = np.zeros(tot, dtype=np.complex128)
        orders = np.zeros(tot, dtype=np.int32)
        flux = np.zeros(th.size)
        ms = np.zeros(th.size)
        check(lib().mlh_batch_solve(self._h, dptr(th), int(bool(refill)), 0, aU.ctypes.data, aD.ctypes.data,
                                    orders.ctypes.data, flux.ctypes.data, ms.ctypes.data))
        cut = np.cumsum([0] + self._nK)
        sp = lambda a: [a[cut[i]:cut[i + 1]] for i in range(len(self._nK))]
        return BatchOutput(sp(aU), sp(aD), sp(orders), flux, ms)

    def get_tuning(self) -> dict:
        t = mlh_tuning()
        check(lib().mlh_batch_get_tuning(self._h, C.byref(t)))
        return {name: getattr(t, name) for name, _ in t._fields_}

    def set_tuning(self, **kw):
        t = mlh_tuning()
        check(lib().mlh_batch_get_tuning(self._h, C.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        check(lib().mlh_batch_set_tuning(self._h, C.byref(t)))

    def autotune(self, thetas, reps: int = 1) -> dict:
        th = np.ascontiguousarray(thetas, dtype=np.float64)
        t = mlh_tuning()
        check(lib().mlh_batch_autotune(self._h, dptr(th), int(reps), C.byref(t)))
        return {name: getattr(t, name) for name, _ in t._fields_}

    def tune_cached(self):
        """The batch's recorded launch choices, if any: (found, choices)."""
        t, found = mlh_tuning(), C.c_int32()
        check(lib().mlh_batch_tune_cached(self._h, C.byref(t), C.byref(found)))
        return bool(found.value), {name: getattr(t, name) for name, _ in t._fields_}


class EfficiencyObjective:
    """J(c, n) = sum over the angles of the zeroth-order reflected efficiency
    of a workloads.ShapeProblem at sine amplitudes c (I x M) and layer
    indices n, as a torch.autograd.Function: the forward pass solves on the
    GPU, the backward pass returns the adjoint gradient (mlh_adjoint):
    dJ/dn_j = omega dJ/dk_j, and dJ/dc_{i,m} from the gradient in the
    interface's cos / sin coefficients (cos_coef = c sin psi, sin_coef =
    c cos psi).  The top layer's index is the incident medium's and gets no
    gradient (zero)."""

    @staticmethod
    def function():
        import torch

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(fctx, c, n, problem, ctx, thetas):
                p = np.concatenate([c.detach().cpu().numpy().ravel(), n.detach().cpu().numpy()])
                st = Stack(ctx, problem.stack(p))
                J, gk, gs = st.adjoint(thetas, shape=True)
                st.close()
                gn = problem.omega * gk
                gn[0] = 0.0
                M = problem.c.shape[1]
                gs = gs.reshape(-1, 2, M)  # per interface: cos then sin
                gc = gs[:, 0, :] * np.sin(problem.psi) + gs[:, 1, :] * np.cos(problem.psi)
                fctx.save_for_backward(torch.as_tensor(gc, dtype=c.dtype), torch.as_tensor(gn, dtype=n.dtype))
                return torch.as_tensor(J, dtype=n.dtype)

            @staticmethod
            def backward(fctx, gout):
                gc, gn = fctx.saved_tensors
                return gout * gc, gout * gn, None, None, None

        return _F
