"""Thin ctypes binding of ``liblddmm.so`` (C ABI in include/lddmm.h).

Only argument marshalling happens here: every field operation runs in the HIP
library.  Torch tensors are used as device buffers and to pick the stream; the
library is loaded from this package directory and a missing or unloadable
library raises immediately (there is no fallback).

Layouts: scalar fields are (N0, N1, N2) tensors, vector fields (3, N0, N1, N2),
contiguous, on the context's device, with the context's dtype.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblddmm.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ENONFINITE, ESTATE, ELINESEARCH = 0, -1, -2, -3, -4, -5, -6, -7
F32, F64 = 0, 1
OP_K, OP_L = 0, 1

_c_double_p = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("nt", ctypes.c_int32),
        ("s", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("sigma2", ctypes.c_double),
        ("mem_budget_bytes", ctypes.c_int64),
        ("checkpoint_every", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


# lddmm_solve_opts.method
METHODS = {"gn_v": 0, "gn_l2": 1, "gd": 2, "newton": 3}


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("gn_iters", ctypes.c_int32),
        ("cg_iters", ctypes.c_int32),
        ("max_halvings", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("c1", ctypes.c_double),
        ("gtol", ctypes.c_double),
        ("eta_max", ctypes.c_double),
    ]


class IterLog(ctypes.Structure):
    _fields_ = [
        ("E", ctypes.c_double),
        ("E_reg", ctypes.c_double),
        ("E_data", ctypes.c_double),
        ("mse_rel", ctypes.c_double),
        ("g_norm", ctypes.c_double),
        ("g_inf_rel", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("cg_iters", ctypes.c_int32),
        ("ls_trials", ctypes.c_int32),
    ]


class SolveReport(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("cg_total", ctypes.c_int32),
        ("hessvecs", ctypes.c_int32),
        ("gradients", ctypes.c_int32),
        ("shoots", ctypes.c_int32),
        ("stop_reason", ctypes.c_int32),
        ("E_first", ctypes.c_double),
        ("E_final", ctypes.c_double),
        ("mse_rel_final", ctypes.c_double),
        ("g_rel_final", ctypes.c_double),
    ]


# name -> (restype, argtypes) of every exported entry point
SIGNATURES = {
    "lddmm_create": (ctypes.c_int, [ctypes.POINTER(Params), _vp, ctypes.POINTER(_vp)]),
    "lddmm_destroy": (ctypes.c_int, [_vp]),
    "lddmm_set_images": (ctypes.c_int, [_vp, _vp, _vp]),
    "lddmm_apply_operator": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "lddmm_dot": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _c_double_p]),
    "lddmm_shoot": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _c_double_p]),
    "lddmm_linearize": (ctypes.c_int, [_vp, _vp, _vp, _c_double_p]),
    "lddmm_gradient": (ctypes.c_int, [_vp, _vp, _vp, _c_double_p]),
    "lddmm_hessvec": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "lddmm_hessvec_newton": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "lddmm_vjp": (ctypes.c_int, [_vp, _vp, _vp]),
    "lddmm_cg_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "lddmm_gn_solve": (
        ctypes.c_int,
        [_vp, _vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveReport), ctypes.POINTER(IterLog), ctypes.c_int],
    ),
    "lddmm_pde_energy": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _c_double_p]),
    "lddmm_pde_gradient": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _c_double_p]),
    "lddmm_pde_hessvec": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp]),
    "lddmm_pde_gn_solve": (
        ctypes.c_int,
        [_vp, ctypes.c_int, _vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveReport), ctypes.POINTER(IterLog),
         ctypes.c_int],
    ),
    "lddmm_pde_displacement": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp]),
    "lddmm_jacobian_det": (ctypes.c_int, [_vp, _vp, _vp, _c_double_p, _c_double_p]),
    "lddmm_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lddmm_profile_read": (
        ctypes.c_int,
        [_vp, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_int64), _c_double_p, ctypes.c_int],
    ),
    "lddmm_set_option": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_int64]),
    "lddmm_get_option": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)]),
    "lddmm_autotune": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _c_double_p]),
    "lddmm_sync": (ctypes.c_int, [_vp]),
    "lddmm_memory_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64)]),
    "lddmm_batch_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(_vp)]),
    "lddmm_batch_destroy": (ctypes.c_int, [_vp]),
    "lddmm_batch_get": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_vp)]),
    "lddmm_batch_sync": (ctypes.c_int, [_vp]),
    "lddmm_batch_gn_solve": (
        ctypes.c_int,
        [_vp, ctypes.POINTER(_vp), ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveReport), ctypes.c_int],
    ),
    "lddmm_batch_hessvec": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int]),
    "lddmm_batch_autotune": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lddmm_apply_operator_noalloc": (
        ctypes.c_int,
        [ctypes.POINTER(ctypes.c_int32), ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp,
         _vp, _vp],
    ),
    "lddmm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lddmm_last_error": (ctypes.c_char_p, [_vp]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblddmm.so once and declare every signature; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class LddmmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class Trace:
    """Gauss-Newton solve outcome: report fields and per-iteration log records."""

    report: dict
    log: list


def apply_operator_noalloc(op, f, alpha, s=2, out=None):
    """K f (op = OP_K) or L f (op = OP_L) without a context and without any
    device allocation by the library (``lddmm_apply_operator_noalloc``): the
    transform's workspace is the library's static per-device array.  f is a
    contiguous float32/float64 scalar (N0, N1, N2) or vector (3, N0, N1, N2)
    field on the current HIP device; out (same shape, dtype, device) may be f
    itself.  Ordered on torch's current stream."""
    lib = load_library()
    if f.dim() not in (3, 4) or (f.dim() == 4 and f.shape[0] != 3):
        raise ValueError("f must be (N0, N1, N2) or (3, N0, N1, N2)")
    if f.dtype not in (torch.float32, torch.float64) or f.device.type != "cuda" or not f.is_contiguous():
        raise ValueError("f must be a contiguous float32/float64 tensor on a HIP device")
    if out is None:
        out = torch.empty_like(f)
    elif out.shape != f.shape or out.dtype != f.dtype or out.device != f.device or not out.is_contiguous():
        raise ValueError("out must match f's shape, dtype and device and be contiguous")
    ncomp = 3 if f.dim() == 4 else 1
    n = (ctypes.c_int32 * 3)(*[int(x) for x in f.shape[-3:]])
    dtype = F32 if f.dtype == torch.float32 else F64
    with torch.cuda.device(f.device):
        st = torch.cuda.current_stream(f.device).cuda_stream
        rc = lib.lddmm_apply_operator_noalloc(n, dtype, float(alpha), int(s), int(op), ncomp, _ptr(f), _ptr(out),
                                              ctypes.c_void_p(st))
    if rc != OK:
        msg = lib.lddmm_last_error(None) or b""
        raise LddmmError(rc, f"apply_operator_noalloc: {lib.lddmm_strerror(rc).decode()}: {msg.decode()}")
    return out


class Registration:
    """One registration problem on one device (a ``lddmm_ctx``).

    n = (N0, N1, N2) grid on [0, 2 pi)^3, nt Heun steps, L = (Id - alpha Lap)^s,
    sigma2 the data-term variance, dtype torch.float32 or torch.float64.
    """

    def __init__(self, n, nt, alpha, s=2, sigma2=1.0, dtype=torch.float32, device="cuda:0", checkpoint_every=0,
                 mem_budget_bytes=0, _handle=None):
        self.lib = load_library()
        self._owned = _handle is None
        self.n = tuple(int(x) for x in n)
        self.nt, self.alpha, self.s, self.sigma2 = int(nt), float(alpha), int(s), float(sigma2)
        self.dtype = dtype
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the library runs on a HIP device only")
        torch.cuda.set_device(self.device)
        if _handle is not None:
            # a batch context: its work runs on a library-owned stream
            self.stream = None
            self._ctx = ctypes.c_void_p(_handle)
            return
        self.stream = torch.cuda.current_stream(self.device)
        p = Params()
        p.n = (ctypes.c_int32 * 3)(*self.n)
        p.nt, p.s = self.nt, self.s
        p.dtype = F32 if dtype == torch.float32 else F64
        p.alpha, p.sigma2 = self.alpha, self.sigma2
        p.checkpoint_every, p.mem_budget_bytes = int(checkpoint_every), int(mem_budget_bytes)
        self._ctx = ctypes.c_void_p()
        rc = self.lib.lddmm_create(ctypes.byref(p), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._ctx))
        if rc != OK:
            raise LddmmError(rc, "lddmm_create: " + self.lib.lddmm_strerror(rc).decode())

    # ---- helpers ----------------------------------------------------------
    def close(self):
        if getattr(self, "_owned", False) and getattr(self, "_ctx", None) is not None and self._ctx.value:
            self.lib.lddmm_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if self.stream is None and rc == OK:
            # batch context: make its results visible to torch's stream
            rc = self.lib.lddmm_sync(self._ctx)
        if rc != OK:
            msg = self.lib.lddmm_last_error(self._ctx) or b""
            raise LddmmError(rc, f"{what}: {self.lib.lddmm_strerror(rc).decode()}: {msg.decode()}")

    def _field(self, t, ncomp, name):
        if self.stream is None:
            # batch context on its own stream: inputs must be complete first
            torch.cuda.current_stream(self.device).synchronize()
        shape = (ncomp,) + self.n if ncomp == 3 else self.n
        if t is None:
            raise ValueError(f"{name} is required")
        if tuple(t.shape) != shape or t.dtype != self.dtype or t.device != self.device or not t.is_contiguous():
            raise ValueError(
                f"{name}: expected contiguous {self.dtype} {shape} on {self.device}, "
                f"got {t.dtype} {tuple(t.shape)} on {t.device}"
            )
        return t

    def empty_vector(self):
        return torch.empty((3,) + self.n, dtype=self.dtype, device=self.device)

    def empty_scalar(self):
        return torch.empty(self.n, dtype=self.dtype, device=self.device)

    # ---- entry points (same names as the C ABI) ----------------------------
    def set_images(self, I0, I1):
        self._check(
            self.lib.lddmm_set_images(self._ctx, _ptr(self._field(I0, 1, "I0")), _ptr(self._field(I1, 1, "I1"))),
            "set_images",
        )

    def apply_operator(self, op, f, out=None):
        ncomp = 3 if f.dim() == 4 else 1
        self._field(f, ncomp, "in")
        out = torch.empty_like(f) if out is None else self._field(out, ncomp, "out")
        self._check(self.lib.lddmm_apply_operator(self._ctx, op, ncomp, _ptr(f), _ptr(out)), "apply_operator")
        return out

    def apply_K(self, f, out=None):
        return self.apply_operator(OP_K, f, out)

    def apply_L(self, f, out=None):
        return self.apply_operator(OP_L, f, out)

    def dot(self, a, b):
        ncomp = 3 if a.dim() == 4 else 1
        r = ctypes.c_double()
        self._check(
            self.lib.lddmm_dot(self._ctx, ncomp, _ptr(self._field(a, ncomp, "a")), _ptr(self._field(b, ncomp, "b")),
                               ctypes.byref(r)),
            "dot",
        )
        return r.value

    def shoot(self, v0, want=("J1", "u1", "v1"), energy=False):
        self._field(v0, 3, "v0")
        J1 = self.empty_scalar() if "J1" in want else None
        u1 = self.empty_vector() if "u1" in want else None
        v1 = self.empty_vector() if "v1" in want else None
        e = ctypes.c_double()
        self._check(
            self.lib.lddmm_shoot(self._ctx, _ptr(v0), _ptr(J1), _ptr(u1), _ptr(v1), ctypes.byref(e) if energy else None),
            "shoot",
        )
        out = {"J1": J1, "u1": u1, "v1": v1}
        if energy:
            out["energy"] = e.value
        return out

    def linearize(self, v0, J1_out=None):
        e = ctypes.c_double()
        J1p = None if J1_out is None else _ptr(self._field(J1_out, 1, "J1"))
        self._check(
            self.lib.lddmm_linearize(self._ctx, _ptr(self._field(v0, 3, "v0")), J1p, ctypes.byref(e)), "linearize"
        )
        return e.value

    def gradient(self, v0, out=None):
        out = self.empty_vector() if out is None else self._field(out, 3, "g")
        e = ctypes.c_double()
        self._check(
            self.lib.lddmm_gradient(self._ctx, _ptr(self._field(v0, 3, "v0")), _ptr(out), ctypes.byref(e)), "gradient"
        )
        return out, e.value

    def hessvec(self, dv, v0=None, out=None, newton=False):
        """Gauss-Newton Hessian-vector product in V (newton=True: the full Newton Hessian)."""
        out = self.empty_vector() if out is None else self._field(out, 3, "hv")
        v0p = None if v0 is None else _ptr(self._field(v0, 3, "v0"))
        fn = self.lib.lddmm_hessvec_newton if newton else self.lib.lddmm_hessvec
        self._check(fn(self._ctx, v0p, _ptr(self._field(dv, 3, "dv")), _ptr(out)), "hessvec")
        return out

    def vjp(self, gbar_J1, out=None):
        out = self.empty_vector() if out is None else self._field(out, 3, "gbar_v0")
        self._check(self.lib.lddmm_vjp(self._ctx, _ptr(self._field(gbar_J1, 1, "gbar_J1")), _ptr(out)), "vjp")
        return out

    def cg_solve(self, g, eta, maxit, out=None):
        out = self.empty_vector() if out is None else self._field(out, 3, "x")
        its = ctypes.c_int()
        self._check(
            self.lib.lddmm_cg_solve(self._ctx, _ptr(self._field(g, 3, "g")), _ptr(out), float(eta), int(maxit),
                                    ctypes.byref(its)),
            "cg_solve",
        )
        return out, its.value

    def gn_solve(self, v0, gn_iters=None, cg_iters=20, max_halvings=10, c1=1e-4, gtol=1e-3, eta_max=0.5,
                 method="gn_v"):
        """Solve from v0 (updated in place); returns a Trace.  method: "gn_v"
        (Gauss-Newton, CG in V), "gn_l2" (Gauss-Newton, PCG in L2 with
        preconditioner K), "gd" (gradient descent in V) or "newton" (Newton-Krylov
        in V on the full Hessian).  gn_iters defaults to 10 (50 for "gd")."""
        self._field(v0, 3, "v0")
        m = METHODS[method]
        if gn_iters is None:
            gn_iters = 50 if method == "gd" else 10
        o = SolveOpts(gn_iters, cg_iters, max_halvings, m, c1, gtol, eta_max)
        rep = SolveReport()
        cap = max(1, gn_iters)
        logs = (IterLog * cap)()
        self._check(
            self.lib.lddmm_gn_solve(self._ctx, _ptr(v0), ctypes.byref(o), ctypes.byref(rep), logs, cap), "gn_solve"
        )
        rd = {k: getattr(rep, k) for k, _ in SolveReport._fields_}
        log = [{k: getattr(logs[i], k) for k, _ in IterLog._fields_} for i in range(min(rep.iters, cap))]
        return Trace(rd, log)

    # ---- PDE-LDDMM (Section 2.3 comparison method) ---------------------------
    def _pde_field(self, t, stationary, name):
        shape = (3,) + self.n if stationary else (self.nt + 1, 3) + self.n
        if t is None:
            raise ValueError(f"{name} is required")
        if tuple(t.shape) != shape or t.dtype != self.dtype or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name}: expected contiguous {self.dtype} {shape} on {self.device}, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")
        if self.stream is None:
            torch.cuda.current_stream(self.device).synchronize()
        return t

    def empty_velocity(self, stationary):
        shape = (3,) + self.n if stationary else (self.nt + 1, 3) + self.n
        return torch.empty(shape, dtype=self.dtype, device=self.device)

    def pde_energy(self, v, stationary=True, m1=True):
        """PDE-LDDMM energy at v (one field, or nt + 1 stacked when not stationary);
        returns (E, m(1) or None).  Becomes the current PDE linearization."""
        self._pde_field(v, stationary, "v")
        out = self.empty_scalar() if m1 else None
        e = ctypes.c_double()
        self._check(self.lib.lddmm_pde_energy(self._ctx, int(bool(stationary)), _ptr(v), _ptr(out), ctypes.byref(e)),
                    "pde_energy")
        return e.value, out

    def pde_gradient(self, v, stationary=True, out=None):
        """L2 gradient of PDE-LDDMM at v; returns (g, E)."""
        self._pde_field(v, stationary, "v")
        out = self.empty_velocity(stationary) if out is None else self._pde_field(out, stationary, "g")
        e = ctypes.c_double()
        self._check(self.lib.lddmm_pde_gradient(self._ctx, int(bool(stationary)), _ptr(v), _ptr(out), ctypes.byref(e)),
                    "pde_gradient")
        return out, e.value

    def pde_hessvec(self, dv, stationary=True, v=None, out=None):
        """Gauss-Newton Hessian of PDE-LDDMM in L2 (v None: the current linearization)."""
        self._pde_field(dv, stationary, "dv")
        if v is not None:
            self._pde_field(v, stationary, "v")
        out = self.empty_velocity(stationary) if out is None else self._pde_field(out, stationary, "hv")
        self._check(self.lib.lddmm_pde_hessvec(self._ctx, int(bool(stationary)), _ptr(v), _ptr(dv), _ptr(out)),
                    "pde_hessvec")
        return out

    def pde_gn_solve(self, v, stationary=True, gn_iters=10, cg_iters=20, max_halvings=10, c1=1e-4, gtol=1e-3,
                     eta_max=0.5):
        """Gauss-Newton-Krylov for PDE-LDDMM from v (updated in place); returns a Trace."""
        self._pde_field(v, stationary, "v")
        o = SolveOpts(gn_iters, cg_iters, max_halvings, 0, c1, gtol, eta_max)
        rep = SolveReport()
        cap = max(1, gn_iters)
        logs = (IterLog * cap)()
        self._check(self.lib.lddmm_pde_gn_solve(self._ctx, int(bool(stationary)), _ptr(v), ctypes.byref(o),
                                                ctypes.byref(rep), logs, cap), "pde_gn_solve")
        rd = {k: getattr(rep, k) for k, _ in SolveReport._fields_}
        log = [{k: getattr(logs[i], k) for k, _ in IterLog._fields_} for i in range(min(rep.iters, cap))]
        return Trace(rd, log)

    def pde_displacement(self, v, stationary=True, out=None):
        """Inverse-map displacement u1 of the PDE-LDDMM flow of v (warped template
        I_0 o (id + u1)); feed it to jacobian_det for det(I + D u1)."""
        self._pde_field(v, stationary, "v")
        out = self.empty_vector() if out is None else self._field(out, 3, "u1")
        self._check(self.lib.lddmm_pde_displacement(self._ctx, int(bool(stationary)), _ptr(v), _ptr(out)),
                    "pde_displacement")
        return out

    def jacobian_det(self, u, out=None):
        out = self.empty_scalar() if out is None else self._field(out, 1, "det")
        mn, mx = ctypes.c_double(), ctypes.c_double()
        self._check(
            self.lib.lddmm_jacobian_det(self._ctx, _ptr(self._field(u, 3, "u")), _ptr(out), ctypes.byref(mn),
                                        ctypes.byref(mx)),
            "jacobian_det",
        )
        return out, mn.value, mx.value

    def profile_enable(self, on=True):
        self._check(self.lib.lddmm_profile_enable(self._ctx, 1 if on else 0), "profile_enable")

    def profile_read(self, cap=64):
        names = (ctypes.c_char_p * cap)()
        counts = (ctypes.c_int64 * cap)()
        ms = (ctypes.c_double * cap)()
        k = self.lib.lddmm_profile_read(self._ctx, names, counts, ms, cap)
        if k < 0:
            self._check(k, "profile_read")
        return {names[i].decode(): (counts[i], ms[i]) for i in range(min(k, cap))}

    def set_option(self, key, value):
        self._check(self.lib.lddmm_set_option(self._ctx, key.encode(), int(value)), f"set_option({key})")

    def get_option(self, key):
        v = ctypes.c_int64()
        self._check(self.lib.lddmm_get_option(self._ctx, key.encode(), ctypes.byref(v)), f"get_option({key})")
        return v.value

    def autotune(self, reps=5):
        """Time the transform variants on this grid and keep the fastest;
        returns (variants tried, ms per K application of a vector field)."""
        tried, ms = ctypes.c_int(), ctypes.c_double()
        self._check(self.lib.lddmm_autotune(self._ctx, int(reps), ctypes.byref(tried), ctypes.byref(ms)), "autotune")
        return tried.value, ms.value

    def sync(self):
        self._check(self.lib.lddmm_sync(self._ctx), "sync")

    def memory_bytes(self):
        b = ctypes.c_int64()
        self._check(self.lib.lddmm_memory_bytes(self._ctx, ctypes.byref(b)), "memory_bytes")
        return b.value


class Batch:
    """Independent registrations, one context per pair on its own stream.

    specs: list of dicts with keys n, nt, alpha, s, sigma2 (dtype shared).
    ``contexts[i]`` is a Registration view of pair i; gn_solve / hessvec run all
    pairs concurrently (one host thread each) or in order.
    """

    def __init__(self, specs, dtype=torch.float32, device="cuda:0"):
        self.lib = load_library()
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        arr = (Params * len(specs))()
        for i, sp in enumerate(specs):
            p = arr[i]
            p.n = (ctypes.c_int32 * 3)(*[int(x) for x in sp["n"]])
            p.nt, p.s = int(sp["nt"]), int(sp.get("s", 2))
            p.dtype = F32 if dtype == torch.float32 else F64
            p.alpha, p.sigma2 = float(sp["alpha"]), float(sp.get("sigma2", 1.0))
        self._b = ctypes.c_void_p()
        rc = self.lib.lddmm_batch_create(arr, len(specs), ctypes.byref(self._b))
        if rc != OK:
            raise LddmmError(rc, "lddmm_batch_create: " + self.lib.lddmm_strerror(rc).decode())
        self.contexts = []
        for i, sp in enumerate(specs):
            h = ctypes.c_void_p()
            self.lib.lddmm_batch_get(self._b, i, ctypes.byref(h))
            self.contexts.append(
                Registration(sp["n"], sp["nt"], sp["alpha"], sp.get("s", 2), sp.get("sigma2", 1.0), dtype=dtype,
                             device=device, _handle=h.value)
            )

    def __len__(self):
        return len(self.contexts)

    def _rc(self, rc, what):
        if rc != OK:
            raise LddmmError(rc, f"{what}: {self.lib.lddmm_strerror(rc).decode()}")

    def _fields(self, ts, name):
        """Check one vector field per pair (count, shape, dtype, device, contiguity)."""
        ts = list(ts)
        if len(ts) != len(self.contexts):
            raise ValueError(f"{name}: {len(ts)} fields for {len(self.contexts)} pairs")
        for i, t in enumerate(ts):
            if t is None:
                raise ValueError(f"{name}[{i}] is required")
            R = self.contexts[i]
            shape = (3,) + R.n
            if tuple(t.shape) != shape or t.dtype != R.dtype or t.device != R.device or not t.is_contiguous():
                raise ValueError(
                    f"{name}[{i}]: expected contiguous {R.dtype} {shape} on {R.device}, "
                    f"got {t.dtype} {tuple(t.shape)} on {t.device}"
                )
        return (_vp * len(ts))(*[t.data_ptr() for t in ts])

    MODES = {"sequential": 0, "threads": 1, "lockstep": 2}

    def _mode(self, concurrent, mode, default):
        if mode is None:
            return self.MODES[default] if concurrent else self.MODES["sequential"]
        if mode not in self.MODES:
            raise ValueError(f"mode must be one of {sorted(self.MODES)}")
        return self.MODES[mode]

    def gn_solve(self, v0s, concurrent=True, gn_iters=None, cg_iters=20, max_halvings=10, c1=1e-4, gtol=1e-3,
                 eta_max=0.5, method="gn_v", mode=None):
        """Solve every pair from its v0 (updated in place).  mode: "sequential",
        "threads" (one host thread per pair, each pair at its own pace; its CG
        iterations replayed from its own graph) or "lockstep" (each phase
        enqueued for all pairs before one wait, CG iterations as one graph
        spanning the pairs); default "threads" (measured faster for whole solves:
        lockstep waits for the slowest pair at every phase), or "sequential" with
        concurrent=False.  Every mode gives bitwise the single-context results."""
        m = self._mode(concurrent, mode, "threads")
        ptrs = self._fields(v0s, "v0s")
        torch.cuda.current_stream(self.device).synchronize()
        if gn_iters is None:
            gn_iters = 50 if method == "gd" else 10
        o = SolveOpts(gn_iters, cg_iters, max_halvings, METHODS[method], c1, gtol, eta_max)
        reps = (SolveReport * len(self.contexts))()
        self._rc(self.lib.lddmm_batch_gn_solve(self._b, ptrs, ctypes.byref(o), reps, m), "batch_gn_solve")
        return [{k: getattr(r, k) for k, _ in SolveReport._fields_} for r in reps]

    def hessvec(self, dvs, hvs, reps=1, concurrent=True, mode=None):
        """reps Gauss-Newton Hv of every pair at its current linearization (modes as
        in gn_solve; "lockstep", the default, replays one graph spanning all pairs
        per round)."""
        m = self._mode(concurrent, mode, "lockstep")
        a = self._fields(dvs, "dvs")
        b = self._fields(hvs, "hvs")
        torch.cuda.current_stream(self.device).synchronize()
        self._rc(self.lib.lddmm_batch_hessvec(self._b, a, b, int(reps), m), "batch_hessvec")

    def autotune(self, reps=5):
        self._rc(self.lib.lddmm_batch_autotune(self._b, int(reps)), "batch_autotune")

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            self.lib.lddmm_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
