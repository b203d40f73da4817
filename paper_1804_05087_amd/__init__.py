"""Stokes-preconditioned Newton-Krylov for plane Couette flow on one MI355X.

Python face of libsp.so (see include/sp.h). ``Plan`` marshals torch tensors
(complex128, canonical layout [3][nx][nz/2+1][ny], on the GPU) to the C ABI;
``PhiFunction`` exposes Phi_dt to torch autograd on packed float64 vectors.
"""
from __future__ import annotations

import ctypes as C
import math

from . import _lib
from ._lib import (SP_FP64, SP_MIXED, SP_OP_PHI, SP_OP_RESIDUAL, SP_STAGE_SOLVE, SP_STAGE_SYNTH,
                   SP_STAGE_XFWD, SP_STAGE_XINV, SP_STAGE_ZLINE, SPError)

__all__ = ["Plan", "PhiFunction", "SPError", "SP_FP64", "SP_MIXED", "SP_OP_PHI",
           "SP_OP_RESIDUAL", "SP_STAGE_SYNTH", "SP_STAGE_XINV", "SP_STAGE_ZLINE", "SP_STAGE_XFWD",
           "SP_STAGE_SOLVE", "couette_box", "hook_step"]


def couette_box():
    """The plane Couette box of the paper's Channelflow runs (Sec. 3.3)."""
    return 2 * math.pi / 1.14, 2 * math.pi / 2.5


def _torch():
    import torch
    return torch


def hook_step(R, g, delta: float):
    """The hookstep subproblem of sp_newton_hookstep on the host (numpy
    arrays): R k x k upper triangular, g the k+1 rotated right-hand side.
    Returns (y, mu, model residual norm)."""
    import numpy as np
    lib = _lib.load()
    Rf = np.asfortranarray(np.asarray(R, dtype=np.float64))
    gv = np.ascontiguousarray(np.asarray(g, dtype=np.float64))
    k = Rf.shape[1]
    if Rf.shape != (k, k) or gv.shape != (k + 1,):
        raise ValueError("R must be k x k and g of length k + 1")
    y = np.zeros(k)
    mu, res = C.c_double(), C.c_double()
    st = lib.sp_hook_step(Rf.ctypes.data, k, gv.ctypes.data, k, float(delta), y.ctypes.data,
                          C.byref(mu), C.byref(res))
    if st != 0:
        raise SPError(st, lib.sp_status_string(st).decode())
    return y, mu.value, res.value


class Plan:
    """A plan for one grid, Reynolds number and BEFE step dt on one GPU."""

    def __init__(self, nx: int, ny: int, nz: int, lx: float, lz: float, re: float, dt: float,
                 wall_upper: float = 1.0, wall_lower: float = -1.0, precision: int = SP_FP64,
                 device=None):
        torch = _torch()
        self.lib = _lib.load()
        dev = torch.device(device if device is not None else "cuda")
        if dev.type != "cuda":
            raise ValueError("Plan needs a GPU device")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.stream = torch.cuda.current_stream(self.device)
        prm = _lib.sp_params(nx, ny, nz, lx, lz, re, dt, wall_upper, wall_lower, precision)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.sp_plan_create(C.byref(prm), C.c_void_p(self.stream.cuda_stream),
                                         C.byref(h))
        if st != 0:
            raise SPError(st, self.lib.sp_status_string(st).decode())
        self.h = h
        self.nx, self.ny, self.nz = nx, ny, nz
        self.lx, self.lz, self.re, self.dt = lx, lz, re, dt
        self.shape = (3, nx, nz // 2 + 1, ny)
        self.packed_n = 3 * ny * (nx - 1) * (nz - 1)
        self.nsteps = 1
        self.scheme = 0
        self._ws = None

    # ------------------------------------------------------------------ helpers
    def _check(self, st: int):
        if st != 0:
            msg = self.lib.sp_last_error(self.h).decode()
            raise SPError(st, f"{self.lib.sp_status_string(st).decode()}: {msg}")

    def _field(self, t, name="field"):
        torch = _torch()
        if t.dtype != torch.complex128 or tuple(t.shape) != self.shape:
            raise ValueError(f"{name} must be complex128 of shape {self.shape}")
        if t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous tensor on {self.device}")
        return C.c_void_p(t.data_ptr())

    def _packed(self, t, name="packed"):
        torch = _torch()
        if t.dtype != torch.float64 or tuple(t.shape) != (self.packed_n,):
            raise ValueError(f"{name} must be float64 of shape ({self.packed_n},)")
        if t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous tensor on {self.device}")
        return C.c_void_p(t.data_ptr())

    def empty(self):
        torch = _torch()
        return torch.empty(self.shape, dtype=torch.complex128, device=self.device)

    def close(self):
        if getattr(self, "h", None):
            self.lib.sp_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ configuration
    def set_dt(self, dt: float):
        self._check(self.lib.sp_plan_set_dt(self.h, dt))
        self.dt = dt

    def set_precision(self, precision: int):
        self._check(self.lib.sp_plan_set_precision(self.h, precision))

    def symmetrize(self, a):
        """In place: project a canonical field onto the shift-reflect
        invariant subspace (EQ1's symmetry group)."""
        self._check(self.lib.sp_symmetrize(self.h, self._field(a, "a")))
        return a

    def set_symmetry(self, on: bool = True):
        """Confine the Newton drivers to the shift-reflect invariant subspace."""
        self._check(self.lib.sp_plan_set_symmetry(self.h, 1 if on else 0))

    def set_advection(self, on: bool = True, host_build: bool = False):
        """Laminar advection (U_lam . grad) u + (u . grad) U_lam in the
        implicit operator of every step (same roots, different Jacobian).
        The per-mode operators are built on the device, or on the host with
        host_build (the reference construction)."""
        self._check(self.lib.sp_plan_set_advection(self.h, (2 if host_build else 1) if on else 0))
        self.advect = bool(on)

    def set_scheme(self, scheme: int):
        """Integrator of the residual operator: 0 = BEFE steps of dt, 1 =
        SBDF2 with implicit step dt (time step 1.5 dt); see set_steps."""
        self._check(self.lib.sp_plan_set_scheme(self.h, int(scheme)))
        self.scheme = int(scheme)

    def set_steps(self, nsteps: int):
        """Residual operator of nsteps BEFE steps of dt: 1 = Stokes operator
        (T = dt), > 1 = time-integration operator with T = nsteps * dt."""
        self._check(self.lib.sp_plan_set_steps(self.h, nsteps))
        self.nsteps = nsteps

    # ------------------------------------------------------------------ operators
    def nonlinear(self, u, out=None):
        out = self.empty() if out is None else out
        self._check(self.lib.sp_nonlinear(self.h, self._field(u, "u"), self._field(out, "out")))
        return out

    def stokes_solve(self, g, out=None, inhomogeneous: bool = False):
        out = self.empty() if out is None else out
        self._check(self.lib.sp_stokes_solve(self.h, self._field(g, "g"), self._field(out, "out"),
                                             1 if inhomogeneous else 0))
        return out

    def befe_step(self, u, out=None):
        out = self.empty() if out is None else out
        self._check(self.lib.sp_befe_step(self.h, self._field(u, "u"), self._field(out, "out")))
        return out

    def befe_step_noalloc(self, u, out):
        """Phi_dt(u) into out with the intermediates in the library's fixed
        per-device scratch (sp_befe_step_noalloc): no device allocation; calls
        that overlap on one device race."""
        self._check(self.lib.sp_befe_step_noalloc(self.h, self._field(u, "u"),
                                                  self._field(out, "out")))
        return out

    def residual(self, u, out=None, norm: bool = False):
        out = self.empty() if out is None else out
        nrm = C.c_double(0.0)
        self._check(self.lib.sp_residual(self.h, self._field(u, "u"), self._field(out, "out"),
                                         C.byref(nrm) if norm else None))
        return (out, nrm.value) if norm else out

    def norm(self, a) -> float:
        nrm = C.c_double(0.0)
        self._check(self.lib.sp_norm(self.h, self._field(a, "a"), C.byref(nrm)))
        return nrm.value

    def linearize(self, u):
        self._check(self.lib.sp_linearize(self.h, self._field(u, "u")))

    def jvp_lin(self, du, op: int = SP_OP_PHI, out=None):
        out = self.empty() if out is None else out
        self._check(self.lib.sp_jvp_lin(self.h, op, self._field(du, "du"), self._field(out, "out")))
        return out

    def jvp(self, u, du, op: int = SP_OP_PHI, out=None):
        out = self.empty() if out is None else out
        self._check(self.lib.sp_jvp(self.h, op, self._field(u, "u"), self._field(du, "du"),
                                    self._field(out, "out")))
        return out

    def vjp_lin(self, w, op: int = SP_OP_PHI, out=None):
        out = self.empty() if out is None else out
        self._check(self.lib.sp_vjp_lin(self.h, op, self._field(w, "w"), self._field(out, "out")))
        return out

    def vjp(self, u, w, op: int = SP_OP_PHI, out=None):
        out = self.empty() if out is None else out
        self._check(self.lib.sp_vjp(self.h, op, self._field(u, "u"), self._field(w, "w"),
                                    self._field(out, "out")))
        return out

    def _batch(self, t, name):
        torch = _torch()
        if (t.dtype != torch.complex128 or t.dim() != 5 or tuple(t.shape[1:]) != self.shape
                or not t.is_contiguous() or t.device != self.device):
            raise ValueError(f"{name} must be a contiguous complex128 (count, *{self.shape}) "
                             f"tensor on {self.device}")
        return C.c_void_p(t.data_ptr())

    def befe_step_batch(self, u, out=None, streams: int = 3):
        """Phi_dt of each of the count fields u[i] (a (count, *shape) tensor),
        up to `streams` of them concurrently (3 with the plan's own stream
        fill the 4 hardware queues a process gets by default)."""
        torch = _torch()
        out = torch.empty_like(u) if out is None else out
        self._check(self.lib.sp_befe_step_batch(self.h, u.shape[0], streams,
                                                self._batch(u, "u"), self._batch(out, "out")))
        return out

    def jvp_lin_batch(self, du, op: int = SP_OP_PHI, out=None, streams: int = 3):
        """The Jacobian action about the base of linearize() on each du[i]."""
        torch = _torch()
        out = torch.empty_like(du) if out is None else out
        self._check(self.lib.sp_jvp_lin_batch(self.h, op, du.shape[0], streams,
                                              self._batch(du, "du"), self._batch(out, "out")))
        return out

    def jacobian_columns(self, op: int = SP_OP_PHI, first: int = 0, count=None, out=None):
        """Columns first .. first+count-1 of the dense Jacobian in the packed
        real basis about the base state of linearize(), as the rows of a
        (count, packed_n) float64 tensor (row c = column first + c), formed on
        the device without host synchronisation."""
        torch = _torch()
        n = self.packed_n
        count = n - first if count is None else count
        if out is None:
            out = torch.empty((count, n), dtype=torch.float64, device=self.device)
        if (out.dtype != torch.float64 or out.dim() != 2 or tuple(out.shape) != (count, n)
                or not out.is_contiguous() or out.device != self.device):
            raise ValueError(f"out must be a contiguous float64 ({count}, {n}) tensor on {self.device}")
        self._check(self.lib.sp_jacobian_columns(self.h, op, first, count, out.data_ptr(), n))
        return out

    def pack(self, a, out=None):
        torch = _torch()
        out = torch.empty(self.packed_n, dtype=torch.float64, device=self.device) \
            if out is None else out
        self._check(self.lib.sp_pack(self.h, self._field(a, "a"), self._packed(out, "out")))
        return out

    def unpack(self, x, out=None):
        out = self.empty() if out is None else out
        self._check(self.lib.sp_unpack(self.h, self._packed(x, "x"), self._field(out, "out")))
        return out

    def time_stage(self, stage: int, u, out=None, reps: int = 100) -> float:
        """Average microseconds per launch of one stage kernel of Phi_dt(u)
        (SP_STAGE_*), launched back to back; out receives Phi_dt(u)."""
        out = self.empty() if out is None else out
        us = C.c_double(0.0)
        self._check(self.lib.sp_time_stage(self.h, int(stage), self._field(u, "u"),
                                           self._field(out, "out"), int(reps), C.byref(us)))
        return us.value

    def profile_enable(self, on: bool = True):
        self._check(self.lib.sp_profile_enable(self.h, 1 if on else 0))

    def profile_read(self, reset: bool = True):
        """{kernel name: (launches, total ms)} since the last reset (synchronises)."""
        nmax = 64
        names = C.create_string_buffer(32 * nmax)
        counts = (C.c_int64 * nmax)()
        ms = (C.c_double * nmax)()
        n = C.c_int32(0)
        self._check(self.lib.sp_profile_read(self.h, nmax, names, counts, ms, C.byref(n),
                                             1 if reset else 0))
        out = {}
        for k in range(n.value):
            nm = names.raw[32 * k: 32 * k + 32].split(b"\0", 1)[0].decode()
            out[nm] = (int(counts[k]), float(ms[k]))
        return out

    def newton_gmres(self, u, max_newton: int = 5, max_krylov: int = 40,
                     gmres_rtol: float = 1e-4, newton_tol: float = 1e-10, jvp_mode: int = 0,
                     fd_eps: float = 1e-7, krylov_fp32: bool = False):
        """Newton-GMRES in place on u; returns the report as a dict.
        krylov_fp32 stores the Krylov basis in FP32."""
        opts = _lib.sp_newton_opts(max_newton, max_krylov, gmres_rtol, newton_tol, jvp_mode,
                                   fd_eps, int(krylov_fp32))
        rep = _lib.sp_newton_report()
        st = self.lib.sp_newton_gmres(self.h, self._field(u, "u"), C.byref(opts), C.byref(rep))
        if st not in (0, _lib.SP_ERR_NOT_CONVERGED):
            self._check(st)
        n = rep.newton_iters
        return {
            "converged": bool(rep.converged),
            "newton_iters": n,
            "total_krylov": rep.total_krylov,
            "total_actions": rep.total_actions,
            "seconds": rep.seconds,
            "res_norm": list(rep.res_norm[: n + 1]),
            "krylov": list(rep.krylov[:n]),
            "gmres_relres": list(rep.gmres_relres[:n]),
        }


    def newton_hookstep(self, u, max_newton: int = 5, max_krylov: int = 40,
                        gmres_rtol: float = 1e-4, newton_tol: float = 1e-10,
                        jvp_mode: int = 0, fd_eps: float = 1e-7, max_trials: int = 10,
                        delta_init: float = 0.0, delta_min: float = 1e-12,
                        delta_max: float = 1e300, krylov_fp32: bool = False):
        """Trust-region Newton-GMRES (hookstep) in place on u; returns the
        report of newton_gmres plus the per-step trials, delta, mu, step_norm
        and rho of the accepted steps."""
        opts = _lib.sp_newton_opts(max_newton, max_krylov, gmres_rtol, newton_tol, jvp_mode,
                                   fd_eps, int(krylov_fp32))
        hook = _lib.sp_hook_opts(max_trials, delta_init, delta_min, delta_max)
        rep = _lib.sp_newton_report()
        hrep = _lib.sp_hook_report()
        st = self.lib.sp_newton_hookstep(self.h, self._field(u, "u"), C.byref(opts),
                                         C.byref(hook), C.byref(rep), C.byref(hrep))
        if st not in (0, _lib.SP_ERR_NOT_CONVERGED):
            self._check(st)
        n = rep.newton_iters
        na = sum(1 for t in hrep.trials[:n] if t > 0)
        out = {
            "converged": bool(rep.converged),
            "newton_iters": n,
            "total_krylov": rep.total_krylov,
            "total_actions": rep.total_actions,
            "seconds": rep.seconds,
            "res_norm": list(rep.res_norm[: n + 1]),
            "krylov": list(rep.krylov[:n]),
            "gmres_relres": list(rep.gmres_relres[:n]),
            "trials": list(hrep.trials[:na]),
            "delta": list(hrep.delta[:na]),
            "mu": list(hrep.mu[:na]),
            "step_norm": list(hrep.step_norm[:na]),
            "rho": list(hrep.rho[:na]),
        }
        if st == _lib.SP_ERR_NOT_CONVERGED:
            out["message"] = self.lib.sp_last_error(self.h).decode()
        return out


def _make_phi_function():
    torch = _torch()

    class PhiFunction(torch.autograd.Function):
        """Phi_dt on packed float64 vectors; backward is the library's VJP."""

        @staticmethod
        def forward(ctx, x, plan):
            u = plan.unpack(x.contiguous())
            y = plan.pack(plan.befe_step(u))
            ctx.plan = plan
            ctx.save_for_backward(x.detach().clone())
            return y

        @staticmethod
        def backward(ctx, gy):
            (x,) = ctx.saved_tensors
            plan = ctx.plan
            u = plan.unpack(x)
            w = plan.unpack(gy.contiguous())
            gx = plan.pack(plan.vjp(u, w, SP_OP_PHI))
            return gx, None

    return PhiFunction


class _LazyPhi:
    _fn = None

    def __getattr__(self, name):
        if _LazyPhi._fn is None:
            _LazyPhi._fn = _make_phi_function()
        return getattr(_LazyPhi._fn, name)


PhiFunction = _LazyPhi()
