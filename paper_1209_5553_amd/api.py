"""Thin torch-facing binding of the EREM C ABI.

Only argument marshalling happens here: tensors are checked (FP64,
contiguous, on the context's device, right length) and their device pointers
are handed to liberem.so together with the context's HIP stream.  Every step
of the computation runs in the library's kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _native as nat


class EremError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{nat.ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def make_opts(**kw) -> nat.Opts:
    """erem_opts with the library defaults, overridden by keyword."""
    o = nat.default_opts()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def leja_points(n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    rc = nat.load().erem_leja_points(n, out.ctypes.data_as(nat._PD))
    if rc != 0:
        raise EremError(rc, "erem_leja_points")
    return out


def phi1_divided_differences(hc: float, hg: float, xi) -> np.ndarray:
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    out = np.zeros(xi.size, dtype=np.float64)
    rc = nat.load().erem_phi1_divided_differences(hc, hg, xi.ctypes.data_as(nat._PD), xi.size,
                                                  out.ctypes.data_as(nat._PD))
    if rc != 0:
        raise EremError(rc, "erem_phi1_divided_differences")
    return out


def phi2_divided_differences(hc: float, hg: float, xi) -> np.ndarray:
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    out = np.zeros(xi.size, dtype=np.float64)
    rc = nat.load().erem_phi2_divided_differences(hc, hg, xi.ctypes.data_as(nat._PD), xi.size,
                                                  out.ctypes.data_as(nat._PD))
    if rc != 0:
        raise EremError(rc, "erem_phi2_divided_differences")
    return out


class EremContext:
    """One grid's EREM state on one HIP device (see include/erem.h)."""

    def __init__(self, nx: int, ny: int, nz: int = 1, dx: float = 1.0, dy: float = 1.0,
                 dz: float = 1.0, device=None):
        self.lib = nat.load()
        if not torch.cuda.is_available():
            raise RuntimeError("EremContext needs a HIP device")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.n = self.nx * self.ny * self.nz
        self.dim = 3 if self.nz > 1 else 2
        g = nat.Grid(self.dim, self.nx, self.ny, self.nz, dx, dy, dz)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            rc = self.lib.erem_create(ctypes.byref(g), ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(h))
        if rc != 0:
            raise EremError(rc, "erem_create")
        self.handle = h
        self.ndir = 7 if self.dim == 3 else 5

    # -- helpers -----------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            self.lib.erem_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if rc != 0:
            msg = self.lib.erem_last_error(self.handle)
            raise EremError(rc, f"{what}: {msg.decode() if msg else ''}")

    def _ptr(self, t, n: int, name: str):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device:
            raise ValueError(f"{name} must be a contiguous float64 tensor on {self.device}")
        if t.numel() != n:
            raise ValueError(f"{name} must hold {n} values, got {t.numel()}")
        return ctypes.c_void_p(t.data_ptr())

    def _new(self, n: int):
        return torch.empty(n, dtype=torch.float64, device=self.device)

    @property
    def face_counts(self):
        nx, ny, nz = self.nx, self.ny, self.nz
        return nz * ny * (nx + 1), nz * (ny + 1) * nx, (nz + 1) * ny * nx

    # -- ABI -----------------------------------------------------------------
    def set_rock(self, logk, poro, lam: float, rhoc_s: float):
        self._check(self.lib.erem_set_rock(self.handle, self._ptr(logk, self.n, "logk"),
                                           self._ptr(poro, self.n, "poro"), lam, rhoc_s),
                    "erem_set_rock")

    def set_fluid(self, law: int, c_f: float, mu0: float, rho0: float):
        self._check(self.lib.erem_set_fluid(self.handle, law, c_f, mu0, rho0), "erem_set_fluid")

    def set_bc(self, p_left, p_right, T_left, T_right, dirichlet_left=True):
        self._check(self.lib.erem_set_bc(self.handle, p_left, p_right, T_left, T_right,
                                         1 if dirichlet_left else 0), "erem_set_bc")

    def assemble_transmissibilities(self, T=None):
        self._check(self.lib.erem_assemble_transmissibilities(self.handle, self._ptr(T, self.n, "T")),
                    "erem_assemble_transmissibilities")

    def solve_pressure(self, rtol=1e-16, max_iter=50000, p=None, warm=False):
        st = nat.Stats()
        self._check(self.lib.erem_solve_pressure(self.handle, rtol, max_iter, int(warm),
                                                 self._ptr(p, self.n, "p"), ctypes.byref(st)),
                    "erem_solve_pressure")
        return st.as_dict()

    def set_pressure_preconditioner(self, kind: str):
        code = {"jacobi": 0, "multigrid": 1}[kind]
        self._check(self.lib.erem_set_pressure_preconditioner(self.handle, code),
                    "erem_set_pressure_preconditioner")

    def set_face_fluxes(self, fx, fy, fz=None):
        nfx, nfy, nfz = self.face_counts
        self._check(self.lib.erem_set_face_fluxes(self.handle, self._ptr(fx, nfx, "fx"),
                                                  self._ptr(fy, nfy, "fy"),
                                                  self._ptr(fz, nfz, "fz")),
                    "erem_set_face_fluxes")

    def get_faces(self):
        nfx, nfy, nfz = self.face_counts
        out = {k: self._new(n) for k, n in
               (("fx", nfx), ("fy", nfy), ("fz", nfz), ("tx", nfx), ("ty", nfy), ("tz", nfz))}
        self._check(self.lib.erem_get_faces(self.handle, *(ctypes.c_void_p(out[k].data_ptr())
                                                           for k in ("fx", "fy", "fz", "tx", "ty", "tz"))),
                    "erem_get_faces")
        return out

    def form_jacobian(self, T):
        self._check(self.lib.erem_form_jacobian(self.handle, self._ptr(T, self.n, "T")),
                    "erem_form_jacobian")

    def get_jacobian(self):
        coef = self._new(self.ndir * self.n)
        F = self._new(self.n)
        self._check(self.lib.erem_get_jacobian(self.handle, ctypes.c_void_p(coef.data_ptr()),
                                               ctypes.c_void_p(F.data_ptr())), "erem_get_jacobian")
        return coef.view(self.ndir, self.n), F

    def set_jacobian(self, coef, F):
        self._check(self.lib.erem_set_jacobian(self.handle, self._ptr(coef, self.ndir * self.n, "coef"),
                                               self._ptr(F, self.n, "F")), "erem_set_jacobian")

    def step_frozen(self, h: float, T, opts: nat.Opts | None = None):
        o = opts if opts is not None else make_opts()
        st = nat.Stats()
        self._check(self.lib.erem_step_frozen(self.handle, h, self._ptr(T, self.n, "T"), ctypes.byref(o),
                                              ctypes.byref(st)), "erem_step_frozen")
        return st.as_dict()

    def phi1_apply(self, h: float, v, out=None, opts: nat.Opts | None = None):
        out = self._new(self.n) if out is None else out
        o = opts if opts is not None else make_opts()
        st = nat.Stats()
        self._check(self.lib.erem_phi1_apply(self.handle, h, self._ptr(v, self.n, "v"),
                                             self._ptr(out, self.n, "out"), ctypes.byref(o),
                                             ctypes.byref(st)), "erem_phi1_apply")
        return out, st.as_dict()

    def step(self, h: float, T, opts: nat.Opts | None = None):
        o = opts if opts is not None else make_opts()
        st = nat.Stats()
        self._check(self.lib.erem_step(self.handle, h, self._ptr(T, self.n, "T"), ctypes.byref(o),
                                       ctypes.byref(st)), "erem_step")
        return st.as_dict()

    def step_nonautonomous(self, h: float, T, T_left: float, T_right: float, dT_left_dt: float,
                           dT_right_dt: float, opts: nat.Opts | None = None):
        """One non-autonomous EREM step in place on T
        (erem_step_nonautonomous): boundary temperatures at t_n and their
        rates; the context keeps T_left and T_right afterwards."""
        o = opts if opts is not None else make_opts()
        st = nat.Stats()
        self._check(self.lib.erem_step_nonautonomous(
            self.handle, h, T_left, T_right, dT_left_dt, dT_right_dt, self._ptr(T, self.n, "T"),
            ctypes.byref(o), ctypes.byref(st)), "erem_step_nonautonomous")
        return st.as_dict()

    def face_fluxes_from_pressure(self, p):
        """Face fluxes of the given pressure (erem_face_fluxes_from_pressure)."""
        self._check(self.lib.erem_face_fluxes_from_pressure(self.handle, self._ptr(p, self.n, "p")),
                    "erem_face_fluxes_from_pressure")

    def step_pressure(self, h: float, p, T, alpha_b: float, beta_f: float, opts: nat.Opts | None = None):
        """EREM step of the transient pressure in place on p
        (erem_step_pressure) at the temperature T (T^n)."""
        o = opts if opts is not None else make_opts()
        st = nat.Stats()
        self._check(self.lib.erem_step_pressure(self.handle, h, self._ptr(p, self.n, "p"), self._ptr(T, self.n, "T"),
                                                alpha_b, beta_f, ctypes.byref(o), ctypes.byref(st)),
                    "erem_step_pressure")
        return st.as_dict()

    ROS_SCHEMES = {"rosm1": 0, "rosm05": 1, "ros2": 2, "ros3p": 3}

    def shifted_solve(self, sigma: float, b, x, rtol: float = 1e-13, max_iter: int = 10000):
        """x = (sigma I - J)^{-1} b for the context's J (erem_shifted_solve)."""
        st = nat.Stats()
        self._check(self.lib.erem_shifted_solve(self.handle, sigma, self._ptr(b, self.n, "b"),
                                                self._ptr(x, self.n, "x"), rtol, max_iter, ctypes.byref(st)),
                    "erem_shifted_solve")
        return st.as_dict()

    def step_rosenbrock(self, h: float, T, scheme: str = "ros2", lin_rtol: float = 1e-13):
        """One Rosenbrock-type step in place (erem_step_rosenbrock); scheme
        one of rosm1, rosm05, ros2, ros3p."""
        st = nat.Stats()
        self._check(self.lib.erem_step_rosenbrock(self.handle, h, self.ROS_SCHEMES[scheme],
                                                  self._ptr(T, self.n, "T"), lin_rtol, ctypes.byref(st)),
                    "erem_step_rosenbrock")
        return st.as_dict()

    ROS_ALPHA = {"rosm1": (0.0,), "rosm05": (0.0,), "ros2": (0.0, 1.0), "ros3p": (0.0, 1.0, 1.0)}

    def step_rosenbrock_nonautonomous(self, h: float, T, scheme: str, T_left_stage, T_right_stage,
                                      dT_left_dt: float, dT_right_dt: float, lin_rtol: float = 1e-13):
        """Non-autonomous Rosenbrock-type step in place
        (erem_step_rosenbrock_nonautonomous): boundary temperatures at the
        stage times t_n + ROS_ALPHA[scheme][i] h and their rates at t_n."""
        n = len(self.ROS_ALPHA[scheme])
        tl = np.ascontiguousarray(T_left_stage, dtype=np.float64)
        tr = np.ascontiguousarray(T_right_stage, dtype=np.float64)
        if tl.size != n or tr.size != n:
            raise ValueError(f"{scheme} takes {n} stage values")
        st = nat.Stats()
        self._check(self.lib.erem_step_rosenbrock_nonautonomous(
            self.handle, h, self.ROS_SCHEMES[scheme], tl.ctypes.data_as(nat._PD), tr.ctypes.data_as(nat._PD),
            dT_left_dt, dT_right_dt, self._ptr(T, self.n, "T"), lin_rtol, ctypes.byref(st)),
            "erem_step_rosenbrock_nonautonomous")
        return st.as_dict()

    def step_theta(self, h: float, T, theta: float = 0.5, newton_rtol: float = 1e-13,
                   lin_rtol: float = 1e-13, max_newton: int = 30):
        """One theta-Euler step with Newton's method in place (erem_step_theta)."""
        st = nat.Stats()
        self._check(self.lib.erem_step_theta(self.handle, h, theta, self._ptr(T, self.n, "T"), newton_rtol,
                                             lin_rtol, max_newton, ctypes.byref(st)), "erem_step_theta")
        return st.as_dict()

    def coupled_step(self, h: float, T, p_rtol: float = 1e-16, opts: nat.Opts | None = None,
                     tape: nat.Tape | None = None, record: bool = True):
        """One sequential coupled step in place on T (erem_coupled_step).
        Returns (stats, tape): the tape of the choices used, replayed when
        ``tape`` is given."""
        o = opts if opts is not None else make_opts()
        st = nat.Stats()
        out = nat.Tape() if record else None
        self._check(self.lib.erem_coupled_step(
            self.handle, h, self._ptr(T, self.n, "T"), p_rtol, ctypes.byref(o),
            ctypes.byref(tape) if tape is not None else None,
            ctypes.byref(out) if out is not None else None, ctypes.byref(st)), "erem_coupled_step")
        return st.as_dict(), out

    def coupled_step_adjoint(self, h: float, T, tape: nat.Tape, Tbar, logk_bar, p_rtol: float = 1e-16,
                             opts: nat.Opts | None = None, ckpt_stride: int = 1):
        """Adjoint of one coupled step at T (erem_coupled_step_adjoint):
        Tbar (in: d/dT^{n+1}, out: d/dT^n) in place, logk_bar accumulated."""
        o = opts if opts is not None else make_opts()
        st = nat.Stats()
        self._check(self.lib.erem_coupled_step_adjoint(
            self.handle, h, self._ptr(T, self.n, "T"), p_rtol, ctypes.byref(o), ctypes.byref(tape),
            int(ckpt_stride), self._ptr(Tbar, self.n, "Tbar"), self._ptr(logk_bar, self.n, "logk_bar"),
            ctypes.byref(st)), "erem_coupled_step_adjoint")
        return st.as_dict()

    def profile(self, enable: bool = True, stride: int = 1):
        """Per-launch event timing on (one launch in ``stride``) or off."""
        self._check(self.lib.erem_profile(self.handle, int(stride) if enable else 0), "erem_profile")

    def profile_read(self):
        kt = nat.KernelTimes()
        self._check(self.lib.erem_profile_read(self.handle, ctypes.byref(kt)), "erem_profile_read")
        return kt.as_dict()

    # -- convenience -----------------------------------------------------------
    @classmethod
    def from_problem(cls, prob, device=None):
        """Context loaded with a paper_1209_5553_amd.inputs.Problem (rock,
        fluid, boundary conditions); fluxes are not computed yet."""
        ctx = cls(prob.nx, prob.ny, prob.nz, prob.dx, prob.dy, prob.dz, device=device)
        dev = ctx.device
        ctx._logk = torch.as_tensor(prob.logk, dtype=torch.float64, device=dev).contiguous()
        ctx._poro = torch.as_tensor(prob.poro, dtype=torch.float64, device=dev).contiguous()
        ctx.set_rock(ctx._logk, ctx._poro, prob.lam, prob.rhoc_s)
        ctx.lam, ctx.rhoc_s = prob.lam, prob.rhoc_s
        ctx.set_fluid(prob.law, prob.c_f, prob.mu0, prob.rho0)
        ctx.set_bc(prob.p_left, prob.p_right, prob.T_left, prob.T_right,
                   getattr(prob, "dirichlet_left", True))
        return ctx

    def pressure_and_fluxes(self, T=None, rtol=1e-16, p=None, warm=False, max_iter=50000):
        """Transmissibilities at T, steady pressure and face fluxes."""
        self.assemble_transmissibilities(T)
        return self.solve_pressure(rtol=rtol, max_iter=max_iter, p=p, warm=warm)


class EremBatch:
    """Many independent linear problems advanced in one persistent launch
    (see the erem_batch_* functions of include/erem.h).

    ``problems`` are paper_1209_5553_amd.inputs.Problem records with a
    constant fluid law.  Temperatures are one packed FP64 tensor; use
    :meth:`pack` / :meth:`unpack` to convert from / to per-problem arrays.
    The batch owns a non-default HIP stream so that its launch can be
    captured in a hipGraph.
    """

    def __init__(self, problems, device=None):
        self.lib = nat.load()
        if not torch.cuda.is_available():
            raise RuntimeError("EremBatch needs a HIP device")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.problems = list(problems)
        n = len(self.problems)
        grids = (nat.Grid * n)(*[nat.Grid(2, p.nx, p.ny, 1, p.dx, p.dy, p.dz) for p in self.problems])
        self.stream = torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        rc = self.lib.erem_batch_create(n, grids, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise EremError(rc, "erem_batch_create")
        self.handle = h
        off = (ctypes.c_int64 * (n + 1))()
        self._check(self.lib.erem_batch_offsets(self.handle, off), "erem_batch_offsets")
        self.offsets = [int(v) for v in off]
        self.ntot = self.offsets[-1]
        keep = []
        for i, p in enumerate(self.problems):
            if p.law != nat.LAW_CONSTANT:
                raise ValueError("the batched form needs a constant fluid law (linear problems)")
            logk = torch.as_tensor(p.logk, dtype=torch.float64, device=self.device).contiguous()
            poro = torch.as_tensor(p.poro, dtype=torch.float64, device=self.device).contiguous()
            T0 = torch.as_tensor(p.T0, dtype=torch.float64, device=self.device).contiguous()
            keep.append((logk, poro, T0))
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            self._check(self.lib.erem_batch_set_problem(
                self.handle, i, ctypes.c_void_p(logk.data_ptr()), ctypes.c_void_p(poro.data_ptr()),
                p.lam, p.rhoc_s, p.c_f, p.mu0, p.rho0, p.p_left, p.p_right, p.T_left, p.T_right,
                ctypes.c_void_p(T0.data_ptr())), f"erem_batch_set_problem({i})")
        del keep

    def _check(self, rc, what):
        if rc != 0:
            msg = self.lib.erem_batch_last_error(self.handle)
            raise EremError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "handle", None):
            self.lib.erem_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def pack(self, arrays):
        flat = np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in arrays])
        assert flat.size == self.ntot
        return torch.as_tensor(flat, dtype=torch.float64, device=self.device).clone()

    def unpack(self, T):
        host = T.detach().cpu().numpy()
        return [host[self.offsets[i]:self.offsets[i + 1]] for i in range(len(self.problems))]

    def _ptr(self, T):
        if T.dtype != torch.float64 or not T.is_contiguous() or T.device != self.device or T.numel() != self.ntot:
            raise ValueError(f"T must be a contiguous float64 tensor of {self.ntot} values on {self.device}")
        return ctypes.c_void_p(T.data_ptr())

    def prepare(self, h: float, opts: nat.Opts | None = None):
        o = opts if opts is not None else make_opts(m_max=128)
        self._check(self.lib.erem_batch_prepare(self.handle, h, ctypes.byref(o)), "erem_batch_prepare")

    def autotune(self, T, nsteps: int = 1) -> int:
        ch = ctypes.c_int32(-1)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(self.lib.erem_batch_autotune(self.handle, self._ptr(T), nsteps, ctypes.byref(ch)),
                    "erem_batch_autotune")
        return ch.value

    def set_tile_shape(self, shape: int):
        self._check(self.lib.erem_batch_set_tile_shape(self.handle, int(shape)), "erem_batch_set_tile_shape")

    def profile(self, stride: int):
        """Time every stride-th work launch of later runs (0: off)."""
        self._check(self.lib.erem_batch_profile(self.handle, int(stride)), "erem_batch_profile")

    def run(self, T, nsteps: int, use_graph: bool = True):
        st = nat.BatchStats()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(self.lib.erem_batch_run(self.handle, self._ptr(T), nsteps, 1 if use_graph else 0,
                                            ctypes.byref(st)), "erem_batch_run")
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return st.as_dict()
