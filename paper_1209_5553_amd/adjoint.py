"""Differentiable sequential coupled EREM run (torch.autograd.Function).

The forward pass takes ``nsteps`` coupled steps (steady pressure, then the
EREM temperature step of Eq. EERM, Sec. 3.2.2) through the C ABI, keeping
every T^n (one FP64 vector per step) and the tape of every step (its
Gershgorin interval, substep count and Newton-Leja degrees).  The backward
pass walks the steps in reverse and calls erem_coupled_step_adjoint, which
recomputes the step from T^n with the taped choices, runs the Newton-Leja
recurrence backwards with the transposed stencil of J over the stored (or
segment-wise recomputed) iterates, and chains through the heat operator,
the face fluxes, the pressure system and the TPFA mobility to d/dT^n and
d/dlog K.  Only argument marshalling happens here.
"""
from __future__ import annotations

import torch

from .api import EremContext, make_opts


class CoupledRun(torch.autograd.Function):
    """T^N = run(T0, log K) for a context set up with
    :meth:`EremContext.from_problem`; differentiable in T0 and log K."""

    @staticmethod
    def forward(fctx, T0, logk, ectx: EremContext, h: float, nsteps: int, opts, p_rtol: float,
                ckpt_stride: int, tapes_in):
        ectx.set_rock(logk.detach().contiguous(), ectx._poro, ectx.lam, ectx.rhoc_s)
        T = T0.detach().clone().contiguous()
        states, tapes = [], []
        for n in range(nsteps):
            states.append(T.clone())
            _, tape = ectx.coupled_step(h, T, p_rtol=p_rtol, opts=opts,
                                        tape=None if tapes_in is None else tapes_in[n])
            tapes.append(tape)
        fctx.ectx, fctx.h, fctx.opts, fctx.p_rtol = ectx, h, opts, p_rtol
        fctx.ckpt_stride, fctx.tapes = ckpt_stride, tapes
        fctx.logk = logk.detach().clone().contiguous()
        fctx.save_for_backward(*states)
        fctx.last_tapes = tapes
        return T

    @staticmethod
    def backward(fctx, gT):
        ectx = fctx.ectx
        states = fctx.saved_tensors
        ectx.set_rock(fctx.logk, ectx._poro, ectx.lam, ectx.rhoc_s)
        Tbar = gT.detach().to(torch.float64).contiguous().clone()
        kbar = torch.zeros_like(Tbar)
        for n in range(len(states) - 1, -1, -1):
            ectx.coupled_step_adjoint(fctx.h, states[n], fctx.tapes[n], Tbar, kbar, p_rtol=fctx.p_rtol,
                                      opts=fctx.opts, ckpt_stride=fctx.ckpt_stride)
        return Tbar, kbar, None, None, None, None, None, None, None


def coupled_run(ectx: EremContext, T0, logk, h: float, nsteps: int, opts=None, p_rtol: float = 1e-16,
                ckpt_stride: int = 1, tapes=None):
    """Differentiable T^N.  ``tapes`` (one per step) replays recorded
    choices, e.g. for finite differences with the discrete choices frozen."""
    o = opts if opts is not None else make_opts()
    return CoupledRun.apply(T0, logk, ectx, h, nsteps, o, p_rtol, ckpt_stride, tapes)


def run_with_tapes(ectx: EremContext, T0, logk, h: float, nsteps: int, opts=None, p_rtol: float = 1e-16,
                   tapes=None):
    """Forward only: (T^N, tapes).  With ``tapes`` the steps replay them."""
    o = opts if opts is not None else make_opts()
    ectx.set_rock(logk.contiguous(), ectx._poro, ectx.lam, ectx.rhoc_s)
    T = T0.clone().contiguous()
    out = []
    for n in range(nsteps):
        _, tape = ectx.coupled_step(h, T, p_rtol=p_rtol, opts=o, tape=None if tapes is None else tapes[n])
        out.append(tape)
    return T, out
