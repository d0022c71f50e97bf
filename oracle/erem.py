"""Oracle: the exponential Rosenbrock-Euler step and the sequential coupled step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

EREM (Eq. EERM):  T^{n+1} = T^n + h phi1(h J_n) G(T^n),  J_n = D_T G(T^n).

For a linear autonomous problem (constant capacity, frozen fluxes) G(T) =
J T + g with constant J and g, the linearised ODE is the ODE itself and EREM
reproduces the exact flow (Eq. exactnu with constant forcing; stability
function R(z) = e^z, Sec. 3.2.3): T(t) = T0 + t phi1(t J) G(T0).

The coupled step follows the sequential (Trotter) approach of Sec. 3.2.2:
first the pressure with the fluid properties at T^n (here the steady,
incompressible pressure equation), then one EREM temperature step with the
resulting face fluxes frozen.
"""
from __future__ import annotations

import copy

import numpy as np

from . import physics as ph
from . import phi as phimod


class Discretisation:
    """All space-discrete objects of one problem at a given temperature.

    ``problem`` is any object with the attributes nx, ny, nz, dx, dy, dz,
    logk, poro, law, lam, rhoc_s, c_f, mu0, rho0, p_left, p_right, T_left,
    T_right (a plain record; no behaviour is used).
    """

    def __init__(self, problem, T, fluxes=None, layered=False):
        self.prob = problem
        self.g = ph.grid_of(problem)
        T = np.asarray(T, dtype=np.float64)
        if fluxes is None and layered:
            mob = ph.mobility(T, problem.logk, problem.law, problem.rho0, problem.mu0)
            self.trans = ph.tpfa_transmissibilities(mob, self.g)
            self.p = None
            fluxes = ph.layered_x_fluxes(mob, self.g, problem.p_left, problem.p_right)
        elif fluxes is None:
            mob = ph.mobility(T, problem.logk, problem.law, problem.rho0, problem.mu0)
            self.trans = ph.tpfa_transmissibilities(mob, self.g)
            self.p = ph.solve_pressure(self.trans, self.g, problem.p_left, problem.p_right)
            fluxes = ph.face_fluxes(self.p, self.trans, self.g,
                                    problem.p_left, problem.p_right)
        else:
            self.trans = None
            self.p = None
        self.fluxes = fluxes
        A, b = ph.heat_operator(fluxes, self.g, problem.lam, problem.c_f,
                                problem.T_left, problem.T_right,
                                getattr(problem, "dirichlet_left", True))
        self.model = ph.HeatModel(A, b, self.g, problem.poro, problem.law,
                                  problem.rho0, problem.c_f, problem.rhoc_s)


def erem_increment(model: ph.HeatModel, T, h, tier: str = "dense"):
    """h phi1(h J(T)) G(T) by the dense (tier A) or sparse (tier B) action."""
    G = model.G(T)
    if tier == "dense":
        return phimod.hphi1_action_dense(model.J(T), G, h)
    return phimod.hphi1_action_taylor(model.J_sparse(T), G, h)


def erem_step(model: ph.HeatModel, T, h, tier: str = "dense"):
    """One EREM step (Eq. EERM) for the frozen-flux heat model."""
    T = np.asarray(T, dtype=np.float64)
    return T + erem_increment(model, T, h, tier)


def run_linear(problem, nsteps=None, h=None, tier: str = "dense", fluxes=None,
               layered=False):
    """EREM steps of a problem whose fluxes and capacity do not depend on T
    (pressure solved once at the initial temperature)."""
    nsteps = problem.nsteps if nsteps is None else nsteps
    h = problem.h if h is None else h
    T = np.asarray(problem.T0, dtype=np.float64).copy()
    disc = Discretisation(problem, T, fluxes=fluxes, layered=layered)
    for _ in range(nsteps):
        T = erem_step(disc.model, T, h, tier)
    return T, disc


def coupled_step(problem, T, h=None, tier: str = "dense"):
    """Sequential step: steady pressure with rho(T^n), mu(T^n), then EREM."""
    h = problem.h if h is None else h
    disc = Discretisation(problem, T)
    return erem_step(disc.model, T, h, tier), disc


def run_coupled(problem, nsteps=None, h=None, tier: str = "dense"):
    nsteps = problem.nsteps if nsteps is None else nsteps
    T = np.asarray(problem.T0, dtype=np.float64).copy()
    for _ in range(nsteps):
        T, _ = coupled_step(problem, T, h, tier)
    return T


# --------------------------------------------------------------------------
# Non-autonomous EREM (Sec. 3.2.3, Eq. nEERMg)
# --------------------------------------------------------------------------

def _at_boundary(problem, T_left, T_right):
    """A copy of the problem record with the boundary temperatures replaced."""
    q = copy.copy(problem)
    q.T_left = float(T_left)
    q.T_right = float(T_right)
    return q


def time_derivative(disc: Discretisation, T, dT_left, dT_right):
    """D_t G(T, t) when the boundary temperatures move at the rates dT_left,
    dT_right.  R(T, t) = A T + b(t) and b is linear and homogeneous in
    (T_left, T_right) (Sec. 3.1 boundary fluxes), so D_t b is the boundary
    vector assembled with the rates in place of the temperatures, and
    D_t G = D_t b / (V C(T)) (the capacity does not depend on t)."""
    prob = disc.prob
    _, bt = ph.heat_operator(disc.fluxes, disc.g, prob.lam, prob.c_f, dT_left, dT_right,
                             getattr(prob, "dirichlet_left", True))
    return bt / (disc.g.volume * disc.model.capacity(np.asarray(T, dtype=np.float64)))


def nonautonomous_step(problem, T, h, T_left, T_right, dT_left, dT_right, fluxes,
                       tier: str = "dense"):
    """One step of Eq. nEERMg for the frozen-flux heat model whose boundary
    temperatures at t_n are (T_left, T_right), moving at (dT_left, dT_right):

        T^{n+1} = T^n + h phi1(h J) G(T^n, t_n) + h^2 phi2(h J) D_t G(T^n, t_n),
        J = D_T G(T^n, t_n).
    """
    T = np.asarray(T, dtype=np.float64)
    disc = Discretisation(_at_boundary(problem, T_left, T_right), T, fluxes=fluxes)
    model = disc.model
    G = model.G(T)
    Gt = time_derivative(disc, T, dT_left, dT_right)
    if tier == "dense":
        inc = phimod.nonautonomous_action_dense(model.J(T), G, Gt, h)
    else:
        inc = phimod.nonautonomous_action_taylor(model.J_sparse(T), G, Gt, h)
    return T + inc


def run_nonautonomous(problem, schedule, nsteps=None, h=None, t0: float = 0.0,
                      tier: str = "dense", fluxes=None):
    """Steps of Eq. nEERMg from problem.T0 at t0; ``schedule(t)`` returns
    (T_left, T_right, dT_left/dt, dT_right/dt) at time t.  The face fluxes are
    those of the pressure solved once at T0 (as in run_linear) unless given."""
    nsteps = problem.nsteps if nsteps is None else nsteps
    h = problem.h if h is None else h
    T = np.asarray(problem.T0, dtype=np.float64).copy()
    if fluxes is None:
        fluxes = Discretisation(problem, T).fluxes
    t = t0
    for _ in range(nsteps):
        Tl, Tr, dTl, dTr = schedule(t)
        T = nonautonomous_step(problem, T, h, Tl, Tr, dTl, dTr, fluxes, tier)
        t += h
    return T, fluxes
