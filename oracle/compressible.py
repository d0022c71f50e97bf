"""Oracle: the compressible pressure ODE and its EREM step (Sec. 2 Eq.
masscon4, Sec. 3.2.2 Eq. spaceheat3 and Eq. EERM1), and the sequential step
that advances temperature and pressure one after the other.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The mass balance of a slightly compressible fluid in a slightly compressible
rock, per cell of the TPFA discretisation (Sec. 3.1), is

    V rho S dp/dt = -(A p - b) + V rho phi alpha_f dT/dt,
    S = phi beta_f + phi_0 alpha_b,    alpha_f = -rho'(T) / rho,

with A p = b the steady TPFA pressure system (mobility rho K / mu at T,
Dirichlet x faces), so

    dp/dt = G4(T, p) = G3(p) + (phi alpha_f / S) G2,   G3 = (b - A p) / (V rho S),

G2 = dT/dt the right-hand side of the energy equation (Eq. spaceheat3).
Readings (the paper's state tables are not given): phi = phi_0 in S and in
the expansivity term (phi_0 alpha_b (p - p_0) is at most a few per mille
here), rho = rho(T) of the workload's law (no pressure dependence in the
flux term), beta_f and alpha_b constants.  The EREM step of the pressure
(Eq. EERM1) is p + h phi1(h J_p) G4 with J_p = D_p G4; the sequential
scheme (Sec. 3.2.2) evaluates G2 at (T^n, p^n) and keeps it fixed in p, so
J_p = -diag(1/(V rho S)) A.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import erem as oerem
from . import phi as phimod
from . import physics as ph


def alpha_f(T, law):
    """Thermal expansivity -rho'(T) / rho(T) of the fluid law [1/K]."""
    return -ph.density_dT(T, law) / ph.density(T, law)


def storage(poro, alpha_b, beta_f):
    """S = phi beta_f + phi_0 alpha_b with phi = phi_0 (reading above)."""
    return np.asarray(poro, dtype=np.float64) * (beta_f + alpha_b)


def pressure_rhs(problem, T, p, G2, alpha_b, beta_f):
    """(G4, J_p) at (T, p): the right-hand side of Eq. spaceheat3 and its
    p-Jacobian with G2 held fixed (sparse)."""
    g = ph.grid_of(problem)
    T = np.asarray(T, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    mob = ph.mobility(T, problem.logk, problem.law, problem.rho0, problem.mu0)
    trans = ph.tpfa_transmissibilities(mob, g)
    A, b = ph.pressure_matrix(trans, g, problem.p_left, problem.p_right)
    S = storage(problem.poro, alpha_b, beta_f)
    D = g.volume * ph.density(T, problem.law, problem.rho0) * S
    G3 = (b - A @ p) / D
    G4 = G3 + np.asarray(problem.poro) * alpha_f(T, problem.law) / S * np.asarray(G2, dtype=np.float64)
    Jp = (-sp.diags(1.0 / D) @ A).tocsr()
    return G4, Jp


def pressure_step(problem, T, p, G2, h, alpha_b, beta_f, tier: str = "dense"):
    """p^{n+1} = p^n + h phi1(h J_p) G4(T^n, p^n) (Eq. EERM1)."""
    G4, Jp = pressure_rhs(problem, T, p, G2, alpha_b, beta_f)
    if tier == "dense":
        inc = phimod.hphi1_action_dense(Jp.toarray(), G4, h)
    else:
        inc = phimod.hphi1_action_taylor(Jp, G4, h)
    return np.asarray(p, dtype=np.float64) + inc


def sequential_step(problem, T, p, h, alpha_b, beta_f, tier: str = "dense"):
    """One step of the sequential scheme (Sec. 3.2.2) with a transient
    pressure: the face fluxes of p^n with the mobility at T^n, the EREM
    temperature step (Eq. EERM) with them, then the EREM pressure step
    (Eq. EERM1) with G2 = G(T^n, p^n).  Returns (T^{n+1}, p^{n+1})."""
    g = ph.grid_of(problem)
    T = np.asarray(T, dtype=np.float64)
    mob = ph.mobility(T, problem.logk, problem.law, problem.rho0, problem.mu0)
    trans = ph.tpfa_transmissibilities(mob, g)
    fluxes = ph.face_fluxes(np.asarray(p, dtype=np.float64), trans, g, problem.p_left, problem.p_right)
    disc = oerem.Discretisation(problem, T, fluxes=fluxes)
    G2 = disc.model.G(T)
    T1 = oerem.erem_step(disc.model, T, h, tier)
    p1 = pressure_step(problem, T, p, G2, h, alpha_b, beta_f, tier)
    return T1, p1


def steady_pressure(problem, T):
    """The steady pressure at T (the initial pressure of the workload)."""
    g = ph.grid_of(problem)
    mob = ph.mobility(np.asarray(T, dtype=np.float64), problem.logk, problem.law, problem.rho0, problem.mu0)
    trans = ph.tpfa_transmissibilities(mob, g)
    return np.asarray(ph.solve_pressure(trans, g, problem.p_left, problem.p_right), dtype=np.float64)


def run_sequential(problem, nsteps, h, alpha_b, beta_f, p0=None, tier: str = "dense"):
    """nsteps sequential steps from (T0, p0), p0 the steady pressure at T0
    unless given."""
    T = np.asarray(problem.T0, dtype=np.float64).copy()
    p = steady_pressure(problem, T) if p0 is None else np.asarray(p0, dtype=np.float64).copy()
    for _ in range(nsteps):
        T, p = sequential_step(problem, T, p, h, alpha_b, beta_f, tier)
    return T, p
