"""Pins of the oracle's compressible pressure ODE and its EREM step
(Sec. 2 Eq. masscon4, Sec. 3.2.2 Eq. spaceheat3, Eq. EERM1): the expansivity
against a difference quotient of the density law, the steady pressure as a
fixed point, mass balance of G3 against the boundary fluxes, the exact flow
of the affine pressure ODE by the eigen-decomposition of its symmetrised
operator, and the agreement of the dense and sparse tiers."""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import compressible as oc
from oracle import physics as ph
from paper_1209_5553_amd import inputs

AB, BF = inputs.ALPHA_B, inputs.BETA_F


def test_expansivity_is_minus_dlogrho_dT():
    T = np.linspace(10.0, 90.0, 9)
    eps = 1e-3
    fd = -(ph.density(T + eps, 1) - ph.density(T - eps, 1)) / (2 * eps) / ph.density(T, 1)
    assert np.allclose(oc.alpha_f(T, 1), fd, rtol=1e-9)
    assert np.all(oc.alpha_f(T, 0) == 0.0)


def test_steady_pressure_is_a_fixed_point():
    """Constant law (alpha_f = 0) and the steady pressure: G4 = 0 and the
    EREM step leaves p unchanged."""
    prob = inputs.compressible_problem(6, seed=1)
    prob.law = 0
    p = oc.steady_pressure(prob, prob.T0)
    G2 = np.random.default_rng(0).standard_normal(prob.n)
    G4, _ = oc.pressure_rhs(prob, prob.T0, p, G2, AB, BF)
    scale = prob.p_left / (prob.h)
    assert np.abs(G4).max() <= 1e-9 * scale
    p1 = oc.pressure_step(prob, prob.T0, p, G2, prob.h, AB, BF)
    assert np.abs(p1 - p).max() <= 1e-9 * prob.p_left


def test_g3_balances_the_boundary_fluxes():
    """sum_i V rho S G3_i = inflow through x = 0 - outflow through x = nx
    (interior fluxes cancel), for any p."""
    prob = inputs.compressible_problem(6, seed=2)
    rng = np.random.default_rng(1)
    p = rng.uniform(0.0, 1e6, prob.n)
    g = ph.grid_of(prob)
    G4, _ = oc.pressure_rhs(prob, prob.T0, p, np.zeros(prob.n), AB, BF)
    D = g.volume * ph.density(prob.T0, prob.law) * oc.storage(prob.poro, AB, BF)
    mob = ph.mobility(prob.T0, prob.logk, prob.law, prob.rho0, prob.mu0)
    fx, _, _ = ph.face_fluxes(p, ph.tpfa_transmissibilities(mob, g), g, prob.p_left, prob.p_right)
    net = fx[:, :, 0].sum() - fx[:, :, -1].sum()
    assert (D * G4).sum() == pytest.approx(net, rel=1e-10)


def test_pressure_step_is_the_exact_flow_of_the_affine_ode():
    """With T and G2 fixed the pressure ODE is affine, p' = -D^{-1}(A p - b) + s,
    and EREM is its exact flow; the reference is p* + D^{-1/2} V e^{h L} V^T
    D^{1/2} (p0 - p*) with D^{-1/2} A D^{-1/2} = -V L V^T (eigh) and
    A p* = b + D s."""
    prob = inputs.compressible_problem(5, seed=3)
    g = ph.grid_of(prob)
    rng = np.random.default_rng(4)
    T = prob.T0 + rng.uniform(-5.0, 5.0, prob.n)
    G2 = rng.standard_normal(prob.n) * 1e-6
    p0 = rng.uniform(0.0, 1e6, prob.n)
    h = 50 * prob.h
    got = oc.pressure_step(prob, T, p0, G2, h, AB, BF)
    mob = ph.mobility(T, prob.logk, prob.law, prob.rho0, prob.mu0)
    A, b = ph.pressure_matrix(ph.tpfa_transmissibilities(mob, g), g, prob.p_left, prob.p_right)
    A = A.toarray()
    S = oc.storage(prob.poro, AB, BF)
    D = g.volume * ph.density(T, prob.law) * S
    s = prob.poro * oc.alpha_f(T, prob.law) / S * G2
    pstar = np.linalg.solve(A, b + D * s)
    Dh = np.sqrt(D)
    lam, V = sl.eigh(A / Dh[:, None] / Dh[None, :])
    q0 = Dh * (p0 - pstar)
    ref = pstar + (V @ (np.exp(-h * lam) * (V.T @ q0))) / Dh
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref - p0).max()
    assert h * lam.max() > 10.0          # a stiff case: the step is far from linear


def test_tiers_agree_and_sequential_step_runs():
    prob = inputs.compressible_problem(6, seed=5)
    p0 = oc.steady_pressure(prob, prob.T0)
    G2 = np.random.default_rng(6).standard_normal(prob.n) * 1e-6
    a = oc.pressure_step(prob, prob.T0, p0, G2, prob.h, AB, BF, tier="dense")
    b = oc.pressure_step(prob, prob.T0, p0, G2, prob.h, AB, BF, tier="taylor")
    assert np.abs(a - b).max() <= 1e-11 * np.abs(a - p0).max()
    T1, p1 = oc.sequential_step(prob, prob.T0, p0, prob.h, AB, BF)
    assert np.all(np.isfinite(T1)) and np.all(np.isfinite(p1))
    assert T1.reshape(prob.shape)[:, :, 0].mean() < prob.T0.reshape(prob.shape)[:, :, 0].mean()  # cooled by injection
