"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test pins one part of the oracle to something other than itself: a hand
worked example (tests/golden), a closed form, an invariant, a library routine
the case reduces to, or brute force on a tiny input.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import erem, phi, physics as ph
from paper_1209_5553_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- phi1 scalar

def test_phi1_scalar_against_high_precision():
    """phi1(z) = (e^z - 1)/z (Sec. 3.2.2) against 50-digit mpmath."""
    mpmath.mp.dps = 50
    zs = [0.0, 1e-300, 1e-12, -1e-8, 1e-3, -0.5, 2.0, -30.0, -700.0, 40.0]
    got = phi.phi1_scalar(np.array(zs))
    for z, g in zip(zs, got):
        if z == 0.0:
            ref = mpmath.mpf(1)
        else:
            zz = mpmath.mpf(z)
            ref = mpmath.expm1(zz) / zz
        assert abs(g - float(ref)) <= 4e-16 * abs(float(ref)), (z, g, ref)


def test_phi_recurrence_integral_definition():
    """phi1(z) = int_0^1 e^{(1-s) z} ds (Sec. 3.2.3 integral form), quadrature."""
    mpmath.mp.dps = 30
    for z in (-40.0, -3.0, -0.1, 0.7):
        ref = mpmath.quad(lambda s: mpmath.exp((1 - s) * z), [0, 1])
        assert abs(phi.phi1_scalar(np.array([z]))[0] - float(ref)) < 1e-15 * abs(float(ref)) + 1e-300


# ------------------------------------------------------------- dense exp, phi1

@pytest.mark.parametrize("seed,scale", [(0, 0.3), (1, 5.0), (2, 80.0)])
def test_expm_taylor_matches_scipy(seed, scale):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((30, 30)) * scale / 6.0
    A -= np.diag(np.abs(A).sum(axis=1))          # stable, like a transport Jacobian
    E = phi.expm_taylor(A)
    R = sl.expm(A)
    assert np.abs(E - R).max() <= 1e-12 * max(1.0, np.abs(R).max())


def test_expm_taylor_nonnormal_jordan_block():
    """exp(lam I + N) = e^lam sum N^k/k! exactly for a nilpotent shift N."""
    n, lam = 8, -3.0
    J = lam * np.eye(n) + np.diag(np.ones(n - 1), -1) * 5.0
    E = phi.expm_taylor(J)
    ref = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1):
            k = i - j
            ref[i, j] = math.exp(lam) * 5.0 ** k / math.factorial(k)
    assert np.abs(E - ref).max() <= 1e-13 * np.abs(ref).max()


def test_phi1_matrix_diagonal_closed_form():
    lam = np.array([-250.0, -7.5, -1.0, -1e-9, 0.0, 0.3])
    M = np.diag(lam)
    P = phi.phi1_matrix(M)
    ref = np.diag(phi.phi1_scalar(lam))
    assert np.abs(P - ref).max() <= 1e-13 * np.abs(ref).max()   # ~9 squarings of eps-level error


def test_phi1_matrix_nilpotent_series():
    """phi1(N) = sum_k N^k/(k+1)! for nilpotent N (definition as a series)."""
    n = 6
    N = np.diag(np.full(n - 1, 2.0), 1)
    ref = np.zeros((n, n))
    Nk = np.eye(n)
    for k in range(n):
        ref += Nk / math.factorial(k + 1)
        Nk = Nk @ N
    assert np.abs(phi.phi1_matrix(N) - ref).max() <= 1e-14 * np.abs(ref).max()


def test_phi1_action_diagonal_closed_form():
    """h phi1(h J) v = (e^{h lam} - 1)/lam v for diagonal J (closed form)."""
    rng = np.random.default_rng(3)
    lam = -np.geomspace(1e-9, 3e-4, 40)
    v = rng.standard_normal(40)
    h = 1e6
    got = phi.hphi1_action_dense(np.diag(lam), v, h)
    ref = np.expm1(h * lam) / lam * v
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    gotB = phi.hphi1_action_taylor(sp.diags(lam), v, h)
    assert np.abs(gotB - ref).max() <= 1e-13 * np.abs(ref).max()


def test_phi1_of_zero_is_identity():
    """phi1(0) = I: with J = 0 the EREM increment is exactly h v."""
    v = np.linspace(-3, 7, 17)
    h = 2.5e5
    assert np.array_equal(phi.hphi1_action_dense(np.zeros((17, 17)), v, h), h * v)
    assert np.allclose(phi.hphi1_action_taylor(sp.csr_matrix((17, 17)), v, h), h * v,
                       rtol=0, atol=1e-15 * h * 7)


# ----------------------------------------------------------------- TPFA, Darcy

def test_tpfa_two_cells_hand_example():
    gd = _golden("tpfa_2cells.json")
    g = ph.Grid(2, 1)
    tr = ph.tpfa_transmissibilities(np.array(gd["k"]), g)
    assert np.allclose(tr["tx"].ravel(), gd["tx"], rtol=1e-15)
    assert tr["t_left"].item() == pytest.approx(gd["t_left"], rel=1e-15)
    assert tr["t_right"].item() == pytest.approx(gd["t_right"], rel=1e-15)
    p = ph.solve_pressure(tr, g, 1.0, 0.0)
    assert np.allclose(p, gd["p"], rtol=1e-14)
    fx, fy, fz = ph.face_fluxes(p, tr, g, 1.0, 0.0)
    assert np.allclose(fx.ravel(), gd["flux"], rtol=1e-14)


def test_strip_flux_is_the_series_closed_form():
    """One row of cells is a chain of resistances 1/tau in series between the
    two Dirichlet faces: every face carries (p_left - p_right) / sum(1/tau).
    A long strip with a strong permeability contrast is ill-conditioned for
    the pressure, so this pins the flux accuracy of the pressure solve."""
    g = ph.Grid(700, 1)
    rng = np.random.default_rng(11)
    k = np.exp(2.0 * rng.standard_normal(g.n))
    tr = ph.tpfa_transmissibilities(k, g)
    p_left, p_right = 6.0e4, 0.0
    p = ph.solve_pressure(tr, g, p_left, p_right)
    fx, _, _ = ph.face_fluxes(p, tr, g, p_left, p_right)
    res = (1.0 / np.asarray(tr["t_left"], dtype=np.longdouble).ravel()).sum() \
        + (1.0 / np.asarray(tr["tx"], dtype=np.longdouble).ravel()).sum() \
        + (1.0 / np.asarray(tr["t_right"], dtype=np.longdouble).ravel()).sum()
    q = float((p_left - p_right) / res)
    # the strip's condition number (~1e10) bounds the flux accuracy of a
    # solve at ~1e-11; a dropped or misplaced boundary term costs O(1)
    assert np.abs(fx.ravel() - q).max() <= 1e-10 * abs(q)
    # the refined residual is at the extended-precision floor
    A, rhs = ph.pressure_matrix(tr, g, p_left, p_right)
    A = A.tocsr()
    rows = np.repeat(np.arange(g.n), np.diff(A.indptr))
    Ap = np.zeros(g.n, dtype=np.longdouble)
    np.add.at(Ap, rows, A.data.astype(np.longdouble) * p[A.indices])
    scale = (np.abs(A).astype(np.longdouble) @ np.abs(p)).max()
    assert np.abs(rhs - Ap).max() <= 64 * np.finfo(np.longdouble).eps * scale


def test_layered_pressure_is_linear_and_fluxes_analytic():
    """Mobility depending on z only: each layer carries k A dp/(nx dx) and
    the TPFA pressure is linear in x (no transverse flow)."""
    g = ph.Grid(6, 5, 4)
    rng = np.random.default_rng(7)
    layers = 10.0 ** rng.uniform(-2, 1, g.nz)
    k = np.broadcast_to(layers[:, None, None], g.shape).ravel()
    tr = ph.tpfa_transmissibilities(k, g)
    p = ph.solve_pressure(tr, g, 3.0, 1.0)
    x = np.arange(g.nx)
    lin = 3.0 - 2.0 * (x + 0.5) / g.nx
    assert np.abs(p.reshape(g.shape) - lin[None, None, :]).max() < 1e-13
    f_direct = ph.face_fluxes(p, tr, g, 3.0, 1.0)
    f_anal = ph.layered_x_fluxes(k, g, 3.0, 1.0)
    for a, b in zip(f_direct, f_anal):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(f_anal[0]).max()


def test_pressure_fluxes_are_divergence_free():
    prob = inputs.linear_problem(16, seed=4)
    d = erem.Discretisation(prob, prob.T0)
    fx, fy, fz = d.fluxes
    div = (fx[:, :, 1:] - fx[:, :, :-1]) + (fy[:, 1:, :] - fy[:, :-1, :])
    assert np.abs(div).max() <= 1e-12 * np.abs(fx).max()
    assert fx[:, :, 0].min() > 0 and fx[:, :, -1].min() > 0   # left-to-right flow


def test_water_laws_against_handbook():
    """Law 1 reproduces tabulated water properties within ~1 % (viscosity
    1.002e-3 Pa s at 20 C, 3.54e-4 at 80 C; density 1000 at 20 C)."""
    assert ph.viscosity(20.0, 1) == pytest.approx(1.002e-3, rel=0.01)
    assert ph.viscosity(80.0, 1) == pytest.approx(3.54e-4, rel=0.015)
    assert ph.density(20.0, 1) == pytest.approx(1000.0, rel=1e-15)
    assert ph.density(80.0, 1) < ph.density(20.0, 1)


# ----------------------------------------------------------- heat operator, J

def test_heat_operator_three_cells_hand_example():
    gd = _golden("heat_operator_3cells.json")
    g = ph.Grid(3, 1)
    fx = np.full((1, 1, 4), 2.0)
    fy = np.zeros((1, 2, 3))
    fz = np.zeros((2, 1, 3))
    A, b = ph.heat_operator((fx, fy, fz), g, lam=1.0, c_f=1.0, T_left=10.0, T_right=99.0)
    assert np.array_equal(A.toarray(), np.array(gd["A"]))
    assert np.array_equal(b, np.array(gd["b"]))


def test_heat_operator_conserves_energy_with_closed_boundaries():
    """Any interior face fluxes, no boundary flux: column sums of A vanish, so
    w^T G(T) = 0 for w = V C (total energy is an invariant)."""
    rng = np.random.default_rng(11)
    g = ph.Grid(7, 5, 3)
    fl = inputs.random_interior_fluxes(rng, g.nx, g.ny, g.nz)
    A, b = ph.heat_operator(fl, g, lam=2.5, c_f=4200.0, T_left=80.0, T_right=20.0,
                            dirichlet_left=False)
    colsum = np.asarray(A.sum(axis=0)).ravel()
    assert np.abs(colsum).max() <= 1e-12 * abs(A).max()
    assert np.all(b == 0.0)
    off = A - sp.diags(A.diagonal())
    assert off.min() >= 0.0                  # upwind: nonnegative couplings


def test_solenoidal_flux_generator_is_divergence_free():
    fx, fy, fz = inputs.random_solenoidal_fluxes(np.random.default_rng(3), 9, 7)
    div = (fx[:, :, 1:] - fx[:, :, :-1]) + (fy[:, 1:, :] - fy[:, :-1, :])
    assert np.abs(div).max() <= 1e-15
    assert np.all(fx[:, :, 0] == 0) and np.all(fx[:, :, -1] == 0)
    assert np.all(fy[:, 0, :] == 0) and np.all(fy[:, -1, :] == 0)
    g = ph.Grid(9, 7)
    A, b = ph.heat_operator((fx, fy, fz), g, 2.5, 4200.0, 80.0, 20.0, dirichlet_left=False)
    rowsum = np.asarray(A.sum(axis=1)).ravel()
    assert np.abs(rowsum).max() <= 1e-12 * abs(A).max()   # and so beta <= 0 up to rounding


@pytest.mark.parametrize("cell", [(1.0, 1.0, 1.0), (2.0, 0.5, 3.0)])
def test_jacobian_matches_central_differences(cell):
    """J = D_T G (Eq. linear), including the temperature-dependent capacity,
    on unit and on non-unit cells (cell volume != 1)."""
    import dataclasses
    prob = dataclasses.replace(inputs.coupled_problem(8, seed=2), dx=cell[0], dy=cell[1], dz=cell[2])
    T = np.random.default_rng(5).uniform(20.0, 80.0, prob.n)
    d = erem.Discretisation(prob, T)
    J = d.model.J(T)
    eps = 1e-4
    Jfd = np.zeros_like(J)
    for j in range(prob.n):
        e = np.zeros(prob.n)
        e[j] = eps
        Jfd[:, j] = (d.model.G(T + e) - d.model.G(T - e)) / (2 * eps)
    assert np.abs(J - Jfd).max() <= 1e-7 * np.abs(J).max()


def test_gershgorin_interval_contains_spectrum():
    rng = np.random.default_rng(8)
    for _ in range(5):
        M = rng.standard_normal((12, 12))
        a, b = ph.gershgorin_interval(M)
        ev = np.linalg.eigvals(M)
        assert a - 1e-12 <= ev.real.min() and ev.real.max() <= b + 1e-12
    lam = np.array([-4.0, -1.0, 0.5])
    assert ph.gershgorin_interval(np.diag(lam)) == (-4.0, 0.5)
    prob = inputs.linear_problem(8)
    d = erem.Discretisation(prob, prob.T0)
    Js = d.model.J_sparse(prob.T0)
    a1, b1 = ph.gershgorin_interval(Js)
    a2, b2 = ph.gershgorin_interval(Js.toarray())
    assert a1 == pytest.approx(a2, rel=1e-14) and abs(b1 - b2) <= 1e-14 * abs(a2)


# ------------------------------------------------------------------ EREM step

def test_tier_b_matches_expm_multiply_and_tier_a():
    prob = inputs.linear_problem(16, seed=1)
    d = erem.Discretisation(prob, prob.T0)
    Js = d.model.J_sparse(prob.T0)
    G = d.model.G(prob.T0)
    h = prob.h
    N = prob.n
    aug = sp.bmat([[h * Js, sp.csr_matrix(h * G[:, None])],
                   [sp.csr_matrix((1, N)), sp.csr_matrix((1, 1))]]).tocsr()
    e = np.zeros(N + 1)
    e[-1] = 1.0
    ref = spla.expm_multiply(aug, e)[:N]
    b = phi.hphi1_action_taylor(Js, G, h)
    a = phi.hphi1_action_dense(Js.toarray(), G, h)
    scale = np.abs(ref).max()
    assert np.abs(b - ref).max() <= 1e-12 * scale
    assert np.abs(a - ref).max() <= 1e-12 * scale


def test_erem_exact_for_linear_problems():
    """EREM is exact in time for a linear autonomous problem (Eq. exactnu,
    R(z) = e^z): ten steps of h equal one step of 10 h."""
    prob = inputs.linear_problem(12, seed=2)
    T10, d = erem.run_linear(prob, nsteps=10)
    T1 = erem.erem_step(d.model, prob.T0, 10 * prob.h)
    assert np.abs(T10 - T1).max() <= 1e-12 * np.abs(T1).max()


def test_erem_scalar_problem_exact():
    """y' = lam y + g: one EREM step reproduces the exact solution."""
    lam, g0, y0, h = -3e-6, 2e-5, 20.0, 7e5
    T = erem.erem_step(_ScalarModel(lam, g0), np.array([y0]), h)
    exact = -g0 / lam + (y0 + g0 / lam) * math.exp(lam * h)
    assert T[0] == pytest.approx(exact, rel=1e-14)


class _ScalarModel:
    def __init__(self, lam, g):
        self.lam, self.g = lam, g

    def G(self, T):
        return self.lam * T + self.g

    def J(self, T):
        return np.array([[self.lam]])


def test_erem_steady_limit_is_injection_temperature():
    """h -> infinity: T + h phi1(hJ) G -> -J^{-1} g, the steady state; with
    the only heat source at T_left it is T_left in every cell."""
    prob = inputs.linear_problem(8, seed=3)
    d = erem.Discretisation(prob, prob.T0)
    T = erem.erem_step(d.model, prob.T0, 1e12)
    assert np.abs(T - prob.T_left).max() <= 1e-9 * prob.T_left


def test_erem_conserves_energy_with_closed_boundaries():
    rng = np.random.default_rng(21)
    prob = inputs.linear_problem(10, seed=5)
    prob.dirichlet_left = False
    fl = inputs.random_interior_fluxes(rng, prob.nx, prob.ny, prob.nz, scale=3e-3)
    T0 = rng.uniform(20.0, 80.0, prob.n)
    d = erem.Discretisation(prob, T0, fluxes=fl)
    T1 = erem.erem_step(d.model, T0, prob.h)
    w = d.g.volume * d.model.capacity(T0)
    assert abs(w @ T1 - w @ T0) <= 1e-14 * abs(w @ T0)
    assert np.abs(T1 - T0).max() > 1e-3          # something did move


def test_coupled_step_runs_and_heats_from_the_left():
    prob = inputs.coupled_problem(16, seed=0)
    T1, d = erem.coupled_step(prob, prob.T0)
    assert T1.min() >= prob.T0.min() - 1e-9
    assert T1.max() <= prob.T_left + 1e-9
    Tg = T1.reshape(prob.shape)
    assert Tg[0, :, 0].mean() > Tg[0, :, -1].mean()
