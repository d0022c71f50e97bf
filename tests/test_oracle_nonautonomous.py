"""Pins of the oracle's phi2 and of its non-autonomous EREM step
(Sec. 3.2.3, Eq. nEERMg) against facts fixed by the paper and by mathematics:
high-precision closed forms, the integral definition of phi2, the recurrence
linking phi2 to phi1, the paper's reduction of the non-autonomous step to the
autonomous one on the time-augmented system, exactness for forcing linear in
t, and second-order convergence otherwise (against an implicit Runge-Kutta
integration of the same ODE)."""
import mpmath
import numpy as np
import pytest
import scipy.linalg as sl
from scipy.integrate import solve_ivp

from oracle import erem, phi, physics as ph
from paper_1209_5553_amd import inputs


def _mp_phi2(z):
    z = mpmath.mpf(z)
    if abs(z) < mpmath.mpf("1e-8"):     # series: the closed form cancels
        return sum(z ** k / mpmath.factorial(k + 2) for k in range(12))
    return (mpmath.expm1(z) - z) / (z * z)


def test_phi2_scalar_against_high_precision():
    """phi2(z) = (e^z - 1 - z)/z^2, phi2(0) = 1/2, across the series switch."""
    mpmath.mp.dps = 60
    zs = [0.0, 1e-300, 1e-12, -1e-6, 0.3, -0.999, 0.999, 1.0, -1.0, 2.0, -30.0, -700.0, 40.0]
    got = phi.phi2_scalar(np.array(zs))
    for z, g in zip(zs, got):
        ref = float(_mp_phi2(z))
        assert g == pytest.approx(ref, rel=2e-15, abs=0.0), z


def test_action_of_zero_matrix():
    """phi1(0) = 1 and phi2(0) = 1/2: the increment is h f + h^2 g / 2."""
    rng = np.random.default_rng(0)
    f, g = rng.standard_normal(5), rng.standard_normal(5)
    h = 3.0
    got = phi.nonautonomous_action_dense(np.zeros((5, 5)), f, g, h)
    assert np.allclose(got, h * f + 0.5 * h * h * g, rtol=1e-15, atol=1e-15)
    got_b = phi.nonautonomous_action_taylor(np.zeros((5, 5)), f, g, h)
    assert np.allclose(got_b, h * f + 0.5 * h * h * g, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("m", [-3.1e-6, -4.0e-8, 2.5e-7, -7.0e-5])
def test_action_1x1_closed_form(m):
    """N = 1: h phi1(h m) f + h^2 phi2(h m) g with the scalar closed forms in
    50-digit arithmetic (h = 1e6 s as in the workloads)."""
    mpmath.mp.dps = 50
    h, f, g = 1.0e6, 2.3e-6, -4.1e-13
    z = mpmath.mpf(h) * mpmath.mpf(m)
    ref = (mpmath.mpf(h) * (mpmath.expm1(z) / z) * mpmath.mpf(f)
           + mpmath.mpf(h) ** 2 * _mp_phi2(z) * mpmath.mpf(g))
    for fn in (phi.nonautonomous_action_dense, phi.nonautonomous_action_taylor):
        got = fn(np.array([[m]]), np.array([f]), np.array([g]), h)[0]
        assert got == pytest.approx(float(ref), rel=1e-13), fn.__name__


def _random_matrix(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) * 0.6
    M -= np.diag(np.abs(M).sum(axis=1))      # spectrum in the left half plane
    M[0, 0] += 1.5                           # and one growing mode
    return M, rng.standard_normal(n), rng.standard_normal(n)


def test_action_integral_definition():
    """phi_i(Z) = int_0^1 e^{(1-s)Z} s^{i-1}/(i-1)! ds (Sec. 3.2.3): the
    increment is int_0^1 e^{(1-s) hM} (h f + s h^2 g) ds, evaluated by
    40-point Gauss-Legendre quadrature with scipy's Pade exponential."""
    M, f, g = _random_matrix(7, 1)
    h = 0.8
    x, w = np.polynomial.legendre.leggauss(40)
    s = 0.5 * (x + 1.0)
    w = 0.5 * w
    ref = np.zeros(7)
    for si, wi in zip(s, w):
        ref += wi * (sl.expm((1.0 - si) * h * M) @ (h * f + si * h * h * g))
    got = phi.nonautonomous_action_dense(M, f, g, h)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_phi2_phi1_recurrence_on_a_matrix():
    """Z phi2(Z) = phi1(Z) - I (the recurrence with phi1(0) = 1): with
    w = h^2 phi2(hM) g, M w = h phi1(hM) g - h g, the right side from the
    phi1 oracle alone."""
    M, _, g = _random_matrix(9, 2)
    h = 0.7
    w = phi.nonautonomous_action_dense(M, np.zeros(9), g, h)
    rhs = phi.hphi1_action_dense(M, g, h) - h * g
    assert np.abs(M @ w - rhs).max() <= 1e-13 * np.abs(rhs).max()


def _heat(problem, T, Tl, Tr):
    """Disc. of the problem at temperature T with boundary (Tl, Tr)."""
    q = erem._at_boundary(problem, Tl, Tr)
    return erem.Discretisation(q, T, fluxes=erem.Discretisation(problem, problem.T0).fluxes)


def test_tiers_agree_on_a_heat_operator():
    prob = inputs.linear_problem(8, seed=3)
    T = np.asarray(prob.T0, dtype=np.float64)
    d = _heat(prob, T, 61.0, 20.0)
    rng = np.random.default_rng(4)
    g = rng.standard_normal(prob.n) * 1e-12
    f = d.model.G(T)
    a = phi.nonautonomous_action_dense(d.model.J(T), f, g, prob.h)
    b = phi.nonautonomous_action_taylor(d.model.J_sparse(T), f, g, prob.h)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def _water_problem(n=6, seed=5):
    """Water laws (temperature-dependent capacity, so J carries the
    -R C'/(V C^2) diagonal) and a non-uniform temperature."""
    prob = inputs.coupled_problem(n, seed=seed)
    rng = np.random.default_rng(seed)
    prob.T0 = 20.0 + 60.0 * rng.random(prob.n)
    return prob


def test_step_is_autonomous_erem_of_the_time_augmented_system():
    """Sec. 3.2.3: with y_hat = (y, t) the system is autonomous, with
    Jacobian [[J, D_t f], [0, 0]] and right-hand side [f; 1]; the EREM step
    (Eq. EERM, the phi1 oracle) of it has the non-autonomous step as its top
    block."""
    prob = _water_problem()
    T = prob.T0
    fl = erem.Discretisation(prob, T).fluxes
    sched = inputs.InjectorSchedule()
    t = 3.3e6
    Tl, Tr, dTl, dTr = sched(t)
    got = erem.nonautonomous_step(prob, T, prob.h, Tl, Tr, dTl, dTr, fl)
    d = erem.Discretisation(erem._at_boundary(prob, Tl, Tr), T, fluxes=fl)
    N = prob.n
    J = d.model.J(T)
    Jh = np.zeros((N + 1, N + 1))
    Jh[:N, :N] = J
    Jh[:N, N] = erem.time_derivative(d, T, dTl, dTr)
    Gh = np.append(d.model.G(T), 1.0)
    ref = T + phi.hphi1_action_dense(Jh, Gh, prob.h)[:N]
    assert np.abs((got - T) - (ref - T)).max() <= 1e-12 * np.abs(ref - T).max()


@pytest.mark.parametrize("t", [0.0, 2.7e6, 1.1e7])
def test_time_derivative_is_the_derivative_of_G(t):
    """D_t G against a central difference of G(T, t) in t (the boundary
    temperatures from the schedule), on a water-law problem."""
    prob = _water_problem(seed=6)
    T = prob.T0
    fl = erem.Discretisation(prob, T).fluxes
    sched = inputs.InjectorSchedule(ramp=3e-6)

    def G(tt):
        Tl, Tr, _, _ = sched(tt)
        return erem.Discretisation(erem._at_boundary(prob, Tl, Tr), T, fluxes=fl).model.G(T)

    eps = 2.0e3
    fd = (G(t + eps) - G(t - eps)) / (2 * eps)
    Tl, Tr, dTl, dTr = sched(t)
    d = erem.Discretisation(erem._at_boundary(prob, Tl, Tr), T, fluxes=fl)
    got = erem.time_derivative(d, T, dTl, dTr)
    assert np.count_nonzero(got) > 0
    assert np.abs(got - fd).max() <= 1e-7 * np.abs(got).max()


def _reference_solution(prob, fl, sched, t0, t1, T0):
    """The ODE dT/dt = G(T, t) of the constant-capacity problem integrated by
    Radau IIA (scipy) to rtol 1e-13, with G affine in T and t."""
    Tl, Tr, _, _ = sched(t0)
    d0 = erem.Discretisation(erem._at_boundary(prob, 0.0, 0.0), T0, fluxes=fl)
    A = d0.model.A.toarray()
    VC = d0.g.volume * d0.model.capacity(T0)       # constant laws: C does not depend on T
    _, bl = ph.heat_operator(fl, d0.g, prob.lam, prob.c_f, 1.0, 0.0)
    _, br = ph.heat_operator(fl, d0.g, prob.lam, prob.c_f, 0.0, 1.0)
    J = A / VC[:, None]

    def rhs(t, T):
        Tl, Tr, _, _ = sched(t)
        return (A @ T + Tl * bl + Tr * br) / VC

    sol = solve_ivp(rhs, (t0, t1), T0, method="Radau", jac=lambda t, T: J,
                    rtol=1e-13, atol=1e-11)
    assert sol.success
    return sol.y[:, -1]


def test_forcing_linear_in_time_is_integrated_exactly():
    """For G affine in T and in t (constant laws, injection temperature a
    linear ramp) the step of Eq. nEERMg is the exact flow: three steps against
    an implicit Runge-Kutta integration to 1e-13.  Dropping the phi2 term
    (the autonomous step at frozen boundary data) misses by far more."""
    prob = inputs.linear_problem(6, seed=7)
    sched = inputs.InjectorSchedule(swing=0.0, ramp=2.0e-5, mean=30.0)
    got, fl = erem.run_nonautonomous(prob, sched, nsteps=3)
    ref = _reference_solution(prob, fl, sched, 0.0, 3 * prob.h, prob.T0)
    scale = np.abs(ref - prob.T0).max()
    err = np.abs(got - ref).max() / scale
    assert err <= 1e-9, err
    # the same steps without the phi2 term
    T = prob.T0.copy()
    t = 0.0
    for _ in range(3):
        Tl, Tr, _, _ = sched(t)
        d = erem.Discretisation(erem._at_boundary(prob, Tl, Tr), T, fluxes=fl)
        T = erem.erem_step(d.model, T, prob.h)
        t += prob.h
    assert np.abs(T - ref).max() / scale > 1e3 * max(err, 1e-12)


def test_sinusoidal_injection_converges_at_second_order():
    """Eq. nEERMg is of order two: halving h over a fixed horizon (3e6 s of
    the default 2e7 s injection period) cuts the error against the implicit
    Runge-Kutta reference by about four."""
    prob = inputs.linear_problem(6, seed=8)
    sched = inputs.InjectorSchedule()
    horizon = 3.0e6
    fl = erem.Discretisation(prob, prob.T0).fluxes
    ref = _reference_solution(prob, fl, sched, 0.0, horizon, prob.T0)
    errs = []
    for n in (8, 16, 32):
        T, _ = erem.run_nonautonomous(prob, sched, nsteps=n, h=horizon / n, fluxes=fl)
        errs.append(np.abs(T - ref).max() / np.abs(ref - prob.T0).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.4 < r1 < 4.6 and 3.4 < r2 < 4.6, errs
