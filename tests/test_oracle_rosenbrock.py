"""Pins of the oracle's Rosenbrock-type methods (Eq. ROS, Eq. ROSf, Eq. ROSMh,
Tables ros2 and ros3) and of its theta-Euler scheme (Eq. temscheme).

They rest on what the paper and the theory of these methods fix: the
stability functions the paper states (Sec. 3.2.3), L- and A-stability, the
orders of convergence (ROSM(1) and theta = 1 first order, ROSM(1/2), ROS2(1)
and theta = 1/2 second, ROS3p third, the embedded solutions one lower) on a
non-autonomous problem with a known solution and on a nonlinear autonomous
one against a high-order reference, conservation of a linear invariant, and
the Newton residual of the implicit scheme.  A mistyped table entry breaks an
order condition and fails the order pins.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import erem
from oracle import rosenbrock as ros
from paper_1209_5553_amd import inputs


def _scalar(lam):
    return (lambda y, t: lam * y), (lambda y, t: np.array([[lam]])), None


def _complex_as_real(x, y):
    """y' = (x + i y) y written as a real 2 x 2 system."""
    A = np.array([[x, -y], [y, x]])
    return (lambda v, t: A @ v), (lambda v, t: A), None


@pytest.mark.parametrize("gamma", [1.0, 0.5])
def test_rosm_stability_function(gamma):
    """R(z) = (1 + (1 - gamma) z) / (1 - gamma z) for ROSM (Sec. 3.2.3)."""
    for z in (-0.3, -5.0, -1e6, 1.5):
        f, J, _ = _scalar(z)
        got = ros.rosenbrock_step(f, J, None, np.array([1.0]), 0.0, 1.0, ros.rosm_table(gamma))[0]
        assert got == pytest.approx((1 + (1 - gamma) * z) / (1 - gamma * z), rel=1e-14)


@pytest.mark.parametrize("theta", [1.0, 0.5, 0.3])
def test_theta_euler_stability_function(theta):
    """R(z) = (1 + z (1 - theta)) / (1 - theta z) (Sec. 3.2.3)."""
    for z in (-0.3, -5.0, -1e4, 1.5):
        f, J, _ = _scalar(z)
        got, _ = ros.theta_euler_step(f, J, np.array([1.0]), 0.0, 1.0, theta)
        assert got[0] == pytest.approx((1 + z * (1 - theta)) / (1 - theta * z), rel=1e-13)


def test_ros2_is_l_stable_and_ros3p_a_stable():
    """ROS2(1) is L-stable, ROS3p A-stable (Sec. 3.2.3): |R(z)| <= 1 on the
    closed left half plane, and R(z) -> 0 for ROS2(1) as z -> -inf."""
    for table in (ros.ROS2, ros.ROS3P):
        for x in (-1e-3, -0.5, -3.0, -40.0, -1e4):
            for yv in (0.0, 0.7, 5.0, 100.0):
                f, J, _ = _complex_as_real(x, yv)
                v = ros.rosenbrock_step(f, J, None, np.array([1.0, 0.0]), 0.0, 1.0, table)
                assert np.hypot(*v) <= 1.0 + 1e-12, (table.name, x, yv)
        # the imaginary axis itself
        f, J, _ = _complex_as_real(0.0, 3.0)
        v = ros.rosenbrock_step(f, J, None, np.array([1.0, 0.0]), 0.0, 1.0, table)
        assert np.hypot(*v) <= 1.0 + 1e-12
    f, J, _ = _scalar(-1e10)
    assert abs(ros.rosenbrock_step(f, J, None, np.array([1.0]), 0.0, 1.0, ros.ROS2)[0]) < 1e-9


def _pr_problem(lam=-2.0):
    """Prothero-Robinson: y' = lam (y - sin t) + cos t, exact y = sin t;
    non-autonomous, so the alpha_i and gamma_i columns are exercised."""
    f = lambda y, t: lam * (y - np.sin(t)) + np.cos(t)
    J = lambda y, t: np.array([[lam]])
    ft = lambda y, t: np.array([-lam * np.cos(t) - np.sin(t)])
    return f, J, ft


def _pendulum():
    """Autonomous and nonlinear: y1' = y2, y2' = -sin(y1) - 0.3 y2 + 0.5 y1 y2."""
    f = lambda y, t: np.array([y[1], -np.sin(y[0]) - 0.3 * y[1] + 0.5 * y[0] * y[1]])
    J = lambda y, t: np.array([[0.0, 1.0], [-np.cos(y[0]) + 0.5 * y[1], -0.3 + 0.5 * y[0]]])
    return f, J, None


def _errors(method, prob, y0, T, ref, ns):
    f, J, ft = prob
    out = []
    for n in ns:
        y, t, h = np.array(y0, dtype=np.float64), 0.0, T / n
        for _ in range(n):
            y = method(f, J, ft, y, t, h)
            t += h
        out.append(np.abs(y - ref).max())
    return np.array(out)


METHODS = {
    "ROSM(1)": (lambda f, J, ft, y, t, h: ros.rosenbrock_step(f, J, ft, y, t, h, ros.rosm_table(1.0)), 1),
    "ROSM(1/2)": (lambda f, J, ft, y, t, h: ros.rosenbrock_step(f, J, ft, y, t, h, ros.rosm_table(0.5)), 2),
    "ROS2(1)": (lambda f, J, ft, y, t, h: ros.rosenbrock_step(f, J, ft, y, t, h, ros.ROS2), 2),
    "ROS3p": (lambda f, J, ft, y, t, h: ros.rosenbrock_step(f, J, ft, y, t, h, ros.ROS3P), 3),
    "ROS2(1) embedded": (lambda f, J, ft, y, t, h: ros.rosenbrock_step(f, J, ft, y, t, h, ros.ROS2, True)[1], 1),
    "ROS3p embedded": (lambda f, J, ft, y, t, h: ros.rosenbrock_step(f, J, ft, y, t, h, ros.ROS3P, True)[1], 2),
    "theta 1/2": (lambda f, J, ft, y, t, h: ros.theta_euler_step(f, J, y, t, h, 0.5)[0], 2),
    "theta 1": (lambda f, J, ft, y, t, h: ros.theta_euler_step(f, J, y, t, h, 1.0)[0], 1),
}


def _observed_order(errs):
    return np.log2(errs[:-1] / errs[1:])


@pytest.mark.parametrize("name", list(METHODS))
def test_order_on_prothero_robinson(name):
    method, p = METHODS[name]
    errs = _errors(method, _pr_problem(), [0.0], 1.0, np.sin(1.0), [16, 32, 64, 128])
    q = _observed_order(errs)
    assert np.all(np.abs(q[1:] - p) < 0.25), (errs, q)


@pytest.mark.parametrize("name", list(METHODS))
def test_order_on_a_nonlinear_autonomous_system(name):
    method, p = METHODS[name]
    prob = _pendulum()
    y0 = [1.0, 0.2]
    sol = solve_ivp(lambda t, y: prob[0](y, t), (0.0, 2.0), y0, method="DOP853", rtol=1e-13, atol=1e-15)
    errs = _errors(method, prob, y0, 2.0, sol.y[:, -1], [20, 40, 80, 160])
    q = _observed_order(errs)
    assert np.all(np.abs(q[1:] - p) < 0.25), (errs, q)


def _closed_problem(seed):
    rng = np.random.default_rng(seed)
    prob = inputs.linear_problem(10, seed=seed)
    prob.dirichlet_left = False
    fl = inputs.random_interior_fluxes(rng, prob.nx, prob.ny, prob.nz, scale=3e-3)
    prob.T0 = rng.uniform(20.0, 80.0, prob.n)
    return prob, fl


@pytest.mark.parametrize("table", [ros.ROS2, ros.ROS3P, ros.rosm_table(1.0)], ids=lambda t: t.name)
def test_rosenbrock_conserves_energy_with_closed_boundaries(table):
    """With closed boundaries and a constant capacity, w^T G = 0 and w^T J = 0
    for w = V C; a Rosenbrock-type step with the exact Jacobian keeps w^T T."""
    prob, fl = _closed_problem(22)
    T1, _ = ros.run_rosenbrock(prob, table, nsteps=2, fluxes=fl)
    w = prob.dx * prob.dy * prob.dz * erem.Discretisation(prob, prob.T0, fluxes=fl).model.capacity(prob.T0)
    assert abs(w @ T1 - w @ prob.T0) <= 1e-13 * abs(w @ prob.T0)
    assert np.abs(T1 - prob.T0).max() > 1e-3


def test_theta_euler_conserves_energy_and_solves_its_equation():
    """theta = 1/2 on the closed problem keeps w^T T; on a water-law problem
    (capacity depends on T, so the equation is nonlinear) the returned X
    satisfies F(X) = 0 to rounding, after a few Newton iterations."""
    prob, fl = _closed_problem(23)
    T1, _, its = ros.run_theta_euler(prob, 0.5, nsteps=2, fluxes=fl)
    w = erem.Discretisation(prob, prob.T0, fluxes=fl).model.capacity(prob.T0)
    assert abs(w @ T1 - w @ prob.T0) <= 1e-13 * abs(w @ prob.T0)
    wp = inputs.coupled_problem(8, seed=3)
    wp.T0 = 20.0 + 60.0 * np.random.default_rng(3).random(wp.n)
    fl2 = erem.Discretisation(wp, wp.T0).fluxes
    ode = ros.HeatODE(wp, fl2)
    for theta in (0.5, 1.0):
        X, it = ros.theta_euler_step(ode.f, ode.jac, wp.T0, 0.0, wp.h, theta)
        F = X - wp.h * theta * ode.f(X, wp.h) - wp.h * (1 - theta) * ode.f(wp.T0, 0.0) - wp.T0
        assert np.abs(F).max() <= 1e-11 * np.abs(X).max(), theta
        assert 2 <= it <= 8
