"""Oracle: the Rosenbrock-type methods and the theta-Euler scheme that the
paper compares EREM with (Sec. 3.2.1, Sec. 3.2.2, Sec. 3.2.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every linear system is solved exactly (sparse LU), so the schemes are their
definitions:

* ROSM(gamma) (Eq. ROS; with a time-dependent right-hand side Eq. ROSf):
      y+ = y + tau (I - tau gamma J)^{-1} [f(y, t) + gamma tau D_t f(y, t)].
* s-stage Rosenbrock-type methods (Eq. ROSMh): for i = 1..s
      (I / (tau gamma) - J) k_i = f(y + sum_{j<i} a_ij k_j, t + alpha_i tau)
                                  - sum_{j<i} (c_ij / tau) k_j + tau gamma_i D_t f(y, t),
      y+ = y + sum_i b_i k_i,   embedded y1 = y + sum_i bhat_i k_i,
  with J = D_y f(y, t) and the coefficients of Table ros2 (ROS2(1)) and
  Table ros3 (ROS3p) as printed.  The tables list c_ii = 1/gamma on the
  diagonal; the stage equations use only j < i.
* theta-Euler (Eq. temscheme): X = T^{n+1} solves
      F(X) = X - tau theta G(X, t+) - tau (1 - theta) G(T^n, t_n) - T^n = 0,
  by Newton's method, (I - tau theta J(X_k)) dX = -F(X_k), until the update
  is below a relative tolerance.

The schemes act on plain callables (f(y, t), its Jacobian and D_t f), so
they can be pinned on scalar and small ODEs; the heat wrappers below supply
the callables of the frozen-flux heat model.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import erem as oerem


@dataclasses.dataclass(frozen=True)
class RosTable:
    """Coefficients of an s-stage Rosenbrock-type method (Eq. ROSMh)."""
    name: str
    gamma: float
    a: tuple          # a[i][j], j < i
    c: tuple          # c[i][j], j < i
    gam: tuple        # gamma_i of the D_t f term
    alpha: tuple      # alpha_i of the stage times
    b: tuple
    bhat: tuple

    @property
    def stages(self) -> int:
        return len(self.b)


# Table ros2 (ROS2(1)), as printed.
ROS2 = RosTable(
    name="ROS2(1)",
    gamma=1.707106781186547,
    a=((), (5.857864376269050e-01,)),
    c=((), (1.171572875253810e+00,)),
    gam=(1.707106781186547, -1.707106781186547),
    alpha=(0.0, 1.0),
    b=(8.786796564403575e-01, 2.928932188134525e-01),
    bhat=(5.857864376269050e-01, 0.0),
)

# Table ros3 (ROS3p), as printed.
ROS3P = RosTable(
    name="ROS3p",
    gamma=7.886751345948129e-01,
    a=((), (1.267949192431123,), (1.267949192431123, 0.0)),
    c=((), (1.607695154586736,), (3.464101615137755, 1.732050807568877)),
    gam=(7.886751345948129e-01, -2.113248654051871e-01, -1.077350269189626),
    alpha=(0.0, 1.0, 1.0),
    b=(2.0, 5.773502691896258e-01, 4.226497308103742e-01),
    bhat=(2.113248654051871, 1.0, 4.226497308103742e-01),
)


def rosm_table(gamma: float) -> RosTable:
    """ROSM(gamma) (Eq. ROS / ROSf) as a one-stage method of Eq. ROSMh:
    (I/(tau gamma) - J) k = f + tau gamma D_t f and y+ = y + k / gamma."""
    return RosTable(name=f"ROSM({gamma:g})", gamma=gamma, a=((),), c=((),), gam=(gamma,),
                    alpha=(0.0,), b=(1.0 / gamma,), bhat=(0.0,))


def _solve(M, rhs):
    if sp.issparse(M):
        return spla.spsolve(sp.csc_matrix(M), rhs)
    return np.linalg.solve(M, rhs)


def rosenbrock_step(f, jac, dfdt, y, t, tau, table: RosTable, embedded: bool = False):
    """One step of Eq. ROSMh.  f(y, t) -> array; jac(y, t) -> matrix (dense or
    sparse); dfdt(y, t) -> array, or None for an autonomous problem.
    Returns y+ (and the embedded y1 when ``embedded``)."""
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    J = jac(y, t)
    eye = sp.identity(n, format="csr") if sp.issparse(J) else np.eye(n)
    M = eye / (tau * table.gamma) - J
    ft = dfdt(y, t) if dfdt is not None else None
    ks = []
    for i in range(table.stages):
        yi = y.copy()
        for j in range(i):
            yi = yi + table.a[i][j] * ks[j]
        rhs = np.asarray(f(yi, t + table.alpha[i] * tau), dtype=np.float64).copy()
        for j in range(i):
            rhs -= (table.c[i][j] / tau) * ks[j]
        if ft is not None:
            rhs += tau * table.gam[i] * ft
        ks.append(_solve(M, rhs))
    yn = y.copy()
    for bi, k in zip(table.b, ks):
        yn = yn + bi * k
    if not embedded:
        return yn
    y1 = y.copy()
    for bi, k in zip(table.bhat, ks):
        y1 = y1 + bi * k
    return yn, y1


def theta_euler_step(f, jac, y, t, tau, theta: float, rtol: float = 1e-13, max_newton: int = 30):
    """One step of Eq. temscheme solved by Newton's method from X_0 = y.
    Returns (X, Newton iterations)."""
    y = np.asarray(y, dtype=np.float64)
    fy = np.asarray(f(y, t), dtype=np.float64)
    if theta == 0.0:
        return y + tau * fy, 0
    X = y.copy()
    for it in range(1, max_newton + 1):
        F = X - tau * theta * np.asarray(f(X, t + tau)) - tau * (1.0 - theta) * fy - y
        J = jac(X, t + tau)
        eye = sp.identity(y.size, format="csr") if sp.issparse(J) else np.eye(y.size)
        dX = _solve(eye - tau * theta * J, -F)
        X = X + dX
        if np.abs(dX).max() <= rtol * max(np.abs(X).max(), 1e-300):
            return X, it
    raise RuntimeError("theta-Euler Newton iteration did not converge")


# --------------------------------------------------------------------------
# The frozen-flux heat model as callables
# --------------------------------------------------------------------------

class HeatODE:
    """f(T, t) = G(T, t) of the frozen-flux heat model (Sec. 3.1) with
    boundary temperatures from ``schedule(t)`` -> (T_left, T_right,
    dT_left/dt, dT_right/dt), or the problem's constant ones."""

    def __init__(self, problem, fluxes, schedule=None):
        self.prob, self.fluxes, self.schedule = problem, fluxes, schedule

    def _disc(self, T, t):
        if self.schedule is None:
            return oerem.Discretisation(self.prob, T, fluxes=self.fluxes)
        Tl, Tr, _, _ = self.schedule(t)
        return oerem.Discretisation(oerem._at_boundary(self.prob, Tl, Tr), T, fluxes=self.fluxes)

    def f(self, T, t):
        return self._disc(T, t).model.G(np.asarray(T, dtype=np.float64))

    def jac(self, T, t):
        return self._disc(T, t).model.J_sparse(np.asarray(T, dtype=np.float64))

    def dfdt(self, T, t):
        if self.schedule is None:
            return None
        _, _, dTl, dTr = self.schedule(t)
        return oerem.time_derivative(self._disc(T, t), T, dTl, dTr)


def run_rosenbrock(problem, table: RosTable, nsteps=None, h=None, fluxes=None, schedule=None,
                   t0: float = 0.0):
    """Steps of Eq. ROSMh from problem.T0 with the fluxes of the pressure at T0
    (as run_linear) unless given."""
    nsteps = problem.nsteps if nsteps is None else nsteps
    h = problem.h if h is None else h
    T = np.asarray(problem.T0, dtype=np.float64).copy()
    if fluxes is None:
        fluxes = oerem.Discretisation(problem, T).fluxes
    ode = HeatODE(problem, fluxes, schedule)
    t = t0
    for _ in range(nsteps):
        T = rosenbrock_step(ode.f, ode.jac, ode.dfdt if schedule is not None else None, T, t, h, table)
        t += h
    return T, fluxes


def run_theta_euler(problem, theta: float, nsteps=None, h=None, fluxes=None, rtol: float = 1e-13):
    """Steps of Eq. temscheme from problem.T0 (autonomous boundary data).
    Returns (T, fluxes, Newton iterations per step)."""
    nsteps = problem.nsteps if nsteps is None else nsteps
    h = problem.h if h is None else h
    T = np.asarray(problem.T0, dtype=np.float64).copy()
    if fluxes is None:
        fluxes = oerem.Discretisation(problem, T).fluxes
    ode = HeatODE(problem, fluxes)
    its = []
    for n in range(nsteps):
        T, it = theta_euler_step(ode.f, ode.jac, T, n * h, h, theta, rtol=rtol)
        its.append(it)
    return T, fluxes, its


def coupled_step_scheme(problem, T, scheme: str, h=None):
    """The sequential coupled step (Sec. 3.2.2) with a comparison scheme for
    the temperature: steady pressure at T^n, then one step of ROSM(1)
    ('rosm1'), ROSM(1/2) ('rosm05'), ROS2(1) ('ros2'), ROS3p ('ros3p') or
    theta-Euler ('theta05', 'theta1') with the fluxes frozen."""
    h = problem.h if h is None else h
    fl = oerem.Discretisation(problem, T).fluxes
    ode = HeatODE(problem, fl)
    tables = {"rosm1": rosm_table(1.0), "rosm05": rosm_table(0.5), "ros2": ROS2, "ros3p": ROS3P}
    if scheme in tables:
        return rosenbrock_step(ode.f, ode.jac, None, T, 0.0, h, tables[scheme])
    theta = {"theta05": 0.5, "theta1": 1.0}[scheme]
    return theta_euler_step(ode.f, ode.jac, T, 0.0, h, theta)[0]
