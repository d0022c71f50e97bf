"""Seeded synthetic inputs for the EREM heat-transport workloads.

This module only draws random fields and fixes workload parameters; it holds
none of the method's arithmetic (no transmissibilities, no Jacobian, no phi1).
Both the CPU oracle (through the tests) and the HIP path consume exactly the
arrays produced here.

Cell ordering everywhere: flat index = x + nx * (y + ny * z), i.e. numpy
shape (nz, ny, nx) in C order.  Units are SI, temperatures in degrees C.

Recipes (the paper's own reservoirs, Sec. 5, are not reproducible: grids, well
models and state-law tables are not given; these synthetic fields stand in):

* log-normal permeability: i.i.d. N(0,1) on the cell grid, Gaussian-smoothed
  with standard deviation ``corr`` cells (reflecting boundary, truncated at
  4 sigma), re-standardised to mean 0 and standard deviation ``sigma_logk``,
  exponentiated and scaled so that the arithmetic mean of K is ``mean_k``.
* layered permeability (3D): one N(0,1) draw per z-layer, affinely mapped so
  that log10 K spans exactly ``decades`` decades, then scaled to mean ``mean_k``.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy import ndimage

# Physical parameters shared by every workload (unit cells, thickness 1 m).
POROSITY = 0.2            # [-]
LAMBDA_EFF = 2.5          # bulk thermal conductivity [W/m/K]
RHOC_ROCK = 2.4e6         # rock volumetric heat capacity [J/m^3/K]
C_FLUID = 4200.0          # fluid specific heat [J/kg/K]; rho0*c_f = 4.2e6 J/m^3/K
RHO0 = 1000.0             # reference fluid density [kg/m^3]
MU0 = 1.0e-3              # constant viscosity of the linear workloads [Pa s]
T_INITIAL = 20.0          # [C]
T_INJECT = 80.0           # left-edge injection temperature [C]
STEP_H = 1.0e6            # EREM time step [s]
# Pressure drop of the coupled workloads: Peclet number
# (rho c)_f * mean(K) * dp / (mu(20 C) * lambda) = 100 with mean(K) = 1e-12 m^2
# and mu(20 C) ~ 1.0055e-3 Pa s gives dp ~ 5.99e4 Pa; 6.0e4 is used.
DP_COUPLED = 6.0e4        # [Pa]
DP_LINEAR = 1.0e6         # [Pa]

LAW_CONSTANT = 0          # rho = RHO0, mu = MU0
LAW_WATER = 1             # rho(T) = 1000 (1 - 3e-4 (T - 20)), mu(T) = 2.414e-5 * 10**(247.8 / (T + 133))

C3_SIDES = (64, 96, 128, 192, 256)


@dataclasses.dataclass
class Problem:
    """One heat-transport problem on a Cartesian grid of unit cells."""
    name: str
    nx: int
    ny: int
    nz: int
    logk: np.ndarray          # natural log of permeability [m^2], flat, float64
    poro: np.ndarray          # porosity per cell, flat, float64
    T0: np.ndarray            # initial temperature per cell, flat, float64
    law: int = LAW_CONSTANT
    lam: float = LAMBDA_EFF
    rhoc_s: float = RHOC_ROCK
    c_f: float = C_FLUID
    mu0: float = MU0
    rho0: float = RHO0
    p_left: float = DP_LINEAR
    p_right: float = 0.0
    T_left: float = T_INJECT
    T_right: float = T_INITIAL
    dirichlet_left: bool = True   # False: adiabatic x = 0 face (closed-system tests)
    h: float = STEP_H
    nsteps: int = 10
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0

    @property
    def dim(self) -> int:
        return 3 if self.nz > 1 else 2

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


def lognormal_field(rng: np.random.Generator, shape, sigma_logk: float,
                    corr: float, mean_k: float = 1e-12) -> np.ndarray:
    """Natural-log permeability of a smoothed log-normal field (flat)."""
    z = rng.standard_normal(shape)
    z = ndimage.gaussian_filter(z, sigma=corr, mode="reflect", truncate=4.0)
    z = (z - z.mean()) / z.std() * sigma_logk
    k = np.exp(z)
    k *= mean_k / k.mean()
    return np.log(k).ravel().astype(np.float64)


def layered_field(rng: np.random.Generator, nx: int, ny: int, nz: int,
                  decades: float = 3.0, mean_k: float = 1e-12) -> np.ndarray:
    """Natural-log permeability constant per z-layer spanning ``decades``."""
    zl = rng.standard_normal(nz)
    log10k = (zl - zl.min()) / (zl.max() - zl.min()) * decades
    k_layer = 10.0 ** log10k
    k = np.broadcast_to(k_layer[:, None, None], (nz, ny, nx)).astype(np.float64)
    k = k * (mean_k / k.mean())
    return np.log(k).ravel().copy()


def _uniform(n: int, value: float) -> np.ndarray:
    return np.full(n, value, dtype=np.float64)


def linear_problem(n: int = 32, seed: int = 0, sigma_logk: float = 1.0,
                   corr: float = 4.0, nsteps: int = 10,
                   name: str | None = None) -> Problem:
    """2D n x n heat transport with a fixed Darcy field (constant viscosity).

    With n = 32 this is the 32x32 FP64 workload (10 steps of 1e6 s).
    """
    rng = np.random.default_rng(seed)
    logk = lognormal_field(rng, (n, n), sigma_logk, corr)
    N = n * n
    return Problem(name=name or f"linear2d_{n}", nx=n, ny=n, nz=1, logk=logk,
                   poro=_uniform(N, POROSITY), T0=_uniform(N, T_INITIAL),
                   law=LAW_CONSTANT, p_left=DP_LINEAR, nsteps=nsteps)


def coupled_problem(n: int = 512, seed: int = 0, nsteps: int = 100,
                    name: str | None = None) -> Problem:
    """2D n x n sequential pressure/temperature problem with water laws.

    n = 512 is the coupled workload (100 steps); n = 256 with 20 steps is the
    adjoint workload.  sigma_logK = 2, correlation width 16 cells.
    """
    rng = np.random.default_rng(seed)
    logk = lognormal_field(rng, (n, n), 2.0, 16.0)
    N = n * n
    return Problem(name=name or f"coupled2d_{n}", nx=n, ny=n, nz=1, logk=logk,
                   poro=_uniform(N, POROSITY), T0=_uniform(N, T_INITIAL),
                   law=LAW_WATER, p_left=DP_COUPLED, nsteps=nsteps)


def adjoint_problem(n: int = 256, seed: int = 0, nsteps: int = 20, structured_T0: bool = True,
                    name: str | None = None) -> Problem:
    """The adjoint workload: the coupled problem of side n (water laws,
    sigma_logK = 2, corr 16), 20 steps.

    With the uniform 20 C start the injected heat penetrates only a few
    metres in 20 steps of 1e6 s (thermal front speed ~3.5e-10 m/s at the
    workload's Peclet number, conduction length ~4 m), so the producer-block
    temperature and all its sensitivities are exactly those of a uniform
    state.  ``structured_T0`` gives the start a smooth temperature structure
    instead: T0 = 20 + 60 * (1 + tanh z) / 2 with z a smoothed N(0, 1) field
    (Gaussian, 8 cells, re-standardised; drawn after the permeability from
    the same generator), so that the objective depends on T0 near the
    producer and, through the pressure field and the advection of that
    structure, on log K everywhere."""
    rng = np.random.default_rng(seed)
    logk = lognormal_field(rng, (n, n), 2.0, 16.0)
    N = n * n
    if structured_T0:
        z = rng.standard_normal((n, n))
        z = ndimage.gaussian_filter(z, sigma=8.0, mode="reflect", truncate=4.0)
        z = (z - z.mean()) / z.std()
        T0 = (T_INITIAL + 60.0 * 0.5 * (1.0 + np.tanh(z))).ravel().astype(np.float64)
    else:
        T0 = _uniform(N, T_INITIAL)
    return Problem(name=name or f"adjoint2d_{n}", nx=n, ny=n, nz=1, logk=logk,
                   poro=_uniform(N, POROSITY), T0=T0, law=LAW_WATER, p_left=DP_COUPLED,
                   nsteps=nsteps)


def injector_problem(n: int = 512, seed: int = 0, nsteps: int = 20,
                     name: str | None = None) -> Problem:
    """2D n x n heat transport with a fixed Darcy field and a time-varying
    injection temperature (the non-autonomous workload): the permeability of
    the coupled workload (sigma_logK = 2, correlation 16 cells, same seed),
    constant fluid laws, the coupled pressure drop (Peclet ~ 100); the
    injection temperature follows InjectorSchedule()."""
    rng = np.random.default_rng(seed)
    logk = lognormal_field(rng, (n, n), 2.0, 16.0)
    N = n * n
    return Problem(name=name or f"injector2d_{n}", nx=n, ny=n, nz=1, logk=logk,
                   poro=_uniform(N, POROSITY), T0=_uniform(N, T_INITIAL),
                   law=LAW_CONSTANT, p_left=DP_COUPLED, nsteps=nsteps)


# Compressible (transient-pressure) workload: the paper's bulk rock
# compressibility (Sec. 5, first experiment) and the compressibility of water.
ALPHA_B = 1.0e-7          # [1/Pa]
BETA_F = 4.5e-10          # [1/Pa]
DARCY = 9.869233e-13      # [m^2]


def compressible_problem(n: int = 50, seed: int = 0, nsteps: int = 20,
                         name: str | None = None) -> Problem:
    """3D n^3 sequential problem with a transient pressure (compressible rock
    and fluid), standing in for the paper's first reservoir (Sec. 5):
    1 km x 1 km x 0.1 km (cells 1000/n x 1000/n x 100/n m), two layers - the
    upper half (z index >= n/2) K = 0.01 D, phi = 0.2, the lower half
    K = 0.1 D, phi = 0.4 - each with a log-normal perturbation (sigma 0.5,
    correlation 2 cells) of its permeability; water laws; T0 = 60 C at z = 0
    rising 3 C per 10 m; injection at 10 C through x = 0 with p_left = 1 MPa,
    p_right = 0 (Dirichlet faces stand in for the wells); h = 2e4 s.  The
    initial pressure is linear_pressure(): linear in x between the boundary
    values, so the first steps relax it toward the steady pressure of the
    heterogeneous field."""
    rng = np.random.default_rng(seed)
    dx, dz = 1000.0 / n, 100.0 / n
    pert = lognormal_field(rng, (n, n, n), 0.5, 2.0, mean_k=1.0).reshape(n, n, n)
    zc = np.arange(n)
    upper = (zc >= n // 2)[:, None, None]
    k = np.where(upper, 0.01 * DARCY, 0.1 * DARCY) * np.exp(pert)
    poro = np.where(upper, 0.2, 0.4) * np.ones((n, n, n))
    zm = (zc + 0.5) * dz
    T0 = np.broadcast_to((60.0 + 0.3 * zm)[:, None, None], (n, n, n))
    return Problem(name=name or f"compressible3d_{n}", nx=n, ny=n, nz=n,
                   logk=np.log(k).ravel().astype(np.float64), poro=poro.ravel().astype(np.float64),
                   T0=T0.ravel().astype(np.float64).copy(), law=LAW_WATER, p_left=1.0e6,
                   T_left=10.0, T_right=60.0, h=2.0e4, nsteps=nsteps, dx=dx, dy=dx, dz=dz)


def linear_pressure(problem: Problem) -> np.ndarray:
    """Initial pressure of the compressible workload: p_left + (p_right -
    p_left) (x + 1/2) / nx at cell centres (flat, float64)."""
    xs = (np.arange(problem.nx) + 0.5) / problem.nx
    row = problem.p_left + (problem.p_right - problem.p_left) * xs
    return np.broadcast_to(row, (problem.nz, problem.ny, problem.nx)).ravel().astype(np.float64).copy()


@dataclasses.dataclass(frozen=True)
class InjectorSchedule:
    """Boundary temperatures at time t for the non-autonomous problems and
    their exact time derivatives: the injected temperature
    T_left(t) = mean + swing sin(2 pi t / period) + ramp t (20 C to 80 C over
    a period of 20 steps by default), T_right constant.  Calling it returns
    (T_left, T_right, dT_left/dt, dT_right/dt)."""
    mean: float = 50.0
    swing: float = 30.0
    period: float = 20 * STEP_H
    ramp: float = 0.0
    T_right: float = T_INITIAL

    def __call__(self, t: float):
        w = 2.0 * np.pi / self.period
        Tl = self.mean + self.swing * np.sin(w * t) + self.ramp * t
        dTl = self.swing * w * np.cos(w * t) + self.ramp
        return float(Tl), float(self.T_right), float(dTl), 0.0


def producer_ring(nx: int, ny: int, block: int = 4, ring: int = 2):
    """Flat indices of the producer block and ``ring`` cells around it
    (inside the grid), for checks of d/dT0 where it is not negligible."""
    ys = np.arange(max(0, ny // 2 - block // 2 - ring), min(ny, ny // 2 + block // 2 + ring))
    xs = np.arange(max(0, nx - block - ring), nx)
    return (xs[None, :] + nx * ys[:, None]).ravel()


def layered3d_problem(n: int = 128, seed: int = 0, nsteps: int = 10,
                      name: str | None = None) -> Problem:
    """3D n^3 7-point heat transport, layered permeability (3 decades)."""
    rng = np.random.default_rng(seed)
    logk = layered_field(rng, n, n, n)
    N = n ** 3
    return Problem(name=name or f"layered3d_{n}", nx=n, ny=n, nz=n, logk=logk,
                   poro=_uniform(N, POROSITY), T0=_uniform(N, T_INITIAL),
                   law=LAW_CONSTANT, p_left=DP_LINEAR, nsteps=nsteps)


def batch_problem(seed: int, nsteps: int = 50, sides=C3_SIDES) -> Problem:
    """One realisation of the ragged batch: side drawn first, then the field."""
    rng = np.random.default_rng(seed)
    n = int(rng.choice(np.asarray(sides)))
    logk = lognormal_field(rng, (n, n), 1.0, 4.0)
    N = n * n
    return Problem(name=f"batch_{seed}_{n}", nx=n, ny=n, nz=1, logk=logk,
                   poro=_uniform(N, POROSITY), T0=_uniform(N, T_INITIAL),
                   law=LAW_CONSTANT, p_left=DP_LINEAR, nsteps=nsteps)


def producer_cells(nx: int, ny: int, block: int = 4):
    """Flat indices of the block x block producer cells at the right edge,
    centred vertically (x in [nx-block, nx-1], y in [ny/2-block/2, ny/2+block/2-1])."""
    ys = np.arange(ny // 2 - block // 2, ny // 2 + block // 2)
    xs = np.arange(nx - block, nx)
    return (xs[None, :] + nx * ys[:, None]).ravel()


def fd_cells(N: int, count: int = 50, seed: int = 1) -> np.ndarray:
    return np.random.default_rng(seed).choice(N, count, replace=False)


def random_solenoidal_fluxes(rng: np.random.Generator, nx: int, ny: int, scale: float = 1e-2):
    """Divergence-free 2D mass fluxes with no boundary flux, from a random
    stream function psi on the (nx+1) x (ny+1) grid nodes that vanishes on
    the boundary: F_x = psi(x, y+1) - psi(x, y), F_y = psi(x, y) - psi(x+1, y)."""
    psi = np.zeros((ny + 1, nx + 1))
    psi[1:-1, 1:-1] = rng.standard_normal((ny - 1, nx - 1)) * scale
    fx = (psi[1:, :] - psi[:-1, :])[None, :, :]            # (1, ny, nx+1)
    fy = (psi[:, :-1] - psi[:, 1:])[None, :, :]            # (1, ny+1, nx)
    fz = np.zeros((2, ny, nx))
    return fx, fy, fz


def random_interior_fluxes(rng: np.random.Generator, nx: int, ny: int, nz: int,
                           scale: float = 1e-3):
    """Arbitrary mass fluxes [kg/s] on interior faces, zero on every boundary
    face (positive along +x, +y, +z).  Shapes: fx (nz, ny, nx+1),
    fy (nz, ny+1, nx), fz (nz+1, ny, nx)."""
    fx = np.zeros((nz, ny, nx + 1))
    fy = np.zeros((nz, ny + 1, nx))
    fz = np.zeros((nz + 1, ny, nx))
    fx[:, :, 1:-1] = rng.standard_normal((nz, ny, nx - 1)) * scale
    fy[:, 1:-1, :] = rng.standard_normal((nz, ny - 1, nx)) * scale
    if nz > 1:
        fz[1:-1, :, :] = rng.standard_normal((nz - 1, ny, nx)) * scale
    return fx, fy, fz
