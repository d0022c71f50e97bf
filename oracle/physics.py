"""Oracle: finite-volume (TPFA + upwind) discretisation of the heat/flow model.

TEST INFRASTRUCTURE ONLY (see the package docstring): plain FP64 numpy/scipy,
written from the paper, sharing no code with the HIP path.

What is modelled (paper Sec. 2 and Sec. 3.1, local-equilibrium limit he -> inf,
so that T_s = T_f = T, no gravity, no heat sources):

    C(T) dT/dt = div(lambda grad T) - div(c_f rho v T)        (energy)
    div(rho K / mu grad p) = 0,  rho v = -(rho K / mu) grad p  (steady mass balance)

with C(T) = phi rho(T) c_f + (1 - phi) (rho c)_s.  Space discretisation: cell
centred control volumes on a Cartesian grid; two-point flux with the harmonic
mean transmissibility of Sec. 3.1 (tau_sigma = |sigma| k_i k_j / (k_i d_j +
k_j d_i)), Dirichlet half-cell fluxes |sigma| k_i (X_sigma - X_i) / d_i on
Dirichlet faces, and upwind advection X_{sigma,+} (Sec. 3.1: the cell's own
value on outflow, the neighbour's or the boundary value on inflow).

Boundary conditions (reading of the workload text, since the paper's
reservoirs are not reproducible): pressure Dirichlet p_left on the x = 0 face
and p_right on the x = nx face, no flow elsewhere; temperature Dirichlet
T_left (conduction and advective inflow) on x = 0, advective outflow (or
inflow at T_right) with no conduction on x = nx, no flux elsewhere.

Array conventions: cell arrays are flat with index x + nx*(y + ny*z); face
flux arrays include boundary faces: fx (nz, ny, nx+1), fy (nz, ny+1, nx),
fz (nz+1, ny, nx), positive along +x/+y/+z, in kg/s.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

LAW_CONSTANT = 0
LAW_WATER = 1


# --------------------------------------------------------------------------
# Fluid state laws
# --------------------------------------------------------------------------

def density(T, law, rho0=1000.0):
    """Fluid density [kg/m^3].  Law 1 is the linearised water density
    1000 (1 - 3e-4 (T - 20)) used by the coupled workloads in place of the
    paper's rational law (Sec. 5); law 0 is constant."""
    T = np.asarray(T, dtype=np.float64)
    if law == LAW_WATER:
        return 1000.0 * (1.0 - 3.0e-4 * (T - 20.0))
    return np.full_like(T, rho0)


def density_dT(T, law):
    T = np.asarray(T, dtype=np.float64)
    if law == LAW_WATER:
        return np.full_like(T, -0.3)
    return np.zeros_like(T)


def viscosity(T, law, mu0=1.0e-3):
    """Fluid viscosity [Pa s].  Law 1: 2.414e-5 * 10**(247.8 / (T + 133))
    (the high-temperature branch shape of the paper's Sec. 5 law, applied on
    the whole range by the coupled workloads); law 0 is constant."""
    T = np.asarray(T, dtype=np.float64)
    if law == LAW_WATER:
        return 2.414e-5 * 10.0 ** (247.8 / (T + 133.0))
    return np.full_like(T, mu0)


def heat_capacity(T, poro, law, rho0, c_f, rhoc_s):
    """Bulk volumetric heat capacity C = phi rho(T) c_f + (1 - phi)(rho c)_s,
    the left-hand coefficient of the local-equilibrium energy equation
    (Sec. 2, sum of the two lines of Eq. heat with T_s = T_f)."""
    return poro * density(T, law, rho0) * c_f + (1.0 - poro) * rhoc_s


def heat_capacity_dT(T, poro, law, c_f):
    return poro * density_dT(T, law) * c_f


# --------------------------------------------------------------------------
# Grid helpers
# --------------------------------------------------------------------------

class Grid:
    def __init__(self, nx, ny, nz=1, dx=1.0, dy=1.0, dz=1.0):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx, self.dy, self.dz = float(dx), float(dy), float(dz)

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def volume(self):
        return self.dx * self.dy * self.dz

    def index(self):
        return np.arange(self.n).reshape(self.shape)


def grid_of(problem) -> Grid:
    return Grid(problem.nx, problem.ny, problem.nz,
                problem.dx, problem.dy, problem.dz)


# --------------------------------------------------------------------------
# TPFA transmissibilities (Sec. 3.1)
# --------------------------------------------------------------------------

def tpfa_transmissibilities(kcell, g: Grid):
    """Two-point transmissibilities of a scalar cell coefficient ``kcell``.

    Interior face sigma = i|j:  tau = |sigma| k_i k_j / (k_i d_j + k_j d_i),
    with d_i = d_j = half the cell width normal to the face (Sec. 3.1).
    Dirichlet half-cell on the x = 0 and x = nx faces: |sigma| k_i / d_i.

    Returns dict with tx (nz, ny, nx-1), ty (nz, ny-1, nx), tz (nz-1, ny, nx),
    t_left (nz, ny), t_right (nz, ny).
    """
    k = np.asarray(kcell, dtype=np.float64).reshape(g.shape)
    ax, ay, az = g.dy * g.dz, g.dx * g.dz, g.dx * g.dy
    hx, hy, hz = g.dx / 2.0, g.dy / 2.0, g.dz / 2.0

    def harmonic(ki, kj, area, di, dj):
        return area * ki * kj / (ki * dj + kj * di)

    tx = harmonic(k[:, :, :-1], k[:, :, 1:], ax, hx, hx)
    ty = harmonic(k[:, :-1, :], k[:, 1:, :], ay, hy, hy)
    tz = harmonic(k[:-1, :, :], k[1:, :, :], az, hz, hz)
    t_left = ax * k[:, :, 0] / hx
    t_right = ax * k[:, :, -1] / hx
    return dict(tx=tx, ty=ty, tz=tz, t_left=t_left, t_right=t_right)


def interior_faces(g: Grid):
    """(i, j) flat cell pairs of the interior faces, per axis, lower cell first."""
    idx = g.index()
    return {
        "x": (idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel()),
        "y": (idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel()),
        "z": (idx[:-1, :, :].ravel(), idx[1:, :, :].ravel()),
    }


# --------------------------------------------------------------------------
# Steady pressure and face fluxes
# --------------------------------------------------------------------------

def pressure_matrix(trans, g: Grid, p_left, p_right):
    """TPFA matrix of -div(m grad p) with Dirichlet x-faces: for each cell,
    sum_sigma tau_sigma (p_i - p_neighbour) = 0 where the neighbour of a
    Dirichlet face is the boundary value.  Returns (A, rhs), A SPD."""
    N = g.n
    faces = interior_faces(g)
    rows, cols, vals = [], [], []
    diag = np.zeros(N)
    for axis, key in (("x", "tx"), ("y", "ty"), ("z", "tz")):
        i, j = faces[axis]
        t = trans[key].ravel()
        rows += [i, j]
        cols += [j, i]
        vals += [-t, -t]
        np.add.at(diag, i, t)
        np.add.at(diag, j, t)
    idx = g.index()
    left = idx[:, :, 0].ravel()
    right = idx[:, :, -1].ravel()
    rhs = np.zeros(N)
    np.add.at(diag, left, trans["t_left"].ravel())
    np.add.at(diag, right, trans["t_right"].ravel())
    np.add.at(rhs, left, trans["t_left"].ravel() * p_left)
    np.add.at(rhs, right, trans["t_right"].ravel() * p_right)
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A, rhs


def solve_pressure(trans, g: Grid, p_left, p_right, refinements: int = 3):
    """Steady pressure: the solution of the TPFA system A p = rhs.

    A sparse direct solve, then iterative refinement with the residual
    rhs - A p formed in extended precision (np.longdouble): on long strips
    with strong permeability contrasts the forward error of a float64 solve
    alone grows with the condition number, and the face fluxes are
    differences of nearly equal pressures.  Returns the pressure in
    np.longdouble (face_fluxes takes the differences in that precision)."""
    A, rhs = pressure_matrix(trans, g, p_left, p_right)
    A = A.tocsr()
    lu = spla.splu(A.tocsc())
    p = lu.solve(rhs).astype(np.longdouble)
    data = A.data.astype(np.longdouble)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    b = rhs.astype(np.longdouble)
    for _ in range(refinements):
        Ap = np.zeros(A.shape[0], dtype=np.longdouble)
        np.add.at(Ap, rows, data * p[A.indices])
        p = p + lu.solve((b - Ap).astype(np.float64)).astype(np.longdouble)
    return p


def face_fluxes(p, trans, g: Grid, p_left, p_right):
    """Face mass fluxes F = tau (p_upstream_side - p_downstream_side), oriented
    along +x/+y/+z, boundary faces included (Darcy's law in TPFA form)."""
    P = np.asarray(p).reshape(g.shape)
    nz, ny, nx = g.shape
    fx = np.zeros((nz, ny, nx + 1))
    fy = np.zeros((nz, ny + 1, nx))
    fz = np.zeros((nz + 1, ny, nx))
    fx[:, :, 1:-1] = trans["tx"] * (P[:, :, :-1] - P[:, :, 1:])
    fx[:, :, 0] = trans["t_left"] * (p_left - P[:, :, 0])
    fx[:, :, -1] = trans["t_right"] * (P[:, :, -1] - p_right)
    fy[:, 1:-1, :] = trans["ty"] * (P[:, :-1, :] - P[:, 1:, :])
    fz[1:-1, :, :] = trans["tz"] * (P[:-1, :, :] - P[1:, :, :])
    return fx, fy, fz  # float64 arrays: differences taken in P's precision


def layered_x_fluxes(kcell, g: Grid, p_left, p_right):
    """Face mass fluxes when the mobility ``kcell`` is constant in x and y on
    every z-layer and may vary with z only: each layer carries the uniform
    flux k A (p_left - p_right) / (nx dx) through its series of nx cells
    (half cells at both Dirichlet faces), with no transverse flow, which is
    the exact TPFA solution of that case."""
    k = np.asarray(kcell, dtype=np.float64).reshape(g.shape)
    nz, ny, nx = g.shape
    ax = g.dy * g.dz
    layer = k[:, 0, 0]
    q = layer * ax * (p_left - p_right) / (nx * g.dx)
    fx = np.broadcast_to(q[:, None, None], (nz, ny, nx + 1)).copy()
    fy = np.zeros((nz, ny + 1, nx))
    fz = np.zeros((nz + 1, ny, nx))
    return fx, fy, fz


def mobility(T, logk, law, rho0, mu0):
    """Cell mass mobility rho(T) K / mu(T)  [kg s / m^3 ... per Pa]."""
    return density(T, law, rho0) * np.exp(logk) / viscosity(T, law, mu0)


# --------------------------------------------------------------------------
# Heat operator: R(T) = A T + b,  G(T) = R(T) / (V C(T))
# --------------------------------------------------------------------------

def heat_operator(fluxes, g: Grid, lam, c_f, T_left, T_right, dirichlet_left=True):
    """Assemble the conductive + upwind advective energy balance.

    For every cell i:  R_i = sum_sigma [ tau_sigma (T_nb - T_i)  (conduction)
                                        - c_f F_{i,sigma} T_{sigma,+} ]  (advection)
    where F_{i,sigma} is the mass flux out of i, T_{sigma,+} = T_i if
    F_{i,sigma} >= 0 and the neighbour (or boundary) value otherwise
    (Sec. 3.1 upwind rule).  Conduction uses the TPFA transmissibility of the
    uniform conductivity lam; the x = 0 face is a Dirichlet half-cell at
    T_left (unless ``dirichlet_left`` is False: adiabatic x = 0 face).
    Returns (A csr, b) with R(T) = A T + b.
    """
    fx, fy, fz = fluxes
    N = g.n
    cond = tpfa_transmissibilities(np.full(N, lam), g)
    faces = interior_faces(g)
    rows, cols, vals = [], [], []
    diag = np.zeros(N)
    b = np.zeros(N)
    interior_flux = {
        "x": fx[:, :, 1:-1].ravel(),
        "y": fy[:, 1:-1, :].ravel(),
        "z": fz[1:-1, :, :].ravel(),
    }
    for axis, key in (("x", "tx"), ("y", "ty"), ("z", "tz")):
        i, j = faces[axis]
        if i.size == 0:
            continue
        tau = cond[key].ravel()
        f = interior_flux[axis]                 # mass flux from i to j
        out_i = np.maximum(f, 0.0) * c_f        # i -> j carries c_f F T_i
        out_j = np.maximum(-f, 0.0) * c_f       # j -> i carries c_f |F| T_j
        # conduction
        np.add.at(diag, i, -tau)
        np.add.at(diag, j, -tau)
        # advection: outflow removes from the upwind cell, inflow adds to the other
        np.add.at(diag, i, -out_i)
        np.add.at(diag, j, -out_j)
        rows += [i, j]
        cols += [j, i]
        vals += [tau + out_j, tau + out_i]
    idx = g.index()
    left = idx[:, :, 0].ravel()
    right = idx[:, :, -1].ravel()
    # x = 0 face: conduction half-cell to T_left and advection
    if dirichlet_left:
        tl = cond["t_left"].ravel()
        np.add.at(diag, left, -tl)
        np.add.at(b, left, tl * T_left)
    f_in = fx[:, :, 0].ravel()                  # +x oriented: > 0 enters cell
    np.add.at(diag, left, -np.maximum(-f_in, 0.0) * c_f)     # outflow through x = 0
    np.add.at(b, left, np.maximum(f_in, 0.0) * c_f * T_left)  # inflow at T_left
    # x = nx face: advection only
    f_out = fx[:, :, -1].ravel()                # +x oriented: > 0 leaves cell
    np.add.at(diag, right, -np.maximum(f_out, 0.0) * c_f)
    np.add.at(b, right, np.maximum(-f_out, 0.0) * c_f * T_right)
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A, b


class HeatModel:
    """Semi-discrete energy equation dT/dt = G(T) for frozen face fluxes."""

    def __init__(self, A, b, g: Grid, poro, law, rho0, c_f, rhoc_s):
        self.A, self.b, self.g = A, b, g
        self.poro = np.asarray(poro, dtype=np.float64)
        self.law, self.rho0, self.c_f, self.rhoc_s = law, rho0, c_f, rhoc_s

    def capacity(self, T):
        return heat_capacity(T, self.poro, self.law, self.rho0, self.c_f, self.rhoc_s)

    def G(self, T):
        """G(T) = R(T) / (V C(T)), the right-hand side of Eq. spaceheat2."""
        return (self.A @ T + self.b) / (self.g.volume * self.capacity(T))

    def J(self, T):
        """Jacobian D_T G (Eq. linear): row-scale A by 1/(V C) and add the
        diagonal -R_i C'(T_i) / (V C_i^2) from the temperature-dependent
        capacity.  Returned as a dense array (small grids only)."""
        return self.J_sparse(T).toarray()

    def J_sparse(self, T):
        C = self.capacity(T)
        VC = self.g.volume * C
        R = self.A @ T + self.b
        dC = heat_capacity_dT(T, self.poro, self.law, self.c_f)
        # d/dT_i of R_i / (V C(T_i)) through C:  -R_i C'(T_i) / (V C_i^2)
        return (sp.diags(1.0 / VC) @ self.A + sp.diags(-R * dC / (VC * C))).tocsr()


def gershgorin_interval(J):
    """Real interval [alpha, beta] covering the Gershgorin discs of the rows
    of J: alpha = min_i (J_ii - R_i), beta = max_i (J_ii + R_i) with
    R_i = sum_{j != i} |J_ij| (Sec. 4.2 spectral focal interval estimate)."""
    if sp.issparse(J):
        Jc = J.tocsr()
        d = Jc.diagonal()
        absrow = np.asarray(abs(Jc).sum(axis=1)).ravel()
    else:
        Jd = np.asarray(J)
        d = np.diag(Jd)
        absrow = np.abs(Jd).sum(axis=1)
    r = absrow - np.abs(d)
    return float(np.min(d - r)), float(np.max(d + r))
