"""Oracle: dense reverse-mode sensitivities of the sequential coupled EREM run.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Small grids only: every
step forms dense N x N matrices and exponentials of order 2(N+1).

Forward map of one step (the sequential approach of Sec. 3.2.2 with the
steady incompressible pressure equation, TPFA and upwinding of Sec. 3.1):

    m   = rho(T) e^{logK} / mu(T)                    cell mass mobility
    t   = TPFA harmonic transmissibilities of m      (Sec. 3.1)
    A_p(t) p = r(t)                                  steady pressure, Dirichlet x faces
    F   = t (p_i - p_j), boundary half cells         Darcy face mass fluxes
    R   = A_h(F) T + b(F)                            conduction + upwind advection
    G   = R / (V C(T)),  J = D_T G                   (Eq. spaceheat2, Eq. linear)
    T+  = T + eta [exp(Atil)]_{0:N, N},  Atil = [[h J, h G / eta], [0, 0]]

The last line is h phi1(hJ) G (Eq. EERM) read off the augmented exponential;
eta is an exact power of two that balances the last column (a fixed choice
of the evaluation, not a function of the inputs for differentiation).

Reverse sweep (adjoint) of one step, given Tbar+ = d objective / d T+:

* exponential: for L(X) = <W, exp(X)> the gradient is the Frechet derivative
  L_exp(X^T, W), the top-right block of exp([[X^T, W], [0, X^T]]) (the
  block-triangular identity for Frechet derivatives of matrix functions);
  here W = eta [Tbar+; 0] e_{N+1}^T, so Jbar = h Abar[:N, :N] and
  Gbar = (h / eta) Abar[:N, N].
* G and J as functions of R, A_h, C(T) (C' = phi c_f rho' is constant in T
  because the density law is affine in T).
* A_h and b are linear in each face flux for a fixed upwind direction; the
  derivative with respect to one face flux is taken as the exact difference
  of the heat operator at the flux doubled and at the flux itself (doubling
  keeps the upwind direction, conduction cancels exactly).
* fluxes, the pressure system (adjoint solve A_p lambda = pbar, A_p
  symmetric), the harmonic means and the mobility law, written out
  analytically.

Upwind directions, eta and the exponential's internal scaling are fixed
choices at the evaluation point; the derivative is that of the smooth map on
the region where they do not change.

Pins (tests/test_oracle_adjoint.py): frechet_exp against
scipy.linalg.expm_frechet; the whole-run gradient against central finite
differences (Richardson-extrapolated) of ``run_forward`` along random
directions of T0 and log K.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla

from . import physics as ph
from . import phi as phimod


def frechet_exp(X, E):
    """Frechet derivative L_exp(X, E) = d/ds exp(X + s E) at s = 0, as the
    top-right block of exp([[X, E], [0, X]]).  E is rescaled by an exact power
    of two so that both blocks have comparable norms."""
    X = np.asarray(X, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    n = X.shape[0]
    ne = np.abs(E).sum(axis=0).max() if n else 0.0
    if ne == 0.0:
        return np.zeros_like(X)
    nx_ = np.abs(X).sum(axis=0).max()
    beta = 2.0 ** round(math.log2(max(nx_, 1e-300) / ne)) if nx_ > 0 else 1.0 / ne
    big = np.zeros((2 * n, 2 * n))
    big[:n, :n] = X
    big[n:, n:] = X
    big[:n, n:] = beta * E
    return phimod.expm_taylor(big)[:n, n:] / beta


def _pow2(x: float) -> float:
    if x <= 0.0 or not np.isfinite(x):
        return 1.0
    return 2.0 ** round(math.log2(x))


def step_forward(problem, T, h):
    """One coupled step with every intermediate kept (dict)."""
    g = ph.grid_of(problem)
    N = g.n
    T = np.asarray(T, dtype=np.float64)
    logk = np.asarray(problem.logk, dtype=np.float64).ravel()
    m = ph.mobility(T, logk, problem.law, problem.rho0, problem.mu0)
    trans = ph.tpfa_transmissibilities(m, g)
    Ap, rhs = ph.pressure_matrix(trans, g, problem.p_left, problem.p_right)
    p = spla.spsolve(Ap.tocsc(), rhs)
    fluxes = ph.face_fluxes(p, trans, g, problem.p_left, problem.p_right)
    dl = getattr(problem, "dirichlet_left", True)
    Ah, b = ph.heat_operator(fluxes, g, problem.lam, problem.c_f, problem.T_left,
                             problem.T_right, dl)
    model = ph.HeatModel(Ah, b, g, problem.poro, problem.law, problem.rho0,
                         problem.c_f, problem.rhoc_s)
    C = model.capacity(T)
    R = Ah @ T + b
    G = model.G(T)
    J = model.J(T)
    eta = _pow2(float(np.abs(h * G).max()))
    Atil = np.zeros((N + 1, N + 1))
    Atil[:N, :N] = h * J
    Atil[:N, N] = h * G / eta
    E = phimod.expm_taylor(Atil)
    T_next = T + eta * E[:N, N]
    return dict(g=g, T=T, logk=logk, m=m, trans=trans, Ap=Ap, p=p, fluxes=fluxes,
                Ah=Ah.toarray(), b=b, C=C, R=R, G=G, J=J, eta=eta, Atil=Atil,
                T_next=T_next, dirichlet_left=dl)


def run_forward(problem, T0, logk, nsteps, h):
    """T^N of ``nsteps`` coupled steps from T0 with permeability exp(logk)."""
    prob = _with_logk(problem, logk)
    T = np.asarray(T0, dtype=np.float64).copy()
    for _ in range(nsteps):
        T = step_forward(prob, T, h)["T_next"]
    return T


class _Rec:
    pass


def _with_logk(problem, logk):
    """A plain record copy of ``problem`` with another log-permeability."""
    r = _Rec()
    for k in ("nx", "ny", "nz", "dx", "dy", "dz", "poro", "law", "lam", "rhoc_s", "c_f",
              "mu0", "rho0", "p_left", "p_right", "T_left", "T_right"):
        setattr(r, k, getattr(problem, k))
    r.dirichlet_left = getattr(problem, "dirichlet_left", True)
    r.logk = np.asarray(logk, dtype=np.float64).ravel()
    return r


def _flux_derivatives(st, problem):
    """d A_h / d F_sigma and d b / d F_sigma for every face with nonzero flux,
    as (axis, face index, dA (N x N dense), db (N))."""
    g = st["g"]
    fx, fy, fz = st["fluxes"]
    dl = st["dirichlet_left"]
    out = []
    for axis, arr in (("x", fx), ("y", fy), ("z", fz)):
        flat = arr.ravel()
        for f_idx in np.nonzero(flat != 0.0)[0]:
            f = flat[f_idx]
            mod = [fx.copy(), fy.copy(), fz.copy()]
            k = {"x": 0, "y": 1, "z": 2}[axis]
            mod[k].reshape(-1)[f_idx] = 2.0 * f
            A2, b2 = ph.heat_operator(tuple(mod), g, problem.lam, problem.c_f, problem.T_left,
                                      problem.T_right, dl)
            dA = (A2.toarray() - st["Ah"]) / f
            db = (b2 - st["b"]) / f
            out.append((axis, int(f_idx), dA, db))
    return out


def step_adjoint(problem, st, h, Tbar_next):
    """Reverse sweep of one coupled step: returns (Tbar, logkbar) with
    Tbar = (dT+/dT)^T Tbar_next and logkbar = (dT+/dlogK)^T Tbar_next."""
    g = st["g"]
    N = g.n
    V = g.volume
    T, C, R, Ah = st["T"], st["C"], st["R"], st["Ah"]
    eta = st["eta"]
    Tbar_next = np.asarray(Tbar_next, dtype=np.float64)
    # T+ = T + eta exp(Atil)[:N, N]
    W = np.zeros((N + 1, N + 1))
    W[:N, N] = eta * Tbar_next
    Abar = frechet_exp(st["Atil"].T, W)
    Jbar = h * Abar[:N, :N]
    Gbar = (h / eta) * Abar[:N, N]
    Tbar = Tbar_next.copy()
    # G = R / (V C),  J = A_h / (V C) (rows) - diag(R C' / (V C^2))
    dC = ph.heat_capacity_dT(T, problem.poro, problem.law, problem.c_f)
    VC = V * C
    jd = np.diag(Jbar)
    Rbar = Gbar / VC - jd * dC / (V * C * C)
    Ahbar = Jbar / VC[:, None]
    Cbar = (-Gbar * R / (V * C * C)
            - (Jbar * Ah).sum(axis=1) / (V * C * C)
            + jd * 2.0 * R * dC / (V * C ** 3))
    # R = A_h T + b
    Ahbar = Ahbar + np.outer(Rbar, T)
    bbar = Rbar
    Tbar += Ah.T @ Rbar
    Tbar += Cbar * dC
    # face fluxes -> A_h, b
    fbar = {"x": np.zeros(st["fluxes"][0].size), "y": np.zeros(st["fluxes"][1].size),
            "z": np.zeros(st["fluxes"][2].size)}
    for axis, f_idx, dA, db in _flux_derivatives(st, problem):
        fbar[axis][f_idx] = float((Ahbar * dA).sum() + bbar @ db)
    # fluxes F = t (p_i - p_j) (+ boundary half cells), t from the mobility
    nz, ny, nx = g.shape
    P = st["p"].reshape(g.shape)
    tr = st["trans"]
    fxb = fbar["x"].reshape(nz, ny, nx + 1)
    fyb = fbar["y"].reshape(nz, ny + 1, nx)
    fzb = fbar["z"].reshape(nz + 1, ny, nx)
    pbar = np.zeros(g.shape)
    tbar = {k: np.zeros_like(v) for k, v in tr.items()}
    # interior x faces: f = tx (p_l - p_r)
    fi = fxb[:, :, 1:-1]
    dp = P[:, :, :-1] - P[:, :, 1:]
    tbar["tx"] += fi * dp
    pbar[:, :, :-1] += fi * tr["tx"]
    pbar[:, :, 1:] -= fi * tr["tx"]
    fi = fyb[:, 1:-1, :]
    dp = P[:, :-1, :] - P[:, 1:, :]
    tbar["ty"] += fi * dp
    pbar[:, :-1, :] += fi * tr["ty"]
    pbar[:, 1:, :] -= fi * tr["ty"]
    fi = fzb[1:-1, :, :]
    dp = P[:-1, :, :] - P[1:, :, :]
    tbar["tz"] += fi * dp
    pbar[:-1, :, :] += fi * tr["tz"]
    pbar[1:, :, :] -= fi * tr["tz"]
    # boundary: f_left = tL (p_left - p_0), f_right = tR (p_last - p_right)
    fl = fxb[:, :, 0]
    tbar["t_left"] += fl * (problem.p_left - P[:, :, 0])
    pbar[:, :, 0] -= fl * tr["t_left"]
    fr = fxb[:, :, -1]
    tbar["t_right"] += fr * (P[:, :, -1] - problem.p_right)
    pbar[:, :, -1] += fr * tr["t_right"]
    # pressure: A_p p = r;  lambda = A_p^{-1} pbar (A_p symmetric)
    lam = spla.spsolve(st["Ap"].tocsc(), pbar.ravel()).reshape(g.shape)
    tbar["tx"] -= (lam[:, :, :-1] - lam[:, :, 1:]) * (P[:, :, :-1] - P[:, :, 1:])
    tbar["ty"] -= (lam[:, :-1, :] - lam[:, 1:, :]) * (P[:, :-1, :] - P[:, 1:, :])
    tbar["tz"] -= (lam[:-1, :, :] - lam[1:, :, :]) * (P[:-1, :, :] - P[1:, :, :])
    tbar["t_left"] += lam[:, :, 0] * (problem.p_left - P[:, :, 0])
    tbar["t_right"] += lam[:, :, -1] * (problem.p_right - P[:, :, -1])
    # harmonic means: t = a k_i k_j / (k_i d + k_j d); boundary t = a k / d
    k = st["m"].reshape(g.shape)
    ax, ay, az = g.dy * g.dz, g.dx * g.dz, g.dx * g.dy
    hx, hy, hz = g.dx / 2.0, g.dy / 2.0, g.dz / 2.0
    kbar = np.zeros(g.shape)

    def harm_bar(tb, ki, kj, area, d, sl_i, sl_j):
        s = ki + kj
        kbar[sl_i] += tb * area * kj * kj / (d * s * s)
        kbar[sl_j] += tb * area * ki * ki / (d * s * s)

    harm_bar(tbar["tx"], k[:, :, :-1], k[:, :, 1:], ax, hx,
             (slice(None), slice(None), slice(None, -1)), (slice(None), slice(None), slice(1, None)))
    harm_bar(tbar["ty"], k[:, :-1, :], k[:, 1:, :], ay, hy,
             (slice(None), slice(None, -1), slice(None)), (slice(None), slice(1, None), slice(None)))
    harm_bar(tbar["tz"], k[:-1, :, :], k[1:, :, :], az, hz,
             (slice(None, -1), slice(None), slice(None)), (slice(1, None), slice(None), slice(None)))
    kbar[:, :, 0] += tbar["t_left"] * ax / hx
    kbar[:, :, -1] += tbar["t_right"] * ax / hx
    # mobility m = rho(T) e^{logK} / mu(T)
    kb = kbar.ravel()
    mflat = st["m"]
    logkbar = kb * mflat
    if problem.law == ph.LAW_WATER:
        rho = ph.density(T, problem.law, problem.rho0)
        dlog_rho = ph.density_dT(T, problem.law) / rho
        dlog_mu = -math.log(10.0) * 247.8 / (T + 133.0) ** 2
        Tbar += kb * mflat * (dlog_rho - dlog_mu)
    return Tbar, logkbar


def gradient(problem, T0, logk, nsteps, h, Tbar_final):
    """Gradient of <Tbar_final, T^N> with respect to T0 and log K: forward
    steps with every state kept, then the reverse sweep."""
    prob = _with_logk(problem, logk)
    T = np.asarray(T0, dtype=np.float64).copy()
    states = []
    for _ in range(nsteps):
        st = step_forward(prob, T, h)
        states.append(st)
        T = st["T_next"]
    Tbar = np.asarray(Tbar_final, dtype=np.float64).copy()
    logkbar = np.zeros(T.size)
    for st in reversed(states):
        Tbar, lb = step_adjoint(prob, st, h, Tbar)
        logkbar += lb
    return T, Tbar, logkbar
