"""Pins of the oracle's dense adjoint (oracle/adjoint.py).

* frechet_exp against scipy.linalg.expm_frechet (the library routine the
  block-exponential identity reduces to);
* the whole-run gradient of <c, T^N> with respect to T0 and log K against
  Richardson-extrapolated central differences of the oracle's own forward
  run, along random directions, for the water-law coupled physics and for
  the constant-law linear physics.
"""
import dataclasses

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import adjoint as oadj
from paper_1209_5553_amd import inputs


@pytest.mark.parametrize("seed,scale", [(0, 0.3), (1, 4.0), (2, 40.0)])
def test_frechet_exp_matches_scipy(seed, scale):
    rng = np.random.default_rng(seed)
    n = 9
    X = scale * rng.standard_normal((n, n)) / np.sqrt(n)
    X[np.tril_indices(n, -2)] *= 0.1          # non-normal
    E = rng.standard_normal((n, n))
    _, L = sl.expm_frechet(X, E)
    got = oadj.frechet_exp(X, E)
    assert np.abs(got - L).max() <= 1e-11 * np.abs(L).max()


def test_frechet_exp_linear_in_direction_and_zero():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((6, 6))
    E = rng.standard_normal((6, 6))
    assert np.array_equal(oadj.frechet_exp(X, np.zeros((6, 6))), np.zeros((6, 6)))
    a = oadj.frechet_exp(X, 3.0 * E)
    b = 3.0 * oadj.frechet_exp(X, E)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def _fd(f, x, v, eps):
    d1 = (f(x + eps * v) - f(x - eps * v)) / (2 * eps)
    d2 = (f(x + 0.5 * eps * v) - f(x - 0.5 * eps * v)) / eps
    return (4.0 * d2 - d1) / 3.0


def _tiny(kind):
    if kind == "water":
        p = inputs.coupled_problem(6, seed=3, nsteps=2)
        p = dataclasses.replace(p, nx=5, ny=4, logk=p.logk.reshape(6, 6)[:4, :5].ravel().copy(),
                                poro=p.poro[:20].copy(), T0=p.T0[:20].copy())
    else:
        p = inputs.linear_problem(4, seed=5, nsteps=2)
        p = dataclasses.replace(p, nx=4, ny=3, logk=p.logk.reshape(4, 4)[:3, :4].ravel().copy(),
                                poro=p.poro[:12].copy(), T0=p.T0[:12].copy(), dx=2.0, dy=0.5)
    return p


@pytest.mark.parametrize("kind", ["water", "linear"])
def test_adjoint_gradient_matches_finite_differences(kind):
    p = _tiny(kind)
    N = p.nx * p.ny
    rng = np.random.default_rng(11)
    T0 = rng.uniform(20.0, 70.0, N)
    logk = np.asarray(p.logk, dtype=np.float64)
    c = rng.standard_normal(N)
    # the linear problem's advection flushes T0 within one step of 1e6 s:
    # a shorter step keeps d T^N / d T0 of order one
    h, nsteps = (p.h if kind == "water" else 2.0e3), 2
    TN, gT, gK = oadj.gradient(p, T0, logk, nsteps, h, c)
    ref = oadj.run_forward(p, T0, logk, nsteps, h)
    assert np.abs(TN - ref).max() == 0.0

    def obj_T(x):
        return float(c @ oadj.run_forward(p, x, logk, nsteps, h))

    def obj_K(x):
        return float(c @ oadj.run_forward(p, T0, x, nsteps, h))

    for trial in range(2):
        v = rng.standard_normal(N)
        fdT = _fd(obj_T, T0, v, 1e-2)
        assert abs(gT @ v - fdT) <= 1e-7 * max(abs(fdT), np.abs(gT).sum() * 1e-3), (trial, gT @ v, fdT)
        w = rng.standard_normal(N)
        fdK = _fd(obj_K, logk, w, 1e-3)
        assert abs(gK @ w - fdK) <= 1e-7 * max(abs(fdK), np.abs(gK).sum() * 1e-3), (trial, gK @ w, fdK)


def test_adjoint_gradient_is_nontrivial_in_both_inputs():
    """Guards the FD pin against a vacuous pass: both gradients are O(1)
    relative to the objective's scale, and log K matters only through the
    pressure (zero for the constant-law problem only if fluxes vanish)."""
    p = _tiny("water")
    N = p.nx * p.ny
    c = np.ones(N) / N
    _, gT, gK = oadj.gradient(p, np.full(N, 20.0), p.logk, 2, p.h, c)
    assert np.abs(gT).max() > 1e-3
    assert np.abs(gK).max() > 1e-6
