"""CPU checks of the C ABI library: it loads, exports every declared symbol,
and its host-side numerics (Leja points, divided differences) match brute
force and high-precision references.  No device work is done here."""
import ctypes
import math
import os
import re

import mpmath
import numpy as np
import pytest

from paper_1209_5553_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "erem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(erem_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return nat.load()


def test_library_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(nat.SIGNATURES), set(names) ^ set(nat.SIGNATURES)


def test_default_opts(lib):
    o = nat.default_opts()
    assert (o.method, o.precision, o.p_order, o.m_max, o.krylov_m) == (0, 0, 2, 256, 10)
    assert o.tol_r == 1e-12 and o.tol_a == 0.0 and o.rho_max == 64.0


def test_create_rejects_bad_grids_without_device_work(lib):
    h = ctypes.c_void_p()
    bad = [nat.Grid(4, 8, 8, 1, 1, 1, 1), nat.Grid(2, 8, 8, 2, 1, 1, 1),
           nat.Grid(2, 0, 8, 1, 1, 1, 1), nat.Grid(3, 8, 8, 8, -1, 1, 1)]
    for g in bad:
        assert lib.erem_create(ctypes.byref(g), None, ctypes.byref(h)) == -1
    assert lib.erem_create(None, None, ctypes.byref(h)) == -1


def test_batch_create_rejects_bad_grids_without_device_work(lib):
    """The batched form takes 2D grids only, at least one of them, each with
    positive sides and spacings: anything else is EREM_EINVAL before any
    device call, and no handle is returned."""
    h = ctypes.c_void_p(1)
    good = nat.Grid(2, 8, 8, 1, 1, 1, 1)
    bad = [nat.Grid(3, 8, 8, 8, 1, 1, 1), nat.Grid(2, 8, 8, 2, 1, 1, 1), nat.Grid(2, 0, 8, 1, 1, 1, 1),
           nat.Grid(2, 8, 0, 1, 1, 1, 1), nat.Grid(2, 8, 8, 1, 0, 1, 1), nat.Grid(2, 70000, 8, 1, 1, 1, 1)]
    for g in bad:
        grids = (nat.Grid * 2)(good, g)
        assert lib.erem_batch_create(2, grids, None, ctypes.byref(h)) == -1
        assert not h.value
        h = ctypes.c_void_p(1)
    grids = (nat.Grid * 1)(good)
    assert lib.erem_batch_create(0, grids, None, ctypes.byref(h)) == -1
    assert lib.erem_batch_create(1, None, None, ctypes.byref(h)) == -1
    assert lib.erem_batch_create(1, grids, None, None) == -1


def _leja(n):
    out = np.zeros(n)
    assert nat.load().erem_leja_points(n, out.ctypes.data_as(nat._PD)) == 0
    return out


def test_leja_first_points_closed_form():
    """xi0 = 2 (Sec. 4.2 sets xi0 = beta), xi1 = -2, xi2 = 0, xi3 = +2/sqrt(3)
    (the tie +-2/sqrt(3) of |x (x^2 - 4)| takes the larger point)."""
    xi = _leja(4)
    assert xi[0] == 2.0 and xi[1] == -2.0
    assert abs(xi[2]) < 1e-15
    assert xi[3] == pytest.approx(2.0 / math.sqrt(3.0), abs=1e-14)


def test_leja_points_maximise_node_polynomial_brute_force():
    """Eq. lejaa: every new point maximises prod |x - xi_k| over [-2, 2];
    compare with a brute-force search on a 10^6-point grid (first 30 points)."""
    xi = _leja(30)
    grid = np.linspace(-2.0, 2.0, 1_000_001)
    logp = np.zeros_like(grid)
    for j in range(1, 30):
        logp += np.log(np.abs(grid - xi[j - 1]) + 1e-300)
        best = grid[np.argmax(logp)]
        val_here = np.sum(np.log(np.abs(xi[j] - xi[:j])))
        # the library's point is at least as good as the grid maximum
        assert val_here >= logp.max() - 1e-9, j
        if j != 3:   # j = 3 is the symmetric tie
            assert abs(best - xi[j]) < 1e-4, (j, best, xi[j])
    assert len(set(np.round(xi, 12))) == 30
    assert np.all(np.abs(xi) <= 2.0)


def _dd_reference(hc, hg, xi, n, dps=80):
    """Divided differences of g(x) = phi1(hc + hg x) by the recursive
    definition (Eq. div), in 80-digit arithmetic."""
    mpmath.mp.dps = dps

    def g(x):
        z = mpmath.mpf(hc) + mpmath.mpf(hg) * x
        return mpmath.mpf(1) if z == 0 else mpmath.expm1(z) / z

    pts = [mpmath.mpf(float(v)) for v in xi[:n]]
    table = [g(p) for p in pts]
    out = [table[0]]
    for k in range(1, n):
        table = [(table[i + 1] - table[i]) / (pts[i + k] - pts[i]) for i in range(n - k)]
        out.append(table[0])
    return np.array([float(v) for v in out])


@pytest.mark.parametrize("hc,hg", [(-128.0, 64.0), (-3.7, 1.9), (-0.5, 0.25), (-30.0, 16.0)])
def test_divided_differences_against_high_precision_recursion(hc, hg):
    n = 40
    xi = _leja(n)
    got = np.zeros(n)
    assert nat.load().erem_phi1_divided_differences(hc, hg, xi.ctypes.data_as(nat._PD), n,
                                                    got.ctypes.data_as(nat._PD)) == 0
    ref = _dd_reference(hc, hg, xi, n)
    scale = np.abs(ref).max()
    # eps-level errors amplified by ~log2(norm) squarings
    assert np.abs(got - ref).max() <= 4e-14 * scale, np.abs(got - ref).max() / scale


def test_divided_differences_phi1_equals_exp_with_zero_node():
    """phi1[z_0..z_k] = exp[0, z_0, .., z_k] (divided-difference identity)."""
    mpmath.mp.dps = 60
    n = 12
    xi = _leja(n)
    hc, hg = -5.3, 2.5          # keeps every node z_k = hc + hg xi_k away from 0
    got = np.zeros(n)
    nat.load().erem_phi1_divided_differences(hc, hg, xi.ctypes.data_as(nat._PD), n,
                                             got.ctypes.data_as(nat._PD))
    z = [mpmath.mpf(0)] + [mpmath.mpf(hc) + mpmath.mpf(hg) * mpmath.mpf(float(v)) for v in xi]
    table = [mpmath.exp(v) for v in z]
    exp_dd = [table[0]]
    for k in range(1, n + 1):
        table = [(table[i + 1] - table[i]) / (z[i + k] - z[i]) for i in range(len(table) - 1)]
        exp_dd.append(table[0])
    # g[xi_0..xi_k] = hg^k phi1[z_0..z_k] = hg^k exp[0, z_0..z_k]
    for k in range(n):
        ref = float(exp_dd[k + 1] * mpmath.mpf(hg) ** k)
        assert got[k] == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_divided_differences_degenerate_interval():
    """hg = 0: g is constant in xi, so d_0 = phi1(hc) and d_k = 0 for k > 0."""
    xi = _leja(8)
    got = np.zeros(8)
    nat.load().erem_phi1_divided_differences(-3.0, 0.0, xi.ctypes.data_as(nat._PD), 8,
                                             got.ctypes.data_as(nat._PD))
    assert got[0] == pytest.approx(math.expm1(-3.0) / -3.0, rel=1e-15)
    assert np.all(got[1:] == 0.0)


def test_host_numerics_argument_validation(lib):
    out = np.zeros(4)
    assert lib.erem_leja_points(-1, out.ctypes.data_as(nat._PD)) == -1
    assert lib.erem_leja_points(5000, out.ctypes.data_as(nat._PD)) == -1
    assert lib.erem_phi1_divided_differences(float("nan"), 1.0, out.ctypes.data_as(nat._PD), 4,
                                             out.ctypes.data_as(nat._PD)) == -1


def _dd2_reference(hc, hg, xi, n, dps=80):
    """Divided differences of g(x) = phi2(hc + hg x), phi2(z) =
    (e^z - 1 - z)/z^2 (Sec. 3.2.3), by the recursive definition in 80 digits
    (series where the closed form would cancel)."""
    mpmath.mp.dps = dps

    def g(x):
        z = mpmath.mpf(hc) + mpmath.mpf(hg) * x
        if abs(z) < mpmath.mpf("1e-20"):
            return sum(z ** k / mpmath.factorial(k + 2) for k in range(6))
        return (mpmath.expm1(z) - z) / (z * z)

    pts = [mpmath.mpf(float(v)) for v in xi[:n]]
    table = [g(p) for p in pts]
    out = [table[0]]
    for k in range(1, n):
        table = [(table[i + 1] - table[i]) / (pts[i + k] - pts[i]) for i in range(n - k)]
        out.append(table[0])
    return np.array([float(v) for v in out])


@pytest.mark.parametrize("hc,hg", [(-128.0, 64.0), (-3.7, 1.9), (-0.5, 0.25), (-30.0, 16.0)])
def test_phi2_divided_differences_against_high_precision_recursion(hc, hg):
    n = 40
    xi = _leja(n)
    got = np.zeros(n)
    assert nat.load().erem_phi2_divided_differences(hc, hg, xi.ctypes.data_as(nat._PD), n,
                                                    got.ctypes.data_as(nat._PD)) == 0
    ref = _dd2_reference(hc, hg, xi, n)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 4e-14 * scale, np.abs(got - ref).max() / scale


def test_phi2_divided_differences_degenerate_interval():
    """hg = 0: d_0 = phi2(hc), the rest 0."""
    xi = _leja(8)
    got = np.zeros(8)
    nat.load().erem_phi2_divided_differences(-3.0, 0.0, xi.ctypes.data_as(nat._PD), 8,
                                             got.ctypes.data_as(nat._PD))
    assert got[0] == pytest.approx((math.expm1(-3.0) + 3.0) / 9.0, rel=1e-15)
    assert np.all(got[1:] == 0.0)
    assert nat.load().erem_phi2_divided_differences(1.0, float("inf"), xi.ctypes.data_as(nat._PD), 8,
                                                    got.ctypes.data_as(nat._PD)) == -1
