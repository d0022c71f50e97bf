"""Pins of the oracle's material laws and of the scaling of its right-hand sides.

The other pins (conservation, linear exactness, the steady limit, J against
finite differences of G, the pressure mass balance) hold for any heat
capacity, mobility or storage coefficient, so they cannot see a mistake in
those laws.  These tests compare them with values worked by hand from the
formulas of Sec. 2 (tests/golden/material_laws.json): the local-equilibrium
capacity C = phi rho c_f + (1 - phi)(rho c)_s, the mass mobility rho K / mu of
Eq. darcy with Eq. masscon2, the storage S = phi beta_f + phi_0 alpha_b of
Eq. masscon4, G = R / (V C) of the energy balance and G4 = (b - A p)/(V rho S)
+ (phi alpha_f / S) G2 of the pressure equation, on one- and three-cell grids
with non-unit cells.  The last tests plant typical mistakes in the oracle
(on the CPU) and check that these pins catch each of them.
"""
import json
import os

import numpy as np
import pytest

from oracle import compressible as ocomp
from oracle import erem as oerem
from oracle import physics as ph
from paper_1209_5553_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "material_laws.json")
RTOL = 1e-14


def _load():
    with open(GOLDEN) as f:
        return json.load(f)


def _close(got, ref, rtol=RTOL):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return bool(np.all(np.abs(got - ref) <= rtol * np.maximum(np.abs(ref), 1e-300)))


def _one_cell_problem(gd, **kw):
    n = 1
    base = dict(name="one_cell", nx=gd["nx"], ny=gd["ny"], nz=gd["nz"], logk=np.full(n, kw.pop("logk", 0.0)),
                poro=np.full(n, kw.pop("poro")), T0=np.full(n, kw.pop("T", 20.0)),
                dx=gd["dx"], dy=gd["dy"], dz=gd["dz"])
    base.update(kw)
    return inputs.Problem(**base)


def check_heat_capacity(gold):
    bad = []
    for c in gold["heat_capacity"]["cases"]:
        T = np.array([c["T"]])
        C = ph.heat_capacity(T, np.array([c["poro"]]), c["law"], c["rho0"], c["c_f"], c["rhoc_s"])
        dC = ph.heat_capacity_dT(T, np.array([c["poro"]]), c["law"], c["c_f"])
        if not _close(C, c["C"]):
            bad.append(("C", c, C))
        if not (np.abs(dC - c["dC"]) <= 1e-12 * max(1.0, abs(c["dC"]))).all():
            bad.append(("dC", c, dC))
    return bad


def check_mobility(gold):
    bad = []
    for c in gold["mobility"]["cases"]:
        m = ph.mobility(np.array([c["T"]]), np.array([c["logk"]]), c["law"], c["rho0"], c["mu0"])
        if not _close(m, c["mobility"], 1e-13):
            bad.append(("mobility", c, m))
    return bad


def check_storage(gold):
    bad = []
    for c in gold["storage"]["cases"]:
        S = ocomp.storage(np.array([c["poro"]]), c["alpha_b"], c["beta_f"])
        if not _close(S, c["S"]):
            bad.append(("S", c, S))
    return bad


def check_heat_rhs(gold):
    bad = []
    c = gold["heat_rhs_one_cell"]
    gd = c["grid"]
    prob = _one_cell_problem(gd, poro=c["poro"], T=c["T"], law=inputs.LAW_CONSTANT, lam=c["lam"], c_f=c["c_f"],
                             rho0=c["rho0"], rhoc_s=c["rhoc_s"], T_left=c["T_left"], T_right=c["T_right"])
    fx = np.full((1, 1, 2), c["flux"])
    fy = np.zeros((1, 2, 1))
    fz = np.zeros((2, 1, 1))
    disc = oerem.Discretisation(prob, prob.T0, fluxes=(fx, fy, fz))
    T = np.array([c["T"]])
    R = disc.model.A @ T + disc.model.b
    G = disc.model.G(T)
    if not _close(R, c["R"]):
        bad.append(("R one cell", R))
    if not _close(G, c["G"]):
        bad.append(("G one cell", G))

    c3 = gold["heat_rhs_three_cells"]
    with open(os.path.join(os.path.dirname(GOLDEN), "heat_operator_3cells.json")) as f:
        op = json.load(f)
    A = np.asarray(op["A"])
    b = np.asarray(op["b"])
    import scipy.sparse as sp
    model = ph.HeatModel(sp.csr_matrix(A), b, ph.Grid(3, 1, 1), np.full(3, c3["poro"]), inputs.LAW_CONSTANT,
                         c3["rho0"], c3["c_f"], c3["rhoc_s"])
    G3 = model.G(np.asarray(c3["T"]))
    if not _close(G3, c3["G"], 4e-16 * 16):
        bad.append(("G three cells", G3))
    return bad


def check_pressure_rhs(gold):
    bad = []
    c = gold["pressure_rhs_one_cell"]
    for case in c["cases"]:
        prob = _one_cell_problem(c["grid"], poro=c["poro"], logk=c["logk"], T=case["T"], law=case["law"],
                                 p_left=c["p_left"], p_right=c["p_right"])
        G4, _ = ocomp.pressure_rhs(prob, prob.T0, np.array([c["p"]]), np.array([c["G2"]]), c["alpha_b"],
                                   c["beta_f"])
        if not _close(G4, case["G4"], 1e-13):
            bad.append(("G4", case, G4))
    return bad


CHECKS = (check_heat_capacity, check_mobility, check_storage, check_heat_rhs, check_pressure_rhs)


@pytest.mark.parametrize("check", CHECKS, ids=lambda f: f.__name__)
def test_material_law_pin(check):
    assert check(_load()) == []


def _all_failures():
    gold = _load()
    return [f for check in CHECKS for f in check(gold)]


def test_planted_capacity_porosity_swap_is_caught(monkeypatch):
    def swapped(T, poro, law, rho0, c_f, rhoc_s):
        return (1.0 - poro) * ph.density(T, law, rho0) * c_f + poro * rhoc_s
    monkeypatch.setattr(ph, "heat_capacity", swapped)
    assert _all_failures()


def test_planted_capacity_without_fluid_density_is_caught(monkeypatch):
    def no_rho(T, poro, law, rho0, c_f, rhoc_s):
        return poro * c_f + (1.0 - poro) * rhoc_s
    monkeypatch.setattr(ph, "heat_capacity", no_rho)
    assert _all_failures()


def test_planted_mobility_without_density_is_caught(monkeypatch):
    def no_rho(T, logk, law, rho0, mu0):
        return np.exp(logk) / ph.viscosity(T, law, mu0)
    monkeypatch.setattr(ph, "mobility", no_rho)
    assert _all_failures()


def test_planted_storage_without_reference_porosity_is_caught(monkeypatch):
    def no_phi0(poro, alpha_b, beta_f):
        return np.asarray(poro, dtype=np.float64) * beta_f + alpha_b
    monkeypatch.setattr(ocomp, "storage", no_phi0)
    assert _all_failures()


def test_planted_rhs_without_cell_volume_is_caught(monkeypatch):
    def G_no_volume(self, T):
        return (self.A @ T + self.b) / self.capacity(T)
    monkeypatch.setattr(ph.HeatModel, "G", G_no_volume)
    assert _all_failures()


def test_planted_viscosity_exponent_base_is_caught(monkeypatch):
    def mu_e(T, law, mu0=1.0e-3):
        T = np.asarray(T, dtype=np.float64)
        if law == ph.LAW_WATER:
            return 2.414e-5 * np.exp(247.8 / (T + 133.0))
        return np.full_like(T, mu0)
    monkeypatch.setattr(ph, "viscosity", mu_e)
    assert _all_failures()
