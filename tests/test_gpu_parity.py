"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerance: 1e-10 relative (max norm) for temperatures after EREM steps and
phi1 actions (the FP64 target); assembly quantities that involve no
iteration (transmissibilities, stencil, G) agree to 1e-13.
"""
import numpy as np
import pytest

from oracle import erem as oerem
from oracle import phi as ophi
from oracle import physics as oph
from paper_1209_5553_amd import inputs

from gpu_util import rel_inf, sparse_to_stencil, stencil_to_sparse

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _ctx(prob):
    from paper_1209_5553_amd.api import EremContext
    return EremContext.from_problem(prob, device="cuda:0")


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0").clone()


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _oracle_fluxes_to_dev(torch, disc):
    fx, fy, fz = disc.fluxes
    return _dev(torch, fx.ravel()), _dev(torch, fy.ravel()), _dev(torch, fz.ravel())


# --------------------------------------------------------------- a1 / a2

def test_transmissibilities_and_fluxes(torch_mod):
    torch = torch_mod
    prob = inputs.linear_problem(32)
    _say(f"transmissibilities {prob.name}")
    ctx = _ctx(prob)
    st = ctx.pressure_and_fluxes(rtol=1e-16)
    faces = {k: v.cpu().numpy() for k, v in ctx.get_faces().items()}
    disc = oerem.Discretisation(prob, prob.T0)
    g = disc.g
    tx = faces["tx"].reshape(g.nz, g.ny, g.nx + 1)
    assert rel_inf(tx[:, :, 1:-1], disc.trans["tx"]) <= 1e-13
    assert rel_inf(tx[:, :, 0], disc.trans["t_left"]) <= 1e-13
    assert rel_inf(tx[:, :, -1], disc.trans["t_right"]) <= 1e-13
    ty = faces["ty"].reshape(g.nz, g.ny + 1, g.nx)
    assert rel_inf(ty[:, 1:-1, :], disc.trans["ty"]) <= 1e-13
    assert np.all(ty[:, 0, :] == 0) and np.all(ty[:, -1, :] == 0)
    for name, ref in zip(("fx", "fy"), disc.fluxes[:2]):
        got = faces[name].reshape(ref.shape)
        assert rel_inf(got, ref) <= TOL, (name, rel_inf(got, ref), st)
    assert st["est_err"] <= 1e-14


@pytest.mark.parametrize("n", [64, 96, 33])
def test_multigrid_and_jacobi_pressure_agree(torch_mod, n):
    """Both preconditioners reach the same (double-double refined) pressure
    and fluxes; the multigrid one in far fewer iterations."""
    torch = torch_mod
    prob = inputs.coupled_problem(n, seed=5)
    T = _dev(torch, np.random.default_rng(2).uniform(20, 80, prob.n))
    res = {}
    for kind in ("jacobi", "multigrid"):
        ctx = _ctx(prob)
        ctx.set_pressure_preconditioner(kind)
        p = torch.zeros(prob.n, dtype=torch.float64, device="cuda:0")
        st = ctx.pressure_and_fluxes(T, rtol=1e-16, p=p)
        res[kind] = (p.cpu().numpy(), ctx.get_faces()["fx"].cpu().numpy(), st["iterations"])
        _say(f"pressure n={n} {kind}: {st}")
    assert rel_inf(res["multigrid"][0], res["jacobi"][0]) <= 1e-13
    assert rel_inf(res["multigrid"][1], res["jacobi"][1]) <= 1e-12
    assert res["multigrid"][2] * 5 < res["jacobi"][2]
    disc = oerem.Discretisation(prob, T.cpu().numpy())
    assert rel_inf(res["multigrid"][1].reshape(disc.fluxes[0].shape), disc.fluxes[0]) <= TOL


@pytest.mark.parametrize("shape", [(150, 37), (37, 150), (700, 3), (3, 700), (65, 17)])
def test_multigrid_pressure_ragged_shapes(torch_mod, shape):
    """Non-square grids above one workgroup's coarse level (the CG iteration
    runs inside the finest multigrid legs, tiles ragged at both edges): the
    refined pressure and fluxes match the oracle's direct solve."""
    import dataclasses
    torch = torch_mod
    nx, ny = shape
    rng = np.random.default_rng(nx * 1000 + ny)
    base = inputs.coupled_problem(8, seed=5)
    N = nx * ny
    prob = dataclasses.replace(base, name=f"coupled{nx}x{ny}", nx=nx, ny=ny,
                               logk=inputs.lognormal_field(rng, (ny, nx), 2.0, 8.0),
                               poro=np.full(N, base.poro[0]), T0=np.full(N, base.T0[0]))
    T = _dev(torch, rng.uniform(20, 80, N))
    ctx = _ctx(prob)
    p = torch.zeros(N, dtype=torch.float64, device="cuda:0")
    st = ctx.pressure_and_fluxes(T, rtol=1e-16, p=p)
    _say(f"pressure {nx}x{ny}: {st}")
    disc = oerem.Discretisation(prob, T.cpu().numpy())
    faces = ctx.get_faces()
    # each flux array relative to its own largest entry, except on the thin
    # strips (3 cells across): their transverse fluxes are differences of
    # nearly equal pressures, known to the oracle's conditioning-limited
    # accuracy only in absolute terms, so they are measured against the
    # field's largest flux
    strip = min(nx, ny) <= 3
    field_scale = max(np.abs(f).max() for f in disc.fluxes[:2])
    for name, ref in zip(("fx", "fy"), disc.fluxes[:2]):
        got = faces[name].cpu().numpy().reshape(ref.shape)
        scale = field_scale if strip else np.abs(ref).max()
        err = np.abs(got - ref).max() / scale
        _say(f"  {name}: max error / {'field' if strip else 'own'} scale = {err:.2e}")
        assert err <= TOL, (name, err)
    assert st["est_err"] <= 1e-14


def test_multigrid_pressure_3d_layered_is_analytic(torch_mod):
    torch = torch_mod
    prob = inputs.layered3d_problem(24, seed=3)
    ctx = _ctx(prob)
    st = ctx.pressure_and_fluxes(rtol=1e-16)
    g = oph.grid_of(prob)
    mob = oph.mobility(prob.T0, prob.logk, prob.law, prob.rho0, prob.mu0)
    fx, fy, fz = oph.layered_x_fluxes(mob, g, prob.p_left, prob.p_right)
    faces = ctx.get_faces()
    _say(f"3D multigrid pressure: {st}")
    assert rel_inf(faces["fx"].cpu().numpy().reshape(fx.shape), fx) <= 1e-12
    assert np.abs(faces["fy"].cpu().numpy()).max() <= 1e-12 * np.abs(fx).max()
    assert np.abs(faces["fz"].cpu().numpy()).max() <= 1e-12 * np.abs(fx).max()


# -------------------------------------------------------------------- a3/a4

@pytest.mark.parametrize("kind", ["linear32", "coupled24", "layered3d"])
def test_jacobian_stencil_and_G(torch_mod, kind):
    torch = torch_mod
    if kind == "linear32":
        prob = inputs.linear_problem(32)
        T = prob.T0.copy()
        T[::7] += 13.0
    elif kind == "coupled24":
        prob = inputs.coupled_problem(24, seed=3)
        T = np.random.default_rng(1).uniform(20, 80, prob.n)
    else:
        prob = inputs.layered3d_problem(9, seed=2)
        T = np.random.default_rng(2).uniform(20, 80, prob.n)
    _say(f"jacobian {kind}")
    disc = oerem.Discretisation(prob, T)
    ctx = _ctx(prob)
    ctx.set_face_fluxes(*_oracle_fluxes_to_dev(torch, disc))
    ctx.form_jacobian(_dev(torch, T))
    coef, F = ctx.get_jacobian()
    coef = coef.cpu().numpy()
    Jref = disc.model.J_sparse(T)
    ref = sparse_to_stencil(Jref, prob.nx, prob.ny, prob.nz)
    assert rel_inf(coef, ref) <= 1e-13
    assert rel_inf(F.cpu().numpy(), disc.model.G(T)) <= 1e-13
    a, b = oph.gershgorin_interval(Jref)
    out, st = ctx.phi1_apply(1.0, _dev(torch, np.ones(prob.n)))
    assert st["alpha"] == pytest.approx(a, rel=1e-13)
    assert abs(st["beta"] - b) <= 1e-13 * abs(a)


# ---------------------------------------------------------------------- a6

def test_phi1_apply_matches_dense_oracle(torch_mod):
    torch = torch_mod
    prob = inputs.linear_problem(32)
    _say("phi1 apply 32x32")
    disc = oerem.Discretisation(prob, prob.T0)
    ctx = _ctx(prob)
    ctx.set_face_fluxes(*_oracle_fluxes_to_dev(torch, disc))
    ctx.form_jacobian(_dev(torch, prob.T0))
    rng = np.random.default_rng(0)
    v = rng.standard_normal(prob.n)
    J = disc.model.J(prob.T0)
    for h in (1e4, 1e6, 3e6):
        out, st = ctx.phi1_apply(h, _dev(torch, v))
        ref = ophi.phi1_action_dense(J, v, h)
        err = rel_inf(out.cpu().numpy(), ref)
        _say(f"  h={h:g} m={st['m_total']} s={st['substeps']} err={err:.2e}")
        assert err <= TOL


def test_diagonal_closed_form(torch_mod):
    """Diagonal J: phi1(hJ) v = (e^{h lam} - 1)/(h lam) v (closed form)."""
    torch = torch_mod
    nx, ny = 40, 9
    N = nx * ny
    from paper_1209_5553_amd.api import EremContext
    ctx = EremContext(nx, ny)
    lam = -np.geomspace(1e-9, 2e-4, N)
    np.random.default_rng(4).shuffle(lam)
    coef = np.zeros((5, N))
    coef[0] = lam
    v = np.random.default_rng(5).standard_normal(N)
    ctx.set_jacobian(_dev(torch, coef.ravel()), _dev(torch, v))
    for h in (1e5, 1e6):
        out, st = ctx.phi1_apply(h, _dev(torch, v))
        ref = ophi.phi1_scalar(h * lam) * v
        err = rel_inf(out.cpu().numpy(), ref)
        _say(f"diagonal h={h:g} m={st['m_total']} s={st['substeps']} err={err:.2e}")
        assert err <= 1e-12


def test_newton_interpolation_is_exact_at_the_nodes(torch_mod):
    """J = diag(c + gamma xi_k), k < N: the Newton polynomial through the
    Leja nodes (Eq. approle) reproduces phi1 at every eigenvalue, so the
    result is exact to rounding whatever the stop rule."""
    torch = torch_mod
    from paper_1209_5553_amd.api import EremContext, leja_points, make_opts
    nx, ny = 4, 4
    N = nx * ny
    xi = leja_points(N)
    c, gam = -2.0e-5, 9.0e-6
    lam = c + gam * xi
    coef = np.zeros((5, N))
    coef[0] = lam
    ctx = EremContext(nx, ny)
    v = np.linspace(1.0, 2.0, N)
    ctx.set_jacobian(_dev(torch, coef.ravel()), _dev(torch, v))
    h = 1e6
    out, st = ctx.phi1_apply(h, _dev(torch, v), opts=make_opts(rho_max=0.0))
    ref = ophi.phi1_scalar(h * lam) * v
    _say(f"node exactness m={st['m_total']} s={st['substeps']}")
    assert st["substeps"] == 1
    assert rel_inf(out.cpu().numpy(), ref) <= 1e-13


def test_phi1_of_zero_matrix_is_identity(torch_mod):
    torch = torch_mod
    from paper_1209_5553_amd.api import EremContext
    ctx = EremContext(7, 5)
    v = np.arange(35, dtype=np.float64) - 11.0
    ctx.set_jacobian(_dev(torch, np.zeros(5 * 35)), _dev(torch, v))
    out, st = ctx.phi1_apply(3.0e5, _dev(torch, v))
    assert np.array_equal(out.cpu().numpy(), v)


# ------------------------------------------------------------- EREM steps

def _run_gpu_linear(torch, prob, nsteps, h=None, opts=None, fluxes=None):
    ctx = _ctx(prob)
    if fluxes is None:
        ctx.pressure_and_fluxes(rtol=1e-16)
    else:
        ctx.set_face_fluxes(*fluxes)
    T = _dev(torch, prob.T0)
    stats = [ctx.step(prob.h if h is None else h, T, opts) for _ in range(nsteps)]
    torch.cuda.synchronize()
    return T.cpu().numpy(), stats


def test_linear_32x32_ten_steps(torch_mod):
    """The 32x32 FP64 workload: 10 EREM steps of 1e6 s against the dense oracle."""
    torch = torch_mod
    prob = inputs.linear_problem(32)
    _say("32x32 x 10 steps")
    T_gpu, stats = _run_gpu_linear(torch, prob, prob.nsteps)
    T_ref, _ = oerem.run_linear(prob)
    err = rel_inf(T_gpu, T_ref)
    inc = rel_inf(T_gpu - prob.T0, T_ref - prob.T0)
    _say(f"  err={err:.2e} inc={inc:.2e} m={[s['m_total'] for s in stats]}")
    assert err <= TOL and inc <= TOL


def test_first_step_increment_32x32(torch_mod):
    """One step from the uniform start, where the front is sharp."""
    torch = torch_mod
    prob = inputs.linear_problem(32)
    T_gpu, st = _run_gpu_linear(torch, prob, 1)
    T_ref, _ = oerem.run_linear(prob, nsteps=1)
    assert rel_inf(T_gpu - prob.T0, T_ref - prob.T0) <= TOL


def test_linear_exactness_on_gpu(torch_mod):
    """Ten GPU steps of h equal one GPU step of 10 h (EREM is exact for
    linear problems, R(z) = e^z), and both equal the oracle."""
    torch = torch_mod
    prob = inputs.linear_problem(24, seed=6)
    T10, _ = _run_gpu_linear(torch, prob, 10)
    T1, _ = _run_gpu_linear(torch, prob, 1, h=10 * prob.h)
    assert rel_inf(T10 - prob.T0, T1 - prob.T0) <= TOL
    disc = oerem.Discretisation(prob, prob.T0)
    Tref = oerem.erem_step(disc.model, prob.T0, 10 * prob.h)
    assert rel_inf(T1, Tref) <= TOL


# Steps after the first are enqueued right behind the assembly: the substep
# count is predicted from the previous step's interval width and the Leja
# coefficients are formed on the device; the interval read back afterwards
# confirms the prediction, else the step runs again on it.

def _lam_steps(torch, prob, factors, h, opts=None):
    """Steps with the conductivity scaled by each factor in turn (the
    interval and the substep count change with it), each from a fresh seeded
    temperature field (so that no step starts near the steady state) against
    the oracle step from the same field with that conductivity."""
    import dataclasses
    ctx = _ctx(prob)
    ctx.pressure_and_fluxes(rtol=1e-16)
    rng = np.random.default_rng(17)
    out = []
    for f in factors:
        lam = prob.lam * f
        ctx.set_rock(ctx._logk, ctx._poro, lam, prob.rhoc_s)
        start = rng.uniform(20.0, 80.0, prob.n)
        T = _dev(torch, start)
        st = ctx.step(h, T, opts)
        model = oerem.Discretisation(dataclasses.replace(prob, lam=lam), start).model
        a, b = oph.gershgorin_interval(model.J_sparse(start))
        Tref = oerem.erem_step(model, start, h)
        got = T.cpu().numpy()
        err, inc = rel_inf(got, Tref), rel_inf(got - start, Tref - start)
        _say(f"  lam x{f:g}: s={st['substeps']} m={st['m_total']} restarts={st['restarts']} "
             f"err={err:.2e} inc={inc:.2e}")
        assert err <= TOL and inc <= TOL
        assert st["alpha"] == pytest.approx(a, rel=1e-13)
        assert abs(st["beta"] - b) <= 1e-13 * abs(a)
        out.append(st)
    return out


def test_predicted_substeps_follow_interval_changes(torch_mod):
    """24x24: the substep count goes 3, 3, 4, 4, 5, 10, 3, 3 as the
    conductivity changes; every change is a failed prediction that falls back
    to the interval read back, every repeat a held one."""
    torch = torch_mod
    prob = inputs.linear_problem(24, seed=6)
    _say("predicted substeps 24x24, conductivity x1 1 4 4 16 64 1 0.25")
    sts = _lam_steps(torch, prob, (1, 1, 4, 4, 16, 64, 1, 0.25), prob.h)
    assert [s["substeps"] for s in sts] == [3, 3, 4, 4, 5, 10, 3, 3]


def test_predicted_step_budget_restart(torch_mod):
    """One substep (rho_max = 0) at h / 64: the degree is about 20, so the
    second and third steps' budgets (the previous degree plus one group) are
    formed on the device; when the conductivity grows 256-fold the degree
    grows to about 38, past the third step's budget of 28 terms, and the
    predicted evaluation restarts with the full budget; the fourth step's
    budget (44 terms) is more than the device forms and takes the
    synchronous path."""
    torch = torch_mod
    from paper_1209_5553_amd.api import make_opts
    prob = inputs.linear_problem(24, seed=6)
    _say("predicted step 24x24, one substep, conductivity x1 1 256 256")
    sts = _lam_steps(torch, prob, (1, 1, 256, 256), prob.h / 64, make_opts(rho_max=0.0))
    assert all(s["substeps"] == 1 for s in sts)
    assert sts[1]["restarts"] == 0 and sts[2]["restarts"] >= 1
    assert sts[2]["m_total"] > 28


def test_energy_conserved_with_closed_boundaries(torch_mod):
    torch = torch_mod
    rng = np.random.default_rng(31)
    prob = inputs.linear_problem(20, seed=7)
    prob.dirichlet_left = False
    prob.T0 = rng.uniform(20.0, 80.0, prob.n)
    # incompressible circulation (stream function), closed boundaries: the
    # Gershgorin interval stays in the left half-plane as for real flows
    fl = inputs.random_solenoidal_fluxes(rng, prob.nx, prob.ny, scale=1e-2)
    T_gpu, stats = _run_gpu_linear(torch, prob, 3, fluxes=tuple(_dev(torch, f.ravel()) for f in fl))
    w = oph.heat_capacity(prob.T0, prob.poro, prob.law, prob.rho0, prob.c_f, prob.rhoc_s)
    drift = abs(w @ T_gpu - w @ prob.T0) / abs(w @ prob.T0)
    _say(f"conservation drift {drift:.2e} stats {stats[-1]}")
    assert drift <= 1e-13
    assert np.abs(T_gpu - prob.T0).max() > 1e-3


@pytest.mark.parametrize("shape", [(70, 5), (1, 33), (33, 1), (1, 1), (129, 3)])
def test_ragged_and_degenerate_shapes(torch_mod, shape):
    torch = torch_mod
    nx, ny = shape
    rng = np.random.default_rng(nx * 100 + ny)
    logk = np.log(1e-12) + 0.7 * rng.standard_normal(nx * ny)
    prob = inputs.Problem(name=f"shape{nx}x{ny}", nx=nx, ny=ny, nz=1, logk=logk,
                          poro=np.full(nx * ny, 0.2), T0=np.full(nx * ny, 20.0), nsteps=2)
    _say(f"shape {shape}")
    T_gpu, _ = _run_gpu_linear(torch, prob, 2)
    T_ref, _ = oerem.run_linear(prob, nsteps=2)
    assert rel_inf(T_gpu - prob.T0, T_ref - prob.T0) <= TOL


def test_small_layered_3d(torch_mod):
    torch = torch_mod
    prob = inputs.layered3d_problem(10, seed=1, nsteps=2)
    _say("layered 3D 10^3")
    T_gpu, _ = _run_gpu_linear(torch, prob, 2)
    T_ref, _ = oerem.run_linear(prob, nsteps=2, layered=True)
    assert rel_inf(T_gpu - prob.T0, T_ref - prob.T0) <= TOL


def test_coupled_steps_match_oracle(torch_mod):
    """Sequential pressure / temperature steps with the water laws (48x48)."""
    torch = torch_mod
    prob = inputs.coupled_problem(48, seed=2, nsteps=3)
    _say("coupled 48x48 x 3")
    ctx = _ctx(prob)
    T = _dev(torch, prob.T0)
    p = torch.zeros(prob.n, dtype=torch.float64, device="cuda:0")
    for n in range(prob.nsteps):
        ctx.pressure_and_fluxes(T, rtol=1e-16, p=p, warm=n > 0)
        ctx.step(prob.h, T)
    T_gpu = T.cpu().numpy()
    T_ref = oerem.run_coupled(prob)
    err = rel_inf(T_gpu - prob.T0, T_ref - prob.T0)
    _say(f"  inc err {err:.2e}")
    assert err <= TOL


def test_coupled_steps_with_extrapolated_pressure_start_match_oracle(torch_mod):
    """The same sequential steps with each pressure solve started from the
    linear extrapolation of the last two pressures (warm = 2): the solve
    reaches the same tolerance, so the steps match the oracle as before."""
    torch = torch_mod
    prob = inputs.coupled_problem(48, seed=2, nsteps=4)
    ctx = _ctx(prob)
    T = _dev(torch, prob.T0)
    p = torch.zeros(prob.n, dtype=torch.float64, device="cuda:0")
    its = []
    for n in range(prob.nsteps):
        st = ctx.pressure_and_fluxes(T, rtol=1e-16, p=p if n == 0 else None, warm=2 if n > 0 else 0)
        its.append(st["iterations"])
        ctx.step(prob.h, T)
    T_ref = oerem.run_coupled(prob)
    err = rel_inf(T.cpu().numpy() - prob.T0, T_ref - prob.T0)
    _say(f"coupled 48x48 x 4, extrapolated pressure starts: CG iterations {its}, increment err {err:.2e}")
    assert err <= TOL


def test_coupled_512_one_step_full_size(torch_mod):
    """The 512x512 coupled workload at full size: one step against the
    sparse (tier B) oracle."""
    torch = torch_mod
    prob = inputs.coupled_problem(512)
    _say("coupled 512x512 one step")
    ctx = _ctx(prob)
    T = _dev(torch, prob.T0)
    st_p = ctx.pressure_and_fluxes(T, rtol=1e-16)
    st = ctx.step(prob.h, T)
    T_gpu = T.cpu().numpy()
    T_ref, _ = oerem.coupled_step(prob, prob.T0, tier="taylor")
    err = rel_inf(T_gpu, T_ref)
    inc = rel_inf(T_gpu - prob.T0, T_ref - prob.T0)
    _say(f"  pcg it={st_p['iterations']} m={st['m_total']} s={st['substeps']} err={err:.2e} inc={inc:.2e}")
    assert err <= TOL and inc <= TOL


# ---------------------------------------------------------------- Krylov

def _krylov_opts(m=10, **kw):
    from paper_1209_5553_amd.api import make_opts
    return make_opts(method=1, krylov_m=m, max_substeps=4096, **kw)


def test_krylov_phi1_apply_matches_dense_oracle(torch_mod):
    """Arnoldi (Alg. alg:al2) + phi1 of the augmented Hessenberg matrix
    (Eq. approphi), m = 10 as in the paper, against the oracle."""
    torch = torch_mod
    prob = inputs.linear_problem(32)
    disc = oerem.Discretisation(prob, prob.T0)
    ctx = _ctx(prob)
    ctx.set_face_fluxes(*_oracle_fluxes_to_dev(torch, disc))
    ctx.form_jacobian(_dev(torch, prob.T0))
    J = disc.model.J(prob.T0)
    v = np.random.default_rng(9).standard_normal(prob.n)
    for m in (10, 30):
        out, st = ctx.phi1_apply(prob.h, _dev(torch, v), opts=_krylov_opts(m))
        err = rel_inf(out.cpu().numpy(), ophi.phi1_action_dense(J, v, prob.h))
        _say(f"krylov m={m}: arnoldi steps={st['m_total']} substeps={st['substeps']} err={err:.2e}")
        assert err <= TOL


def test_krylov_full_dimension_is_exact(torch_mod):
    """With m = N the Krylov space is the whole space (happy breakdown): one
    substep reproduces phi1(hJ) v exactly (to rounding)."""
    torch = torch_mod
    prob = inputs.linear_problem(3, seed=2)
    disc = oerem.Discretisation(prob, prob.T0)
    ctx = _ctx(prob)
    ctx.set_face_fluxes(*_oracle_fluxes_to_dev(torch, disc))
    ctx.form_jacobian(_dev(torch, prob.T0))
    v = np.linspace(1.0, 3.0, prob.n)
    out, st = ctx.phi1_apply(prob.h, _dev(torch, v), opts=_krylov_opts(prob.n))
    ref = ophi.phi1_action_dense(disc.model.J(prob.T0), v, prob.h)
    _say(f"krylov m=N: {st}")
    assert st["substeps"] == 1
    assert rel_inf(out.cpu().numpy(), ref) <= 1e-12


def test_krylov_erem_32x32_ten_steps(torch_mod):
    torch = torch_mod
    prob = inputs.linear_problem(32)
    T_gpu, stats = _run_gpu_linear(torch, prob, prob.nsteps, opts=_krylov_opts(10))
    T_ref, _ = oerem.run_linear(prob)
    err = rel_inf(T_gpu - prob.T0, T_ref - prob.T0)
    _say(f"krylov EREM 10 steps: inc err {err:.2e}, last {stats[-1]}")
    assert err <= TOL


def test_krylov_and_leja_agree_on_coupled_step(torch_mod):
    torch = torch_mod
    prob = inputs.coupled_problem(64, seed=4)
    res = []
    for opts in (None, _krylov_opts(10)):
        ctx = _ctx(prob)
        T = _dev(torch, prob.T0)
        ctx.pressure_and_fluxes(T, rtol=1e-16)
        ctx.step(prob.h, T, opts)
        res.append(T.cpu().numpy())
    assert rel_inf(res[1] - prob.T0, res[0] - prob.T0) <= TOL


def test_krylov_ragged_grid_matches_taylor_oracle_and_repeats_bitwise(torch_mod):
    """Arnoldi across many 64 x 4 cell bands with ragged edges (200 x 70,
    m = 30): phi1(hJ) v against the oracle's sparse Taylor action (tier B),
    and a second evaluation is bit-for-bit the first (every inner product is
    reduced in a fixed order)."""
    torch = torch_mod
    nx, ny = 200, 70
    rng = np.random.default_rng(77)
    logk = np.log(1e-12) + 0.8 * rng.standard_normal(nx * ny)
    prob = inputs.Problem(name="krylov200x70", nx=nx, ny=ny, nz=1, logk=logk,
                          poro=np.full(nx * ny, 0.2), T0=np.full(nx * ny, 20.0), nsteps=1)
    disc = oerem.Discretisation(prob, prob.T0)
    ctx = _ctx(prob)
    ctx.set_face_fluxes(*_oracle_fluxes_to_dev(torch, disc))
    ctx.form_jacobian(_dev(torch, prob.T0))
    v = rng.standard_normal(prob.n)
    outs = []
    for _ in range(2):
        out, st = ctx.phi1_apply(prob.h, _dev(torch, v), opts=_krylov_opts(30))
        outs.append(out.cpu().numpy())
    ref = ophi.hphi1_action_taylor(disc.model.J_sparse(prob.T0), v, prob.h) / prob.h
    err = rel_inf(outs[0], ref)
    _say(f"krylov 200x70 m=30: arnoldi steps={st['m_total']} substeps={st['substeps']} err={err:.2e}")
    assert err <= TOL
    assert np.array_equal(outs[0], outs[1])


def test_krylov_3d_matches_dense_oracle(torch_mod):
    """The 7-point Arnoldi pass on a 10^3 layered grid against the dense
    phi1 (tier A)."""
    torch = torch_mod
    prob = inputs.layered3d_problem(10, seed=5)
    disc = oerem.Discretisation(prob, prob.T0)
    ctx = _ctx(prob)
    ctx.set_face_fluxes(*_oracle_fluxes_to_dev(torch, disc))
    ctx.form_jacobian(_dev(torch, prob.T0))
    v = np.random.default_rng(12).standard_normal(prob.n)
    out, st = ctx.phi1_apply(prob.h, _dev(torch, v), opts=_krylov_opts(20))
    err = rel_inf(out.cpu().numpy(), ophi.phi1_action_dense(disc.model.J(prob.T0), v, prob.h))
    _say(f"krylov 10^3 m=20: arnoldi steps={st['m_total']} substeps={st['substeps']} err={err:.2e}")
    assert err <= TOL


# ------------------------------------------------------- mixed precision

MIXED_TOL = 1e-5


def test_mixed_phi1_apply_matches_dense_oracle(torch_mod):
    """FP32 stencil / vectors / accumulation, FP64 divided differences, norms
    and update: within 1e-5 of the FP64 oracle."""
    torch = torch_mod
    from paper_1209_5553_amd.api import make_opts
    prob = inputs.linear_problem(32)
    disc = oerem.Discretisation(prob, prob.T0)
    ctx = _ctx(prob)
    ctx.set_face_fluxes(*_oracle_fluxes_to_dev(torch, disc))
    ctx.form_jacobian(_dev(torch, prob.T0))
    G = disc.model.G(prob.T0)
    out, st = ctx.phi1_apply(prob.h, _dev(torch, G), opts=make_opts(precision=1, tol_r=1e-7))
    ref = ophi.phi1_action_dense(disc.model.J(prob.T0), G, prob.h)
    err = rel_inf(out.cpu().numpy(), ref)
    _say(f"mixed phi1 m={st['m_total']} s={st['substeps']} err={err:.2e}")
    assert err <= MIXED_TOL


def test_mixed_steps_layered_3d_vs_oracle_and_fp64(torch_mod):
    torch = torch_mod
    from paper_1209_5553_amd.api import make_opts
    prob = inputs.layered3d_problem(12, seed=4, nsteps=3)
    T64, _ = _run_gpu_linear(torch, prob, 3)
    T32, _ = _run_gpu_linear(torch, prob, 3, opts=make_opts(precision=1, tol_r=1e-7))
    T_ref, _ = oerem.run_linear(prob, nsteps=3, layered=True)
    e32 = rel_inf(T32, T_ref)
    _say(f"mixed 3D err vs oracle {e32:.2e}, fp64 err {rel_inf(T64, T_ref):.2e}")
    assert rel_inf(T64, T_ref) <= TOL
    assert e32 <= MIXED_TOL
    assert rel_inf(T32 - prob.T0, T_ref - prob.T0) <= MIXED_TOL


def test_mixed_vs_fp64_full_size_layered_128(torch_mod):
    """The 128^3 layered workload, 10 steps: mixed precision against the FP64
    GPU path on the same inputs (the FP64 path is itself checked against the
    oracle on smaller grids and by linear exactness)."""
    torch = torch_mod
    from paper_1209_5553_amd.api import make_opts
    prob = inputs.layered3d_problem(128)
    _say("layered 128^3 x 10, FP64 and mixed")
    T64, s64 = _run_gpu_linear(torch, prob, prob.nsteps)
    T32, s32 = _run_gpu_linear(torch, prob, prob.nsteps, opts=make_opts(precision=1, tol_r=1e-7))
    err = rel_inf(T32, T64)
    inc = rel_inf(T32 - prob.T0, T64 - prob.T0)
    _say(f"  m64={s64[-1]['m_total']} m32={s32[-1]['m_total']} err={err:.2e} inc={inc:.2e}")
    assert err <= MIXED_TOL and inc <= MIXED_TOL


def test_full_size_layered_128_fp64_and_mixed_vs_oracle(torch_mod):
    """The 128^3 layered workload at full size against the oracle's sparse
    action (tier B, exact layered fluxes), one step, on every cell: FP64
    within 1e-10 and mixed precision within 1e-5, on T and on the increment."""
    torch = torch_mod
    from paper_1209_5553_amd.api import make_opts
    prob = inputs.layered3d_problem(128)
    _say("layered 128^3, one step: FP64 and mixed on the GPU, then the oracle (about 30 s)")
    T64, s64 = _run_gpu_linear(torch, prob, 1)
    T32, s32 = _run_gpu_linear(torch, prob, 1, opts=make_opts(precision=1, tol_r=1e-7))
    T_ref, _ = oerem.run_linear(prob, nsteps=1, tier="taylor", layered=True)
    e64, i64 = rel_inf(T64, T_ref), rel_inf(T64 - prob.T0, T_ref - prob.T0)
    e32, i32 = rel_inf(T32, T_ref), rel_inf(T32 - prob.T0, T_ref - prob.T0)
    _say(f"  m64={s64[-1]['m_total']} m32={s32[-1]['m_total']}: FP64 err {e64:.2e} inc {i64:.2e}; "
         f"mixed err {e32:.2e} inc {i32:.2e}")
    assert e64 <= TOL and i64 <= TOL
    assert e32 <= MIXED_TOL and i32 <= MIXED_TOL


def test_linear_exactness_full_size_layered_128(torch_mod):
    """Property at full size: ten steps of h equal one step of 10 h."""
    torch = torch_mod
    prob = inputs.layered3d_problem(128)
    T10, _ = _run_gpu_linear(torch, prob, 10)
    T1, _ = _run_gpu_linear(torch, prob, 1, h=10 * prob.h)
    assert rel_inf(T10 - prob.T0, T1 - prob.T0) <= TOL


# ------------------------------------------------------------ error paths

def test_error_paths_leave_T_unchanged(torch_mod):
    torch = torch_mod
    from paper_1209_5553_amd.api import EremError, make_opts
    prob = inputs.linear_problem(32)
    ctx = _ctx(prob)
    ctx.pressure_and_fluxes()
    T = _dev(torch, prob.T0)
    T0 = T.clone()
    with pytest.raises(EremError) as e:
        ctx.step(prob.h, T, make_opts(m_max=5, max_substeps=1, rho_max=0.0))
    assert e.value.code == -4
    assert torch.equal(T, T0)
    with pytest.raises(EremError) as e:
        ctx.step(0.0, T)
    assert e.value.code == -1
    Tn = T.clone()
    Tn[5] = float("nan")
    with pytest.raises(EremError) as e:
        ctx.step(prob.h, Tn)
    assert e.value.code == -5
    assert torch.isnan(Tn[5]) and torch.equal(Tn[:5], T0[:5])


def test_step_is_deterministic(torch_mod):
    torch = torch_mod
    prob = inputs.linear_problem(32)
    a, _ = _run_gpu_linear(torch, prob, 2)
    b, _ = _run_gpu_linear(torch, prob, 2)
    assert np.array_equal(a, b)


def test_coupled_512_steps_are_bitwise_reproducible(torch_mod):
    """Three steps of the 512x512 coupled workload (multigrid-preconditioned
    CG pressure with warm starts, assembly, Leja step), run twice in fresh
    contexts: every inner product is summed from per-band partials in a
    fixed order, so the two runs agree bit for bit (with 1024 blocks,
    atomically accumulated sums would not)."""
    torch = torch_mod
    prob = inputs.coupled_problem(512)
    runs = []
    for r in range(2):
        ctx = _ctx(prob)
        T = _dev(torch, prob.T0)
        p = torch.zeros(prob.n, dtype=torch.float64, device="cuda:0")
        iters = []
        for n in range(3):
            st = ctx.pressure_and_fluxes(T, rtol=1e-16, p=p if n == 0 else None, warm=n > 0)
            iters.append(st["iterations"])
            ctx.step(prob.h, T)
        torch.cuda.synchronize()
        runs.append((T.clone(), ctx.get_faces()["fx"].clone()))
        _say(f"coupled 512 run {r}: CG iterations {iters}")
    assert torch.equal(runs[0][0], runs[1][0])
    assert torch.equal(runs[0][1], runs[1][1])
