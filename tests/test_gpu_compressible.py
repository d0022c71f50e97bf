"""GPU parity of the transient (compressible) pressure step and the
sequential temperature + pressure step (Eq. masscon4, Eq. spaceheat3,
Eq. EERM1, Sec. 3.2.2) through the C ABI against the CPU oracle.

Per step: transmissibilities at T^n, the fluxes of p^n, the EREM temperature
step (Newton-Leja), then the EREM pressure step - Krylov (m = 10, the
paper's pairing) or Newton-Leja.  Both sides start from the workload's
initial pressure (linear in x).  Tolerance: 1e-10 relative (max norm) on T^n - T^0 and on
p^n - p^0."""
import numpy as np
import pytest

from oracle import compressible as oc
from paper_1209_5553_amd import inputs

from gpu_util import rel_inf

pytestmark = pytest.mark.gpu

TOL = 1e-10
AB, BF = inputs.ALPHA_B, inputs.BETA_F


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _popts(method):
    from paper_1209_5553_amd.api import make_opts
    if method == "krylov":
        return make_opts(method=1, krylov_m=10, max_substeps=4096, tol_r=1e-14)
    return make_opts(tol_r=1e-14, max_substeps=4096)


def _run_gpu(torch, prob, p0, nsteps, method):
    from paper_1209_5553_amd.api import EremContext
    ctx = EremContext.from_problem(prob, device="cuda:0")
    T = torch.as_tensor(prob.T0, dtype=torch.float64, device="cuda:0").clone()
    p = torch.as_tensor(p0, dtype=torch.float64, device="cuda:0").clone()
    stats = []
    for _ in range(nsteps):
        Tn = T.clone()
        ctx.assemble_transmissibilities(T)
        ctx.face_fluxes_from_pressure(p)
        st_T = ctx.step(prob.h, T)
        st_p = ctx.step_pressure(prob.h, p, Tn, AB, BF, _popts(method))
        stats.append((st_T, st_p))
    torch.cuda.synchronize()
    return T.cpu().numpy(), p.cpu().numpy(), stats


@pytest.mark.parametrize("method", ["krylov", "leja"])
@pytest.mark.parametrize("n", [8, 12])
def test_sequential_compressible_steps_match_oracle(torch_mod, n, method):
    prob = inputs.compressible_problem(n, seed=n)
    p0 = inputs.linear_pressure(prob)
    nsteps = 3
    _say(f"compressible {n}^3 ({prob.n} cells), pressure by {method}, {nsteps} steps")
    T, p, stats = _run_gpu(torch_mod, prob, p0, nsteps, method)
    _say(f"  last step: temperature {stats[-1][0]}; pressure {stats[-1][1]}")
    tier = "dense" if prob.n <= 700 else "taylor"
    Tr, pr = oc.run_sequential(prob, nsteps, prob.h, AB, BF, p0=p0, tier=tier)
    eT = rel_inf(T - prob.T0, Tr - prob.T0)
    ep = rel_inf(p - p0, pr - p0)
    _say(f"  rel err: T increment {eT:.2e}, p increment {ep:.2e} (max |dp| {np.abs(pr - p0).max():.3e} Pa)")
    assert eT <= TOL and ep <= TOL


def test_pressure_step_alone_with_water_law_2d(torch_mod):
    """A 2D grid with a random temperature field (alpha_f and rho vary) and
    a pressure away from steady state: one pressure step, G2 from the
    temperature step's assembly, Krylov."""
    torch = torch_mod
    from paper_1209_5553_amd.api import EremContext
    prob = inputs.coupled_problem(20, seed=7)
    rng = np.random.default_rng(7)
    prob.T0 = 20.0 + 60.0 * rng.random(prob.n)
    prob.dx = prob.dy = 50.0
    p0 = rng.uniform(0.0, prob.p_left, prob.n)
    h = 2.0e4
    ctx = EremContext.from_problem(prob, device="cuda:0")
    T = torch.as_tensor(prob.T0, dtype=torch.float64, device="cuda:0").clone()
    p = torch.as_tensor(p0, dtype=torch.float64, device="cuda:0").clone()
    ctx.assemble_transmissibilities(T)
    ctx.face_fluxes_from_pressure(p)
    ctx.form_jacobian(T)
    st = ctx.step_pressure(h, p, T, AB, BF, _popts("krylov"))
    torch.cuda.synchronize()
    import oracle.physics as ph
    from oracle import erem as oerem
    g = ph.grid_of(prob)
    mob = ph.mobility(prob.T0, prob.logk, prob.law, prob.rho0, prob.mu0)
    fl = ph.face_fluxes(p0, ph.tpfa_transmissibilities(mob, g), g, prob.p_left, prob.p_right)
    G2 = oerem.Discretisation(prob, prob.T0, fluxes=fl).model.G(prob.T0)
    ref = oc.pressure_step(prob, prob.T0, p0, G2, h, AB, BF, tier="dense")
    err = rel_inf(p.cpu().numpy() - p0, ref - p0)
    _say(f"2D pressure step: {st}, rel err {err:.2e}")
    assert err <= TOL


def test_full_size_compressible_50(torch_mod):
    """The 50^3 workload (125 000 cells, the pressure system size of the
    paper's first reservoir), one sequential step, every cell vs tier B."""
    prob = inputs.compressible_problem(50)
    p0 = inputs.linear_pressure(prob)
    T, p, stats = _run_gpu(torch_mod, prob, p0, 1, "krylov")
    _say(f"compressible 50^3: {stats}")
    Tr, pr = oc.run_sequential(prob, 1, prob.h, AB, BF, p0=p0, tier="taylor")
    eT = rel_inf(T - prob.T0, Tr - prob.T0)
    ep = rel_inf(p - p0, pr - p0)
    _say(f"  rel err: T increment {eT:.2e}, p increment {ep:.2e}")
    assert eT <= TOL and ep <= TOL


def test_bad_arguments_are_rejected(torch_mod):
    torch = torch_mod
    from paper_1209_5553_amd.api import EremContext, EremError
    prob = inputs.compressible_problem(6, seed=1)
    ctx = EremContext.from_problem(prob, device="cuda:0")
    T = torch.as_tensor(prob.T0, dtype=torch.float64, device="cuda:0").clone()
    p = torch.zeros_like(T)
    with pytest.raises(EremError):        # no transmissibilities yet
        ctx.face_fluxes_from_pressure(p)
    ctx.assemble_transmissibilities(T)
    ctx.face_fluxes_from_pressure(p)
    with pytest.raises(EremError):        # no G2 yet
        ctx.step_pressure(prob.h, p, T, AB, BF)
    ctx.form_jacobian(T)
    with pytest.raises(EremError):
        ctx.step_pressure(prob.h, p, T, 0.0, 0.0)
    torch.cuda.synchronize()
    assert torch.count_nonzero(p).item() == 0


def test_pressure_operator_is_not_taken_for_the_heat_operator(torch_mod):
    """After erem_step_pressure the context's stencil and right-hand side are
    J_p and G4: a second pressure step (which needs G2 = dT/dt) and every
    call that needs the heat Jacobian are rejected, with their outputs left
    unchanged, until erem_form_jacobian forms J and G2 again."""
    torch = torch_mod
    from paper_1209_5553_amd.api import EremContext, EremError
    prob = inputs.compressible_problem(6, seed=2)
    ctx = EremContext.from_problem(prob, device="cuda:0")
    T = torch.as_tensor(prob.T0, dtype=torch.float64, device="cuda:0").clone()
    p = torch.as_tensor(inputs.linear_pressure(prob), device="cuda:0").clone()
    ctx.assemble_transmissibilities(T)
    ctx.face_fluxes_from_pressure(p)
    ctx.form_jacobian(T)
    ctx.step_pressure(prob.h, p, T, AB, BF, _popts("leja"))
    p1 = p.clone()
    T1 = T.clone()
    with pytest.raises(EremError):        # G2 was overwritten by G4
        ctx.step_pressure(prob.h, p, T, AB, BF, _popts("leja"))
    with pytest.raises(EremError):
        ctx.step_frozen(prob.h, T)
    out = torch.zeros_like(T)
    with pytest.raises(EremError):
        ctx.phi1_apply(prob.h, T, out)
    with pytest.raises(EremError):
        ctx.get_jacobian()
    x = torch.zeros_like(T)
    with pytest.raises(EremError):
        ctx.shifted_solve(1.0 / prob.h, T, x)
    torch.cuda.synchronize()
    assert torch.equal(p, p1) and torch.equal(T, T1)
    assert torch.count_nonzero(out).item() == 0 and torch.count_nonzero(x).item() == 0
    ctx.form_jacobian(T)                  # J and G2 again: the pressure step runs
    ctx.step_pressure(prob.h, p, T, AB, BF, _popts("leja"))
    torch.cuda.synchronize()
    assert not torch.equal(p, p1)


def test_mixed_precision_pressure_close_to_fp64(torch_mod):
    """The Newton-Leja pressure passes in FP32 (the a10 form) stay within
    1e-5 of the FP64 GPU result on the increment."""
    from paper_1209_5553_amd.api import make_opts
    prob = inputs.compressible_problem(12, seed=21)
    p0 = inputs.linear_pressure(prob)

    def run(opts):
        from paper_1209_5553_amd.api import EremContext
        torch = torch_mod
        ctx = EremContext.from_problem(prob, device="cuda:0")
        T = torch.as_tensor(prob.T0, dtype=torch.float64, device="cuda:0").clone()
        p = torch.as_tensor(p0, dtype=torch.float64, device="cuda:0").clone()
        for _ in range(2):
            Tn = T.clone()
            ctx.assemble_transmissibilities(T)
            ctx.face_fluxes_from_pressure(p)
            ctx.step(prob.h, T)
            st = ctx.step_pressure(prob.h, p, Tn, AB, BF, opts)
        torch.cuda.synchronize()
        return p.cpu().numpy(), st

    p64, _ = run(make_opts(tol_r=1e-14, max_substeps=4096))
    p32, st = run(make_opts(precision=1, tol_r=1e-7, max_substeps=4096))
    err = rel_inf(p32 - p0, p64 - p0)
    _say(f"mixed-precision pressure: {st}, rel err vs FP64 {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 1, 1), (1, 4, 3)])
def test_compressible_degenerate_and_thin_grids(torch_mod, shape):
    """One cell (the pressure Jacobian is a scalar: the closed form replaces
    the Newton passes) and thin grids, the pressure by Leja; a long step
    (h = 1e7 s) so that T and p move by more than their last bits."""
    nx, ny, nz = shape
    base = inputs.compressible_problem(4, seed=31)
    rng = np.random.default_rng(nx + 10 * ny + 100 * nz)
    N = nx * ny * nz
    prob = inputs.Problem(name=f"thin_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                          logk=np.log(1e-13 * np.exp(rng.normal(0.0, 0.5, N))), poro=np.full(N, 0.3),
                          T0=60.0 + rng.random(N), law=inputs.LAW_WATER, p_left=1.0e6, T_left=10.0,
                          T_right=60.0, h=1.0e7, dx=base.dx, dy=base.dy, dz=base.dz)
    p0 = inputs.linear_pressure(prob)
    T, p, stats = _run_gpu(torch_mod, prob, p0, 2, "leja")
    _say(f"compressible {shape}: {stats[-1][1]}")
    Tr, pr = oc.run_sequential(prob, 2, prob.h, AB, BF, p0=p0, tier="dense")
    eT = rel_inf(T - prob.T0, Tr - prob.T0)
    ep = rel_inf(p - p0, pr - p0)
    _say(f"  rel err: T {eT:.2e}, p {ep:.2e} (max |dT| {np.abs(Tr - prob.T0).max():.3e} K, "
         f"max |dp| {np.abs(pr - p0).max():.3e} Pa)")
    assert eT <= TOL and ep <= TOL


def test_ten_sequential_steps_16(torch_mod):
    """Ten sequential steps on a 16^3 compressible grid (the pressure relaxes
    from its linear start), Krylov for the pressure as the paper pairs it."""
    prob = inputs.compressible_problem(16, seed=16)
    p0 = inputs.linear_pressure(prob)
    T, p, stats = _run_gpu(torch_mod, prob, p0, 10, "krylov")
    Tr, pr = oc.run_sequential(prob, 10, prob.h, AB, BF, p0=p0, tier="taylor")
    eT = rel_inf(T - prob.T0, Tr - prob.T0)
    ep = rel_inf(p - p0, pr - p0)
    _say(f"compressible 16^3 x 10: {stats[-1][1]}, rel err T {eT:.2e}, p {ep:.2e}")
    assert eT <= TOL and ep <= TOL
