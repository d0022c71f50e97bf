"""GPU parity of the batched form (many ragged problems, one graph launch).

Each realisation of the batch must equal the oracle to 1e-10 (small grids,
and sampled realisations of the full 256-problem workload), the
single-problem HIP path to 1e-12, and in FP32 the oracle to 1e-5; graph and
host-driven runs agree bit for bit.
"""
import numpy as np
import pytest

from oracle import erem as oerem
from paper_1209_5553_amd import inputs

from gpu_util import rel_inf

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _single(torch, prob, nsteps, opts=None):
    from paper_1209_5553_amd.api import EremContext
    ctx = EremContext.from_problem(prob, device="cuda:0")
    ctx.pressure_and_fluxes(rtol=1e-16)
    T = torch.as_tensor(prob.T0, dtype=torch.float64, device="cuda:0").clone()
    for _ in range(nsteps):
        ctx.step(prob.h, T, opts)
    torch.cuda.synchronize()
    return T.cpu().numpy()


def _small_problems():
    out = []
    for i, n in enumerate((16, 24, 9, 32)):
        p = inputs.linear_problem(n, seed=10 + i)
        out.append(p)
    return out


def test_batch_small_matches_oracle(torch_mod):
    torch = torch_mod
    from paper_1209_5553_amd.api import EremBatch, make_opts
    probs = _small_problems()
    nsteps = 4
    b = EremBatch(probs, device="cuda:0")
    b.prepare(probs[0].h, make_opts(m_max=256))
    T = b.pack([p.T0 for p in probs])
    st = b.run(T, nsteps, use_graph=False)
    _say(f"small batch: {st}")
    got = b.unpack(T)
    for p, Tg in zip(probs, got):
        Tref, _ = oerem.run_linear(p, nsteps=nsteps)
        assert rel_inf(Tg - p.T0, Tref - p.T0) <= 1e-10, p.name


@pytest.mark.parametrize("shape", list(range(8)))
def test_batch_every_tile_shape_matches_oracle(torch_mod, shape):
    """Every tile shape, on sides that span several 64 x 16 tiles with
    ragged tails (70 x 70) and on grids smaller than one tile."""
    torch = torch_mod
    from paper_1209_5553_amd.api import EremBatch, make_opts
    probs = _small_problems() + [inputs.linear_problem(70, seed=20)]
    nsteps = 3
    b = EremBatch(probs, device="cuda:0")
    b.prepare(probs[0].h, make_opts(m_max=256))
    b.set_tile_shape(shape)
    T = b.pack([p.T0 for p in probs])
    st = b.run(T, nsteps, use_graph=False)
    _say(f"tile shape {shape}: {st}")
    assert st["tile_shape"] == shape and st["failed"] == 0
    for p, Tg in zip(probs, b.unpack(T)):
        Tref, _ = oerem.run_linear(p, nsteps=nsteps)
        assert rel_inf(Tg - p.T0, Tref - p.T0) <= 1e-10, (shape, p.name)


def test_batch_matches_single_problem_path(torch_mod):
    """Ragged sides drawn as in the 256-realisation workload (first 8 seeds)."""
    torch = torch_mod
    from paper_1209_5553_amd.api import EremBatch, make_opts
    probs = [inputs.batch_problem(s) for s in range(8)]
    nsteps = 5
    b = EremBatch(probs, device="cuda:0")
    b.prepare(probs[0].h, make_opts(m_max=128))
    T = b.pack([p.T0 for p in probs])
    st = b.run(T, nsteps, use_graph=False)
    _say(f"ragged batch: sides {[p.nx for p in probs]} {st}")
    for p, Tg in zip(probs, b.unpack(T)):
        Ts = _single(torch, p, nsteps, make_opts(m_max=128))
        assert rel_inf(Tg - p.T0, Ts - p.T0) <= 1e-12, p.name


def test_batch_graph_replay_and_fp32(torch_mod):
    torch = torch_mod
    from paper_1209_5553_amd.api import EremBatch, make_opts
    probs = [inputs.batch_problem(s) for s in range(8, 14)]
    nsteps = 3
    b = EremBatch(probs, device="cuda:0")
    b.prepare(probs[0].h, make_opts(m_max=128))
    T0 = b.pack([p.T0 for p in probs])
    Ta = T0.clone()
    sa = b.run(Ta, nsteps, use_graph=True)
    Tb = Ta.clone()
    Tb.copy_(T0)
    sb = b.run(Tb, nsteps, use_graph=True)   # new pointer: captured again
    Tc = T0.clone()
    sc = b.run(Tc, nsteps, use_graph=False)
    _say(f"graph runs: {sa} {sb} plain {sc}")
    assert sa["graph"] == 1 and sb["graph"] == 1 and sc["graph"] == 0
    assert torch.equal(Ta, Tb)
    assert torch.equal(Ta, Tc)      # fixed-order reductions: the same bits either way
    Td = T0.clone()
    b.run(Td, nsteps, use_graph=True)
    for _ in range(2):              # replays with eager work and syncs between them
        Td.copy_(T0)
        torch.cuda.synchronize()
        sd = b.run(Td, nsteps, use_graph=True)
        assert sd["graph"] == 1 and torch.equal(Td, Ta)
    # FP32 Newton passes
    b.prepare(probs[0].h, make_opts(m_max=128, precision=1, tol_r=1e-7))
    Tf = T0.clone()
    sf = b.run(Tf, nsteps, use_graph=False)
    _say(f"fp32 batch: {sf}")
    for g64, g32, p in zip(b.unpack(Ta), b.unpack(Tf), probs):
        assert rel_inf(g32, g64) <= 1e-5 and rel_inf(g32 - p.T0, g64 - p.T0) <= 1e-5


def test_batch_autotune_picks_a_shape_and_results_agree(torch_mod):
    torch = torch_mod
    from paper_1209_5553_amd.api import EremBatch, make_opts
    probs = [inputs.batch_problem(s) for s in range(20, 24)]
    b = EremBatch(probs, device="cuda:0")
    b.prepare(probs[0].h, make_opts(m_max=128))
    T0 = b.pack([p.T0 for p in probs])
    shape = b.autotune(T0, nsteps=1)
    assert shape in range(8)
    assert torch.equal(T0, b.pack([p.T0 for p in probs]))   # autotune leaves T alone
    T = T0.clone()
    st = b.run(T, 2, use_graph=False)
    _say(f"autotuned shape {shape}: {st}")
    assert st["tile_shape"] == shape
    for p, Tg in zip(probs, b.unpack(T)):
        Ts = _single(torch, p, 2, make_opts(m_max=128))
        assert rel_inf(Tg - p.T0, Ts - p.T0) <= 1e-12


def test_batch_graph_budget_exceeded_continues_from_host(torch_mod):
    """A graph captured for a start that needs almost no Newton terms (each
    realisation's steady state, where G(T) = 0 up to rounding), replayed on
    the workload's start: the run goes on with launches from the host where
    the graph's passes end, with the same result, bit for bit, as a run
    without the graph, and the oracle's."""
    import scipy.sparse.linalg as spla
    torch = torch_mod
    from paper_1209_5553_amd.api import EremBatch, make_opts
    probs = [inputs.batch_problem(s) for s in range(30, 34)]
    nsteps = 2
    b = EremBatch(probs, device="cuda:0")
    b.prepare(probs[0].h, make_opts(m_max=256))
    steady = []
    for p in probs:
        m = oerem.Discretisation(p, p.T0).model
        steady.append(spla.spsolve(m.A.tocsc(), -m.b))
    T = b.pack(steady)
    sg = b.run(T, nsteps, use_graph=True)           # calibrated and captured on the steady start
    T.copy_(b.pack([p.T0 for p in probs]))
    sr = b.run(T, nsteps, use_graph=True)           # same array: the same graph, too short
    Te = b.pack([p.T0 for p in probs])
    se = b.run(Te, nsteps, use_graph=False)
    _say(f"steady start {sg}; workload start through the graph {sr}; without {se}")
    assert sr["graph"] == 1 and sr["failed"] == 0
    assert sr["passes"] > sg["passes"]               # launched past the end of the graph
    assert torch.equal(T, Te)
    for p, Tg in zip(probs, b.unpack(Te)):
        Tref, _ = oerem.run_linear(p, nsteps=nsteps, tier="taylor")
        assert rel_inf(Tg - p.T0, Tref - p.T0) <= 1e-10, p.name


@pytest.fixture(scope="module")
def full_batch(torch_mod):
    """The full workload's 256 realisations (seeds 0..255) set up once."""
    from paper_1209_5553_amd.api import EremBatch
    probs = [inputs.batch_problem(s) for s in range(256)]
    b = EremBatch(probs, device="cuda:0")
    _say(f"256 problems set up ({b.ntot} cells)")
    yield probs, b
    b.close()


def _sample_of(probs):
    """The smallest and the largest realisation and two drawn at random."""
    sides = np.array([p.nx for p in probs])
    rnd = np.random.default_rng(7).choice(len(probs), 2, replace=False)
    return [int(np.argmin(sides)), int(np.argmax(sides))] + [int(i) for i in rnd]


def test_batch_256_first_steps_match_oracle(torch_mod, full_batch):
    """The full 256-realisation launch, 3 steps, FP64 and FP32 Newton passes:
    the smallest, the largest and two random realisations on every cell
    against the oracle's sparse action (1e-10 FP64, 1e-5 FP32)."""
    from paper_1209_5553_amd.api import make_opts
    probs, b = full_batch
    nsteps = 3
    T0 = b.pack([p.T0 for p in probs])
    b.prepare(probs[0].h, make_opts(m_max=128))
    T64 = T0.clone()
    st = b.run(T64, nsteps, use_graph=True)
    _say(f"256 x {nsteps} FP64: {st}")
    assert st["failed"] == 0
    b.prepare(probs[0].h, make_opts(m_max=128, precision=1, tol_r=1e-7))
    T32 = T0.clone()
    st = b.run(T32, nsteps, use_graph=True)
    _say(f"256 x {nsteps} FP32: {st}")
    assert st["failed"] == 0
    g64, g32 = b.unpack(T64), b.unpack(T32)
    for i in _sample_of(probs):
        p = probs[i]
        Tref, _ = oerem.run_linear(p, nsteps=nsteps, tier="taylor")
        e64 = rel_inf(g64[i] - p.T0, Tref - p.T0)
        e32 = rel_inf(g32[i] - p.T0, Tref - p.T0)
        _say(f"realisation {i} (side {p.nx}): FP64 increment err {e64:.3e}, FP32 {e32:.3e}, "
             f"FP32 T err {rel_inf(g32[i], Tref):.3e}")
        assert e64 <= 1e-10, i
        assert e32 <= 1e-5 and rel_inf(g32[i], Tref) <= 1e-5, i


def test_batch_256_realisations_full_size(torch_mod, full_batch):
    """The full workload: 256 realisations (seeds 0..255), 50 steps in one
    graph launch; sampled realisations against the single-problem path."""
    torch = torch_mod
    from paper_1209_5553_amd.api import make_opts
    probs, b = full_batch
    b.prepare(probs[0].h, make_opts(m_max=128))
    T = b.pack([p.T0 for p in probs])
    _say("prepared; running 256 x 50 in one graph launch")
    st = b.run(T, 50, use_graph=True)
    _say(f"256 x 50: {st}")
    assert st["failed"] == 0
    got = b.unpack(T)
    sides = np.array([p.nx for p in probs])
    for i in _sample_of(probs):
        Ts = _single(torch, probs[i], 50, make_opts(m_max=128))
        err = rel_inf(got[i] - probs[i].T0, Ts - probs[i].T0)
        _say(f"realisation {i} (side {sides[i]}): rel err {err:.3e}")
        assert err <= 1e-12, i


def _rect_problem(nx, ny, seed):
    rng = np.random.default_rng(seed)
    logk = np.log(1e-12) + 0.7 * rng.standard_normal(nx * ny)
    return inputs.Problem(name=f"rect{nx}x{ny}", nx=nx, ny=ny, nz=1, logk=logk,
                          poro=np.full(nx * ny, 0.2), T0=np.full(nx * ny, 20.0), nsteps=2)


@pytest.mark.parametrize("shape", [0, 5, 7])
def test_batch_degenerate_and_rectangular_problems_match_oracle(torch_mod, shape):
    """Two cells, a single row and a single column, and rectangles ragged in
    both directions (65 x 17, 130 x 3, 3 x 130, one exact 64 x 16 tile) in
    one batch, for a four-term and both eight-term tile shapes: every
    realisation against the oracle.  The stiff thin grids (h (beta - alpha)
    up to 5500) run at the 64-substep cap."""
    from paper_1209_5553_amd.api import EremBatch, make_opts
    sides = [(2, 1), (1, 40), (40, 1), (65, 17), (130, 3), (3, 130), (64, 16)]
    probs = [_rect_problem(nx, ny, seed=40 + i) for i, (nx, ny) in enumerate(sides)]
    nsteps = 2
    b = EremBatch(probs, device="cuda:0")
    b.prepare(probs[0].h, make_opts(m_max=256))
    b.set_tile_shape(shape)
    T = b.pack([p.T0 for p in probs])
    st = b.run(T, nsteps, use_graph=True)
    _say(f"degenerate batch, shape {shape}: {st}")
    assert st["failed"] == 0
    for p, Tg in zip(probs, b.unpack(T)):
        Tref, _ = oerem.run_linear(p, nsteps=nsteps)
        assert rel_inf(Tg - p.T0, Tref - p.T0) <= 1e-10, (shape, p.name)


def test_batch_problem_over_the_term_budget_fails_alone(torch_mod):
    """Substeps capped at two: a stiff two-cell problem (h (beta - alpha)
    about 1200) cannot meet the tolerance within m_max terms of a substep of
    600, while a workload realisation (one substep) converges.  The run
    reports the failure, the failed problem keeps its initial temperatures,
    and the other one is bit for bit what it is in a batch of its own."""
    torch = torch_mod
    from paper_1209_5553_amd.api import EremBatch, EremError, make_opts
    p_hard = _rect_problem(2, 1, seed=47)
    p_easy = inputs.batch_problem(41)
    opts = make_opts(m_max=128, max_substeps=2)
    solo = EremBatch([p_easy], device="cuda:0")
    solo.prepare(p_easy.h, opts)
    solo.set_tile_shape(5)
    Ts = solo.pack([p_easy.T0])
    st = solo.run(Ts, 1, use_graph=False)
    assert st["failed"] == 0
    b = EremBatch([p_hard, p_easy], device="cuda:0")
    b.prepare(p_easy.h, opts)
    b.set_tile_shape(5)
    T = b.pack([p_hard.T0, p_easy.T0])
    with pytest.raises(EremError) as ei:
        b.run(T, 1, use_graph=False)
    _say(f"over budget: {ei.value}")
    assert "ENOCONV" in str(ei.value) or "ENONFINITE" in str(ei.value)
    hard, easy = b.unpack(T)
    assert np.array_equal(hard, p_hard.T0)
    assert np.array_equal(easy, solo.unpack(Ts)[0])


def test_batch_rejects_a_degenerate_interval(torch_mod):
    """A one-cell problem has J = c I (alpha = beta): the batched form, which
    fixes one Leja interval per problem, refuses it at prepare with
    EREM_EINVAL (the single-problem path takes the closed form instead)."""
    from paper_1209_5553_amd.api import EremBatch, EremError, make_opts
    probs = [_rect_problem(1, 1, seed=3), _rect_problem(16, 16, seed=4)]
    b = EremBatch(probs, device="cuda:0")
    with pytest.raises(EremError) as ei:
        b.prepare(probs[0].h, make_opts(m_max=128))
    assert "EINVAL" in str(ei.value)


def test_batch_wide_substeps_match_oracle(torch_mod):
    """The benchmark's FP64 setting, substep intervals up to 96 wide
    (rho_max = 96, m_max = 128): the realisations of the workload with the
    widest substeps at that setting (h (beta - alpha) of 96.0, 95.9, 186.0,
    183.8 and 208.1, seeds 205, 118, 207, 94 and 74) after three steps
    against the oracle on every cell."""
    from paper_1209_5553_amd.api import EremBatch, make_opts
    seeds = (205, 118, 207, 94, 74)
    probs = [inputs.batch_problem(s) for s in seeds]
    nsteps = 3
    b = EremBatch(probs, device="cuda:0")
    b.prepare(probs[0].h, make_opts(m_max=128, rho_max=96.0))
    T = b.pack([p.T0 for p in probs])
    st = b.run(T, nsteps, use_graph=True)
    _say(f"rho_max 96: {st}")
    assert st["failed"] == 0
    for s, p, Tg in zip(seeds, probs, b.unpack(T)):
        Tref, _ = oerem.run_linear(p, nsteps=nsteps, tier="taylor")
        err = rel_inf(Tg - p.T0, Tref - p.T0)
        _say(f"seed {s} (side {p.nx}): increment err {err:.2e}")
        assert err <= 1e-10, s
