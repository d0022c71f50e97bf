"""GPU parity of the batched persistent form (many ragged problems, one launch).

Each realisation of the batch must equal the single-problem HIP path (which
the oracle pins) to 1e-12, the oracle itself to 1e-10 on small grids, and the
FP32 variant the FP64 one to 1e-5.
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


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4])
def test_batch_every_tile_shape_matches_oracle(torch_mod, shape):
    """Every workgroup shape, on sides that span several 64 x 16 tiles with
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
    assert sa["graph"] == 1 and sb["graph"] == 1
    assert torch.equal(Ta, Tb)
    assert rel_inf(Ta.cpu().numpy(), Tc.cpu().numpy()) <= 1e-14
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
    assert shape in (0, 1, 2, 3, 4)
    assert torch.equal(T0, b.pack([p.T0 for p in probs]))   # autotune leaves T alone
    T = T0.clone()
    st = b.run(T, 2, use_graph=False)
    _say(f"autotuned shape {shape}: {st}")
    assert st["tile_shape"] == shape
    for p, Tg in zip(probs, b.unpack(T)):
        Ts = _single(torch, p, 2, make_opts(m_max=128))
        assert rel_inf(Tg - p.T0, Ts - p.T0) <= 1e-12


def test_batch_256_realisations_full_size(torch_mod):
    """The full workload: 256 realisations (seeds 0..255), 50 steps in one
    graph launch; sampled realisations against the single-problem path."""
    torch = torch_mod
    from paper_1209_5553_amd.api import EremBatch, make_opts
    probs = [inputs.batch_problem(s) for s in range(256)]
    b = EremBatch(probs, device="cuda:0")
    _say("256 problems set up")
    b.prepare(probs[0].h, make_opts(m_max=128))
    T = b.pack([p.T0 for p in probs])
    _say("prepared; running 256 x 50 in one graph launch")
    st = b.run(T, 50, use_graph=True)
    _say(f"256 x 50: {st}")
    assert st["failed"] == 0
    got = b.unpack(T)
    sides = np.array([p.nx for p in probs])
    sample = [int(np.argmin(sides)), int(np.argmax(sides)), 17, 130]
    for i in sample:
        Ts = _single(torch, probs[i], 50, make_opts(m_max=128))
        err = rel_inf(got[i] - probs[i].T0, Ts - probs[i].T0)
        _say(f"realisation {i} (side {sides[i]}): rel err {err:.3e}")
        assert err <= 1e-12, i
