"""The allocation-free evaluation erem_phi1_apply_noalloc against the
existing entry point it is a variant of (erem_set_jacobian + erem_phi1_apply)
on the same stencil and vector, through the C ABI: two calls in a row, the
second on a smaller grid (the scratch array keeps the first call's
contents), at the parity bar of the FP64 path (1e-10 relative, max norm);
and the limits rejected with EREM_EINVAL and the output left alone."""
import ctypes

import numpy as np
import pytest

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


def _problem_operator(torch, prob, T):
    """J (stencil) and G of a problem at T, from the library's assembly."""
    from paper_1209_5553_amd.api import EremContext
    ctx = EremContext.from_problem(prob, device="cuda:0")
    ctx.pressure_and_fluxes(T, rtol=1e-16)
    ctx.form_jacobian(T)
    coef, F = ctx.get_jacobian()
    torch.cuda.synchronize()
    return coef.contiguous().clone(), F.clone()


def _reference(torch, prob, coef, v, h, opts):
    """The existing entry points: erem_set_jacobian, then erem_phi1_apply."""
    from paper_1209_5553_amd.api import EremContext
    ctx = EremContext(prob.nx, prob.ny, prob.nz, prob.dx, prob.dy, prob.dz, device="cuda:0")
    ctx.set_jacobian(coef, torch.zeros_like(v))
    out, st = ctx.phi1_apply(h, v, opts=opts)
    torch.cuda.synchronize()
    return out, st


def _noalloc(torch, prob, coef, v, h, opts, out=None):
    from paper_1209_5553_amd import _native as nat
    lib = nat.load()
    grid = nat.Grid(3 if prob.nz > 1 else 2, prob.nx, prob.ny, prob.nz, prob.dx, prob.dy, prob.dz)
    out = torch.empty_like(v) if out is None else out
    st = nat.Stats()
    stream = torch.cuda.current_stream()
    rc = lib.erem_phi1_apply_noalloc(ctypes.byref(grid), ctypes.c_void_p(coef.data_ptr()), h,
                                     ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                     ctypes.byref(opts), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(st))
    return rc, out, st.as_dict()


def test_noalloc_matches_phi1_apply_twice_second_smaller(torch_mod):
    torch = torch_mod
    from paper_1209_5553_amd.api import make_opts
    opts = make_opts()
    cases = [inputs.coupled_problem(96, seed=4), inputs.linear_problem(40, seed=9)]
    for i, prob in enumerate(cases):
        rng = np.random.default_rng(50 + i)
        T = torch.as_tensor(rng.uniform(20.0, 80.0, prob.n), dtype=torch.float64, device="cuda:0")
        coef, F = _problem_operator(torch, prob, T)
        ref, st_ref = _reference(torch, prob, coef, F, prob.h, opts)
        rc, got, st = _noalloc(torch, prob, coef, F, prob.h, opts)
        torch.cuda.synchronize()
        assert rc == 0, rc
        err = rel_inf(got.cpu().numpy(), ref.cpu().numpy())
        _say(f"call {i + 1}: {prob.nx}x{prob.ny} ({prob.n} cells) m={st['m_total']} s={st['substeps']} "
             f"(phi1_apply m={st_ref['m_total']} s={st_ref['substeps']}), rel err {err:.2e}, "
             f"bitwise {torch.equal(got, ref)}")
        assert err <= 1e-10
        assert st["substeps"] == st_ref["substeps"] and st["m_total"] == st_ref["m_total"]


def test_noalloc_3d_after_2d(torch_mod):
    """A 7-point stencil after the 2D calls (one-term passes, other block count)."""
    torch = torch_mod
    from paper_1209_5553_amd.api import make_opts
    prob = inputs.layered3d_problem(20, seed=2)
    T = torch.as_tensor(np.random.default_rng(1).uniform(20.0, 80.0, prob.n), dtype=torch.float64,
                        device="cuda:0")
    coef, F = _problem_operator(torch, prob, T)
    opts = make_opts()
    ref, _ = _reference(torch, prob, coef, F, prob.h, opts)
    rc, got, st = _noalloc(torch, prob, coef, F, prob.h, opts)
    torch.cuda.synchronize()
    assert rc == 0
    err = rel_inf(got.cpu().numpy(), ref.cpu().numpy())
    _say(f"3D 20^3: m={st['m_total']} s={st['substeps']} rel err {err:.2e}")
    assert err <= 1e-10


def test_noalloc_limits_are_rejected(torch_mod):
    torch = torch_mod
    from paper_1209_5553_amd.api import make_opts
    prob = inputs.linear_problem(24, seed=1)
    T = torch.as_tensor(prob.T0, dtype=torch.float64, device="cuda:0")
    coef, F = _problem_operator(torch, prob, T)
    out = torch.full_like(F, 7.0)
    rc, _, _ = _noalloc(torch, prob, coef, F, prob.h, make_opts(m_max=300), out)
    assert rc == -1
    rc, _, _ = _noalloc(torch, prob, coef, F, prob.h, make_opts(precision=1, tol_r=1e-7), out)
    assert rc == -1
    big = inputs.Problem(name="big", nx=1024, ny=512, nz=1, logk=np.zeros(1), poro=np.zeros(1),
                         T0=np.zeros(1))
    rc, _, _ = _noalloc(torch, big, coef, F, prob.h, make_opts(), out)
    assert rc == -1
    rc, _, _ = _noalloc(torch, prob, coef, F, prob.h, make_opts(m_max=8, max_substeps=1, rho_max=0.0), out)
    assert rc == -4
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
