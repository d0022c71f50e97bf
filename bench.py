#!/usr/bin/env python3
"""Benchmark of the MI355X EREM path (one GPU).

Default workload: the batched form, 256 linear heat-transport realisations
(seeds 0..255, square grids with sides drawn from {64, 96, 128, 192, 256},
7.16 M cells in all, log-normal permeability sigma = 1 / correlation 4
cells, 1 MPa pressure drop), 50 EREM steps of h = 1e6 s each with the
real-Leja phi1 (FP64), replayed from one hipGraph; a step is one EREM step
of all 256 realisations.  This is the largest single-GPU workload and the
one whose Newton passes do not fit the 256 MB Infinity Cache.  Inputs are
synthetic (seeded generators) and already resident in HBM when timing
starts.

Other workloads (--workload): coupled512 (the 512 x 512 sequential coupled
problem: TPFA transmissibilities at T^n, steady pressure, EREM temperature
step), linear32, layered128 and layered256 (3D, --precision mixed for the
FP32 Newton passes), injector512 (the non-autonomous step with the phi2
term), compressible50 (the sequential step with a transient pressure,
--pressure-method leja|krylov), adjoint256 (a coupled step and its
adjoint).  --scheme runs the coupled workload with a comparison scheme
instead of EREM (ROSM(1), ROSM(1/2), ROS2(1), ROS3p, theta-Euler 1/2 or 1
with Newton's method).

Prints ONE JSON line: steps/s over the timed steps, the roofline of the
dominant kernel (HIP-event timing of a sample of the launches inside the
timed region, one in PROFILE_STRIDE), the Leja term kernel's own figures,
the measured copy and triad bandwidth of the device beside its 8 TB/s
peak, and the CPU oracle timed on a bounded sample beside it (with the
GPU/oracle agreement on that sample).

Roofline labels: "achieved" is the algorithmic bytes of a launch (one pass
per Newton term; see LEJA_BYTES) over its measured duration.  A kernel whose
per-launch working set fits the 256 MB Infinity Cache, or that moves fewer
bytes than its algorithmic count (the four-term passes keep the
intermediate terms on chip), has "bound": "effective": its rate is not an
HBM rate and can exceed the HBM peak.  "hbm" then gives the memory-side
rate: the counter-measured bytes ("traffic") over the same duration.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "EREM steps/s & Leja SpMV GB/s (% of HBM peak) at 1e-10 rel. err vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
MALL_BYTES = 256e6      # Infinity Cache: working sets below this are cache-resident
# Kernel timing inside the timed region: HIP events around one launch in
# PROFILE_STRIDE (Newton terms and CG iterations whose index is a multiple of
# it), which keeps the event overhead out of most of the timed steps.
PROFILE_STRIDE = 4

# Algorithmic bytes per cell per launch (one pass per launch; stencil
# structure implicit; halo re-reads counted once).
LEJA_BYTES = {2: {"f64": 72, "f32": 36}, 3: {"f64": 88, "f32": 44}}
PCG_A_BYTES = {2: 48, 3: 64}    # read z, p_old, face transmissibilities; write p_new, q
PCG_B_BYTES = {2: 48, 3: 48}    # read x, p_new, r, q; write x, r (multigrid-preconditioned)
# One BiCGSTAB iteration of the comparison schemes (three kernels): K1 reads
# r, p, v (with halos), the stencil and rhat and writes p, v; K2 reads r, v
# and the stencil and writes s, t; K3 reads x, p, s, t, the diagonal and rhat
# and writes x, r.
BICG_BYTES = {2: 88 + 72 + 64, 3: 104 + 88 + 64}
SCHEMES = ("erem", "rosm1", "rosm05", "ros2", "ros3p", "theta05", "theta1")
# One multigrid V-cycle per finest cell: on the finest level the four passes
# (two-sweep smoothing, residual + restriction, prolongation + sweep, sweep)
# read b, diag, faces and the iterate and write one vector each (~180 B);
# the coarser levels add a third of that (2 x 2 aggregation).
MG_BYTES = {2: 240, 3: 240}
# On 2D grids a whole Chronopoulos-Gear CG iteration runs inside the finest
# legs of the V-cycle: the first down leg reads w, s_old, z, p, x and writes
# r_new, s, p, x (r itself is the cycle's right-hand side); the last up leg
# also writes w = A z.
CG_FUSED_BYTES = 80


def mg_bytes(times, dim):
    """Algorithmic bytes per cell of one preconditioner application."""
    fused = times["pcg_a_launches"] == 0 and times["mg_cycles"] > 0
    return MG_BYTES[dim] + (CG_FUSED_BYTES if fused else 0)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    from paper_1209_5553_amd import inputs
    if name == "coupled512":
        prob = inputs.coupled_problem(512)
        desc = ("coupled 2D 512x512: TPFA steady pressure (water laws, sigma_logK=2, corr 16, "
                "Pe~100) + EREM-Leja temperature step, h=1e6 s")
        return prob, desc, True
    if name == "linear32":
        prob = inputs.linear_problem(32)
        desc = "linear 2D 32x32 heat transport, fixed Darcy field, EREM-Leja, h=1e6 s"
        return prob, desc, False
    if name == "injector512":
        prob = inputs.injector_problem(512)
        desc = ("non-autonomous 2D 512x512 heat transport, fixed Darcy field (sigma_logK=2, corr 16, "
                "Pe~100), injection temperature 50+30 sin(2 pi t / 20h) C: EREM-Leja with the phi2 "
                "term (Eq. nEERMg), h=1e6 s")
        return prob, desc, False
    if name == "compressible50":
        prob = inputs.compressible_problem(50)
        desc = ("sequential 3D 50^3 (1 km x 1 km x 0.1 km, two layers 0.01/0.1 D, water laws) with a transient "
                "pressure (alpha_b=1e-7, beta_f=4.5e-10 1/Pa): fluxes of p^n, EREM-Leja temperature step, "
                "EREM pressure step (Eq. EERM1), h=2e4 s")
        return prob, desc, False
    if name in ("layered128", "layered256"):
        n = int(name[len("layered"):])
        prob = inputs.layered3d_problem(n)
        desc = f"linear 3D {n}^3 7-point heat transport, layered K (3 decades), EREM-Leja, h=1e6 s"
        return prob, desc, False
    raise SystemExit(f"unknown workload {name}")


def schedule_of(name):
    """Boundary schedule of a non-autonomous workload, else None."""
    from paper_1209_5553_amd import inputs
    return inputs.InjectorSchedule() if name == "injector512" else None


def gpu_run(prob, coupled, steps, warmup, rtol_p, mixed=False, sched=None, scheme="erem", pmethod="leja",
            rho_max=None):
    import torch
    from paper_1209_5553_amd.api import EremContext, make_opts

    ctx = EremContext.from_problem(prob, device="cuda:0")
    dev = ctx.device
    T = torch.as_tensor(prob.T0, dtype=torch.float64, device=dev).clone()
    p = torch.zeros(prob.n, dtype=torch.float64, device=dev)
    extra = {} if rho_max is None else {"rho_max": rho_max}
    opts = make_opts(precision=1, tol_r=1e-7, **extra) if mixed else make_opts(**extra)
    state = {"n": 0, "last": None, "pcg": 0}

    comp = prob.name.startswith("compressible")
    if comp:
        from paper_1209_5553_amd import inputs
        pc = torch.as_tensor(inputs.linear_pressure(prob), device=dev)
        Tn = torch.empty_like(T)
        popts = (make_opts(method=1, krylov_m=10, max_substeps=4096, tol_r=1e-14) if pmethod == "krylov"
                 else make_opts(tol_r=1e-14, max_substeps=4096))
    elif not coupled:
        st = ctx.pressure_and_fluxes(rtol=rtol_p)

    def one_step():
        if comp:
            # transmissibilities at T^n, fluxes of p^n, temperature, then pressure at T^n
            Tn.copy_(T)
            ctx.assemble_transmissibilities(T)
            ctx.face_fluxes_from_pressure(pc)
            state["last"] = ctx.step(prob.h, T, opts)
            state["plast"] = ctx.step_pressure(prob.h, pc, Tn, inputs.ALPHA_B, inputs.BETA_F, popts)
            state["n"] += 1
            return
        if coupled:
            # the pressure stays resident in the context: after the first
            # step each solve starts from the linear extrapolation of the
            # last two pressures
            sp = ctx.pressure_and_fluxes(T, rtol=rtol_p, p=p if state["n"] == 0 else None,
                                         warm=2 if state["n"] > 0 else 0)
            state["pcg"] += sp["iterations"]
        if sched is not None:
            # boundary temperatures and their rates at t_n = n h
            state["last"] = ctx.step_nonautonomous(prob.h, T, *sched(state["n"] * prob.h), opts)
        elif scheme.startswith("theta"):
            state["last"] = ctx.step_theta(prob.h, T, 0.5 if scheme == "theta05" else 1.0)
        elif scheme != "erem":
            state["last"] = ctx.step_rosenbrock(prob.h, T, scheme)
        else:
            state["last"] = ctx.step(prob.h, T, opts)
        state["n"] += 1

    snapshots = {}
    for w in range(warmup):
        one_step()
        if state["n"] <= 3:
            snapshots[state["n"]] = T.clone()
            if comp:
                snapshots[("p", state["n"])] = pc.clone()
    log(f"warmup done ({warmup} steps), last stats {state['last']}")
    torch.cuda.synchronize()
    ctx.profile(True, stride=PROFILE_STRIDE)
    state["pcg"] = 0
    m_total = 0
    lin_total = 0
    pm_total = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step()
        m_total += state["last"]["m_total"]
        lin_total += state["last"]["iterations"]
        if comp:
            pm_total += state["plast"]["m_total"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    times = ctx.profile_read()
    ctx.profile(False)
    log(f"timed {steps} steps in {t1 - t0:.3f} s; kernel times {times}")
    snaps = {k: v.cpu().numpy() for k, v in snapshots.items()}
    return dict(elapsed=t1 - t0, times=times, m_per_step=m_total / steps, lin_per_step=lin_total / steps,
                pressure_m_per_step=pm_total / steps if comp else None, plast=state.get("plast"),
                pcg_per_step=state["pcg"] / steps, last=state["last"], snapshots=snaps,
                T_final=T.cpu().numpy())


def cpu_baseline(prob, coupled, nsteps, gpu_snaps, sched=None, scheme="erem"):
    """The oracle as it stands, on a bounded sample: the first `nsteps` steps
    of the same workload (tier-B sparse action; SuperLU pressure with extended-precision refinement)."""
    from threadpoolctl import threadpool_limits

    from oracle import erem as oerem
    if prob.n > 4_000_000:
        return cpu_baseline_scaled(prob)
    # the dense tier (small linear grids) runs its matrix products on every
    # host core the GPU's share allows; the sparse tiers are single-threaded
    dense = (not coupled and sched is None and not prob.name.startswith("compressible") and prob.n <= 4096)
    threads = min(16, os.cpu_count() or 1) if dense else 1
    with threadpool_limits(limits=threads):
        T = np.asarray(prob.T0, dtype=np.float64).copy()
        t0 = time.perf_counter()
        if coupled and scheme != "erem":
            from oracle import rosenbrock as oros
            for _ in range(nsteps):
                T = oros.coupled_step_scheme(prob, T, scheme)
        elif coupled:
            for _ in range(nsteps):
                T, _ = oerem.coupled_step(prob, T, tier="taylor")
        elif sched is not None:
            T, _ = oerem.run_nonautonomous(prob, sched, nsteps=nsteps, tier="taylor")
        elif prob.name.startswith("compressible"):
            from oracle import compressible as ocomp
            from paper_1209_5553_amd import inputs
            T, P = ocomp.run_sequential(prob, nsteps, prob.h, inputs.ALPHA_B, inputs.BETA_F,
                                        p0=inputs.linear_pressure(prob), tier="taylor")
        else:
            tier = "dense" if dense else "taylor"
            layered = prob.nz > 1
            T, _ = oerem.run_linear(prob, nsteps=nsteps, tier=tier, layered=layered)
        t1 = time.perf_counter()
    out = {"value": nsteps / (t1 - t0), "unit": "steps/s", "cores": threads, "kind": "oracle",
           "sample": f"first {nsteps} steps of the same workload from T0 "
                     f"({'SuperLU pressure refined in extended precision + ' if coupled else ''}"
                     + (f"{scheme} with sparse LU stage solves" if scheme != "erem" else
                        "temperature and pressure by the substepped Taylor action of their augmented exponentials"
                        if prob.name.startswith("compressible") else
                        ("dense augmented exponential (Taylor scaling and squaring)" if dense else
                         f"substepped Taylor action of the augmented exponential"
                         f"{' with the two extra rows of the phi2 term' if sched else ''}"))
                     + f", FP64, {threads} thread{'s' if threads > 1 else ''})",
           "seconds": t1 - t0, **cpu_info()}
    if ("p", nsteps) in gpu_snaps:
        from paper_1209_5553_amd import inputs
        p0 = inputs.linear_pressure(prob)
        out["gpu_pressure_increment_rel_err"] = float(np.abs((gpu_snaps[("p", nsteps)] - p0) - (P - p0)).max()
                                                      / np.abs(P - p0).max())
    if nsteps in gpu_snaps:
        Tg = gpu_snaps[nsteps]
        out["gpu_rel_err"] = float(np.abs(Tg - T).max() / np.abs(T).max())
        out["gpu_increment_rel_err"] = float(np.abs((Tg - prob.T0) - (T - prob.T0)).max()
                                             / np.abs(T - prob.T0).max())
    return out


def cpu_baseline_scaled(prob):
    """Grids too large for a bounded oracle run (the 256^3 layered workload):
    one oracle step of the same recipe at half the side (1/8 of the cells),
    scaled by the cell count."""
    from threadpoolctl import threadpool_limits

    from oracle import erem as oerem
    from paper_1209_5553_amd import inputs
    small = inputs.layered3d_problem(prob.nx // 2)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oerem.run_linear(small, nsteps=1, tier="taylor", layered=True)
        t1 = time.perf_counter()
    scale = prob.n / small.n
    return {"value": 1.0 / ((t1 - t0) * scale), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 step of the same recipe on {small.nx}^3 ({small.n} cells, substepped Taylor action, "
                      f"FP64, 1 thread), scaled by the cell count ({scale:.0f}x); no GPU comparison at this size",
            "seconds": t1 - t0, **cpu_info()}


# Reverse Newton-Leja term (adjoint): read s_k, q_{k-1}, the stencil, ubar,
# the five Jbar accumulators; write Jbar and s_{k-1}.
ADJ_REV_BYTES = 8 + 8 + 40 + 8 + 80 + 8


BATCH_RHO_MAX = 96.0   # widest substep interval h (beta - alpha) / s of the batched FP64 passes


def bench_batch(args, mixed):
    """256 realisations (seeds 0..255, sides from {64, 96, 128, 192, 256}),
    50 EREM steps per run.  The timed region holds `steps` runs replayed
    from the hipGraph and one more run enqueued from the host in which every
    PROFILE_STRIDE-th work launch is timed by its dispatch's events (the
    roofline's launch duration); value counts all of them."""
    import torch
    from paper_1209_5553_amd import inputs
    from paper_1209_5553_amd.api import EremBatch, make_opts

    nprob, nst = 256, 50
    probs = [inputs.batch_problem(s) for s in range(nprob)]
    b = EremBatch(probs, device="cuda:0")
    # FP64 passes on substep intervals up to 96 wide (the single-problem
    # default is 64): fewer, longer substeps need about 15% fewer Newton terms
    # and stay within 1e-12 of the oracle on the widest realisations; FP32
    # passes keep their cap of 32
    opts = (make_opts(m_max=128, precision=1, tol_r=1e-7) if mixed
            else make_opts(m_max=128, rho_max=BATCH_RHO_MAX))
    b.prepare(probs[0].h, opts)
    T0 = b.pack([p.T0 for p in probs])
    if args.tile_shape is None:
        shape = b.autotune(T0, nsteps=5)
    else:
        shape = args.tile_shape
        b.set_tile_shape(shape)
    log(f"batch: {nprob} problems, {b.ntot} cells, "
        f"{'autotuned' if args.tile_shape is None else 'requested'} tile shape {shape}")
    T = T0.clone()
    for _ in range(max(1, args.warmup)):
        T.copy_(T0)
        st = b.run(T, nst, use_graph=True)
    log(f"warmup done: {st}")
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        T.copy_(T0)
        runs.append(b.run(T, nst, use_graph=True))
    T.copy_(T0)
    b.profile(PROFILE_STRIDE)
    prof = b.run(T, nst, use_graph=True)      # enqueued from the host while profiling
    b.profile(0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"graph runs {[round(r['ms'], 3) for r in runs]} ms; profiled run {prof}")
    nruns = len(runs) + 1
    passes = prof["passes"]
    avg_work_s = prof["work_ms"] * 1e-3 / max(prof["work_timed"], 1)
    byts = prof["leja_bytes"]
    kname = "k_bt_work"
    tr = _traffic("batch256", args.precision, f"{kname}/shape{shape}")   # counters are per tile shape
    roof = roofline_entry(kname, byts / passes, avg_work_s, int(passes),
                          traffic=None if tr is None else tr / passes,
                          working_set=(36 if mixed else 72) * b.ntot)
    roof["bytes_rule"] = (f"Newton terms only (start and finish passes not counted): sum over problems of "
                          f"terms x cells x {36 if mixed else 72} B, spread over the {passes} work launches of a run")
    roof["timing"] = (f"dispatch events of every {PROFILE_STRIDE}th work launch of the host-enqueued run "
                      f"({prof['work_timed']} launches)")
    roof["share_of_run"] = round(avg_work_s * passes / (prof["ms"] * 1e-3), 4)
    desc = (f"batched: {nprob} linear 2D realisations (seeds 0..{nprob - 1}, sides from {list(inputs.C3_SIDES)}), "
            f"{nst} EREM-Leja steps each per run, hipGraph replays")
    line = {
        "metric": METRIC, "value": round(nst * nruns / elapsed, 3), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / (nst * nruns), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic (seeded generators)",
        "config": {"workload": desc, "cells": int(b.ntot), "problems": nprob, "steps_per_run": nst,
                   "step_unit": f"one EREM step of all realisations (timed: {len(runs)} graph runs + 1 "
                                f"profiled run, x {nst} steps)",
                   "tile_shape": shape, "tile_shape_from": "autotune" if args.tile_shape is None else "--tile-shape",
                   "tol_r": 1e-7 if mixed else 1e-12, "precision": args.precision,
                   "m_max": 128, "rho_max": 32.0 if mixed else BATCH_RHO_MAX},
        "roofline": roof,
        "leja_terms_per_run": prof["terms_total"],
        "work_launches_per_run": passes,
        "phases_of_longest_problem": prof["phases"],
        "graph_run_ms": round(float(np.mean([r["ms"] for r in runs])), 3) if runs else None,
        "profiled_run_ms": round(prof["ms"], 3),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = batch_cpu_baseline(probs, b, T0)
    b.close()
    return line


CPU_SAMPLE_CELLS = 2_400_000   # about 10-15 s of one host core for the oracle's sparse action


def batch_cpu_baseline(probs, b, T0):
    """Oracle (tier-B action), one step of the leading realisations up to
    CPU_SAMPLE_CELLS cells, scaled to one step of the whole batch by cell
    count; agreement of the GPU's one-step batch on those realisations."""
    from threadpoolctl import threadpool_limits

    from oracle import erem as oerem
    k, cells = 0, 0
    while k < len(probs) and cells < CPU_SAMPLE_CELLS:
        cells += probs[k].n
        k += 1
    sample = probs[:k]
    T1 = T0.clone()
    b.run(T1, 1, use_graph=False)
    got = b.unpack(T1)
    errs = []
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        outs = [oerem.run_linear(p, nsteps=1, tier="taylor")[0] for p in sample]
        t1 = time.perf_counter()
    terr = []
    for i, (p, To) in enumerate(zip(sample, outs)):
        errs.append(float(np.abs((got[i] - p.T0) - (To - p.T0)).max() / np.abs(To - p.T0).max()))
        terr.append(float(np.abs(got[i] - To).max() / np.abs(To).max()))
    cells_sample = sum(p.n for p in sample)
    cells_all = sum(p.n for p in probs)
    per_batch_step = (t1 - t0) * cells_all / cells_sample
    return {"value": 1.0 / per_batch_step, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 EREM step of realisations 0-{k - 1} ({cells_sample} cells, substepped Taylor action, "
                      f"FP64, 1 thread), scaled by cell count to the {cells_all}-cell batch",
            "seconds": t1 - t0, "gpu_rel_err": max(terr), "gpu_increment_rel_err": max(errs), **cpu_info()}


def bench_adjoint(args):
    """256 x 256 water-law coupled problem, 20 steps; one timed step = one
    gradient of the producer-block mean temperature with respect to T0 and
    log K (20 forward steps with tapes, 20 adjoint steps)."""
    import torch
    from paper_1209_5553_amd import inputs
    from paper_1209_5553_amd.adjoint import coupled_run, run_with_tapes
    from paper_1209_5553_amd.api import EremContext

    nst = 20
    prob = inputs.adjoint_problem(256, structured_T0=args.adjoint_start == "structured")
    ctx = EremContext.from_problem(prob, device="cuda:0")
    dev = ctx.device
    prod = torch.as_tensor(inputs.producer_cells(prob.nx, prob.ny), device=dev)
    T0 = torch.as_tensor(prob.T0, dtype=torch.float64, device=dev)
    lk = torch.as_tensor(prob.logk, dtype=torch.float64, device=dev)

    def grad_once():
        a = T0.clone().requires_grad_(True)
        k = lk.clone().requires_grad_(True)
        TN = coupled_run(ctx, a, k, prob.h, nst)
        TN[prod].mean().backward()
        return a.grad, k.grad

    for _ in range(args.warmup):
        grad_once()
    torch.cuda.synchronize()
    # forward alone (same steps, tapes recorded)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_with_tapes(ctx, T0, lk, prob.h, nst)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    ctx.profile(True, stride=PROFILE_STRIDE)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        grad_once()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    times = ctx.profile_read()
    ctx.profile(False)
    log(f"adjoint: forward {fwd:.3f} s, forward + adjoint {elapsed:.3f} s, kernel times {times}")
    N = prob.n
    kern = {
        "adj_rev_term": (times["adj_rev_ms"], times["adj_rev_launches"], ADJ_REV_BYTES * N),
        "leja_term": (times["leja_term_ms"], times["leja_term_launches"], LEJA_BYTES[2]["f64"] * N),
        "pcg_a": (times["pcg_a_ms"], times["pcg_a_launches"], PCG_A_BYTES[2] * N),
        "pcg_b": (times["pcg_b_ms"], times["pcg_b_launches"], PCG_B_BYTES[2] * N),
        "mg_vcycle": (times["mg_ms"], times["mg_cycles"], mg_bytes(times, 2) * N),
    }
    desc = (f"adjoint: coupled 2D 256x256 water laws, {nst} EREM-Leja steps with tapes + {nst} adjoint steps "
            f"(reverse Leja, transposed stencil, stored iterates), gradient of the producer-block mean T "
            f"wrt T0 and log K ({args.adjoint_start} start)")
    dom = max(kern, key=lambda k: kern[k][0])
    line = {
        "metric": METRIC, "value": round(nst * args.steps / elapsed, 3), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / (nst * args.steps), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generators)",
        "config": {"workload": desc, "grid": [prob.nx, prob.ny, 1], "cells": N, "h_s": prob.h,
                   "step_unit": "one coupled step forward plus its adjoint", "tol_r": 1e-12},
        "roofline": _roof(kern, dom, _traffic("adjoint256", "fp64", dom)),
        "adjoint_rev_term": _roof(kern, "adj_rev_term", _traffic("adjoint256", "fp64", "adj_rev_term")),
        "leja": _roof(kern, "leja_term"),
        "forward_only_steps_per_s": round(nst * args.steps / fwd, 3),
        "gradient_cost_in_forward_runs": round(elapsed / fwd, 3),
    }
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle import erem as oerem
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            oerem.coupled_step(prob, np.asarray(prob.T0, dtype=np.float64), tier="taylor")
            t1 = time.perf_counter()
        line["cpu_baseline"] = {"value": 1.0 / (t1 - t0), "unit": "steps/s", "cores": 1, "kind": "oracle",
                                "sample": "1 forward coupled step of the same workload (SuperLU pressure + "
                                          "substepped Taylor action, FP64, 1 thread); the oracle's dense "
                                          "adjoint is limited to grids of a few hundred cells",
                                "seconds": t1 - t0, **cpu_info()}
    return line


# Bytes moved between L2 and memory per launch unit (the unit of "achieved":
# one V-cycle, one Newton term, one batch launch), from rocprofv3 --pmc runs
# of FETCH_SIZE and WRITE_SIZE on these kernels, scaled by what the counters
# read for a plain 512 MiB copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  They
# describe the kernels as measured: reset an entry to None when its kernel
# changes.
TRAFFIC = {
    ("coupled512", "fp64", "mg_vcycle"): 57.55e6,
    ("coupled512", "fp64", "leja_term"): 6.15e6,     # a working 4-term launch moves 24.60 MB
    ("injector512", "fp64", "leja_term"): 6.15e6,    # the same kernel on the same grid: 24.60 MB
    ("layered128", "fp64", "leja_term"): 186.49e6,
    ("compressible50", "fp64", "leja_term"): 11.34e6,   # the 3D one-term kernel on 125 000 cells
    ("layered128", "mixed", "leja_term"): 93.30e6,      # FP32 one-term kernel, 44 B per cell algorithmic
    # batch256: whole-run totals of the work kernel (divided by its launches)
    ("batch256", "fp64", "k_bt_work/shape5"): 213.05e9,   # one 50-step run, substep intervals up to 96
    ("batch256", "mixed", "k_bt_work/shape7"): 174.68e9,  # one 50-step run, FP32 passes
    # layered256: a working launch (the z-neighbour planes are fetched again: 1.16x algorithmic)
    ("layered256", "fp64", "leja_term"): 1714.26e6,
    ("layered256", "mixed", "leja_term"): 742.57e6,    # FP32: exactly its algorithmic bytes
    # one BiCGSTAB iteration (three kernels) of the comparison schemes
    ("coupled512", "fp64", "bicg_iteration"): 66.55e6,
    # adjoint workload (256 x 256): V-cycle + CG iteration, reverse Newton term
    ("adjoint256", "fp64", "mg_vcycle"): 15.69e6,
    ("adjoint256", "fp64", "adj_rev_term"): 11.10e6,
}


def _traffic(workload, precision, kernel):
    return TRAFFIC.get((workload, precision, kernel))


def roofline_entry(name, bytes_per, avg_s, launches, traffic=None, working_set=None):
    """Roofline object of one kernel: algorithmic bytes per launch over the
    average launch duration, against the HBM peak.  The label is "hbm" only
    when the launch's working set exceeds the Infinity Cache and the
    counters show it moving at least its algorithmic bytes; otherwise it is
    "effective" (cache-resident or temporally blocked) and the memory-side
    rate from the counter traffic is given beside it."""
    ach = bytes_per / avg_s / 1e9
    ws = bytes_per if working_set is None else working_set
    resident = ws < MALL_BYTES
    blocked = traffic is not None and traffic < 0.9 * bytes_per
    out = {"kernel": name, "bound": "effective" if (resident or blocked) else "hbm", "achieved": round(ach, 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
           "avg_launch_us": round(avg_s * 1e6, 3), "launches": launches, "bytes_per_launch": bytes_per,
           "working_set_bytes": ws}
    if resident or blocked:
        out["why_effective"] = ("per-launch working set below the 256 MB Infinity Cache" if resident else
                                f"moves {traffic / bytes_per:.2f}x its algorithmic bytes (terms kept on chip)")
    if traffic is not None:
        out["hbm"] = {"achieved": round(traffic / avg_s / 1e9, 1), "frac": round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                      "unit": "GB/s", "source": "FETCH_SIZE + WRITE_SIZE counters per launch over the same duration"}
    return out


def _roof(kern, name, traffic=None):
    ms, n, bytes_per = kern[name]
    if n == 0:
        return None
    avg_s = ms / n * 1e-3
    out = roofline_entry(name, bytes_per, avg_s, n, traffic)
    out["share_of_kernel_time"] = round(ms / max(sum(v[0] for v in kern.values()), 1e-30), 4)
    return out


def cpu_info():
    """Host CPU model and the number of CPUs the process sees."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_cpus": os.cpu_count()}


def hbm_ceiling(nbytes=1 << 30, reps=10):
    """Measured copy (b = a) and triad (c = a + s b) bandwidth of the device on
    arrays of nbytes each, the practical ceiling beside the 8 TB/s peak."""
    import torch
    n = nbytes // 8
    a = torch.rand(n, dtype=torch.float64, device="cuda:0")
    b = torch.rand(n, dtype=torch.float64, device="cuda:0")
    c = torch.empty_like(a)
    res = {}
    for name, fn, moved in (("copy", lambda: b.copy_(a), 2 * nbytes),
                            ("triad", lambda: torch.add(a, b, alpha=1.5, out=c), 3 * nbytes)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) * 1e-3 / reps
        res[name + "_GBs"] = round(moved / s / 1e9, 1)
    res.update({"bytes_per_array": nbytes, "peak_GBs": HBM_PEAK_GBS,
                "triad_frac_of_peak": round(res["triad_GBs"] / HBM_PEAK_GBS, 4),
                "kernels": "torch copy_ and add(out=) on float64 arrays, HIP events, mean of 10"})
    del a, b, c
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch256",
                    choices=["batch256", "coupled512", "linear32", "layered128", "layered256", "injector512",
                             "compressible50", "adjoint256"])
    ap.add_argument("--no-ceiling", action="store_true", help="skip the copy / triad bandwidth measurement")
    ap.add_argument("--rho-max", type=float, default=None,
                    help="single-problem workloads: widest substep interval h (beta - alpha) / s "
                         "(default: the library's)")
    ap.add_argument("--tile-shape", type=int, default=None,
                    help="batch256: use this tile shape (0-7) instead of autotuning (profiler runs)")
    ap.add_argument("--adjoint-start", default="uniform", choices=["uniform", "structured"])
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pressure-rtol", type=float, default=1e-16)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--pressure-method", default="leja", choices=["leja", "krylov"],
                    help="phi1 of the transient pressure step (compressible50)")
    ap.add_argument("--scheme", default="erem", choices=list(SCHEMES),
                    help="temperature scheme of the coupled workloads: EREM or a comparison scheme "
                         "(ROSM(1), ROSM(1/2), ROS2(1), ROS3p, theta-Euler 1/2 or 1 with Newton)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the EREM library runs on one GPU; multi-GPU runs "
              "(--gpus > 1) are not supported.", file=sys.stderr, flush=True)
        sys.exit(2)
    # the first min(3, cpu-steps) GPU steps are kept for the oracle comparison
    args.cpu_steps = max(1, min(args.cpu_steps, 3))
    if not args.no_cpu_baseline and args.warmup < args.cpu_steps:
        args.warmup = args.cpu_steps

    mixed = args.precision == "mixed"
    if args.workload in ("batch256", "adjoint256"):
        line = bench_batch(args, mixed) if args.workload == "batch256" else bench_adjoint(args)
        if not args.no_ceiling:
            line["hbm_ceiling"] = hbm_ceiling()
        print(json.dumps(line), flush=True)
        return

    prob, desc, coupled = make_workload(args.workload)
    log(f"workload {args.workload}: {desc}; N={prob.n}")
    sched = schedule_of(args.workload)
    if args.scheme != "erem" and (not coupled or mixed):
        raise SystemExit("comparison schemes run on the coupled workloads in FP64")
    if args.workload == "compressible50":
        args.cpu_steps = min(args.cpu_steps, 2)
    res = gpu_run(prob, coupled, args.steps, args.warmup, args.pressure_rtol, mixed=mixed, sched=sched,
                  scheme=args.scheme, pmethod=args.pressure_method, rho_max=args.rho_max)
    dim = prob.dim
    N = prob.n
    t = res["times"]
    kern = {
        "leja_term": (t["leja_term_ms"], t["leja_term_launches"],
                      LEJA_BYTES[dim]["f32" if mixed else "f64"] * N),
        "pcg_a": (t["pcg_a_ms"], t["pcg_a_launches"], PCG_A_BYTES[dim] * N),
        "pcg_b": (t["pcg_b_ms"], t["pcg_b_launches"], PCG_B_BYTES[dim] * N),
        "mg_vcycle": (t["mg_ms"], t["mg_cycles"], mg_bytes(t, dim) * N),
        "bicg_iteration": (t["bicg_ms"], t["bicg_iterations"], BICG_BYTES[dim] * N),
    }
    dominant = max(kern, key=lambda k: kern[k][0])

    def roof(name):
        return _roof(kern, name, _traffic(args.workload, args.precision, name))

    steps_s = args.steps / res["elapsed"]
    erem = args.scheme == "erem"
    metric = METRIC if erem else (f"{args.scheme} coupled steps/s (comparison scheme) & BiCGSTAB iteration GB/s "
                                  f"(% of HBM peak) at 1e-10 rel. err vs FP64 oracle")
    line = {
        "metric": metric, "value": round(steps_s, 3), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * res["elapsed"] / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic (seeded generators)",
        "config": {"workload": desc, "grid": [prob.nx, prob.ny, prob.nz], "cells": N, "h_s": prob.h,
                   "tol_r": 1e-7 if mixed else 1e-12, "precision": args.precision, "pressure_rtol": args.pressure_rtol if coupled else None,
                   "scheme": args.scheme, "rho_max": args.rho_max},
        "roofline": roof(dominant),
        "leja": roof("leja_term") if erem else None,
        "bicg": None if erem else roof("bicg_iteration"),
        "leja_terms_per_step": res["m_per_step"],
        "bicg_iterations_per_step": None if erem else res["lin_per_step"],
        "pressure": None if res["plast"] is None else {
            "method": args.pressure_method, "terms_per_step": res["pressure_m_per_step"],
            "substeps": res["plast"]["substeps"],
            "interval_hJp": [res["plast"]["alpha"] * prob.h, res["plast"]["beta"] * prob.h]},
        "substeps": res["last"]["substeps"],
        "pcg_iterations_per_step": res["pcg_per_step"],
        "interval_hJ": [res["last"]["alpha"] * prob.h, res["last"]["beta"] * prob.h] if erem else None,
    }
    if not args.no_cpu_baseline:
        log(f"cpu baseline: {args.cpu_steps} oracle step(s)")
        line["cpu_baseline"] = cpu_baseline(prob, coupled, args.cpu_steps, res["snapshots"], sched, args.scheme)
    if not args.no_ceiling:
        line["hbm_ceiling"] = hbm_ceiling()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
