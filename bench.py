"""Throughput of the gliding-assay micro-step on one MI355X.

Workload (the measured configuration): 256 x 256 periodic grid, 64 orientations, 64
arclength cells (268M bound-motor cells), FP32 storage and arithmetic, a new seeded fluid
field every K = 10 micro-steps, stress/moments/global sums on every exchange.  A "step" is
one micro-step of the whole path: motor column step, s-moments, psi donor-cell update,
and (every 10th) theta-moments, stress and FP64 global sums.  Inputs are resident in HBM
before the timed region.  The headline runs the library's default order, in which the motor
field of the linear model is advanced through the 10 micro-steps of a call in one launch
(every cell of every micro-step is computed; M is read and written once per call); the
same grid with one motor launch per micro-step (the HBM-bound form) is reported beside it,
each with its own roofline.  Also measured: both forms in FP64, 512^2 x 128 x 64 FP32,
128^2 x 64 x 32 FP64, the launch-bound 16^2 x 16 x 16 FP64 case eager and as a replayed HIP
graph, free-motor depletion, motor sub-cycling, the motor force density, the anchor-resolved
model, the adjoint/forward time ratios, the VALU issue rates of the chip, the FP32 error per
output against the FP64 oracle, and the oracle (FP64 C) on bounded samples on the host
cores (all threads at 256^2 x 64 x 64, one thread at 16^2 x 16 x 16 and 128^2 x 64 x 32).

Prints one JSON line.  --gpus N > 1 is refused: this path runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "micro-steps/s + HBM GB/s (% peak), FP32 vs FP64 at 256²×64×64; adjoint/fwd ratio"
CSRC = os.path.join(ROOT, "paper_1908_04279_amd", "csrc")
# rocprofv3 HBM byte counters of the motor kernel, and the sources it is built from (the
# counters count only while those sources are unchanged)
COUNTERS = (os.path.join(ROOT, "profiles", "motor_step_f32_256x256x64x64_counters.txt"),
            ["motor.hip", "device_util.h", "kernels.h"])
# the same for one motor launch per micro-step (16 bytes of the column per lane)
COUNTERS_PLAIN = (os.path.join(ROOT, "profiles", "motor_step_plain_f32_256x256x64x64_counters.txt"),
                  ["motor.hip", "device_util.h", "kernels.h"])
# kernel launches bracketed by HIP events inside the timed region: every EVENT_EVERY-th launch
# of each kernel (an event pair on every launch costs ~14 us per micro-step on MI355X, ~4%)
EVENT_EVERY = 13
# total motors per unit area of the depletion leg: about twice the coarse bound density the
# linear model settles to on this workload, so the free pool is roughly halved
M_TOTAL_BENCH = 0.02
# Motor sub-cycling leg: motors walking 8x faster than the default (v0 = 8), whose stability
# limit (v0/ds + k_off) is then stricter than the psi limit at 256^2, and a motor CFL of 0.4.
SUBSTEP_V0 = 8.0
MOTOR_CFL_BENCH = 0.4
# Anchor-resolved leg (M_b(r0, x, th, s) on the capture ball): 128^2 anchors and filament cells,
# 32 orientations, 32 arclength cells, capture radius 0.1 (13216 tracked cells per filament cell,
# 216.5M in all, runs of at most 7 cells), with depletion: m_total about the median coarse
# density of the seeded state (M_b ~ U[0, k_on/k_off]), so the clamp is active at the start.
R0_BENCH = dict(nx=128, ny=128, ntheta=32, ns=32, rc=0.1)
R0_M_TOTAL = 8.0e-4
R0_COUNTERS = (os.path.join(ROOT, "profiles", "r0_motor_f32_128x128x32x32_counters.txt"),
               ["r0.hip", "r0.h", "device_util.h"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def motor_bytes(p, b, with_m1, nstep=1):
    """Algorithmic HBM bytes of one motor launch over nstep micro-steps: read M, write M, write
    m0 of every micro-step [and m1 of the last]."""
    n_psi = p.nx * p.ny * p.ntheta
    return b * (2 * n_psi * p.ns + n_psi * (nstep + (1 if with_m1 else 0)))


MAX_BLOCK = 16  # micro-steps per temporally blocked motor launch (the library's block)

# Algorithmic floating-point operations of one motor micro-step per cell (FMA = 2), counted on
# the scheme: per Runge-Kutta stage the difference z_l - z_{l-1} (1), the superbee slope (2
# doublings, 2 minima, 1 maximum, the sign test 1: 6), the face value z + sigma/2 (2), the flux
# difference (1), R = -(v0/ds) dh + (src - k_off z) (4) and the stage update (2): 16; two
# stages and the m0 sum (1): 33; m1 on output launches (2) more.
MOTOR_FLOPS_PER_CELL = 33
M1_FLOPS_PER_CELL = 2
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published peak (FP64: 78.6)
FP64_VECTOR_PEAK_TFLOPS = 78.6


def motor_flops(p, with_m1, nstep=1):
    cells = p.nx * p.ny * p.ntheta * p.ns
    return cells * (MOTOR_FLOPS_PER_CELL * nstep + (M1_FLOPS_PER_CELL if with_m1 else 0))


def motor_substeps(p, dt):
    """Motor sub-steps per micro-step, by the rule documented for mmk_params.motor_cfl."""
    cfl = getattr(p, "motor_cfl", 0.0)
    return max(1, math.ceil(dt * (p.v0 / (p.L / p.ns) + p.k_off) / cfl)) if cfl > 0 else 1


def block_plan(p, K, options=None):
    """Motor launches per K-step call and micro-steps in each: blocks of up to MAX_BLOCK for
    the linear model (m_total = 0), unless the motor_block option is 0; else one per
    micro-step."""
    if getattr(p, "m_total", 0.0) > 0 or (options or {}).get("motor_block", 1) == 0:
        return [1] * K
    return [min(MAX_BLOCK, K - d) for d in range(0, K, MAX_BLOCK)]


def psi_bytes(p, b, out):
    """Algorithmic HBM bytes of one psi step: read psi, m0, u, gradu, write psi [read m1,
    write stress and moments]."""
    n_psi = p.nx * p.ny * p.ntheta
    nxy = p.nx * p.ny
    return b * (3 * n_psi + 6 * nxy) + (b * (n_psi + 10 * nxy) if out else 0)


_INPUTS = {}


def fluids_of(p, n):
    """Seeded fluid fields 1 .. n of the grid (host, FP64), generated once per grid."""
    key = ("fluid", p.nx, p.ny, p.lx, p.ly)
    from paper_1908_04279_amd import inputs as gen
    have = _INPUTS.setdefault(key, [])
    for e in range(len(have), n):
        have.append(gen.make_fluid(p.nx, p.ny, p.lx, p.ly, seed=1 + e))
    return have[:n]


def psi0_of(p):
    """Seeded initial filament density of the grid (host, FP64), generated once per grid."""
    key = ("psi0", p.nx, p.ny, p.ntheta, p.lx, p.ly)
    if key not in _INPUTS:
        from paper_1908_04279_amd import inputs as gen
        _INPUTS[key] = gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=0)
    return _INPUTS[key]


def run_forward(p, precision, steps, warmup, K, profile=True, event_every=1, options=None, motor_every=None):
    """One forward leg: warmup, then `steps` micro-steps in calls of K with a new fluid field
    each, timed on the host around the whole; every event_every-th launch of each kernel (of
    the motor kernel every motor_every-th, if given) carries HIP events."""
    import torch
    from paper_1908_04279_amd import inputs as gen
    from paper_1908_04279_amd import mmk

    n_ex = (warmup + steps) // K + 2
    fluids_np = fluids_of(p, n_ex)
    dt = gen.cfl_dt(p, fluids_np)
    ctx = mmk.Context(p, precision=precision, options=options)
    fl = [(torch.as_tensor(u).to(ctx.device, ctx.dtype), torch.as_tensor(g).to(ctx.device, ctx.dtype))
          for u, g in fluids_np]
    ctx.set_state(torch.as_tensor(psi0_of(p)))
    torch.cuda.synchronize()

    def advance(nsteps, e0):
        done, e = 0, e0
        while done < nsteps:
            ctx.set_fluid(*fl[e])
            k = min(K, nsteps - done)
            ctx.step(k, dt)
            done += k
            e += 1
        return e

    log(f"[bench] {p.nx}x{p.ny}x{p.ntheta}x{p.ns} {'FP32' if precision == mmk.FP32 else 'FP64'} "
        f"{options or ''}: warmup {warmup} steps, {steps} timed")
    e = advance(warmup, 0)
    torch.cuda.synchronize()
    if profile:
        ctx.profile(True, every=event_every)
        if motor_every is not None:
            ctx.profile_every("motor_step", motor_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance(steps, e)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    prof = {}
    if profile:
        for name in ("motor_step", "psi_step", "global_sums"):
            ms, n = ctx.profile_read(name)
            prof[name] = (ms, n)
        ctx.profile(False)
    mass, ss = ctx.get_sums()
    ctx.close()
    return dict(elapsed=elapsed, steps=steps, dt=dt, prof=prof, mass=mass, event_every=event_every,
                motor_every=event_every if motor_every is None else motor_every,
                blocks=block_plan(p, K, options), p=p, K=K, precision=precision)


def run_adjoint(name, precision):
    """Forward with tape (checkpoints every C steps, fluid exchange every K) and the
    reverse pass (recompute + reverse kernels), timed separately."""
    import torch
    from paper_1908_04279_amd import inputs as gen
    from paper_1908_04279_amd import mmk
    c = gen.CONFIGS[name]
    p = gen.params_for(name)
    n, K, C = c["steps"], c["K"], c["ckpt"]
    fl_np = gen.fluid_schedule(p.nx, p.ny, -(-n // K), new_each=c["new_fluid_each_exchange"])
    dt = gen.cfl_dt(p, fl_np)
    torch.cuda.reset_peak_memory_stats()
    ctx = mmk.Context(p, precision=precision, ckpt_every=C, max_tape_steps=n)
    fl = [(torch.as_tensor(u).to(ctx.device, ctx.dtype), torch.as_tensor(g).to(ctx.device, ctx.dtype))
          for u, g in fl_np]
    psi0 = torch.as_tensor(gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0)).to(ctx.device, ctx.dtype)
    target = torch.as_tensor(gen.make_target_stress(p.nx, p.ny)).to(ctx.device, ctx.dtype)

    def forward():
        ctx.set_state(psi0)
        ctx.set_fluid(*fl[0])
        ctx.tape_begin(C)
        done, e = 0, 0
        while done < n:
            if e > 0:
                ctx.set_fluid(*fl[e])
            k = min(K, n - done)
            ctx.step(k, dt)
            done += k
            e += 1
        return ctx.get_stress()

    out = {}
    # pair 0: warm-up; pair 1: timed (no events); pair 2: HIP events on every reverse launch
    for rep in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sigma = forward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        d = sigma - target
        g_sigma = torch.stack([d[0], 2 * d[1], d[2]]) / torch.sqrt((d[0] ** 2 + 2 * d[1] ** 2 + d[2] ** 2).sum())
        if rep == 2:
            ctx.profile(True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g_psi0, g_par = ctx.tape_backward(g_sigma.contiguous(), None)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        ctx.tape_end()
        if rep == 1:
            out = dict(forward_s=t1 - t0, backward_s=t3 - t2, g_params=g_par)
    ms_r, n_r = ctx.profile_read("motor_step_reverse")
    ms_p, n_p = ctx.profile_read("psi_step_reverse")
    b = 4 if precision == mmk.FP32 else 8
    n_m = p.nx * p.ny * p.ntheta * p.ns
    rev_bytes = b * (3 * n_m + p.nx * p.ny * p.ntheta)
    out.update(ratio=out["backward_s"] / out["forward_s"], steps=n, ckpt_every=C,
               workspace_gb=ctx.ws_bytes / 1e9,
               peak_device_gb=torch.cuda.max_memory_allocated() / 1e9,
               motor_reverse_avg_us=ms_r / n_r * 1e3,
               motor_reverse_gbs=rev_bytes / (ms_r / n_r / 1e3) / 1e9,
               psi_reverse_avg_us=ms_p / n_p * 1e3)
    ctx.profile(False)
    ctx.close()
    return out


def run_force(p, precision, reps):
    """Motor force density of a seeded state (Eq. (10)), timed over `reps` calls with HIP
    events on the library's stream."""
    import torch
    from paper_1908_04279_amd import inputs as gen
    from paper_1908_04279_amd import mmk
    ctx = mmk.Context(p, precision=precision)
    psi0 = psi0_of(p)
    M0 = torch.rand(p.nx, p.ny, p.ntheta, p.ns, dtype=ctx.dtype, device=ctx.device,
                    generator=torch.Generator(device=ctx.device).manual_seed(5)) * (p.k_on / p.k_off)
    ctx.set_state(torch.as_tensor(psi0), M0)
    for _ in range(2):
        ctx.get_force()
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.get_force()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, n = ctx.profile_read("motor_force")
    ctx.profile(False)
    ctx.close()
    b = 4 if precision == mmk.FP32 else 8
    n_psi = p.nx * p.ny * p.ntheta
    alg = b * (n_psi * p.ns + n_psi + 2 * p.nx * p.ny)   # read M and psi, write the force
    us = ms / n * 1e3
    return {"avg_us": us, "wall_us_per_call": el / reps * 1e6, "algorithmic_bytes": alg,
            "gbs": alg / (us * 1e-6) / 1e9, "frac": alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, "calls": n}


def r0_runs(cells):
    """Number of runs (consecutive l with the same a, b, k) in a tracked-cell table."""
    if len(cells) == 0:
        return 0
    brk = (np.diff(cells[:, 3]) != 1) | np.any(np.diff(cells[:, :3], axis=0) != 0, axis=1)
    return int(np.sum(brk)) + 1


def r0_motor_bytes(p, b, ncell, nrun, depl):
    """Algorithmic HBM bytes of one anchor-resolved motor launch: read and write M_b, write the
    run totals and the marginals m0, m1 [read the anchors' clamp factor and pool]."""
    nxy = p.nx * p.ny
    return b * (2 * ncell * nxy + nrun * nxy + 2 * nxy * p.ntheta + (2 * nxy if depl else 0))


def r0_anchor_bytes(p, b, ncell, nrun):
    """Algorithmic HBM bytes of one launch with one anchor per block (all sub-steps of a depleted
    micro-step): read and write M_b, read psi, write the run totals q0 and q1 by anchor."""
    nxy = p.nx * p.ny
    return b * (2 * ncell * nxy + nxy * p.ntheta + 2 * nrun * nxy)


def r0_marg_bytes(p, b, nrun):
    """The anchor marginals from the run totals: read q0 and q1, write m0 and m1."""
    nxy = p.nx * p.ny
    return b * (2 * nrun * nxy + 2 * nxy * p.ntheta)


def r0_coarse_bytes(p, b, nrun, nsplit):
    """Coarse density, clamp and pool: read the run totals and psi, write and read the FP64
    partial rows, write the clamp factor and pool."""
    nxy = p.nx * p.ny
    return b * (nrun * nxy + nxy * p.ntheta + 2 * nxy) + 2 * 8 * 4 * nsplit * nxy


def r0_counters_traffic():
    """HBM bytes per FP32 anchor-resolved motor launch from the committed rocprofv3 counter
    summary, or None when it is missing or was taken on other kernel sources."""
    path, files = R0_COUNTERS
    if not os.path.exists(path):
        return None
    kv = dict(line.strip().split("=", 1) for line in open(path) if "=" in line and not line.startswith("#"))
    if kv.get("sources_sha256_16") != sources_sha(files):
        return None
    return float(kv["hbm_bytes_per_launch"])


def r0_substeps(args):
    """Fast motors (v0 = SUBSTEP_V0) on the anchor-resolved workload: one motor step per
    micro-step (dt at the motor limit) against motor sub-cycling (dt at the psi limit), as
    simulated time per second; with depletion (one pass per micro-step, or every sub-step its own
    launch after its anchors' clamp) and with linear attachment (the sub-steps in registers); the
    one-pass path also in FP64."""
    from paper_1908_04279_amd import mmk
    keep = ("micro_steps_per_s", "dt", "simulated_time_per_s", "motor_substeps", "motor_avg_us",
            "coarse_avg_us", "psi_avg_us", "onepass")
    d = {"v0": SUBSTEP_V0, "motor_cfl": MOTOR_CFL_BENCH}
    for name, over in (("one_motor_step", dict(v0=SUBSTEP_V0)),
                       ("subcycled", dict(v0=SUBSTEP_V0, motor_cfl=MOTOR_CFL_BENCH)),
                       ("subcycled_launch_per_substep", dict(v0=SUBSTEP_V0, motor_cfl=MOTOR_CFL_BENCH,
                                                             options={"r0_onepass": 0})),
                       ("one_motor_step_linear", dict(v0=SUBSTEP_V0, m_total=0.0)),
                       ("subcycled_linear", dict(v0=SUBSTEP_V0, motor_cfl=MOTOR_CFL_BENCH, m_total=0.0))):
        r = run_r0(mmk.FP32, args.r0_steps, 20, 10, args.event_every, **over)
        d[name] = {k: r[k] for k in keep if k in r}
    # the FP64 variant of the one-pass path (16 FP64 slots a thread)
    r = run_r0(mmk.FP64, args.r0_steps, 20, 10, args.event_every, v0=SUBSTEP_V0, motor_cfl=MOTOR_CFL_BENCH)
    d["subcycled_fp64"] = {k: r[k] for k in keep if k in r}
    d["speedup_simulated_time"] = (d["subcycled"]["simulated_time_per_s"]
                                   / d["one_motor_step"]["simulated_time_per_s"])
    d["speedup_simulated_time_launch_per_substep"] = (d["subcycled_launch_per_substep"]["simulated_time_per_s"]
                                                      / d["one_motor_step"]["simulated_time_per_s"])
    d["speedup_simulated_time_linear"] = (d["subcycled_linear"]["simulated_time_per_s"]
                                          / d["one_motor_step_linear"]["simulated_time_per_s"])
    return d


def run_r0(precision, steps, warmup, K, event_every, options=None, **over):
    """The anchor-resolved micro-step (coarse + pool, motor, psi) on the R0_BENCH workload
    (parameters in `over` replace the defaults: faster motors, motor sub-cycling; `options`:
    library options by name)."""
    import torch
    from paper_1908_04279_amd import inputs as gen
    from paper_1908_04279_amd import mmk
    p = gen.ModelParams(**{**R0_BENCH, "m_total": R0_M_TOTAL, **over})
    cells = mmk.r0_cells(p)
    ncell, nrun = len(cells), r0_runs(cells)
    n_ex = (warmup + steps) // K + 2
    fluids_np = fluids_of(p, n_ex)
    dt = gen.cfl_dt(p, fluids_np)
    ctx = mmk.Context(p, precision=precision, options=options)
    fl = [(torch.as_tensor(u).to(ctx.device, ctx.dtype), torch.as_tensor(g).to(ctx.device, ctx.dtype))
          for u, g in fluids_np]
    psi0 = psi0_of(p)
    Mb0 = torch.rand(ncell, p.nx, p.ny, dtype=ctx.dtype, device=ctx.device,
                     generator=torch.Generator(device=ctx.device).manual_seed(6)) * (p.k_on / p.k_off)
    ctx.set_state(torch.as_tensor(psi0), Mb0)
    del Mb0
    co0, _ = ctx.get_anchors()
    clamped0 = float((co0 > p.m_total).float().mean())

    def advance(nsteps, e0):
        done, e = 0, e0
        while done < nsteps:
            ctx.set_fluid(*fl[e])
            k = min(K, nsteps - done)
            ctx.step(k, dt)
            done += k
            e += 1
        return e

    log(f"[bench] anchor-resolved {'FP32' if precision == mmk.FP32 else 'FP64'}: {ncell} cells per filament "
        f"cell, {nrun} runs, warmup {warmup}")
    e = advance(warmup, 0)
    torch.cuda.synchronize()
    ctx.profile(True, every=event_every)
    t0 = time.perf_counter()
    advance(steps, e)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = {name: ctx.profile_read(name)
            for name in ("r0_motor_step", "r0_coarse", "psi_step", "r0_anchor_step", "r0_marginals")}
    ctx.profile(False)
    # the motor force of the state (anchor-marginal field + spreading), 10 calls
    ctx.get_force()
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(10):
        ctx.get_force()
    ms_f, n_f = ctx.profile_read("motor_force")
    ctx.profile(False)
    co, _ = ctx.get_anchors()
    clamped = float((co > p.m_total).float().mean())
    mass, _ = ctx.get_sums()
    ctx.close()
    b = 4 if precision == mmk.FP32 else 8
    # the library's coarse split: about 4096 blocks of 64 lanes, one anchor per lane
    gx = -(-(p.nx * p.ny) // 64)
    nsplit = max(1, min(-(-4096 // gx), 64, -(-nrun // 4)))
    mb = r0_motor_bytes(p, b, ncell, nrun, True)
    cb = r0_coarse_bytes(p, b, nrun, nsplit)
    ms_m, n_m = prof["r0_motor_step"]
    ms_c, n_c = prof["r0_coarse"]
    ms_p, n_p = prof["psi_step"]
    ms_a, n_a = prof["r0_anchor_step"]
    ms_g, n_g = prof["r0_marginals"]
    us_p = ms_p / n_p * 1e3
    us_m = ms_m / n_m * 1e3 if n_m else None  # none when each micro-step is one launch per anchor
    us_c = ms_c / n_c * 1e3 if n_c else None  # no coarse launches without depletion
    flops = ncell * p.nx * p.ny * (MOTOR_FLOPS_PER_CELL + M1_FLOPS_PER_CELL)
    alu_peak = FP32_VECTOR_PEAK_TFLOPS if b == 4 else FP64_VECTOR_PEAK_TFLOPS
    onepass = None
    if n_a:
        # one launch per micro-step: nsub sub-steps of every cell, each with its clamp's sum
        # (one multiply-add a cell) and its scaling (one multiply)
        us_a, us_g = ms_a / n_a * 1e3, ms_g / n_g * 1e3
        ab, gb = r0_anchor_bytes(p, b, ncell, nrun), r0_marg_bytes(p, b, nrun)
        nsub = motor_substeps(p, dt)
        aflops = ncell * p.nx * p.ny * (nsub * (MOTOR_FLOPS_PER_CELL + 3) + M1_FLOPS_PER_CELL)
        onepass = {"anchor_avg_us": us_a, "anchor_algorithmic_bytes": ab, "anchor_gbs": ab / (us_a * 1e-6) / 1e9,
                   "anchor_frac": ab / (us_a * 1e-6) / 1e9 / HBM_PEAK_GBS,
                   "anchor_alu_frac": aflops / (us_a * 1e-6) / 1e12 / alu_peak,
                   "marginals_avg_us": us_g, "marginals_algorithmic_bytes": gb,
                   "marginals_gbs": gb / (us_g * 1e-6) / 1e9, "timed_launches": [n_a, n_g]}
    return {"workload": f"{p.nx}x{p.ny} anchors and filament cells, {p.ntheta} orientations, {p.ns} arclength "
                        f"cells, capture radius {p.rc}, m_total {p.m_total}",
            "tracked_cells_per_filament_cell": ncell, "Mb_cells": ncell * p.nx * p.ny, "runs": nrun,
            "steps": steps, "micro_steps_per_s": steps / el, "ms_per_step": el / steps * 1e3,
            "dt": dt, "simulated_time_per_s": dt * steps / el,
            "motor_substeps": motor_substeps(p, dt), "motor_avg_us": us_m, "motor_algorithmic_bytes": mb,
            "motor_gbs": mb / (us_m * 1e-6) / 1e9 if us_m else None,
            "motor_frac": mb / (us_m * 1e-6) / 1e9 / HBM_PEAK_GBS if us_m else None,
            "motor_alu_frac": flops / (us_m * 1e-6) / 1e12 / alu_peak if us_m else None,
            "onepass": onepass,
            "motor_traffic": r0_counters_traffic() if b == 4 else None,
            "coarse_avg_us": us_c, "coarse_algorithmic_bytes": cb, "coarse_gbs": cb / (us_c * 1e-6) / 1e9 if us_c else None,
            "psi_avg_us": us_p, "force_avg_us": ms_f / n_f * 1e3,
            "clamped_anchor_fraction_start": clamped0, "clamped_anchor_fraction_end": clamped,
            "mass": mass, "timed_launches": [n_m, n_c, n_p]}


def copy_calibration(nbytes, reps):
    """A plain device copy of known size (for scaling the HBM byte counters)."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": nbytes, "reps": reps}), flush=True)


def sources_sha(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def counters_traffic(n_plain, n_out, steps_per_launch=1, counters=COUNTERS):
    """HBM bytes per motor launch (weighted like `achieved`: n_plain launches without and
    n_out with the m1 output) from a committed rocprofv3 counter summary, or None when it
    is missing, was taken on different kernel sources or on launches of another number of
    micro-steps."""
    path, files = counters
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("sources_sha256_16") != sources_sha(files):
        return None
    try:
        if abs(float(kv.get("micro_steps_per_launch", "1")) - steps_per_launch) > 1e-9:
            return None
        t1 = float(kv["hbm_bytes_per_output_launch"])
        t0 = float(kv["hbm_bytes_per_launch"]) if n_plain else t1
    except (KeyError, ValueError):
        return None
    return (n_plain * t0 + n_out * t1) / max(n_plain + n_out, 1)


def cpu_baseline(p, sample_steps):
    """The FP64 C oracle on the same grid (M0 = 0, fluid seed 1 held fixed), a few micro-steps,
    on the host cores.  Returns the record and the oracle (its state is the FP64 reference of
    the FP32 error report)."""
    from oracle import oracle_a as A
    from paper_1908_04279_amd import inputs as gen
    u, g = fluids_of(p, 1)[0]
    dt = gen.cfl_dt(p, [(u, g)])
    o = A.OracleA(p)
    o.set_state(psi0_of(p))
    o.set_fluid(u, g)
    threads = A.max_threads()
    log(f"[bench] cpu baseline: oracle, {sample_steps} steps, {threads} threads")
    t0 = time.perf_counter()
    o.step(sample_steps, dt)
    el = time.perf_counter() - t0
    rec = dict(value=sample_steps / el, unit="micro-steps/s", cores=threads, kind="oracle",
               sample=f"{sample_steps} FP64 micro-steps of the full {p.nx}x{p.ny}x{p.ntheta}x{p.ns} grid "
                      f"(C oracle, OpenMP over x rows), {el:.1f} s")
    return rec, o, dt


def cpu_oracle_one_thread(name, steps):
    """The FP64 C oracle on one host thread (the analogue of a single-threaded code) on a
    bounded sample of a seeded workload: `steps` micro-steps from its initial state."""
    from oracle import oracle_a as A
    from paper_1908_04279_amd import inputs as gen
    p = gen.params_for(name)
    u, g = fluids_of(p, 1)[0]
    dt = gen.cfl_dt(p, [(u, g)])
    o = A.OracleA(p)
    o.set_state(psi0_of(p))
    o.set_fluid(u, g)
    before = A.max_threads()
    A.set_threads(1)
    try:
        t0 = time.perf_counter()
        o.step(steps, dt)
        el = time.perf_counter() - t0
    finally:
        A.set_threads(before)
    return {"value": steps / el, "unit": "micro-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} FP64 micro-steps of {p.nx}x{p.ny}x{p.ntheta}x{p.ns} on one thread, {el:.2f} s"}


def fp32_errors(p, o, dt, steps):
    """The FP32 path against the FP64 oracle state of the CPU baseline (same inputs, dt and
    steps; one call): norm-wise relative error max|x - ref| / max|ref| per output."""
    import torch
    from paper_1908_04279_amd import mmk
    from oracle import oracle_a as A
    ctx = mmk.Context(p, precision=mmk.FP32)
    ctx.set_state(torch.as_tensor(psi0_of(p)))
    ctx.set_fluid(*map(torch.as_tensor, fluids_of(p, 1)[0]))
    ctx.step(steps, dt)
    psi, M = ctx.get_state()
    m0, m1 = ctx.get_motor_moments()
    stress, mom = ctx.get_stress(), ctx.get_moments()
    mass, ss = ctx.get_sums()
    s_ref, mom_ref = o.get_stress_moments()
    mass_ref, ss_ref = A.global_sums(p, o.psi, s_ref)

    def rel(x, ref):
        x = x.double().cpu().numpy() if hasattr(x, "cpu") else np.asarray(x, dtype=np.float64)
        return float(np.abs(x - ref).max() / np.abs(ref).max())
    names = ["c", "n_x", "n_y", "D_xx", "D_xy", "D_yy", "B"]
    out = {"steps": steps, "grid": f"{p.nx}x{p.ny}x{p.ntheta}x{p.ns}",
           "stress_xx": rel(stress[0], s_ref[0]), "stress_xy": rel(stress[1], s_ref[1]),
           "stress_yy": rel(stress[2], s_ref[2]), "stress": rel(stress, s_ref)}
    for i, n in enumerate(names):
        out[f"moment_{n}"] = rel(mom[i], mom_ref[i])
    # M columns stay equal (M0 = 0): every column against the oracle's
    out.update(psi=rel(psi, o.psi), M=rel(M[0, 0], o.M[0, 0]) if M.numel() else None,
               M_columns_spread=float((M.amax(dim=(0, 1)) - M.amin(dim=(0, 1))).abs().max()),
               m0=rel(m0, o.m0), m1=rel(m1, o.m1), mass=abs(mass - mass_ref) / abs(mass_ref),
               sum_sigma=float(np.abs(np.array(ss) - ss_ref).max() / np.abs(ss_ref).max()))
    ctx.close()
    return out


def run_launch_bound(reps):
    """The 16^2 x 16 x 16 FP64 workload (100 micro-steps per call, fixed fluid): host-timed
    micro-steps/s of repeated calls, eager (mmk_step) and as a replayed HIP graph
    (mmk_step_graph), after two untimed calls each."""
    import torch
    from paper_1908_04279_amd import inputs as gen
    from paper_1908_04279_amd import mmk
    p = gen.params_for("fp64_16x16x16x16")
    K = gen.CONFIGS["fp64_16x16x16x16"]["K"]
    fl = fluids_of(p, 1)
    dt = gen.cfl_dt(p, fl)
    out = {"workload": "16x16 grid, 16 orientations, 16 arclength cells, FP64, 100 micro-steps per call",
           "calls": reps}
    for mode in ("eager", "graph"):
        ctx = mmk.Context(p)
        ctx.set_state(torch.as_tensor(psi0_of(p)))
        ctx.set_fluid(*map(torch.as_tensor, fl[0]))
        run = ctx.step if mode == "eager" else ctx.step_graph
        for _ in range(2):
            run(K, dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            run(K, dt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx.close()
        out[f"{mode}_micro_steps_per_s"] = reps * K / el
        out[f"{mode}_us_per_micro_step"] = el / (reps * K) * 1e6
    out["graph_over_eager"] = out["graph_micro_steps_per_s"] / out["eager_micro_steps_per_s"]
    return out


CALIB_KINDS = {"fma_f32": (0, 2), "add_f32": (1, 1), "max_f32": (2, 1), "med3_f32": (3, 1),
               "fma_f64": (4, 2), "mov_dpp": (5, 0), "cmp_cndmask": (6, 0), "fmac_f32": (7, 2),
               "mul_f32": (8, 1), "sub_f32": (9, 1), "cndmask_sgpr_mask": (10, 0), "mov_b32": (11, 0),
               "min3_f32": (12, 0), "add_f32_dpp": (13, 1), "add_med3_alternating": (14, 0),
               "add_f64": (15, 1), "med3_f32_const0": (16, 0), "fma_f32_const": (17, 2),
               "fma_f32_sgpr": (18, 2), "max_f32_abs": (19, 0), "add_med3_each_other": (20, 0),
               "motor_mix": (21, 0)}


def valu_calibration():
    """Issue rate of single VALU instruction kinds on the whole chip (libmmk_calib): 8192 waves
    (8 per SIMD) of 8 independent chains; wave64 instructions per second, lane operations per
    second and, for the arithmetic kinds, FLOP/s (an FMA counted as 2)."""
    import ctypes as C
    import torch
    path = os.path.join(ROOT, "paper_1908_04279_amd", "libmmk_calib.so")
    if not os.path.exists(path):
        return None
    L = C.CDLL(path)
    f = L.mmk_calib_valu
    f.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]
    f.restype = C.c_int
    blocks, iters = 2048, 4096
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {"waves": blocks * 4, "instructions_per_lane": 64 * iters}
    for name, (kind, flops) in CALIB_KINDS.items():
        ms = C.c_double()
        for rep in range(2):   # the second launch is the measurement
            st = f(kind, blocks, iters, C.c_void_p(out.data_ptr()), stream, C.byref(ms))
            if st != 0:
                return {"error": f"calibration kind {name}: hip error {st}"}
        per_count = 2 if name == "cmp_cndmask" else 1
        wave_insts = blocks * 4 * 64 * iters * per_count
        rate = wave_insts / (ms.value * 1e-3)
        res[name] = {"ms": ms.value, "wave_instructions_per_s": rate, "lane_ops_per_s": rate * 64,
                     "cycles_per_wave_instruction_per_simd": 256 * 4 * 2.4e9 / rate}
        if flops:
            res[name]["tflops"] = rate * 64 * flops / 1e12
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--fp64-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=130)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["all", "fp32", "fp64", "fp32_1", "adjoint", "adjoint64", "depletion", "force",
                                       "substeps", "r0", "r0_fp32", "r0_sub", "r0_sub64", "large", "c2", "launch_bound",
                                       "calib"],
                    default="all",
                    help="restrict to one leg (used for profiler runs)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--depletion-steps", type=int, default=200)
    ap.add_argument("--substep-steps", type=int, default=200)
    ap.add_argument("--r0-steps", type=int, default=200)
    ap.add_argument("--large-steps", type=int, default=20)
    ap.add_argument("--event-every", type=int, default=EVENT_EVERY,
                    help="bracket every N-th launch of each kernel with HIP events (the headline leg's "
                         "motor launches: every one)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    ap.add_argument("--option", action="append", default=[], metavar="NAME=VALUE",
                    help="a context option (mmk_set_option) for the fp32, fp64 and large legs of --only "
                         "(measurements; the default run takes the library's defaults)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this micro-step path runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_04279_amd import inputs as gen
    from paper_1908_04279_amd import mmk
    mmk.lib()   # fail loudly if the HIP library is missing
    torch.cuda.set_device(0)
    if args.copy_calib:
        copy_calibration(args.copy_calib, 10)
        return
    if args.only == "adjoint":
        print(json.dumps({"adjoint_fp32": run_adjoint("adjoint_fp32_256x256x64x32", mmk.FP32)}), flush=True)
        return
    if args.only == "adjoint64":
        print(json.dumps({"adjoint_fp64": run_adjoint("adjoint_fp64_64x64x32x32", mmk.FP64)}), flush=True)
        return
    if args.only == "force":
        print(json.dumps({"force_fp32": run_force(gen.params_for("fp32_256x256x64x64"), mmk.FP32, 10)}),
              flush=True)
        return
    if args.only == "calib":
        print(json.dumps({"valu_calibration": valu_calibration()}), flush=True)
        return
    if args.only == "launch_bound":
        print(json.dumps({"launch_bound_fp64_16x16x16x16": run_launch_bound(50)}), flush=True)
        return

    if args.only in ("r0_sub", "r0_sub64"):  # the depleted sub-cycled anchor-resolved leg alone (profiler runs)
        prec, name = (mmk.FP64, "fp64") if args.only == "r0_sub64" else (mmk.FP32, "fp32")
        print(json.dumps({f"anchor_resolved_subcycled_{name}": run_r0(
            prec, args.r0_steps, 20, 10, args.event_every, v0=SUBSTEP_V0, motor_cfl=MOTOR_CFL_BENCH)}), flush=True)
        return

    if args.only in ("r0", "r0_fp32"):
        r0 = {"anchor_resolved_fp32": run_r0(mmk.FP32, args.r0_steps, 20, 10, args.event_every)}
        if args.only == "r0":
            r0["anchor_resolved_fp64"] = run_r0(mmk.FP64, args.r0_steps, 20, 10, args.event_every)
            r0["anchor_resolved_substeps_fp32"] = r0_substeps(args)
        print(json.dumps(r0), flush=True)
        return

    p = gen.params_for("fp32_256x256x64x64")
    K = 10
    res = {}
    calib = None
    extra = {}
    for kv in args.option:
        name, value = kv.split("=", 1)
        extra[name] = int(value)
    if extra and args.only == "all":
        print("bench.py: --option applies to the single legs of --only", file=sys.stderr)
        sys.exit(2)
    if args.only == "all":
        log("[bench] VALU calibration")
        calib = valu_calibration()
    if args.only in ("all", "depletion"):
        # the same grid with free-motor depletion and the over-binding clamp
        pd = gen.params_for("fp32_256x256x64x64", m_total=M_TOTAL_BENCH)
        res["depletion"] = run_forward(pd, mmk.FP32, args.depletion_steps, min(args.warmup, 20), K,
                                       event_every=args.event_every)
    if args.only in ("all", "substeps"):
        # fast motors on the same grid: one motor step per micro-step (dt at the motor limit)
        # against motor sub-cycling (dt at the psi limit, n motor steps per launch)
        pf = gen.params_for("fp32_256x256x64x64", v0=SUBSTEP_V0)
        ps = gen.params_for("fp32_256x256x64x64", v0=SUBSTEP_V0, motor_cfl=MOTOR_CFL_BENCH)
        res["fast_plain"] = run_forward(pf, mmk.FP32, args.substep_steps, 20, K, event_every=args.event_every)
        res["fast_sub"] = run_forward(ps, mmk.FP32, args.substep_steps, 20, K, event_every=args.event_every)
        # the same with depletion: every sub-step after the clamp of its sub-state, all sub-steps
        # of a micro-step in one launch (one block per (x, y) point), and one launch per sub-step
        pds = gen.params_for("fp32_256x256x64x64", v0=SUBSTEP_V0, motor_cfl=MOTOR_CFL_BENCH, m_total=M_TOTAL_BENCH)
        res["fast_depl_sub"] = run_forward(pds, mmk.FP32, min(args.substep_steps, 100), 10, K,
                                           event_every=args.event_every)
        res["fast_depl_sub_1"] = run_forward(pds, mmk.FP32, min(args.substep_steps, 100), 10, K,
                                             event_every=args.event_every, options={"depl_fused": 0})
    if args.only in ("all", "fp64"):
        res["fp64"] = run_forward(p, mmk.FP64, args.fp64_steps, min(args.warmup, 20), K,
                                  event_every=args.event_every, options=extra or None)
    if args.only in ("all", "fp32"):
        # the headline: runs right after the FP64 leg (the chip at its working clock), every
        # motor launch of the timed region bracketed by HIP events
        res["fp32"] = run_forward(p, mmk.FP32, args.steps, args.warmup, K, event_every=args.event_every,
                                  motor_every=1, options=extra or None)
    if args.only in ("all", "fp32_1"):
        # the same grid with one motor launch per micro-step (HBM-bound): FP32 and FP64
        res["fp32_1"] = run_forward(p, mmk.FP32, args.fp64_steps, 20, K, event_every=args.event_every,
                                    options={**extra, "motor_block": 0})
    if args.only == "all":
        res["fp64_1"] = run_forward(p, mmk.FP64, args.fp64_steps, 20, K, event_every=args.event_every,
                                    options={"motor_block": 0})
    large = {}
    if args.only in ("all", "large"):
        # the largest single-GPU case, 512^2 x 128 x 64 FP32 (2^31 motor cells), both orders
        pl = gen.params_for("fp32_512x512x128x64")
        torch.cuda.reset_peak_memory_stats()
        large["blocked"] = run_forward(pl, mmk.FP32, args.large_steps, 10, K, event_every=args.event_every,
                                       motor_every=1, options=extra or None)
        large["peak_device_gb"] = torch.cuda.max_memory_allocated() / 1e9
        large["one_launch"] = run_forward(pl, mmk.FP32, args.large_steps, 10, K, event_every=args.event_every,
                                          options={**extra, "motor_block": 0}, motor_every=1)
    c2 = None
    if args.only in ("all", "c2"):
        # paper-like scale in FP64: 128^2 x 64 x 32, 1000 micro-steps, a new fluid every 10
        c2 = run_forward(gen.params_for("fp64_128x128x64x32"), mmk.FP64, 1000, 20, K, event_every=args.event_every)

    def summarise(r):
        """Whole-step rate, and the motor kernel's roofline over its timed launches.  A K-step
        call runs the motor launches of r["blocks"] (micro-steps each); the last one of a call
        carries the outputs (m1, stress, moments), as does the psi launch of the call's last
        micro-step.  Launches j = 0, E, 2E, ... of each kernel in the timed region carry HIP
        events (E = r["motor_every"] for the motor kernel, r["event_every"] for psi)."""
        q, Kr = r["p"], r["K"]
        b = 4 if r["precision"] == mmk.FP32 else 8
        calls = r["steps"] // Kr
        blocks = r["blocks"]
        sps = r["steps"] / r["elapsed"]
        launches = [(nb, i == len(blocks) - 1) for _ in range(calls) for i, nb in enumerate(blocks)]
        total = sum(motor_bytes(q, b, out, nb) for nb, out in launches) \
            + (r["steps"] - calls) * psi_bytes(q, b, False) + calls * psi_bytes(q, b, True)
        timed_m = launches[::r["motor_every"]]
        timed_p = list(range(0, r["steps"], r["event_every"]))
        ms_m, n_m = r["prof"]["motor_step"]
        ms_p, n_p = r["prof"]["psi_step"]
        assert n_m == len(timed_m) and n_p == len(timed_p), (n_m, n_p, len(timed_m), len(timed_p))
        n_out = sum(1 for _, out in timed_m if out)
        kb = sum(motor_bytes(q, b, out, nb) for nb, out in timed_m) / n_m
        kf = sum(motor_flops(q, out, nb) for nb, out in timed_m) / n_m
        steps_per_launch = sum(nb for nb, _ in timed_m) / n_m
        return dict(steps_per_s=sps, step_gbs=total / r["elapsed"] / 1e9, avg_us=ms_m / n_m * 1e3,
                    gbs=kb / (ms_m / n_m / 1e3) / 1e9, bytes_per_launch=kb, n_plain=n_m - n_out,
                    tflops=kf / (ms_m / n_m / 1e3) / 1e12, flops_per_launch=kf,
                    n_out=n_out, psi_avg_us=ms_p / n_p * 1e3, timed_launches=n_m, mass=r["mass"],
                    steps_per_launch=steps_per_launch,
                    motor_us_per_step=ms_m / n_m * 1e3 / steps_per_launch, b=b)

    def hbm_roofline(sm, counters=None):
        traffic = counters_traffic(sm["n_plain"], sm["n_out"], sm["steps_per_launch"], counters) \
            if counters and sm["b"] == 4 else None
        return {"bound": "hbm", "achieved": sm["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": sm["gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "motor column step, one launch per micro-step",
                "avg_launch_us": sm["avg_us"], "algorithmic_bytes_per_launch": sm["bytes_per_launch"],
                "timed_launches": sm["timed_launches"], "output_launches_timed": sm["n_out"]}

    def depletion_summary():
        sd = summarise(res["depletion"])
        d = {"m_total": M_TOTAL_BENCH, "micro_steps_per_s": sd["steps_per_s"],
             "ms_per_step": 1e3 / sd["steps_per_s"], "motor_avg_us": sd["avg_us"], "motor_gbs": sd["gbs"],
             "motor_frac": sd["gbs"] / HBM_PEAK_GBS, "psi_avg_us": sd["psi_avg_us"],
             "steps": res["depletion"]["steps"]}
        return d

    def substep_summary():
        """Simulated time per wall second with and without motor sub-cycling (fast motors);
        n per micro-step by the rule documented for mmk_params.motor_cfl."""
        d = {"v0": SUBSTEP_V0, "motor_cfl": MOTOR_CFL_BENCH}
        for key, name in (("fast_plain", "one_motor_step"), ("fast_sub", "subcycled")):
            r = res[key]
            sr = summarise(r)
            rate = SUBSTEP_V0 / (p.L / p.ns) + p.k_off
            n = max(1, math.ceil(r["dt"] * rate / MOTOR_CFL_BENCH)) if key == "fast_sub" else 1
            d[name] = {"dt": r["dt"], "motor_steps_per_micro_step": n, "micro_steps_per_s": sr["steps_per_s"],
                       "simulated_time_per_s": r["dt"] * sr["steps_per_s"],
                       "motor_us_per_micro_step": sr["motor_us_per_step"],
                       "motor_us_per_motor_step": sr["motor_us_per_step"] / n, "psi_avg_us": sr["psi_avg_us"]}
        d["speedup_simulated_time"] = (d["subcycled"]["simulated_time_per_s"]
                                       / d["one_motor_step"]["simulated_time_per_s"])
        for key, name in (("fast_depl_sub", "depleted_subcycled"),
                          ("fast_depl_sub_1", "depleted_subcycled_launch_per_substep")):
            if key in res:
                r = res[key]
                ms_m, n_m = r["prof"]["motor_step"]
                n = max(1, math.ceil(r["dt"] * (SUBSTEP_V0 / (p.L / p.ns) + p.k_off) / MOTOR_CFL_BENCH))
                launches = 1 if key == "fast_depl_sub" else n  # motor launches per micro-step
                d[name] = {"m_total": M_TOTAL_BENCH, "dt": r["dt"], "motor_steps_per_micro_step": n,
                           "micro_steps_per_s": r["steps"] / r["elapsed"],
                           "simulated_time_per_s": r["dt"] * r["steps"] / r["elapsed"],
                           "motor_us_per_micro_step": ms_m / n_m * 1e3 * launches}
        return d

    if args.only == "depletion":
        print(json.dumps({"depletion_fp32": depletion_summary()}), flush=True)
        return
    if args.only == "substeps":
        print(json.dumps({"substeps_fp32": substep_summary()}), flush=True)
        return
    if args.only in ("large", "c2"):
        d = {}
        if large:
            d["fp32_512x512x128x64"] = {k: (summarise(v) if isinstance(v, dict) else v) for k, v in large.items()}
        if c2:
            d["fp64_128x128x64x32"] = summarise(c2)
        print(json.dumps(d), flush=True)
        return

    out = {"metric": METRIC, "unit": "micro-steps/s", "n_gpus": 1, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    main_leg = "fp32" if "fp32" in res else ("fp32_1" if "fp32_1" in res else "fp64")
    s = summarise(res[main_leg])
    blocked = max(res[main_leg]["blocks"]) > 1
    out.update(value=s["steps_per_s"], steps=res[main_leg]["steps"], warmup=args.warmup,
               ms_per_step=1e3 / s["steps_per_s"], dtype="f32" if s["b"] == 4 else "f64",
               config={"workload": "256x256 grid, 64 orientations, 64 arclength cells, "
                                   f"{'FP32' if s['b'] == 4 else 'FP64'}, fluid exchange every 10 steps, "
                                   + ("motor field blocked over the 10 micro-steps of a call"
                                      if blocked else "one motor launch per micro-step"),
                       "nx": p.nx, "ny": p.ny, "ntheta": p.ntheta, "ns": p.ns,
                       "motor_cells": p.nx * p.ny * p.ntheta * p.ns, "K": K})
    if blocked:
        # the blocked launch does 10 micro-steps of arithmetic per read and write of M: the
        # vector ALU bounds it; the roof is the published FP32 (FP64) vector peak, with the
        # chip's measured issue rates beside it
        alu_peak = FP32_VECTOR_PEAK_TFLOPS if s["b"] == 4 else FP64_VECTOR_PEAK_TFLOPS
        traffic = counters_traffic(s["n_plain"], s["n_out"], s["steps_per_launch"]) if s["b"] == 4 else None
        roof = {"bound": "alu", "achieved": s["tflops"], "peak": alu_peak, "unit": "TFLOP/s",
                "frac": s["tflops"] / alu_peak, "traffic": traffic,
                "kernel": "motor column step, 10 micro-steps per launch (temporally blocked)"}
        if calib and "fma_f32" in calib:
            meas = calib["fma_f32" if s["b"] == 4 else "fma_f64"]["tflops"]
            roof.update(measured_fma_peak_tflops=meas, frac_of_measured_fma_peak=s["tflops"] / meas)
    else:
        roof = hbm_roofline(s, COUNTERS_PLAIN)
        roof["achieved"] = s["gbs"]
    roof.update({"avg_launch_us": s["avg_us"], "micro_steps_per_launch": s["steps_per_launch"],
                 "motor_us_per_micro_step": s["motor_us_per_step"],
                 "algorithmic_bytes_per_launch": s["bytes_per_launch"], "hbm_gbs": s["gbs"],
                 "hbm_frac": s["gbs"] / HBM_PEAK_GBS, "algorithmic_flops_per_launch": s["flops_per_launch"],
                 "alu_tflops": s["tflops"], "timed_launches": s["timed_launches"],
                 "output_launches_timed": s["n_out"]})
    out["roofline"] = roof
    out["step_hbm_gbs"] = s["step_gbs"]
    out["step_hbm_frac"] = s["step_gbs"] / HBM_PEAK_GBS
    out["psi_step_avg_us"] = s["psi_avg_us"]
    if "fp32" in res and "fp64" in res:
        s64 = summarise(res["fp64"])
        out["fp64"] = {"micro_steps_per_s": s64["steps_per_s"], "ms_per_step": 1e3 / s64["steps_per_s"],
                       "step_hbm_gbs": s64["step_gbs"], "motor_gbs": s64["gbs"],
                       "motor_tflops": s64["tflops"], "motor_alu_frac": s64["tflops"] / FP64_VECTOR_PEAK_TFLOPS,
                       "motor_avg_us": s64["avg_us"], "psi_avg_us": s64["psi_avg_us"],
                       "steps": res["fp64"]["steps"]}
        out["fp32_over_fp64"] = s["steps_per_s"] / s64["steps_per_s"]
    if "fp32_1" in res and "fp64_1" in res:
        a1, b1 = summarise(res["fp32_1"]), summarise(res["fp64_1"])
        out["one_launch_per_step"] = {
            "fp32_micro_steps_per_s": a1["steps_per_s"], "fp64_micro_steps_per_s": b1["steps_per_s"],
            "fp32_ms_per_step": 1e3 / a1["steps_per_s"], "fp32_step_hbm_gbs": a1["step_gbs"],
            "fp32_step_hbm_frac": a1["step_gbs"] / HBM_PEAK_GBS, "fp64_step_hbm_gbs": b1["step_gbs"],
            "fp64_step_hbm_frac": b1["step_gbs"] / HBM_PEAK_GBS,
            "fp32_psi_avg_us": a1["psi_avg_us"], "fp64_psi_avg_us": b1["psi_avg_us"],
            "fp32_over_fp64": a1["steps_per_s"] / b1["steps_per_s"],
            "roofline": hbm_roofline(a1, COUNTERS_PLAIN), "roofline_fp64": hbm_roofline(b1)}
    if large:
        lb, l1 = summarise(large["blocked"]), summarise(large["one_launch"])
        pl = large["blocked"]["p"]
        out["fp32_512x512x128x64"] = {
            "motor_cells": pl.nx * pl.ny * pl.ntheta * pl.ns, "steps": large["blocked"]["steps"],
            "micro_steps_per_s": lb["steps_per_s"], "step_hbm_gbs": lb["step_gbs"], "motor_avg_us": lb["avg_us"],
            "motor_tflops": lb["tflops"], "psi_avg_us": lb["psi_avg_us"],
            "one_launch_micro_steps_per_s": l1["steps_per_s"], "one_launch_step_hbm_gbs": l1["step_gbs"],
            "one_launch_step_hbm_frac": l1["step_gbs"] / HBM_PEAK_GBS, "one_launch_motor_gbs": l1["gbs"],
            "one_launch_motor_frac": l1["gbs"] / HBM_PEAK_GBS, "one_launch_psi_avg_us": l1["psi_avg_us"],
            "peak_device_gb": large["peak_device_gb"]}
    if c2:
        sc = summarise(c2)
        out["fp64_128x128x64x32"] = {"steps": c2["steps"], "micro_steps_per_s": sc["steps_per_s"],
                                     "ms_per_step": 1e3 / sc["steps_per_s"], "step_hbm_gbs": sc["step_gbs"],
                                     "motor_avg_us": sc["avg_us"], "psi_avg_us": sc["psi_avg_us"]}
    if args.only == "all":
        log("[bench] launch-bound leg")
        out["launch_bound_fp64_16x16x16x16"] = run_launch_bound(50)
        log("[bench] motor force leg")
        out["force_fp32"] = run_force(p, mmk.FP32, 10)
    if "fast_sub" in res:
        out["substeps_fp32"] = substep_summary()
    if args.only == "all":
        out["anchor_resolved_fp32"] = run_r0(mmk.FP32, args.r0_steps, 20, K, args.event_every)
        out["anchor_resolved_fp64"] = run_r0(mmk.FP64, args.r0_steps, 20, K, args.event_every)
        out["anchor_resolved_substeps_fp32"] = r0_substeps(args)
    if "depletion" in res:
        out["depletion_fp32"] = depletion_summary()
        out["depletion_fp32"]["relative_to_linear"] = out["depletion_fp32"]["micro_steps_per_s"] / s["steps_per_s"]
    out["adjoint_over_forward"] = None
    if args.only == "all" and not args.no_adjoint:
        log("[bench] adjoint legs")
        adj32 = run_adjoint("adjoint_fp32_256x256x64x32", mmk.FP32)
        adj64 = run_adjoint("adjoint_fp64_64x64x32x32", mmk.FP64)
        out["adjoint_over_forward"] = adj32["ratio"]
        out["adjoint"] = {"fp32_256x256x64x32_C25": adj32, "fp64_64x64x32x32_C20": adj64}
    if calib:
        out["valu_calibration"] = calib
    if not args.no_cpu_baseline:
        rec, o, dt0 = cpu_baseline(p, args.cpu_steps)
        out["cpu_baseline"] = rec
        log("[bench] FP32 error per output against the oracle")
        out["fp32_error_vs_fp64_oracle"] = fp32_errors(p, o, dt0, args.cpu_steps)
        del o
        if args.only == "all":
            log("[bench] oracle on one thread")
            out["cpu_oracle_one_thread"] = {
                "fp64_16x16x16x16": cpu_oracle_one_thread("fp64_16x16x16x16", 100),
                "fp64_128x128x64x32": cpu_oracle_one_thread("fp64_128x128x64x32", 20)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
