"""Throughput of the gliding-assay micro-step on one MI355X.

Workload (the measured configuration): 256 x 256 periodic grid, 64 orientations, 64
arclength cells (268M bound-motor cells), FP32 storage and arithmetic, a new seeded fluid
field every K = 10 micro-steps, stress/moments/global sums on every exchange.  A "step" is
one micro-step of the whole path: motor column step, s-moments, psi donor-cell update,
and (every 10th) theta-moments, stress and FP64 global sums.  Inputs are resident in HBM
before the timed region.  Also measured: the same grid in FP64, and the oracle (FP64 C,
OpenMP) on a bounded sample of the same grid on the host cores.

Prints one JSON line.  --gpus N > 1 is refused: this path runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "micro-steps/s + HBM GB/s (% peak), FP32 vs FP64 at 256²×64×64; adjoint/fwd ratio"
COUNTERS = os.path.join(ROOT, "profiles", "motor_step_f32_256x256x64x64_counters.txt")
MOTOR_SRC = os.path.join(ROOT, "paper_1908_04279_amd", "csrc", "motor.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def motor_bytes(p, b, with_m1):
    n_psi = p.nx * p.ny * p.ntheta
    return b * (2 * n_psi * p.ns + n_psi * (2 if with_m1 else 1))


def step_bytes(p, b, out):
    """Algorithmic HBM bytes of one micro-step: motor kernel (read M, write M, write m0
    [and m1]) + psi kernel (read psi, m0, u, gradu; write psi [read m1, write stress and
    moments])."""
    n_psi = p.nx * p.ny * p.ntheta
    nxy = p.nx * p.ny
    psi = b * (3 * n_psi + 6 * nxy) + (b * (n_psi + 10 * nxy) if out else 0)
    return motor_bytes(p, b, out) + psi


def run_forward(p, precision, steps, warmup, K, profile=True):
    import torch
    from paper_1908_04279_amd import inputs as gen
    from paper_1908_04279_amd import mmk

    n_ex = (warmup + steps) // K + 2
    log(f"[bench] generating {n_ex} fluid fields for {p.nx}x{p.ny}")
    fluids_np = [gen.make_fluid(p.nx, p.ny, p.lx, p.ly, seed=1 + e) for e in range(n_ex)]
    dt = gen.cfl_dt(p, fluids_np)
    ctx = mmk.Context(p, precision=precision)
    fl = [(torch.as_tensor(u).to(ctx.device, ctx.dtype), torch.as_tensor(g).to(ctx.device, ctx.dtype))
          for u, g in fluids_np]
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=0)
    ctx.set_state(torch.as_tensor(psi0))
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

    log(f"[bench] warmup {warmup} steps")
    e = advance(warmup, 0)
    torch.cuda.synchronize()
    if profile:
        ctx.profile(True)
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
    return dict(elapsed=elapsed, steps=steps, dt=dt, prof=prof, mass=mass)


def counters_traffic(bytes_per_launch):
    """HBM bytes per motor-step launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on a different motor kernel source."""
    if not os.path.exists(COUNTERS):
        return None
    kv = {}
    for line in open(COUNTERS):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k.strip()] = v.strip()
    src_sha = hashlib.sha256(open(MOTOR_SRC, "rb").read()).hexdigest()[:16]
    if kv.get("motor_hip_sha256_16") != src_sha:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(p, sample_steps):
    """The FP64 C oracle on the same grid, a few micro-steps, on the host cores."""
    from oracle import oracle_a as A
    from paper_1908_04279_amd import inputs as gen
    u, g = gen.make_fluid(p.nx, p.ny, p.lx, p.ly, seed=1)
    dt = gen.cfl_dt(p, [(u, g)])
    o = A.OracleA(p)
    o.set_state(gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=0))
    o.set_fluid(u, g)
    threads = A.max_threads()
    log(f"[bench] cpu baseline: oracle, {sample_steps} steps, {threads} threads")
    t0 = time.perf_counter()
    o.step(sample_steps, dt)
    el = time.perf_counter() - t0
    return dict(value=sample_steps / el, unit="micro-steps/s", cores=threads, kind="oracle",
                sample=f"{sample_steps} FP64 micro-steps of the full {p.nx}x{p.ny}x{p.ntheta}x{p.ns} grid "
                       f"(C oracle, OpenMP over x rows), {el:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--fp64-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["all", "fp32", "fp64"], default="all",
                    help="restrict to one leg (used for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this micro-step path runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_04279_amd import inputs as gen
    from paper_1908_04279_amd import mmk
    mmk.lib()   # fail loudly if the HIP library is missing
    torch.cuda.set_device(0)

    p = gen.params_for("c3_fp32_256x256x64x64")
    K = 10
    res = {}
    if args.only in ("all", "fp32"):
        res["fp32"] = run_forward(p, mmk.FP32, args.steps, args.warmup, K)
    if args.only in ("all", "fp64"):
        res["fp64"] = run_forward(p, mmk.FP64, args.fp64_steps, min(args.warmup, 20), K)

    def summarise(r, b):
        n_out = r["steps"] // K
        sps = r["steps"] / r["elapsed"]
        total = (r["steps"] - n_out) * step_bytes(p, b, False) + n_out * step_bytes(p, b, True)
        ms, n = r["prof"]["motor_step"]
        mb = ((n - n_out) * motor_bytes(p, b, False) + n_out * motor_bytes(p, b, True)) / max(n, 1)
        motor_gbs = mb / (ms / n / 1e3) / 1e9
        return dict(steps_per_s=sps, step_gbs=total / r["elapsed"] / 1e9,
                    motor_avg_us=ms / n * 1e3, motor_gbs=motor_gbs, motor_bytes_per_launch=mb,
                    psi_avg_us=r["prof"]["psi_step"][0] / r["prof"]["psi_step"][1] * 1e3,
                    mass=r["mass"])

    out = {"metric": METRIC, "unit": "micro-steps/s", "n_gpus": 1, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    main_leg = "fp32" if "fp32" in res else "fp64"
    b_main = 4 if main_leg == "fp32" else 8
    s = summarise(res[main_leg], b_main)
    out.update(value=s["steps_per_s"], steps=res[main_leg]["steps"], warmup=args.warmup,
               ms_per_step=1e3 / s["steps_per_s"], dtype="f32" if main_leg == "fp32" else "f64",
               config={"workload": "256x256 grid, 64 orientations, 64 arclength cells, "
                                   f"{'FP32' if main_leg == 'fp32' else 'FP64'}, fluid exchange every 10 steps",
                       "nx": p.nx, "ny": p.ny, "ntheta": p.ntheta, "ns": p.ns,
                       "motor_cells": p.nx * p.ny * p.ntheta * p.ns, "K": K})
    traffic = counters_traffic(s["motor_bytes_per_launch"]) if main_leg == "fp32" else None
    out["roofline"] = {"bound": "hbm", "achieved": s["motor_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": s["motor_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                       "kernel": "motor column step", "avg_launch_us": s["motor_avg_us"],
                       "algorithmic_bytes_per_launch": s["motor_bytes_per_launch"]}
    out["step_hbm_gbs"] = s["step_gbs"]
    out["step_hbm_frac"] = s["step_gbs"] / HBM_PEAK_GBS
    out["psi_step_avg_us"] = s["psi_avg_us"]
    if "fp32" in res and "fp64" in res:
        s64 = summarise(res["fp64"], 8)
        out["fp64"] = {"micro_steps_per_s": s64["steps_per_s"], "ms_per_step": 1e3 / s64["steps_per_s"],
                       "step_hbm_gbs": s64["step_gbs"], "motor_gbs": s64["motor_gbs"],
                       "motor_frac": s64["motor_gbs"] / HBM_PEAK_GBS, "motor_avg_us": s64["motor_avg_us"],
                       "steps": res["fp64"]["steps"]}
        out["fp32_over_fp64"] = s["steps_per_s"] / s64["steps_per_s"]
    out["adjoint_over_forward"] = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
