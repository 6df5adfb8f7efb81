"""Seeded synthetic inputs for the gliding-assay micro-step.

This module only *draws* inputs: initial filament densities, fluid fields, random
initial motor densities, target stresses and perturbation directions, plus a step
size picked from the advective CFL bound.  It performs none of the micro-step's own
arithmetic (no motor transport, no flux update, no moments), so both the HIP path's
tests/benchmark and the FP64 oracle's tests can take their inputs from here without
sharing any of the method's code.

Conventions (Cook & Shinar, Sec. 2: Psi(x, p) with p = (cos th, sin th); theta and
s are discretised uniformly):
  * periodic box [0, lx) x [0, ly), cell-centred x_i = (i + 1/2) dx, y_j = (j + 1/2) dy
  * theta_k = k * dth with dth = 2 pi / ntheta
  * arrays are C-contiguous numpy float64:
      psi   [nx][ny][ntheta]
      M     [nx][ny][ntheta][ns]
      u     [2][nx][ny]           (u_x, u_y)
      gradu [4][nx][ny]           (du_x/dx, du_x/dy, du_y/dx, du_y/dy)
      sigma [3][nx][ny]           (xx, xy, yy)

Nothing here is a published benchmark: the paper measures on its own simulations
(a lattice of filament rings whose initial condition it does not give), so these
seeded fields stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass
class ModelParams:
    """Grid and model coefficients of one micro-step problem (defaults: the seeded workloads)."""
    nx: int
    ny: int
    ntheta: int
    ns: int
    lx: float = TWO_PI
    ly: float = TWO_PI
    L: float = 1.0
    k_on: float = 1.0
    k_off: float = 0.5
    v0: float = 1.0
    F: float = 1.0
    sigma_f: float = 1.0
    limiter: int = 0          # 0: superbee-limited MUSCL flux in s, 1: first-order upwind
    m_total: float = 0.0      # total motors per unit area (free-motor depletion); 0: pool of 1
    motor_cfl: float = 0.0    # > 0: the motor step sub-cycles at this CFL number; 0: one step
    rc: float = 0.0           # > 0: anchor-resolved bound motors with this capture radius

    def as_dict(self):
        return asdict(self)


# The five seeded workloads: plain FP64 small case, paper-like FP64 scale, FP32 at
# 256^2 x 64 x 64, the adjoint case, and the largest single-GPU forward case.
CONFIGS = {
    "fp64_16x16x16x16": dict(nx=16, ny=16, ntheta=16, ns=16, steps=100, K=100,
                                precision="fp64", new_fluid_each_exchange=False),
    "fp64_128x128x64x32": dict(nx=128, ny=128, ntheta=64, ns=32, steps=1000, K=10,
                                  precision="fp64", new_fluid_each_exchange=True),
    "fp32_256x256x64x64": dict(nx=256, ny=256, ntheta=64, ns=64, steps=500, K=10,
                                  precision="fp32", new_fluid_each_exchange=True),
    "adjoint_fp64_64x64x32x32": dict(nx=64, ny=64, ntheta=32, ns=32, steps=200, K=200,
                                        ckpt=20, precision="fp64",
                                        new_fluid_each_exchange=False),
    "fp32_512x512x128x64": dict(nx=512, ny=512, ntheta=128, ns=64, steps=200, K=10,
                                   precision="fp32", new_fluid_each_exchange=True),
    "adjoint_fp32_256x256x64x32": dict(nx=256, ny=256, ntheta=64, ns=32, steps=200,
                                          K=10, ckpt=25, precision="fp32",
                                          new_fluid_each_exchange=True),
}


def params_for(name: str, **over) -> ModelParams:
    c = CONFIGS[name]
    kw = dict(nx=c["nx"], ny=c["ny"], ntheta=c["ntheta"], ns=c["ns"])
    kw.update(over)
    return ModelParams(**kw)


def _axes(nx, ny, ntheta, lx, ly):
    x = (np.arange(nx) + 0.5) * (lx / nx)
    y = (np.arange(ny) + 0.5) * (ly / ny)
    th = np.arange(ntheta) * (TWO_PI / ntheta)
    return x, y, th


def _draw_wavevector(rng, n):
    while True:
        k = rng.integers(-2, 3, n)
        if np.any(k != 0):
            return k


def make_psi0(nx, ny, ntheta, lx=TWO_PI, ly=TWO_PI, seed=0, n_modes=4, amp=0.1):
    """Psi0 = 1 + amp * sum_m cos(2 pi a x/lx + 2 pi b y/ly + c th + phi_m), unit mass.

    (a, b, c) are integer wavenumbers in [-2, 2] (redrawn if all zero), phi_m ~ U[0, 2 pi).
    Normalised so that sum(psi) dx dy dth = 1.
    """
    rng = np.random.default_rng(seed)
    x, y, th = _axes(nx, ny, ntheta, lx, ly)
    X, Y, T = np.meshgrid(x, y, th, indexing="ij")
    psi = np.ones((nx, ny, ntheta))
    for _ in range(n_modes):
        a, b, c = _draw_wavevector(rng, 3)
        phi = rng.uniform(0.0, TWO_PI)
        psi += amp * np.cos(TWO_PI * a * X / lx + TWO_PI * b * Y / ly + c * T + phi)
    vol = (lx / nx) * (ly / ny) * (TWO_PI / ntheta)
    psi /= psi.sum() * vol
    return np.ascontiguousarray(psi)


def make_fluid(nx, ny, lx=TWO_PI, ly=TWO_PI, seed=1, n_modes=3, amp=0.1):
    """Divergence-free velocity from a random stream function and its exact gradient.

    stream = sum_m (amp/|k_m|) sin(k_m . x + phi_m), u_x = d stream/dy, u_y = -d stream/dx,
    so each mode has speed amplitude exactly `amp`.  Returns (u[2][nx][ny], gradu[4][nx][ny])
    with gradu = (du_x/dx, du_x/dy, du_y/dx, du_y/dy), evaluated analytically.
    """
    rng = np.random.default_rng(seed)
    x, y, _ = _axes(nx, ny, 1, lx, ly)
    X, Y = np.meshgrid(x, y, indexing="ij")
    u = np.zeros((2, nx, ny))
    g = np.zeros((4, nx, ny))
    for _ in range(n_modes):
        a, b = _draw_wavevector(rng, 2)
        phi = rng.uniform(0.0, TWO_PI)
        kx, ky = TWO_PI * a / lx, TWO_PI * b / ly
        kn = math.hypot(kx, ky)
        arg = kx * X + ky * Y + phi
        c, s = np.cos(arg), np.sin(arg)
        w = amp / kn
        u[0] += w * ky * c          # d/dy of w sin(arg)
        u[1] += -w * kx * c         # -d/dx
        g[0] += -w * ky * kx * s    # d u_x / dx
        g[1] += -w * ky * ky * s    # d u_x / dy
        g[2] += w * kx * kx * s     # d u_y / dx
        g[3] += w * kx * ky * s     # d u_y / dy
    return np.ascontiguousarray(u), np.ascontiguousarray(g)


def fluid_schedule(nx, ny, n_exchanges, lx=TWO_PI, ly=TWO_PI, new_each=True, base_seed=1):
    """One fluid field per exchange; seed base_seed + exchange index (or one fixed field)."""
    out = []
    for e in range(n_exchanges):
        out.append(make_fluid(nx, ny, lx, ly, seed=base_seed + (e if new_each else 0)))
    return out


def make_M0_random(nx, ny, ntheta, ns, k_on=1.0, k_off=0.5, seed=5):
    """Random non-uniform bound-motor density, U[0, k_on/k_off], so columns differ."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(0.0, k_on / k_off, (nx, ny, ntheta, ns)))


def M0_columns_values(cols, ns, k_on=1.0, k_off=0.5):
    """Closed-form bound-motor density whose columns differ (no random draw, so any column can
    be formed on its own): column c (flat index of (x, y, th)) holds
        (1 + (c mod 97) / 97) * (k_on / k_off) * (l + 1/2) / ns,   l = 0 .. ns-1,
    in FP64.  97 is prime, so columns 2^k apart (a wrapped 32-bit offset) hold other values.
    cols: integer array of column indices; returns [len(cols)][ns]."""
    cols = np.asarray(cols, dtype=np.int64)
    w = 1.0 + (cols % 97).astype(np.float64) / 97.0
    ramp = (k_on / k_off) * (np.arange(ns, dtype=np.float64) + 0.5) / ns
    return w[:, None] * ramp[None, :]


def make_M0_columns_device(nx, ny, ntheta, ns, dtype, device, k_on=1.0, k_off=0.5, chunk=1 << 22):
    """M0_columns_values for every column of the grid, formed on the device in FP64 and rounded
    once to `dtype` (the same values as the host form), [nx][ny][ntheta][ns]; built in chunks of
    columns to bound the FP64 temporaries."""
    import torch
    ncol = nx * ny * ntheta
    out = torch.empty((ncol, ns), dtype=dtype, device=device)
    ramp = (k_on / k_off) * (torch.arange(ns, dtype=torch.float64, device=device) + 0.5) / ns
    for c0 in range(0, ncol, chunk):
        c1 = min(ncol, c0 + chunk)
        cols = torch.arange(c0, c1, dtype=torch.int64, device=device)
        w = 1.0 + (cols % 97).to(torch.float64) / 97.0
        out[c0:c1] = (w[:, None] * ramp[None, :]).to(dtype)
    return out.view(nx, ny, ntheta, ns)


def make_Mb0_random(ncell, nx, ny, k_on=1.0, k_off=0.5, seed=6):
    """Random anchor-resolved bound-motor density [ncell][nx][ny], U[0, k_on/k_off]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, k_on / k_off, (ncell, nx, ny))


def make_target_stress(nx, ny, seed=3, scale=1e-3):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(scale * rng.standard_normal((3, nx, ny)))


def make_direction(shape, seed):
    """N(0,1) direction scaled to max |d| = 1."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(shape)
    return np.ascontiguousarray(d / np.abs(d).max())


def cfl_dt(p: ModelParams, fluids, cfl=0.4):
    """Step size from the advective stability limits (one fixed dt per run).

    rate_M   = v0/ds + k_off                            (motor walk + detachment)
    rate_Psi = (max|u_x| + F m_bar)/dx + (max|u_y| + F m_bar)/dy + max sum|gradu|/dth
    with m_bar = L k_on P / k_off the largest steady bound-motor count per filament, P the
    free-motor pool (1, or m_total if larger under depletion).
    dt = cfl / max(rate_M, rate_Psi), minimised over every fluid field of the run; with
    p.motor_cfl > 0 the motor step sub-cycles and rate_M is left out.
    """
    ds = p.L / p.ns
    dx, dy, dth = p.lx / p.nx, p.ly / p.ny, TWO_PI / p.ntheta
    pool = max(1.0, getattr(p, "m_total", 0.0))
    m_bar = p.L * p.k_on * pool / p.k_off if p.k_off > 0 else 0.0
    rate_m = 0.0 if getattr(p, "motor_cfl", 0.0) > 0 else p.v0 / ds + p.k_off
    best = math.inf
    for u, g in fluids:
        rate_psi = ((np.abs(u[0]).max() + p.F * m_bar) / dx
                    + (np.abs(u[1]).max() + p.F * m_bar) / dy
                    + np.abs(g).sum(axis=0).max() / dth)
        best = min(best, cfl / max(rate_m, rate_psi))
    return float(best)
