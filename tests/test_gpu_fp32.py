"""FP32 storage-and-arithmetic path against the FP64 oracle.

Bar: norm-wise relative error <= 1e-5 on stress and moments (the FP32 target); the errors
of psi, M, m0 and the mass drift are printed alongside."""
import numpy as np
import pytest

from paper_1908_04279_amd import inputs as gen
from paper_1908_04279_amd.inputs import ModelParams
from tests.conftest import rel_err
from tests.runners import run_gpu, run_oracle, run_oracle_uniform_columns, seeded_case

pytestmark = pytest.mark.gpu
TOL = 1e-5


def report(g, o, fields):
    errs = {f: rel_err(g[f], o[f]) for f in fields}
    errs["mass"] = abs(g["mass"] - o["mass"]) / abs(o["mass"])
    errs["sum_sigma"] = rel_err(g["sum_sigma"], o["sum_sigma"])
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    return errs


@pytest.mark.parametrize("ns", [16, 32, 64, 128, 20])
def test_random_M0_small_grids(ns):
    p = ModelParams(nx=9, ny=7, ntheta=16, ns=ns)
    psi0, M0, fl, dt = seeded_case(p, n_exchanges=3, M0_kind="random")
    g = run_gpu(p, psi0, M0, fl, 10, 30, dt, precision=1)
    o = run_oracle(p, psi0, M0, fl, 10, 30, dt)
    e = report(g, o, ["psi", "M", "m0", "m1", "stress", "mom"])
    assert e["stress"] <= TOL and e["mom"] <= TOL
    assert e["psi"] <= TOL and e["M"] <= TOL


def test_fp32_16x16x16x16():
    p = gen.params_for("fp64_16x16x16x16")
    psi0, M0, fl, dt = seeded_case(p)
    g = run_gpu(p, psi0, None, fl, 100, 100, dt, precision=1)
    o = run_oracle(p, psi0, np.zeros((16, 16, 16, 16)), fl, 100, 100, dt)
    e = report(g, o, ["psi", "M", "m0", "m1", "stress", "mom"])
    assert e["stress"] <= TOL and e["mom"] <= TOL


def test_fp32_256x256x64x64_full_size():
    """256^2 x 64 x 64 FP32, 500 steps, a new fluid field every 10 steps, against the FP64
    oracle (column decomposition: M0 = 0 gives identical columns)."""
    p = gen.params_for("fp32_256x256x64x64")
    psi0, _, fl, dt = seeded_case(p, n_exchanges=50)
    print("gpu", flush=True)
    g = run_gpu(p, psi0, None, fl, 10, 500, dt, precision=1, want_M=False, keep_ctx=True)
    import torch
    _, M = g["ctx"].get_state()
    print("oracle", flush=True)
    o = run_oracle_uniform_columns(p, psi0, fl, 10, 500, dt)
    col = torch.as_tensor(o["col"], dtype=torch.float64, device=M.device)
    m_err = float((M.double() - col).abs().max() / col.abs().max())
    g["ctx"].close()
    e = report(g, o, ["psi", "m0", "m1", "stress", "mom"])
    print(f"M (all columns vs the oracle column): {m_err:.2e}; mass drift {abs(g['mass'] - 1.0):.2e}", flush=True)
    assert e["stress"] <= TOL and e["mom"] <= TOL
    assert m_err <= TOL and e["psi"] <= TOL


@pytest.mark.parametrize("block", [1, 0])
def test_fp32_s_moments_error_bound(block):
    """The FP32 s-reductions (a lane's cells added pairwise in FP32, the lane partials in FP64,
    one rounding to FP32): m0 and m1 of columns whose cells span nine decades lie within 8 units
    of 2^-24 of the exact sums of the same FP32 cells, relative to the sums of magnitudes (the
    bound of the form is log2(cells a lane) + 2 units); both the blocked launch (16 cells a
    lane) and one launch per step (4 cells a lane)."""
    import math
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=6, ny=5, ntheta=16, ns=64)
    rng = np.random.default_rng(11)
    M0 = (10.0 ** rng.uniform(-6, 3, (p.nx, p.ny, p.ntheta, p.ns))).astype(np.float32)
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=0).astype(np.float32)
    fl = gen.fluid_schedule(p.nx, p.ny, 1, p.lx, p.ly)
    ctx = mmk.Context(p, precision=mmk.FP32, options={"motor_block": block})
    ctx.set_state(torch.as_tensor(psi0), torch.as_tensor(M0))
    ctx.set_fluid(*map(torch.as_tensor, fl[0]))
    ctx.step(3, 1e-4)
    _, M = ctx.get_state()
    m0, m1 = ctx.get_motor_moments()
    M = M.double().cpu().numpy().reshape(-1, p.ns)
    m0 = m0.double().cpu().numpy().ravel()
    m1 = m1.double().cpu().numpy().ravel()
    ctx.close()
    ds = float(np.float32(p.L / p.ns))
    ds2 = float(np.float32((p.L / p.ns) ** 2))
    w = np.arange(p.ns) + 0.5 - p.ns / 2
    u = 2.0 ** -24
    worst0 = worst1 = 0.0
    for c in range(M.shape[0]):
        ex0 = math.fsum(M[c]) * ds
        t1 = M[c] * w                     # exact: FP32 cells times half-integers
        ex1 = math.fsum(t1) * ds2
        worst0 = max(worst0, abs(m0[c] - ex0) / (np.abs(M[c]).sum() * ds))
        worst1 = max(worst1, abs(m1[c] - ex1) / (np.abs(t1).sum() * ds2))
    print(f"m0: {worst0 / u:.2f} u, m1: {worst1 / u:.2f} u", flush=True)
    assert worst0 <= 8 * u and worst1 <= 8 * u
