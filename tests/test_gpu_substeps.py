"""Motor sub-cycling on the GPU (n midpoint steps of dt/n inside one motor launch) against the
FP64 oracle: every column tiling of the motor kernel, both limiters, FP64 1e-12 and FP32
1e-5 (norm-wise relative per field); the refusals; temporal blocking of the motor field
(several micro-steps per launch) against the one-launch-per-step order, bit for bit."""
import numpy as np
import pytest

from oracle import oracle_a as A
from paper_1908_04279_amd import inputs as gen
from paper_1908_04279_amd.inputs import ModelParams
from tests.conftest import rel_err
from tests.runners import run_gpu, run_oracle

pytestmark = pytest.mark.gpu
FIELDS = ["psi", "M", "m0", "m1", "stress", "mom"]


def substep_case(p, n, n_exchanges=2):
    """Seeded state and fluids; motor CFL 0.4 and a dt of n - 1/2 motor limits, so that a
    micro-step takes n motor sub-steps (the psi step stays inside its own limit)."""
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=0)
    M0 = gen.make_M0_random(p.nx, p.ny, p.ntheta, p.ns, p.k_on, p.k_off, seed=5)
    fl = gen.fluid_schedule(p.nx, p.ny, n_exchanges, p.lx, p.ly)
    p.motor_cfl = 0.4
    dt = (n - 0.5) * 0.4 / (p.v0 / (p.L / p.ns) + p.k_off)
    assert dt <= gen.cfl_dt(p, fl)  # the psi limit alone
    assert A.motor_substeps(p, dt) == n
    return psi0, M0, fl, dt


def compare(g, o, tol):
    errs = {f: rel_err(g[f], o[f]) for f in FIELDS}
    errs["mass"] = abs(g["mass"] - o["mass"]) / abs(o["mass"])
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)


@pytest.mark.parametrize("shape,limiter,n", [
    ((6, 5, 16, 64), 0, 2),     # 16 lanes per column (FP64 64 = 32 x 2 cells)
    ((6, 5, 16, 16), 1, 3),     # 8 lanes
    ((7, 4, 32, 8), 0, 5),      # 4 lanes
    ((5, 6, 12, 128), 0, 2),    # cross-row column
    ((9, 3, 16, 20), 0, 7),     # masked generic kernel
    ((4, 4, 8, 5), 1, 4),       # masked, short
])
def test_fp64_against_oracle(shape, limiter, n):
    nx, ny, nt, ns = shape
    # fast motors: the motor limit sits well inside the psi limit, so n sub-steps fit
    p = ModelParams(nx=nx, ny=ny, ntheta=nt, ns=ns, limiter=limiter, k_on=0.9, k_off=0.6, v0=4.0, F=0.8)
    psi0, M0, fl, dt = substep_case(p, n)
    g = run_gpu(p, psi0, M0, fl, 4, 8, dt)
    o = run_oracle(p, psi0, M0, fl, 4, 8, dt)
    compare(g, o, 1e-12)


def test_chunked_blocked_against_oracle():
    """The chunked tiling (16 cells a lane) with sub-cycling inside blocks, FP64, against the
    oracle."""
    p = ModelParams(nx=6, ny=5, ntheta=16, ns=64, k_on=0.9, k_off=0.6, v0=4.0, F=0.8)
    psi0, M0, fl, dt = substep_case(p, 3)
    g = run_gpu(p, psi0, M0, fl, 9, 18, dt, options={"motor_chunks": 4})
    o = run_oracle(p, psi0, M0, fl, 9, 18, dt)
    compare(g, o, 1e-12)


@pytest.mark.parametrize("shape,n", [((20, 18, 64, 64), 3), ((9, 7, 32, 32), 2), ((6, 5, 16, 100), 4)])
def test_fp32_against_fp64_oracle(shape, n):
    nx, ny, nt, ns = shape
    p = ModelParams(nx=nx, ny=ny, ntheta=nt, ns=ns)
    psi0, M0, fl, dt = substep_case(p, n)
    g = run_gpu(p, psi0.astype(np.float32), M0.astype(np.float32), fl, 5, 10, dt, precision=1)
    o = run_oracle(p, psi0.astype(np.float32).astype(np.float64), M0.astype(np.float32).astype(np.float64),
                   fl, 5, 10, dt)
    compare(g, o, 1e-5)


def test_one_substep_is_the_plain_step():
    """A motor_cfl above the step's need (n = 1) gives the same bits as no sub-cycling."""
    p = ModelParams(nx=8, ny=6, ntheta=16, ns=32)
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=0)
    M0 = gen.make_M0_random(p.nx, p.ny, p.ntheta, p.ns, seed=5)
    fl = gen.fluid_schedule(p.nx, p.ny, 1, p.lx, p.ly)
    dt = gen.cfl_dt(p, fl)
    a = run_gpu(p, psi0, M0, fl, 6, 6, dt)
    q = ModelParams(**{**p.as_dict(), "motor_cfl": 10.0})
    assert A.motor_substeps(q, dt) == 1
    b = run_gpu(q, psi0, M0, fl, 6, 6, dt)
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), f


def test_refusals():
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=4, ny=4, ntheta=8, ns=8, motor_cfl=0.4)
    ctx = mmk.Context(p, ckpt_every=4, max_tape_steps=8)
    ctx.set_state(torch.as_tensor(gen.make_psi0(4, 4, 8, seed=0)))
    ctx.set_fluid(*map(torch.as_tensor, gen.make_fluid(4, 4)))
    with pytest.raises(mmk.MMKError) as ei:
        ctx.tape_begin(4)
    assert ei.value.status == mmk.MMK_ERR_UNSUPPORTED
    with pytest.raises(mmk.MMKError) as ei:  # more than 4096 sub-steps
        ctx.step(1, 1.0e4)
    assert ei.value.status == mmk.MMK_ERR_ARG
    ctx.close()


@pytest.mark.parametrize("shape,precision,calls,tiling", [
    ((8, 6, 16, 32), 0, [1, 7, 16, 17, 33], None),   # blocks of 16 with every remainder kind
    ((9, 5, 12, 20), 0, [10, 3], None),              # masked generic kernel
    ((12, 10, 64, 64), 1, [10, 10, 25], None),       # FP32, the default wide tiling (16 cells a lane)
    ((12, 10, 64, 32), 1, [10, 6], None),            # FP32, 8 cells a lane
    ((12, 10, 64, 64), 0, [10, 10, 25], None),       # FP64, 8 cells a lane
    ((12, 10, 64, 64), 1, [10, 7], {"motor_chunks": 2}),   # FP32, chunked tiling (8 cells a lane)
    ((8, 6, 16, 64), 0, [12, 5], {"motor_chunks": 2}),     # FP64, chunked tiling
])
def test_temporal_blocking_is_bitwise_serial(shape, precision, calls, tiling):
    """A run of several mmk_step calls gives the same bits with the motor field blocked over
    up to 16 micro-steps per launch (the default for m_total = 0) and with one launch per
    micro-step (motor_block = 0); also with sub-cycling inside the blocks.  The serial run is
    given the blocked run's column tiling through the motor_lanes option (the blocked default:
    16 cells a lane for FP32 columns of 64, 32 bytes a lane otherwise; a one-launch-per-step
    context would otherwise take 16 bytes, which sums the s-moments in another order)."""
    import torch
    from paper_1908_04279_amd import mmk
    nx, ny, nt, ns = shape
    if tiling is None:
        # the blocked default: 16 cells a lane for FP32 columns of 64, else 32 bytes a lane
        # (lengths without an exact tiling take the masked generic kernel in both runs)
        cpl = (16 if ns == 64 else 8) if precision else 4
        lanes = ns // cpl
        tiling = {"motor_lanes": lanes} if ns % cpl == 0 and lanes >= 2 and lanes & (lanes - 1) == 0 else {}
    for cfl in (0.0, 0.15):
        p = ModelParams(nx=nx, ny=ny, ntheta=nt, ns=ns, motor_cfl=cfl)
        psi0 = gen.make_psi0(nx, ny, nt, p.lx, p.ly, seed=0)
        M0 = gen.make_M0_random(nx, ny, nt, ns, seed=5)
        fl = gen.fluid_schedule(nx, ny, len(calls), p.lx, p.ly)
        dt = gen.cfl_dt(p, fl)
        outs = []
        for block in (1, 0):
            # the blocked run keeps the default tiling; the serial run is given it
            opts = {"motor_block": block, **(tiling if (block == 0 or "motor_chunks" in tiling) else {})}
            ctx = mmk.Context(p, precision=precision, options=opts)
            if precision:
                ctx.set_state(torch.as_tensor(psi0.astype(np.float32)), torch.as_tensor(M0.astype(np.float32)))
            else:
                ctx.set_state(torch.as_tensor(psi0), torch.as_tensor(M0))
            for e, k in enumerate(calls):
                ctx.set_fluid(*map(torch.as_tensor, fl[e]))
                ctx.step(k, dt)
            psi, M = ctx.get_state()
            m0, m1 = ctx.get_motor_moments()
            r = [x.cpu().numpy() for x in (psi, M, m0, m1, ctx.get_stress(), ctx.get_moments())]
            r.append(np.array(ctx.get_sums()[0]))
            ctx.close()
            outs.append(r)
        for x, y in zip(*outs):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("precision,tol", [(0, 1e-14), (1, 1e-6)])
def test_wide_and_narrow_tilings_agree(precision, tol):
    """The default blocked context (64 bytes of the column per lane in FP32, 32 in FP64) against
    one launch per micro-step (16 bytes per lane): the same scheme, only the association of the
    s-sums differs."""
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=12, ny=10, ntheta=64, ns=64)
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=0)
    M0 = gen.make_M0_random(p.nx, p.ny, p.ntheta, p.ns, seed=5)
    fl = gen.fluid_schedule(p.nx, p.ny, 3, p.lx, p.ly)
    dt = gen.cfl_dt(p, fl)
    outs = []
    for block in (1, 0):
        ctx = mmk.Context(p, precision=precision, options={"motor_block": block})
        cast = (lambda a: a.astype(np.float32)) if precision else (lambda a: a)
        ctx.set_state(torch.as_tensor(cast(psi0)), torch.as_tensor(cast(M0)))
        for e in range(3):
            ctx.set_fluid(*map(torch.as_tensor, fl[e]))
            ctx.step(10, dt)
        psi, M = ctx.get_state()
        outs.append([x.double().cpu().numpy() for x in (psi, M, ctx.get_stress(), ctx.get_moments())])
        ctx.close()
    for a, b in zip(*outs):
        assert rel_err(a, b) <= tol


@pytest.mark.parametrize("shape,n,precision,walk,fused", [
    ((6, 5, 16, 64), 2, 0, None, "0"),     # one launch per sub-step; even n: the last sub-step
                                           # lands in the first buffer
    ((6, 5, 16, 64), 2, 0, None, "1"),     # all sub-steps in one launch, 16 lanes per column
    ((7, 4, 32, 8), 3, 0, None, "1"),      # no single-launch tiling for ns = 8: per sub-step
    ((10, 7, 10, 32), 3, 0, None, "1"),    # 10 x 8 lanes, not whole waves: per sub-step
    ((9, 5, 16, 16), 5, 0, None, "1"),     # single launch, 4 lanes per column, one wave a block
    ((12, 10, 64, 32), 4, 0, "1", "1"),    # walking psi kernel
    ((12, 10, 64, 32), 3, 0, "0", "0"),    # LDS-tiled psi kernel
    ((12, 10, 64, 32), 3, 0, "0", "1"),
    ((20, 18, 64, 64), 2, 1, None, "1"),   # FP32 against the FP64 oracle
    ((20, 18, 64, 64), 3, 1, None, "0"),
    ((8, 6, 32, 32), 4, 1, None, "1"),     # FP32, 4 lanes per column
])
def test_depleted_substeps_against_oracle(shape, n, precision, walk, fused):
    """Depletion with sub-cycling: every sub-step takes the clamp and the pool of the current
    sub-state (Alg. 2), m_total between the smallest and the largest coarse density so both
    branches occur; in one launch per micro-step and in one launch per sub-step."""
    opts = {"depl_fused": int(fused)}
    if walk is not None:
        opts["psi_kernel"] = 2 if walk == "1" else 1
    nx, ny, nt, ns = shape
    p = ModelParams(nx=nx, ny=ny, ntheta=nt, ns=ns, k_on=0.9, k_off=0.6, v0=4.0, F=0.8)
    psi0, M0, fl, dt = substep_case(p, n)
    Bv = A.coarse_bound(p, psi0, M0.sum(-1) * (p.L / p.ns))
    p.m_total = float(0.5 * (Bv.min() + Bv.max()))
    assert (Bv > p.m_total).any() and (Bv < p.m_total).any()
    if precision:
        psi0, M0 = psi0.astype(np.float32), M0.astype(np.float32)
    g = run_gpu(p, psi0, M0, fl, 4, 8, dt, precision=precision, options=opts)
    o = run_oracle(p, psi0.astype(np.float64), M0.astype(np.float64), fl, 4, 8, dt)
    compare(g, o, 1e-5 if precision else 1e-12)


@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 2e-6)])
def test_depleted_substeps_one_launch_and_per_substep_agree(precision, tol):
    """The single-launch depleted sub-cycling (one block per (x, y) point) against one launch per
    sub-step: the same scheme; only the association of the coarse-density sum differs."""
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=16, ny=12, ntheta=64, ns=64, k_on=0.9, k_off=0.6, v0=4.0, F=0.8)
    psi0, M0, fl, dt = substep_case(p, 3, n_exchanges=3)
    Bv = A.coarse_bound(p, psi0, M0.sum(-1) * (p.L / p.ns))
    p.m_total = float(0.5 * (Bv.min() + Bv.max()))
    outs = []
    for fused in (1, 0):
        ctx = mmk.Context(p, precision=precision, options={"depl_fused": fused})
        cast = (lambda a: a.astype(np.float32)) if precision else (lambda a: a)
        ctx.set_state(torch.as_tensor(cast(psi0)), torch.as_tensor(cast(M0)))
        for e in range(3):
            ctx.set_fluid(*map(torch.as_tensor, fl[e]))
            ctx.step(6, dt)
        psi, M = ctx.get_state()
        outs.append([x.double().cpu().numpy() for x in (psi, M, ctx.get_stress(), ctx.get_moments())])
        ctx.close()
    for a, b in zip(*outs):
        assert rel_err(a, b) <= tol
