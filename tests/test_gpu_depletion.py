"""Free-motor depletion and the over-binding clamp on the GPU against the FP64 oracle.

Each case picks m_total between the smallest and the largest coarse bound density of the
initial state, so that both the clamped and the unclamped branch occur; the state then
evolves under flow and several fluid exchanges.  Tolerances as for the plain path: FP64
1e-12, FP32 1e-5 (norm-wise relative per field).
"""
import numpy as np
import pytest

from oracle import oracle_a as A
from paper_1908_04279_amd import inputs as gen
from paper_1908_04279_amd.inputs import ModelParams
from tests.conftest import rel_err
from tests.runners import run_gpu, run_oracle

pytestmark = pytest.mark.gpu
FIELDS = ["psi", "M", "m0", "m1", "stress", "mom"]


def depleted_case(p, M0_kind="random", frac=0.5, n_exchanges=3):
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=0)
    M0 = None if M0_kind == "zero" else gen.make_M0_random(p.nx, p.ny, p.ntheta, p.ns, p.k_on, p.k_off, seed=5)
    if M0 is not None:
        Bv = A.coarse_bound(p, psi0, M0.sum(-1) * (p.L / p.ns))
        p.m_total = float(Bv.min() + frac * (Bv.max() - Bv.min()))
        assert (Bv > p.m_total).any() and (Bv < p.m_total).any()
    else:
        p.m_total = 0.01
    fl = gen.fluid_schedule(p.nx, p.ny, n_exchanges, p.lx, p.ly)
    dt = gen.cfl_dt(p, fl)
    return psi0, M0, fl, dt


def compare(g, o, tol):
    errs = {f: rel_err(g[f], o[f]) for f in FIELDS}
    errs["mass"] = abs(g["mass"] - o["mass"]) / abs(o["mass"])
    errs["sum_sigma"] = rel_err(g["sum_sigma"], o["sum_sigma"])
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)


@pytest.mark.parametrize("walk", ["0", "1"])
@pytest.mark.parametrize("shape,limiter", [((5, 7, 12, 16), 0), ((9, 6, 64, 32), 0), ((9, 6, 64, 32), 1),
                                           ((4, 5, 128, 8), 0), ((13, 3, 32, 20), 1)])
def test_fp64_against_oracle(shape, limiter, walk):
    nx, ny, nt, ns = shape
    p = ModelParams(nx=nx, ny=ny, ntheta=nt, ns=ns, limiter=limiter, k_on=0.9, k_off=0.6, v0=1.2, F=0.8)
    psi0, M0, fl, dt = depleted_case(p)
    g = run_gpu(p, psi0, M0, fl, 6, 17, dt, options={"psi_kernel": 2 if walk == "1" else 1})
    o = run_oracle(p, psi0, M0, fl, 6, 17, dt)
    compare(g, o, 1e-12)


def test_fp64_zero_initial_motors():
    p = ModelParams(nx=6, ny=5, ntheta=16, ns=16)
    psi0, M0, fl, dt = depleted_case(p, M0_kind="zero")
    g = run_gpu(p, psi0, M0, fl, 10, 30, dt)
    o = run_oracle(p, psi0, np.zeros((6, 5, 16, 16)), fl, 10, 30, dt)
    compare(g, o, 1e-12)


def test_fp64_64x64x64x32_against_oracle():
    """A grid of several psi tiles in both directions, 40 steps, a new fluid every 10."""
    p = ModelParams(nx=64, ny=64, ntheta=64, ns=32)
    psi0, M0, fl, dt = depleted_case(p, frac=0.3, n_exchanges=4)
    print("gpu run", flush=True)
    g = run_gpu(p, psi0, M0, fl, 10, 40, dt)
    print("oracle run", flush=True)
    o = run_oracle(p, psi0, M0, fl, 10, 40, dt)
    compare(g, o, 1e-12)


@pytest.mark.parametrize("shape", [(20, 18, 64, 64), (6, 5, 16, 16), (9, 7, 128, 32)])
def test_fp32_against_fp64_oracle(shape):
    nx, ny, nt, ns = shape
    p = ModelParams(nx=nx, ny=ny, ntheta=nt, ns=ns)
    psi0, M0, fl, dt = depleted_case(p)
    g = run_gpu(p, psi0.astype(np.float32), M0.astype(np.float32), fl, 10, 30, dt, precision=1)
    o = run_oracle(p, psi0.astype(np.float32).astype(np.float64), M0.astype(np.float32).astype(np.float64),
                   fl, 10, 30, dt)
    compare(g, o, 1e-5)


def test_resume_and_repeat():
    """Bitwise repeatable; a run split by get_state / set_state (which recomputes the coarse
    bound density of the state) agrees with the unsplit run to rounding."""
    p = ModelParams(nx=12, ny=10, ntheta=32, ns=16)
    psi0, M0, fl, dt = depleted_case(p)
    a = run_gpu(p, psi0, M0, fl, 30, 30, dt)
    b = run_gpu(p, psi0, M0, fl, 30, 30, dt)
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), f
    c1 = run_gpu(p, psi0, M0, fl, 15, 15, dt, keep_ctx=True)
    psi, M = c1["ctx"].get_state()
    c1["ctx"].close()
    c2 = run_gpu(p, psi.cpu().numpy(), M.cpu().numpy(), fl, 15, 15, dt)
    for f in FIELDS:
        assert rel_err(c2[f], a[f]) <= 1e-13, f


def test_tape_is_refused_with_depletion():
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=4, ny=4, ntheta=8, ns=8, m_total=0.5)
    ctx = mmk.Context(p, ckpt_every=4, max_tape_steps=8)
    psi0 = gen.make_psi0(4, 4, 8, seed=0)
    ctx.set_state(torch.as_tensor(psi0))
    ctx.set_fluid(*map(torch.as_tensor, gen.make_fluid(4, 4)))
    with pytest.raises(mmk.MMKError) as ei:
        ctx.tape_begin(4)
    assert ei.value.status == mmk.MMK_ERR_UNSUPPORTED
    ctx.close()
