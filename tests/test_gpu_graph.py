"""HIP-graph replay of the K-step loop (mmk_step_graph) against eager mmk_step: the same
kernels with the same arguments, so every output must match bit for bit after every call.
Each replay is followed by the program's own eager work (copies out, a new fluid, a
synchronisation) before the next one, and every replay is checked.  The launch-bound
16^2 x 16 x 16 FP64 workload is also compared with the FP64 oracle (1e-12)."""
import numpy as np
import pytest

from paper_1908_04279_amd import inputs as gen
from paper_1908_04279_amd.inputs import ModelParams
from tests.conftest import rel_err
from tests.runners import run_oracle

pytestmark = pytest.mark.gpu


def outputs(ctx):
    psi, M = ctx.get_state()
    m0, m1 = ctx.get_motor_moments()
    r = [x.cpu().numpy() for x in (psi, M, m0, m1, ctx.get_stress(), ctx.get_moments())]
    r.append(np.array([ctx.get_sums()[0]] + ctx.get_sums()[1]))
    return r


DEPL = {"m_total": 0.05, "motor_cfl": 0.1, "v0": 4.0}


@pytest.mark.parametrize("shape,precision,over,calls,opts", [
    ((16, 16, 16, 16), 0, {}, [100, 100, 100], {}),               # the launch-bound workload
    ((12, 10, 64, 64), 1, {}, [10, 10, 7, 10, 17], {}),           # FP32 blocked motor, odd K
    ((9, 7, 16, 32), 0, {"motor_cfl": 0.15}, [4, 4, 5], {}),      # sub-cycling inside blocks
    ((8, 6, 16, 32), 0, DEPL, [3, 3, 4], {}),                     # depleted, fused sub-steps
    # a launch per sub-step, an even number of them (the copy of M closes each micro-step)
    ((8, 6, 16, 16), 0, {**DEPL, "motor_cfl": 0.2}, [2, 2], {"depl_fused": 0}),
    ((9, 7, 16, 32), 1, {}, [10, 3], {"motor_block": 0}),         # one motor launch per step
])
def test_graph_replays_match_eager_bitwise(shape, precision, over, calls, opts):
    import torch
    from paper_1908_04279_amd import mmk
    nx, ny, nt, ns = shape
    p = ModelParams(nx=nx, ny=ny, ntheta=nt, ns=ns, **over)
    psi0 = gen.make_psi0(nx, ny, nt, p.lx, p.ly, seed=0)
    M0 = gen.make_M0_random(nx, ny, nt, ns, p.k_on, p.k_off, seed=5)
    fl = gen.fluid_schedule(nx, ny, len(calls), p.lx, p.ly)
    dt = gen.cfl_dt(p, fl)
    cast = (lambda a: torch.as_tensor(a.astype(np.float32))) if precision else torch.as_tensor
    ctxs = [mmk.Context(p, precision=precision, options=opts) for _ in range(2)]
    for c in ctxs:
        c.set_state(cast(psi0), cast(M0))
    for e, k in enumerate(calls):
        for c in ctxs:
            c.set_fluid(*map(torch.as_tensor, fl[e]))
        ctxs[0].step(k, dt)
        ctxs[1].step_graph(k, dt)
        torch.cuda.synchronize()
        for a, b in zip(outputs(ctxs[0]), outputs(ctxs[1])):
            assert np.array_equal(a, b), (e, k)
    # a new state between replays of a held graph
    for c in ctxs:
        c.set_state(cast(M0[..., 0].copy()), cast(M0))
        c.step_graph(calls[0], dt) if c is ctxs[1] else c.step(calls[0], dt)
    for a, b in zip(outputs(ctxs[0]), outputs(ctxs[1])):
        assert np.array_equal(a, b)
    for c in ctxs:
        c.close()


def test_graph_fp64_16x16x16x16_against_oracle():
    import torch
    from paper_1908_04279_amd import mmk
    p = gen.params_for("fp64_16x16x16x16")
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0)
    fl = [gen.make_fluid(p.nx, p.ny, seed=1)]
    dt = gen.cfl_dt(p, fl)
    ctx = mmk.Context(p)
    ctx.set_state(torch.as_tensor(psi0))
    ctx.set_fluid(*map(torch.as_tensor, fl[0]))
    for _ in range(4):
        ctx.step_graph(25, dt)
    psi, M = ctx.get_state()
    o = run_oracle(p, psi0, np.zeros((p.nx, p.ny, p.ntheta, p.ns)), fl, 100, 100, dt)
    # the oracle's outputs are those of its last call; four calls of 25 leave the same state
    assert rel_err(psi.cpu().numpy(), o["psi"]) <= 1e-12
    assert rel_err(M.cpu().numpy(), o["M"]) <= 1e-12
    assert rel_err(ctx.get_stress().cpu().numpy(), o["stress"]) <= 1e-12
    ctx.close()


def test_graph_refusals():
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=4, ny=4, ntheta=8, ns=8)
    ctx = mmk.Context(p, ckpt_every=2, max_tape_steps=8)
    with pytest.raises(mmk.MMKError) as ei:
        ctx.step_graph(2, 0.01)
    assert ei.value.status == mmk.MMK_ERR_STATE
    ctx.set_state(torch.as_tensor(gen.make_psi0(4, 4, 8, seed=0)))
    ctx.set_fluid(*map(torch.as_tensor, gen.make_fluid(4, 4)))
    ctx.tape_begin(2)
    with pytest.raises(mmk.MMKError) as ei:
        ctx.step_graph(2, 0.01)
    assert ei.value.status == mmk.MMK_ERR_STATE
    ctx.tape_end()
    with pytest.raises(mmk.MMKError) as ei:
        ctx.step_graph(1, float("nan"))
    assert ei.value.status == mmk.MMK_ERR_ARG
    ctx.step_graph(2, 0.01)
    ctx.close()


@pytest.mark.parametrize("over", [
    dict(rc=0.45, m_total=0.01),                            # coarse pass and motor launch per step
    dict(rc=0.45, m_total=0.01, motor_cfl=0.25, v0=4.0),    # per sub-step (6: an even count, a copy)
    dict(rc=0.45, motor_cfl=0.2, v0=4.0),                   # sub-steps in registers
])
def test_graph_anchor_resolved_matches_eager_bitwise(over):
    """The anchor-resolved model through mmk_step_graph against mmk_step, bit for bit after every
    call (state, marginals, outputs, per-anchor coarse density and pool)."""
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=12, ny=12, ntheta=8, ns=8, **over)
    ncell = len(mmk.r0_cells(p))
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=0)
    Mb0 = gen.make_Mb0_random(ncell, p.nx, p.ny, seed=4)
    fl = gen.fluid_schedule(p.nx, p.ny, 3, p.lx, p.ly)
    dt = gen.cfl_dt(p, fl)
    ctxs = [mmk.Context(p) for _ in range(2)]
    for c in ctxs:
        c.set_state(torch.as_tensor(psi0), torch.as_tensor(Mb0))
    for e, k in enumerate([3, 2, 3]):
        for c in ctxs:
            c.set_fluid(*map(torch.as_tensor, fl[e]))
        ctxs[0].step(k, dt)
        ctxs[1].step_graph(k, dt)
        torch.cuda.synchronize()
        a, b = outputs(ctxs[0]), outputs(ctxs[1])
        a += [x.cpu().numpy() for x in ctxs[0].get_anchors()]
        b += [x.cpu().numpy() for x in ctxs[1].get_anchors()]
        for x, y in zip(a, b):
            assert np.array_equal(x, y), (e, k)
    for c in ctxs:
        c.close()
