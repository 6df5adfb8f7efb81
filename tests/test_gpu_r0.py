"""Anchor-resolved bound motors on the GPU (capture ball of radius rc; Eqs. (4)-(6); Alg. 2) against
the FP64 oracle: every run-register size of the motor kernel (8, 16, 32 cells), ragged grids, both
limiters, linear attachment and depletion with the clamp active, a zero start and an empty tracked
set, at FP64 1e-12 and FP32 1e-5 (norm-wise relative per field); the per-anchor outputs; the motor
force of the anchor-resolved state (Eq. (10) with its r0 integral); the refusals; repeatable bits;
and a sampled check at the benchmark's size and launch configuration."""
import numpy as np
import pytest

from oracle import oracle_a as A
from paper_1908_04279_amd import inputs as gen
from paper_1908_04279_amd.inputs import ModelParams
from tests.conftest import rel_err
from tests.runners import run_r0_gpu, run_r0_oracle

pytestmark = pytest.mark.gpu
FIELDS = ["psi", "M", "m0", "m1", "stress", "mom", "coarse", "free"]


def r0_case(p, depletion, zero_start=False, n_exchanges=2, seed=4):
    """Seeded psi, anchor-resolved state and fluids; with depletion m_total is the median coarse
    density of the initial state, so about half of the anchors start clamped."""
    cells = A.r0_cells(p)
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=0)
    Mb0 = None if zero_start else gen.make_Mb0_random(len(cells), p.nx, p.ny, p.k_on, p.k_off, seed=seed)
    if depletion:
        co = A.r0_coarse(p, cells, psi0, Mb0 if Mb0 is not None else np.zeros((len(cells), p.nx, p.ny)))
        p.m_total = float(np.median(co)) if np.max(co) > 0 else 0.02
    fl = gen.fluid_schedule(p.nx, p.ny, n_exchanges, p.lx, p.ly)
    dt = gen.cfl_dt(p, fl)
    return cells, psi0, Mb0, fl, dt


def compare(g, o, tol, fields=FIELDS):
    errs = {f: rel_err(g[f], o[f]) for f in fields}
    errs["mass"] = abs(g["mass"] - o["mass"]) / abs(o["mass"])
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)


CASES = [
    # kw, depletion, zero start, (K, n)
    (dict(nx=16, ny=16, ntheta=8, ns=8, rc=0.45), False, False, (5, 12)),               # runs <= 8
    (dict(nx=20, ny=18, ntheta=16, ns=16, rc=0.35), True, False, (4, 10)),              # clamp active
    (dict(nx=9, ny=7, ntheta=12, ns=10, rc=0.6, lx=5.0, ly=6.0, limiter=1), True, False, (3, 7)),  # ragged
    (dict(nx=24, ny=22, ntheta=16, ns=24, rc=0.45, v0=1.7), True, False, (6, 9)),       # runs <= 16 / 32
    (dict(nx=14, ny=12, ntheta=8, ns=30, rc=0.5, L=1.2, k_on=0.8, k_off=0.9), False, True, (4, 8)),  # M = 0
    (dict(nx=10, ny=12, ntheta=6, ns=6, rc=0.8, lx=5.5, ly=7.0), True, True, (2, 5)),  # zero start, depleted
]


@pytest.mark.parametrize("kw,depletion,zero_start,Kn", CASES)
def test_fp64_against_oracle(kw, depletion, zero_start, Kn):
    p = ModelParams(**kw)
    cells, psi0, Mb0, fl, dt = r0_case(p, depletion, zero_start)
    runs = np.sum((np.diff(cells[:, 3]) != 1) | np.any(np.diff(cells[:, :3], axis=0) != 0, axis=1)) + 1
    print(f"cells {len(cells)} runs {runs} m_total {p.m_total:.4g}", flush=True)
    K, n = Kn
    g = run_r0_gpu(p, psi0, Mb0, fl, K, n, dt)
    o = run_r0_oracle(p, psi0, Mb0, fl, K, n, dt)
    compare(g, o, 1e-12)


def test_run_lengths_cover_every_kernel():
    """The parity cases hold runs of at most 8, 16 and 32 cells (each register size)."""
    longest = []
    for kw, *_ in CASES:
        c = A.r0_cells(ModelParams(**kw))
        brk = np.nonzero((np.diff(c[:, 3]) != 1) | np.any(np.diff(c[:, :3], axis=0) != 0, axis=1))[0]
        edges = np.concatenate([[0], brk + 1, [len(c)]])
        longest.append(int(np.max(np.diff(edges))))
    assert min(longest) <= 8 and any(8 < m <= 16 for m in longest) and any(16 < m <= 32 for m in longest), longest


def test_empty_tracked_set():
    """An rc that catches no cell: Mb is empty, the marginals are 0 and psi only advects."""
    p = ModelParams(nx=8, ny=8, ntheta=8, ns=4, rc=0.01)
    cells = A.r0_cells(p)
    assert len(cells) == 0
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0)
    fl = gen.fluid_schedule(p.nx, p.ny, 1)
    dt = gen.cfl_dt(p, fl)
    g = run_r0_gpu(p, psi0, None, fl, 3, 3, dt)
    o = run_r0_oracle(p, psi0, None, fl, 3, 3, dt)
    assert g["M"].shape == (0, p.nx, p.ny)
    assert np.all(g["m0"] == 0) and np.all(g["coarse"] == 0)
    compare(g, o, 1e-12, ["psi", "stress", "mom", "free"])


@pytest.mark.parametrize("kw,depletion", [
    (dict(nx=24, ny=20, ntheta=16, ns=16, rc=0.35), True),
    (dict(nx=19, ny=13, ntheta=12, ns=24, rc=0.45, lx=5.0, ly=5.5), False),
    (dict(nx=32, ny=32, ntheta=32, ns=32, rc=0.3), True),
])
def test_fp32_against_fp64_oracle(kw, depletion):
    p = ModelParams(**kw)
    cells, psi0, Mb0, fl, dt = r0_case(p, depletion)
    psi32, Mb32 = psi0.astype(np.float32), Mb0.astype(np.float32)
    g = run_r0_gpu(p, psi32, Mb32, fl, 5, 10, dt, precision=1)
    o = run_r0_oracle(p, psi32.astype(np.float64), Mb32.astype(np.float64), fl, 5, 10, dt)
    compare(g, o, 1e-5)


def test_refusals():
    import torch
    from paper_1908_04279_amd import mmk
    with pytest.raises(mmk.MMKError) as ei:   # rc + L/2 not below half the box
        mmk.Context(ModelParams(nx=8, ny=8, ntheta=4, ns=4, rc=2.7))
    assert "rc + L/2" in str(ei.value)
    with pytest.raises(mmk.MMKError) as ei:   # a run of more than 32 cells
        mmk.Context(ModelParams(nx=8, ny=8, ntheta=4, ns=64, rc=0.5))
    assert "longer than 32" in str(ei.value)
    with pytest.raises(mmk.MMKError) as ei:   # the tape
        mmk.Context(ModelParams(nx=8, ny=8, ntheta=4, ns=8, rc=0.5), ckpt_every=2, max_tape_steps=4)
    assert ei.value.status == mmk.MMK_ERR_UNSUPPORTED
    p = ModelParams(nx=8, ny=8, ntheta=4, ns=8, rc=0.5)
    ctx = mmk.Context(p)
    with pytest.raises(mmk.MMKError) as ei:
        ctx.get_anchors()
    assert ei.value.status == mmk.MMK_ERR_STATE
    ctx.set_state(torch.as_tensor(gen.make_psi0(8, 8, 4, seed=0)))
    with pytest.raises(mmk.MMKError) as ei:
        ctx.tape_begin(2)
    assert ei.value.status == mmk.MMK_ERR_UNSUPPORTED
    ctx.close()
    q = mmk.Context(ModelParams(nx=8, ny=8, ntheta=4, ns=8))
    q.set_state(torch.as_tensor(gen.make_psi0(8, 8, 4, seed=0)))
    with pytest.raises(mmk.MMKError) as ei:   # the anchor-marginal model has no anchors
        q.get_anchors()
    assert ei.value.status == mmk.MMK_ERR_STATE
    q.close()


def test_repeatable_bits():
    p = ModelParams(nx=20, ny=18, ntheta=16, ns=16, rc=0.35)
    cells, psi0, Mb0, fl, dt = r0_case(p, True)
    a = run_r0_gpu(p, psi0, Mb0, fl, 4, 8, dt)
    b = run_r0_gpu(p, psi0, Mb0, fl, 4, 8, dt)
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), f


def test_full_size_sampled():
    """The benchmark's workload (128^2 anchors, 32 orientations, 32 arclength cells, rc = 0.1,
    FP32, depletion with about half of the anchors clamped) and launch configuration, one
    micro-step: at sampled anchors the oracle's coarse density, clamp and pool, and the oracle's
    run step of every run of those anchors, against the GPU's new state; the marginal m0 at
    sampled filament cells against the sum of the GPU's own new state; psi mass conserved."""
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=128, ny=128, ntheta=32, ns=32, rc=0.1)
    cells = A.r0_cells(p)
    nc = len(cells)
    rng = np.random.default_rng(11)
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0).astype(np.float32)
    Mb0 = rng.uniform(0.0, 2.0, (nc, p.nx, p.ny)).astype(np.float32)
    u, G = gen.make_fluid(p.nx, p.ny)
    dt = gen.cfl_dt(p, [(u, G)])
    ds, dx, dy, dth = p.L / p.ns, p.lx / p.nx, p.ly / p.ny, 2 * np.pi / p.ntheta
    psi64, a, b, k = psi0.astype(np.float64), cells[:, 0], cells[:, 1], cells[:, 2]

    def coarse_at(i0, j0):
        xi, xj = (i0 + a) % p.nx, (j0 + b) % p.ny
        return float(np.sum(Mb0[np.arange(nc), xi, xj].astype(np.float64) * psi64[xi, xj, k]) * ds * dx * dy * dth)

    anchors = [(int(rng.integers(p.nx)), int(rng.integers(p.ny))) for _ in range(6)]
    p.m_total = float(np.median([coarse_at(*r) for r in anchors]))
    ctx = mmk.Context(p, precision=mmk.FP32)
    ctx.set_state(torch.as_tensor(psi0), torch.as_tensor(Mb0))
    ctx.set_fluid(torch.as_tensor(u), torch.as_tensor(G))
    co_gpu, _ = ctx.get_anchors()
    ctx.step(1, dt)
    _, Mb1 = ctx.get_state()
    m0, _ = ctx.get_motor_moments()
    mass1, _ = ctx.get_sums()
    Mb1, m0, co_gpu = Mb1.cpu().numpy(), m0.cpu().numpy(), co_gpu.cpu().numpy()
    torch.cuda.synchronize()
    ctx.close()
    # runs: consecutive cells with the same (a, b, k) and consecutive l
    brk = np.nonzero((np.diff(cells[:, 3]) != 1) | np.any(np.diff(cells[:, :3], axis=0) != 0, axis=1))[0]
    edges = np.concatenate([[0], brk + 1, [nc]])
    clamped = 0
    for (i0, j0) in anchors:
        co = coarse_at(i0, j0)
        assert abs(co_gpu[i0, j0] - co) <= 1e-5 * co
        over = co > p.m_total
        clamped += over
        scale, src = (p.m_total / co, 0.0) if over else (1.0, p.k_on * (p.m_total - co))
        for r in range(len(edges) - 1):
            c0, c1 = edges[r], edges[r + 1]
            xi, xj = (i0 + a[c0]) % p.nx, (j0 + b[c0]) % p.ny
            want = A.run_step(p, dt, scale * Mb0[c0:c1, xi, xj].astype(np.float64), src)
            got = Mb1[c0:c1, xi, xj].astype(np.float64)
            assert np.max(np.abs(got - want)) <= 1e-5 * 2.0, (i0, j0, r)
    assert 0 < clamped < len(anchors)
    for _ in range(8):
        i, j, kk = int(rng.integers(p.nx)), int(rng.integers(p.ny)), int(rng.integers(p.ntheta))
        sel = k == kk
        want = float(np.sum(Mb1[sel, i, j].astype(np.float64))) * ds * dx * dy
        assert abs(m0[i, j, kk] - want) <= 1e-5 * abs(want)
    assert abs(mass1 - 1.0) <= 1e-5


@pytest.mark.parametrize("kw,precision", [
    (dict(nx=20, ny=18, ntheta=16, ns=16, rc=0.35), 0),
    (dict(nx=9, ny=7, ntheta=12, ns=10, rc=0.6, lx=5.0, ly=6.0, limiter=1), 0),
    (dict(nx=32, ny=32, ntheta=32, ns=32, rc=0.3), 1),
])
def test_force_against_oracle(kw, precision):
    """get_force of an anchor-resolved state after a few depleted steps: the force of its anchor
    marginal (oracle: the marginal field, then the oracle's force), twice with the same bits."""
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(**kw)
    cells, psi0, Mb0, fl, dt = r0_case(p, True)
    if precision:
        psi0, Mb0 = psi0.astype(np.float32), Mb0.astype(np.float32)
    ctx = mmk.Context(p, precision=precision)
    ctx.set_state(torch.as_tensor(psi0), torch.as_tensor(Mb0))
    ctx.set_fluid(*map(torch.as_tensor, fl[0]))
    ctx.step(4, dt)
    psi, Mb = ctx.get_state()
    f1 = ctx.get_force().double().cpu().numpy()
    f2 = ctx.get_force().double().cpu().numpy()
    torch.cuda.synchronize()
    ctx.close()
    assert np.array_equal(f1, f2)
    want = A.r0_motor_force(p, cells, psi.double().cpu().numpy(), Mb.double().cpu().numpy())
    err = rel_err(f1, want)
    print(f"force rel err {err:.2e}", flush=True)
    assert err <= (1e-5 if precision else 1e-12)


def test_resume_is_bitwise():
    """8 steps in one context give the same bits as 4 steps, get_state, a new context and set_state,
    4 more steps (the state carries everything: set_state rebuilds the run totals and marginals
    with the same sums the motor launch makes)."""
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=20, ny=18, ntheta=16, ns=16, rc=0.35)
    cells, psi0, Mb0, fl, dt = r0_case(p, True)
    a = run_r0_gpu(p, psi0, Mb0, fl, 4, 8, dt)
    ctx = mmk.Context(p)
    ctx.set_state(torch.as_tensor(psi0), torch.as_tensor(Mb0))
    ctx.set_fluid(*map(torch.as_tensor, fl[0]))
    ctx.step(4, dt)
    psi, Mb = ctx.get_state()
    psi, Mb = psi.cpu().numpy(), Mb.cpu().numpy()
    ctx.close()
    b = run_r0_gpu(p, psi, Mb, fl[1:], 4, 4, dt)
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), f


SUBSTEP_CASES = [
    # kw, depletion, motor sub-steps per micro-step, (K, n)
    (dict(nx=16, ny=16, ntheta=8, ns=8, rc=0.45), False, 3, (3, 7)),
    (dict(nx=20, ny=18, ntheta=16, ns=16, rc=0.35), True, 2, (4, 8)),      # even: ends in the other buffer
    (dict(nx=9, ny=7, ntheta=12, ns=10, rc=0.6, lx=5.0, ly=6.0, limiter=1), True, 4, (3, 6)),
    (dict(nx=24, ny=22, ntheta=16, ns=24, rc=0.45, v0=1.7), True, 3, (3, 5)),   # runs <= 16 / 32
    # linear attachment: all sub-steps in registers, one launch per micro-step
    (dict(nx=24, ny=22, ntheta=16, ns=24, rc=0.45, v0=1.7), False, 2, (3, 5)),
    (dict(nx=9, ny=7, ntheta=12, ns=10, rc=0.6, lx=5.0, ly=6.0, limiter=1), False, 5, (3, 6)),
]


def substep_r0_case(p, depletion, nsub):
    """r0_case at the psi limit (motor_cfl > 0 leaves the motor rate out of it), then motor_cfl
    chosen so that a micro-step takes nsub motor sub-steps."""
    p.motor_cfl = 1.0
    cells, psi0, Mb0, fl, dt = r0_case(p, depletion)
    rate = p.v0 / (p.L / p.ns) + p.k_off
    p.motor_cfl = dt * rate / (nsub - 0.5)
    assert A.motor_substeps(p, dt) == nsub
    return cells, psi0, Mb0, fl, dt


@pytest.mark.parametrize("kw,depletion,nsub,Kn", SUBSTEP_CASES)
def test_substeps_fp64_against_oracle(kw, depletion, nsub, Kn):
    """Motor sub-cycling of the runs (Alg. 2's local dt*), with depletion every sub-step after the
    clamp and the pool of its anchor's current sub-state."""
    p = ModelParams(**kw)
    cells, psi0, Mb0, fl, dt = substep_r0_case(p, depletion, nsub)
    K, n = Kn
    g = run_r0_gpu(p, psi0, Mb0, fl, K, n, dt)
    o = run_r0_oracle(p, psi0, Mb0, fl, K, n, dt)
    compare(g, o, 1e-12)


@pytest.mark.parametrize("depletion", [True, False])
def test_substeps_fp32_against_fp64_oracle(depletion):
    p = ModelParams(nx=20, ny=18, ntheta=16, ns=16, rc=0.35)
    cells, psi0, Mb0, fl, dt = substep_r0_case(p, depletion, 3)
    psi32, Mb32 = psi0.astype(np.float32), Mb0.astype(np.float32)
    g = run_r0_gpu(p, psi32, Mb32, fl, 4, 8, dt, precision=1)
    o = run_r0_oracle(p, psi32.astype(np.float64), Mb32.astype(np.float64), fl, 4, 8, dt)
    compare(g, o, 1e-5)


def test_one_substep_is_the_plain_step():
    """motor_cfl so large that n = 1: the same bits as motor_cfl = 0, with depletion."""
    p = ModelParams(nx=20, ny=18, ntheta=16, ns=16, rc=0.35)
    cells, psi0, Mb0, fl, dt = r0_case(p, True)
    outs = []
    for cfl in (0.0, 1e6):
        p.motor_cfl = cfl
        g = run_r0_gpu(p, psi0, Mb0, fl, 3, 6, dt)
        outs.append(g)
    for f in FIELDS:
        assert np.array_equal(outs[0][f], outs[1][f]), f
