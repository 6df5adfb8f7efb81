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


def run_length_max(cells):
    brk = np.nonzero((np.diff(cells[:, 3]) != 1) | np.any(np.diff(cells[:, :3], axis=0) != 0, axis=1))[0]
    return int(np.max(np.diff(np.concatenate([[0], brk + 1, [len(cells)]]))))


def onepass_expected(cells, depletion, nsub, precision, onepass=1):
    """Whether the library takes the one-anchor-per-block launch: depletion with sub-cycling, the
    option on, and the runs within the slots of a thread (16 in FP64, 24 in FP32)."""
    return bool(onepass and depletion and nsub > 1 and run_length_max(cells) <= (24 if precision else 16))


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
    for bad in (-1, 2):   # the one-pass option takes 0 or 1
        with pytest.raises(mmk.MMKError) as ei:
            ctx.set_option("r0_onepass", bad)
        assert ei.value.status == mmk.MMK_ERR_ARG
    assert mmk.lib().mmk_set_option(ctx.h, len(mmk.OPTIONS), 0) == mmk.MMK_ERR_ARG   # no such option
    ctx.profile(True)
    for kid in (-1, len(mmk.KERNEL_IDS)):   # kernel ids 0 .. 9
        with pytest.raises(mmk.MMKError) as ei:
            ctx.profile_read(kid)
        assert ei.value.status == mmk.MMK_ERR_ARG
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


@pytest.mark.parametrize("precision,tol", [(1, 1e-5), (0, 1e-12)])
def test_full_size_sampled_onepass(precision, tol):
    """The sub-cycled benchmark workload (128^2 anchors, 32 orientations, 32 arclength cells,
    rc = 0.1, fast motors v0 = 8 with motor_cfl = 0.4: 3 sub-steps, FP32 and FP64, depletion with
    about half of the anchors clamped at the first sub-step) in its launch configuration (one
    anchor per block, 832 threads of 16 slots),
    one micro-step: at sampled anchors the oracle's sub-steps of every run of the anchor, each after
    the clamp and pool of the anchor's current sub-state (psi of the step's start); the coarse
    density after the step from the GPU's own new state and psi; the marginal m0 at sampled
    filament cells against the sum of the GPU's own new state."""
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=128, ny=128, ntheta=32, ns=32, rc=0.1, v0=8.0, motor_cfl=0.4)
    cells = A.r0_cells(p)
    nc = len(cells)
    rng = np.random.default_rng(12)
    dtype = np.float32 if precision else np.float64
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0).astype(dtype)
    Mb0 = rng.uniform(0.0, 2.0, (nc, p.nx, p.ny)).astype(dtype)
    u, G = (a.astype(dtype) for a in gen.make_fluid(p.nx, p.ny))
    dt = gen.cfl_dt(p, [(u, G)])
    nsub = A.motor_substeps(p, dt)
    assert nsub == 3
    h = dt / nsub
    ds, dx, dy, dth = p.L / p.ns, p.lx / p.nx, p.ly / p.ny, 2 * np.pi / p.ntheta
    a, b, k = cells[:, 0], cells[:, 1], cells[:, 2]

    def at(field, i0, j0):  # the anchor's cells of a [ncell][nx][ny] field
        return field[np.arange(nc), (i0 + a) % p.nx, (j0 + b) % p.ny]

    def coarse(y, psi, i0, j0):
        return float(np.sum(y * psi[(i0 + a) % p.nx, (j0 + b) % p.ny, k].astype(np.float64)) * ds * dx * dy * dth)

    anchors = [(int(rng.integers(p.nx)), int(rng.integers(p.ny))) for _ in range(6)]
    p.m_total = float(np.median([coarse(at(Mb0, *r).astype(np.float64), psi0, *r) for r in anchors]))
    ctx = mmk.Context(p, precision=precision)
    ctx.profile(True)
    ctx.set_state(torch.as_tensor(psi0), torch.as_tensor(Mb0))
    ctx.set_fluid(torch.as_tensor(u), torch.as_tensor(G))
    ctx.step(1, dt)
    psi1, Mb1 = ctx.get_state()
    m0, _ = ctx.get_motor_moments()
    co1, _ = ctx.get_anchors()
    assert onepass_launches(ctx)[0] == 1
    psi1, Mb1, m0, co1 = psi1.cpu().numpy(), Mb1.cpu().numpy(), m0.cpu().numpy(), co1.cpu().numpy()
    torch.cuda.synchronize()
    ctx.close()
    brk = np.nonzero((np.diff(cells[:, 3]) != 1) | np.any(np.diff(cells[:, :3], axis=0) != 0, axis=1))[0]
    edges = np.concatenate([[0], brk + 1, [nc]])
    clamped = 0
    for (i0, j0) in anchors:
        y = at(Mb0, i0, j0).astype(np.float64)
        for q in range(nsub):
            co = coarse(y, psi0, i0, j0)
            over = co > p.m_total
            clamped += over and q == 0
            scale, src = (p.m_total / co, 0.0) if over else (1.0, p.k_on * (p.m_total - co))
            for r in range(len(edges) - 1):
                c0, c1 = edges[r], edges[r + 1]
                y[c0:c1] = A.run_step(p, h, scale * y[c0:c1], src)
        got = at(Mb1, i0, j0).astype(np.float64)
        assert np.max(np.abs(got - y)) <= tol * 2.0, (i0, j0)
        want_co = coarse(got, psi1, i0, j0)
        assert abs(co1[i0, j0] - want_co) <= tol * want_co, (i0, j0)
    assert 0 < clamped < len(anchors)
    for _ in range(8):
        i, j, kk = int(rng.integers(p.nx)), int(rng.integers(p.ny)), int(rng.integers(p.ntheta))
        sel = k == kk
        want = float(np.sum(Mb1[sel, i, j].astype(np.float64))) * ds * dx * dy
        assert abs(m0[i, j, kk] - want) <= tol * abs(want)


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


@pytest.mark.parametrize("nsub", [1, 3])
def test_resume_is_bitwise(nsub):
    """8 steps in one context give the same bits as 4 steps, get_state, a new context and set_state,
    4 more steps (the state carries everything: set_state rebuilds the run totals and marginals
    with the same sums the motor launch makes; with 3 sub-steps the state leaves the first context
    from the anchor layout and enters the second one tiled)."""
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=20, ny=18, ntheta=16, ns=16, rc=0.35)
    cells, psi0, Mb0, fl, dt = r0_case(p, True) if nsub == 1 else substep_r0_case(p, True, nsub)
    a = run_r0_gpu(p, psi0, Mb0, fl, 4, 8, dt)
    assert (a["launches"]["r0_anchor_step"] > 0) == (nsub > 1)
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


@pytest.mark.parametrize("onepass", [1, 0])
@pytest.mark.parametrize("kw,depletion,nsub,Kn", SUBSTEP_CASES)
def test_substeps_fp64_against_oracle(kw, depletion, nsub, Kn, onepass):
    """Motor sub-cycling of the runs (Alg. 2's local dt*), with depletion every sub-step after the
    clamp and the pool of its anchor's current sub-state: one anchor per block (all sub-steps of a
    micro-step in one launch), and one coarse pass and motor launch per sub-step."""
    if not depletion and not onepass:
        pytest.skip("the option selects between the depleted paths only")
    p = ModelParams(**kw)
    cells, psi0, Mb0, fl, dt = substep_r0_case(p, depletion, nsub)
    K, n = Kn
    g = run_r0_gpu(p, psi0, Mb0, fl, K, n, dt, options={"r0_onepass": onepass})
    print(g["launches"], flush=True)
    assert (g["launches"]["r0_anchor_step"] == n) == onepass_expected(cells, depletion, nsub, 0, onepass)
    o = run_r0_oracle(p, psi0, Mb0, fl, K, n, dt)
    compare(g, o, 1e-12)


def onepass_launches(ctx):
    return ctx.profile_read("r0_anchor_step")[1], ctx.profile_read("r0_motor_step")[1]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kw", [
    dict(nx=24, ny=24, ntheta=8, ns=8, rc=0.3),    # runs <= 4: 4 slots a thread, 64 threads
    dict(nx=24, ny=24, ntheta=8, ns=8, rc=0.45),   # runs <= 8: 8 slots a thread, 128 threads
])
def test_onepass_few_slots_against_oracle(kw, precision):
    """The one-pass kernel with 4 and 8 slots a thread (the forms that store each anchor after the
    next one's loads in FP64 as well) and up to 3 anchors per block in turn, against the oracle:
    FP64 1e-12, FP32 against the FP64 oracle 1e-5."""
    p = ModelParams(**kw)
    cells, psi0, Mb0, fl, dt = substep_r0_case(p, True, 3)
    assert run_length_max(cells) <= 8
    if precision:
        psi0, Mb0 = psi0.astype(np.float32), Mb0.astype(np.float32)
    g = run_r0_gpu(p, psi0, Mb0, fl, 3, 6, dt, precision=precision)
    assert g["launches"]["r0_anchor_step"] == 6
    o = run_r0_oracle(p, psi0.astype(np.float64), Mb0.astype(np.float64), fl, 3, 6, dt)
    compare(g, o, 1e-5 if precision else 1e-12)


@pytest.mark.parametrize("kw,precision", [
    (dict(nx=20, ny=18, ntheta=16, ns=16, rc=0.35), 0),           # 16 slots a thread
    (dict(nx=24, ny=22, ntheta=16, ns=24, rc=0.45, v0=1.7), 1),  # runs of 22 cells: 24 slots (FP32)
])
def test_onepass_and_per_substep_paths_agree(kw, precision):
    """The two depleted sub-cycling paths on the same inputs (they differ only in the association of
    the coarse sums and where the run totals are rounded), and which launches each made."""
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(**kw)
    cells, psi0, Mb0, fl, dt = substep_r0_case(p, True, 3)
    assert onepass_expected(cells, True, 3, precision)
    if precision:
        psi0, Mb0 = psi0.astype(np.float32), Mb0.astype(np.float32)
    outs = []
    for onepass in (1, 0):
        ctx = mmk.Context(p, precision=precision, options={"r0_onepass": onepass})
        ctx.profile(True)
        ctx.set_state(torch.as_tensor(psi0), torch.as_tensor(Mb0))
        ctx.set_fluid(*map(torch.as_tensor, fl[0]))
        ctx.step(3, dt)
        ctx.set_fluid(*map(torch.as_tensor, fl[1]))
        ctx.step(2, dt)
        psi, Mb = ctx.get_state()
        m0, m1 = ctx.get_motor_moments()
        co, fr = ctx.get_anchors()
        n8, n6 = onepass_launches(ctx)
        # set_state makes one anchor-resolved motor launch (the totals of the new state)
        assert (n8, n6) == ((5, 1) if onepass else (0, 1 + 5 * 3)), (n8, n6)
        outs.append({k: v.double().cpu().numpy() for k, v in
                     dict(psi=psi, M=Mb, m0=m0, m1=m1, stress=ctx.get_stress(), mom=ctx.get_moments(),
                          coarse=co, free=fr).items()})
        torch.cuda.synchronize()
        ctx.close()
    tol = 2e-6 if precision else 1e-13
    for f in outs[0]:
        err = rel_err(outs[0][f], outs[1][f])
        print(f, f"{err:.2e}", flush=True)
        assert err <= tol, (f, err)


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_onepass_layout_round_trips(precision, tol):
    """One context through every change of the state's layout, against the oracle stepped alongside:
    one-pass steps (anchor layout), get_state, get_anchors and get_force from it (the force leaves
    the layout as it is: the next one-pass call starts from it), steps of the other path (tiled
    again), one-pass steps once more, a get_state/set_state round trip; FP64 1e-12, FP32 (its
    inputs rounded to FP32, the oracle in FP64) 1e-5."""
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=20, ny=18, ntheta=16, ns=16, rc=0.35)
    cells, psi0, Mb0, fl, dt = substep_r0_case(p, True, 3)
    if precision:
        psi0, Mb0 = (a.astype(np.float32).astype(np.float64) for a in (psi0, Mb0))
        fl = [tuple(a.astype(np.float32).astype(np.float64) for a in f) for f in fl]
    ctx = mmk.Context(p, precision=precision)
    o = A.OracleR0(p)
    ctx.set_state(torch.as_tensor(psi0), torch.as_tensor(Mb0))
    o.set_state(psi0, Mb0)

    def check(tag, force=False):
        psi, Mb = ctx.get_state()
        psi, Mb = psi.double().cpu().numpy(), Mb.double().cpu().numpy()
        co, _ = ctx.get_anchors()
        errs = dict(psi=rel_err(psi, o.psi), M=rel_err(Mb, o.Mb), coarse=rel_err(co.double().cpu().numpy(), o.coarse()))
        m0, m1 = ctx.get_motor_moments()
        om0, om1 = o.marginals()
        errs.update(m0=rel_err(m0.double().cpu().numpy(), om0), m1=rel_err(m1.double().cpu().numpy(), om1))
        if force:
            errs["force"] = rel_err(ctx.get_force().double().cpu().numpy(), A.r0_motor_force(p, cells, o.psi, o.Mb))
        print(tag, {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
        for k, v in errs.items():
            assert v <= tol, (tag, k, v)

    for e, (onepass, K) in enumerate([(1, 2), (1, 1), (0, 2), (1, 2)]):
        ctx.set_option("r0_onepass", onepass)
        ctx.set_fluid(*map(torch.as_tensor, fl[e % 2]))
        o.set_fluid(*fl[e % 2])
        ctx.step(K, dt)
        o.step(K, dt)
        check(f"call {e} onepass {onepass}", force=e in (0, 3))
    psi, Mb = ctx.get_state()
    ctx.set_state(psi, Mb)
    ctx.step(1, dt)
    o.step(1, dt)
    check("after set_state")
    torch.cuda.synchronize()
    ctx.close()


def test_onepass_graph_replays_are_bitwise():
    """mmk_step_graph on the one-pass path: the first graph includes the change to the anchor
    layout, later ones start from it; a get_force in between leaves the layout as it is, and a
    get_state/set_state round trip (back to tiled) makes the next call use the first graph again.
    Every replay has the bits of mmk_step in a twin context."""
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=20, ny=18, ntheta=16, ns=16, rc=0.35)
    cells, psi0, Mb0, fl, dt = substep_r0_case(p, True, 2)
    ctxs = [mmk.Context(p), mmk.Context(p)]
    for c in ctxs:
        c.set_state(torch.as_tensor(psi0), torch.as_tensor(Mb0))
        c.set_fluid(*map(torch.as_tensor, fl[0]))
    for r in range(5):
        ctxs[0].step_graph(2, dt)
        ctxs[1].step(2, dt)
        if r in (1, 2):
            fa, fb = (c.get_force().double().cpu().numpy() for c in ctxs)
            assert np.array_equal(fa, fb)
        torch.cuda.synchronize()  # eager work and synchronisation between the replays
        (pa, Ma), (pb, Mbb) = (c.get_state() for c in ctxs)
        assert torch.equal(pa, pb) and torch.equal(Ma, Mbb), r
        assert torch.equal(ctxs[0].get_stress(), ctxs[1].get_stress()), r
        assert torch.equal(ctxs[0].get_motor_moments()[0], ctxs[1].get_motor_moments()[0]), r
        if r == 2:  # set_state clears the step's outputs: after the checks
            for c in ctxs:
                c.set_state(*c.get_state())
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("kw,depletion", [
    (dict(nx=20, ny=18, ntheta=16, ns=16, rc=0.35), True),
    (dict(nx=20, ny=18, ntheta=16, ns=16, rc=0.35), False),
    (dict(nx=24, ny=22, ntheta=16, ns=24, rc=0.45, v0=1.7), True),  # one anchor per block, 24 slots
])
def test_substeps_fp32_against_fp64_oracle(kw, depletion):
    p = ModelParams(**kw)
    cells, psi0, Mb0, fl, dt = substep_r0_case(p, depletion, 3)
    psi32, Mb32 = psi0.astype(np.float32), Mb0.astype(np.float32)
    g = run_r0_gpu(p, psi32, Mb32, fl, 4, 8, dt, precision=1)
    assert (g["launches"]["r0_anchor_step"] == 8) == onepass_expected(cells, depletion, 3, 1)
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
