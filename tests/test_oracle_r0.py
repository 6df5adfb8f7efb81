"""Pins of the oracle's anchor-resolved bound-motor step (Sec. 2: M_b(r0, x, p, s) on the capture
ball B_rc(r0); Eqs. (4)-(6); Alg. 2: per anchor the motor update, the coarse integral, the
clamp and the free pool).

Each pin reaches the oracle by another route: the tracked set by brute force over anchor and
filament positions on the torus, and by its continuum volume; the motor step by the closed form
without walking and by the exact steady profile of a run; a whole micro-step with depletion and
clamp by a pure-Python re-implementation on a tiny grid that knows nothing of the oracle's
cell list or layout.
"""
import math

import numpy as np
import pytest

from oracle import oracle_a as A
from paper_1908_04279_amd import inputs as gen
from paper_1908_04279_amd.inputs import ModelParams


def torus_tracked(p):
    """Tracked (a, b, k, l) by brute force: for the anchor at the centre of cell (0, 0) and every
    filament cell (i, j, k, l) of the periodic box, the motor point (x_i, y_j) + (s_l - L/2) p_k,
    its minimum-image distance to the anchor, and the offset (a, b) of (i, j) from the anchor.
    Also returns the smallest |distance^2 - rc^2| seen (ties would make the test ill-posed)."""
    dx, dy, dth, ds = p.lx / p.nx, p.ly / p.ny, 2 * math.pi / p.ntheta, p.L / p.ns
    ax, ay = 0.5 * dx, 0.5 * dy
    out, margin = set(), np.inf
    for i in range(p.nx):
        for j in range(p.ny):
            a = i if i <= p.nx // 2 else i - p.nx
            b = j if j <= p.ny // 2 else j - p.ny
            for k in range(p.ntheta):
                for l in range(p.ns):
                    t = (l + 0.5) * ds - 0.5 * p.L
                    hx = (i + 0.5) * dx + t * math.cos(k * dth) - ax
                    hy = (j + 0.5) * dy + t * math.sin(k * dth) - ay
                    hx -= p.lx * round(hx / p.lx)
                    hy -= p.ly * round(hy / p.ly)
                    d2 = hx * hx + hy * hy
                    margin = min(margin, abs(d2 - p.rc * p.rc))
                    if d2 <= p.rc * p.rc:
                        out.add((a, b, k, l))
    return out, margin


@pytest.mark.parametrize("kw", [
    dict(nx=12, ny=12, ntheta=8, ns=8, rc=0.45),
    dict(nx=16, ny=10, ntheta=12, ns=10, rc=0.3, L=1.4),
    dict(nx=9, ny=14, ntheta=6, ns=5, rc=0.8, lx=5.0, ly=7.0),
])
def test_cells_are_the_capture_ball(kw):
    p = ModelParams(**kw)
    cells = A.r0_cells(p)
    want, margin = torus_tracked(p)
    assert margin > 1e-9
    got = [tuple(int(v) for v in c) for c in cells]
    assert set(got) == want
    assert got == sorted(got)  # lexicographic (a, b, k, l)


def test_tracked_volume_is_the_continuum_one():
    """Each orientation and arclength point sees the anchors of a disc of area pi rc^2 around its
    motor point, so the tracked set has measure 2 pi * L * pi rc^2 in (x, th, s); the cell count
    times dx dy dth ds approaches it (lattice count of a disc, within a few per cent)."""
    p = ModelParams(nx=96, ny=96, ntheta=16, ns=16, rc=0.4)
    n = len(A.r0_cells(p))
    vol = n * (p.lx / p.nx) * (p.ly / p.ny) * (2 * math.pi / p.ntheta) * (p.L / p.ns)
    want = 2 * math.pi * p.L * math.pi * p.rc ** 2
    assert abs(vol / want - 1) < 0.03, vol / want


def test_window_limit():
    with pytest.raises(ValueError):
        A.r0_cells(ModelParams(nx=8, ny=8, ntheta=4, ns=4, rc=2.7))  # rc + L/2 >= pi
    with pytest.raises(ValueError):
        A.r0_cells(ModelParams(nx=8, ny=8, ntheta=4, ns=4, rc=0.0))


def test_no_walking_closed_form():
    """v0 = 0, linear attachment: every tracked cell is M' = k_on - k_off M, a midpoint step of h
    maps M - c to (M - c) g with g = 1 - k_off h + (k_off h)^2 / 2, c = k_on / k_off; the
    marginal m0 is the brute-force sum over the anchors of the torus."""
    p = ModelParams(nx=10, ny=8, ntheta=8, ns=6, rc=0.5, v0=0.0, k_on=0.7, k_off=1.3)
    cells = A.r0_cells(p)
    Mb0 = gen.make_Mb0_random(len(cells), p.nx, p.ny, p.k_on, p.k_off, seed=2)
    o = A.OracleR0(p)
    o.set_state(gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0), Mb0)
    o.set_fluid(*gen.make_fluid(p.nx, p.ny))
    dt, n = 0.05, 7
    o.step(n, dt)
    g = 1 - p.k_off * dt + 0.5 * (p.k_off * dt) ** 2
    c = p.k_on / p.k_off
    want = c + (Mb0 - c) * g ** n
    assert np.max(np.abs(o.Mb - want)) <= 1e-14 * np.max(np.abs(want))
    m0, _ = o.marginals()
    index = {tuple(int(v) for v in cl): q for q, cl in enumerate(cells)}
    dx, dy, ds = p.lx / p.nx, p.ly / p.ny, p.L / p.ns
    bf = np.zeros((p.nx, p.ny, p.ntheta))
    for i in range(p.nx):
        for j in range(p.ny):
            for i0 in range(p.nx):          # every anchor of the box
                for j0 in range(p.ny):
                    a = (i - i0) % p.nx
                    b = (j - j0) % p.ny
                    a = a if a <= p.nx // 2 else a - p.nx
                    b = b if b <= p.ny // 2 else b - p.ny
                    for k in range(p.ntheta):
                        for l in range(p.ns):
                            q = index.get((a, b, k, l))
                            if q is not None:
                                bf[i, j, k] += o.Mb[q, i, j] * ds * dx * dy
    assert np.max(np.abs(m0 - bf)) <= 1e-14 * np.max(np.abs(bf))


def test_run_steady_profile():
    """First-order flux, linear attachment: a run of n tracked cells has the exact steady state
    c (1 - rho^(t+1)), t = 0..n-1, rho = v0 / (v0 + k_off ds) (no influx at its first cell,
    free outflow at its last), whatever its place on the filament."""
    p = ModelParams(nx=8, ny=8, ntheta=8, ns=12, rc=0.6, v0=0.9, k_on=0.8, k_off=1.1, limiter=1)
    cells = A.r0_cells(p)
    ds = p.L / p.ns
    dt = 0.4 / (p.v0 / ds + p.k_off)
    Mb = np.zeros((len(cells), p.nx, p.ny))
    for _ in range(1500):
        Mb = A.r0_motor_step(p, dt, cells, Mb)
    rho = p.v0 / (p.v0 + p.k_off * ds)
    c = p.k_on / p.k_off
    q = 0
    nrun = 0
    while q < len(cells):
        r = q + 1
        while r < len(cells) and tuple(cells[r, :3]) == tuple(cells[q, :3]) and cells[r, 3] == cells[r - 1, 3] + 1:
            r += 1
        want = c * (1 - rho ** (np.arange(r - q) + 1.0))
        assert np.max(np.abs(Mb[q:r] - want[:, None, None])) <= 1e-13, (q, r)
        nrun += 1
        q = r
    assert nrun > 10


def superbee(a, b):
    if a * b <= 0:
        return 0.0
    r = max(min(2 * abs(a), abs(b)), min(abs(a), 2 * abs(b)))
    return r if b > 0 else -r


def py_run_step(z, dt, v0, src, k_off, ds, limiter):
    """Midpoint RK2 of one run (written afresh: face fluxes, then the update)."""
    def rhs(y):
        n = len(y)
        flux = [0.0] * (n + 1)
        for t in range(n):
            left = y[t - 1] if t > 0 else 0.0
            right = y[t + 1] if t + 1 < n else y[t]
            slope = superbee(y[t] - left, right - y[t]) if limiter == 0 else 0.0
            flux[t + 1] = v0 * y[t] if t == n - 1 else v0 * (y[t] + 0.5 * slope)
        return [-(flux[t + 1] - flux[t]) / ds + src - k_off * y[t] for t in range(n)]
    r1 = rhs(z)
    mid = [z[t] + 0.5 * dt * r1[t] for t in range(len(z))]
    r2 = rhs(mid)
    return [z[t] + dt * r2[t] for t in range(len(z))]


def py_r0_step(p, dt, psi, Mb_of):
    """One micro-step's motor part with depletion, by anchors: Mb_of maps
    (anchor i0, j0, filament i, j, k, l) -> value for tracked configurations only."""
    dx, dy, dth, ds = p.lx / p.nx, p.ly / p.ny, 2 * math.pi / p.ntheta, p.L / p.ns
    coarse = np.zeros((p.nx, p.ny))
    for (i0, j0, i, j, k, l), v in Mb_of.items():
        coarse[i0, j0] += v * psi[i, j, k] * ds * dx * dy * dth
    scale = np.where(coarse > p.m_total, p.m_total / np.maximum(coarse, 1e-300), 1.0)
    src = np.where(coarse > p.m_total, 0.0, p.k_on * (p.m_total - coarse))
    cols = {}
    for key in sorted(Mb_of):
        cols.setdefault(key[:5], []).append(key[5])
    new = {}
    for (i0, j0, i, j, k), ls in cols.items():
        runs, cur = [], [ls[0]]
        for l in ls[1:]:
            if l == cur[-1] + 1:
                cur.append(l)
            else:
                runs.append(cur)
                cur = [l]
        runs.append(cur)
        for run in runs:
            z = [scale[i0, j0] * Mb_of[(i0, j0, i, j, k, l)] for l in run]
            z = py_run_step(z, dt, p.v0, src[i0, j0], p.k_off, ds, p.limiter)
            for l, v in zip(run, z):
                new[(i0, j0, i, j, k, l)] = v
    m0 = np.zeros((p.nx, p.ny, p.ntheta))
    m1 = np.zeros((p.nx, p.ny, p.ntheta))
    for (i0, j0, i, j, k, l), v in new.items():
        m0[i, j, k] += v * ds * dx * dy
        m1[i, j, k] += ((l + 0.5) * ds - 0.5 * p.L) * v * ds * dx * dy
    return new, coarse, m0, m1


@pytest.mark.parametrize("limiter", [0, 1])
def test_micro_step_by_anchors(limiter):
    """Two micro-steps with depletion (about half of the anchors clamped) against the pure-Python
    step organised by anchors, which finds its own tracked set on the torus."""
    p = ModelParams(nx=7, ny=6, ntheta=6, ns=7, rc=0.75, v0=1.1, k_on=0.9, k_off=0.6, limiter=limiter)
    cells = A.r0_cells(p)
    want, margin = torus_tracked(p)
    assert margin > 1e-9 and len(cells) == len(want)
    psi = gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0)
    Mb0 = gen.make_Mb0_random(len(cells), p.nx, p.ny, p.k_on, p.k_off, seed=4)
    coarse0 = A.r0_coarse(p, cells, psi, Mb0)
    p.m_total = float(np.median(coarse0))
    u, G = gen.make_fluid(p.nx, p.ny)
    dt = 0.5 * gen.cfl_dt(p, [(u, G)])
    # the pure-Python state, keyed by anchor and filament configuration
    Mb_of = {}
    for q, (a, b, k, l) in enumerate(cells):
        for i in range(p.nx):
            for j in range(p.ny):
                Mb_of[((i - a) % p.nx, (j - b) % p.ny, i, j, int(k), int(l))] = Mb0[q, i, j]
    ps = psi.copy()
    for _ in range(2):
        Mb_of, coarse, m0, m1 = py_r0_step(p, dt, ps, Mb_of)
        ps = A.psi_step(p, dt, ps, m0, u, G)
    o = A.OracleR0(p)
    o.set_state(psi, Mb0)
    o.set_fluid(u, G)
    o.step(1, dt)
    assert 0.2 < np.mean(coarse0 > p.m_total) < 0.8
    o.step(1, dt)
    got = np.zeros_like(Mb0)
    for (i0, j0, i, j, k, l), v in Mb_of.items():
        a, b = (i - i0) % p.nx, (j - j0) % p.ny
        a = a if a <= p.nx // 2 else a - p.nx
        b = b if b <= p.ny // 2 else b - p.ny
        q = np.nonzero((cells == (a, b, k, l)).all(axis=1))[0]
        assert len(q) == 1
        got[q[0], i, j] = v
    scale = np.max(np.abs(got))
    assert np.max(np.abs(o.Mb - got)) <= 1e-13 * scale
    gm0, gm1 = o.marginals()
    assert np.max(np.abs(gm0 - m0)) <= 1e-13 * np.max(np.abs(m0))
    assert np.max(np.abs(gm1 - m1)) <= 1e-13 * np.max(np.abs(m1))
    assert np.max(np.abs(o.psi - ps)) <= 1e-13 * np.max(np.abs(ps))


def test_clamp_brings_the_anchor_to_its_total():
    """Where the coarse density exceeds m_total the anchor's cells are scaled to the total and
    the pool is 0: with v0 = 0 one step is then a pure decay of the scaled state."""
    p = ModelParams(nx=8, ny=8, ntheta=8, ns=8, rc=0.5, v0=0.0, k_on=0.9, k_off=0.7)
    cells = A.r0_cells(p)
    psi = gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0)
    Mb0 = gen.make_Mb0_random(len(cells), p.nx, p.ny, seed=1)
    coarse = A.r0_coarse(p, cells, psi, Mb0)
    p.m_total = 0.5 * float(np.min(coarse))  # every anchor over-bound
    scale = p.m_total / coarse
    # the clamped state of every anchor carries exactly the total
    clamped = np.empty_like(Mb0)
    for q, (a, b, _, _) in enumerate(cells):
        clamped[q] = Mb0[q] * np.roll(np.roll(scale, a, axis=0), b, axis=1)
    assert np.max(np.abs(A.r0_coarse(p, cells, psi, clamped) / p.m_total - 1)) < 1e-14
    o = A.OracleR0(p)
    o.set_state(psi, Mb0)
    o.set_fluid(np.zeros((2, p.nx, p.ny)), np.zeros((4, p.nx, p.ny)))
    dt = 0.03
    o.step(1, dt)
    g = 1 - p.k_off * dt + 0.5 * (p.k_off * dt) ** 2
    assert np.max(np.abs(o.Mb - clamped * g)) <= 1e-15 * np.max(clamped)


def test_marginal_field_by_brute_force():
    """The anchor-marginal field that the motor force of the anchor-resolved model spreads (the
    r0 integral of Eq. (10)): M(x, k, l) = sum over all anchors of the torus of M_b dx dy, found
    by minimum-image offsets; its s-sum is the marginal m0."""
    p = ModelParams(nx=7, ny=6, ntheta=6, ns=5, rc=0.7)
    cells = A.r0_cells(p)
    Mb = gen.make_Mb0_random(len(cells), p.nx, p.ny, seed=3)
    M = A.r0_marginal_field(p, cells, Mb)
    index = {tuple(int(v) for v in cl): q for q, cl in enumerate(cells)}
    dx, dy = p.lx / p.nx, p.ly / p.ny
    bf = np.zeros((p.nx, p.ny, p.ntheta, p.ns))
    for i in range(p.nx):
        for j in range(p.ny):
            for i0 in range(p.nx):
                for j0 in range(p.ny):
                    a, b = (i - i0) % p.nx, (j - j0) % p.ny
                    a = a if a <= p.nx // 2 else a - p.nx
                    b = b if b <= p.ny // 2 else b - p.ny
                    for k in range(p.ntheta):
                        for l in range(p.ns):
                            q = index.get((a, b, k, l))
                            if q is not None:
                                bf[i, j, k, l] += Mb[q, i, j] * dx * dy
    assert np.max(np.abs(M - bf)) <= 1e-14 * np.max(bf)
    m0, _ = A.r0_marginal(p, cells, Mb)
    assert np.max(np.abs(M.sum(-1) * (p.L / p.ns) - m0)) <= 1e-14 * np.max(m0)


def test_substeps_no_walking_closed_form():
    """Sub-cycling (motor_cfl > 0) without walking, linear attachment: n midpoint steps of
    h = dt/n per micro-step map M - c to (M - c) g^n, g = 1 - k_off h + (k_off h)^2 / 2."""
    p = ModelParams(nx=10, ny=8, ntheta=8, ns=6, rc=0.5, v0=0.0, k_on=0.7, k_off=1.3)
    dt, K = 0.05, 4
    p.motor_cfl = 0.025  # rate k_off: n = ceil(0.05 * 1.3 / 0.025) = 3
    n = A.motor_substeps(p, dt)
    assert n == 3
    cells = A.r0_cells(p)
    Mb0 = gen.make_Mb0_random(len(cells), p.nx, p.ny, p.k_on, p.k_off, seed=2)
    o = A.OracleR0(p)
    o.set_state(gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0), Mb0)
    o.set_fluid(*gen.make_fluid(p.nx, p.ny))
    o.step(K, dt)
    h = dt / n
    g = 1 - p.k_off * h + 0.5 * (p.k_off * h) ** 2
    c = p.k_on / p.k_off
    want = c + (Mb0 - c) * g ** (n * K)
    assert np.max(np.abs(o.Mb - want)) <= 1e-14 * np.max(np.abs(want))


def test_one_substep_is_the_plain_step():
    """motor_cfl so large that n = 1: the same bits as motor_cfl = 0, with depletion."""
    p = ModelParams(nx=7, ny=6, ntheta=6, ns=7, rc=0.75, v0=1.1, k_on=0.9, k_off=0.6)
    cells = A.r0_cells(p)
    psi = gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0)
    Mb0 = gen.make_Mb0_random(len(cells), p.nx, p.ny, p.k_on, p.k_off, seed=4)
    p.m_total = float(np.median(A.r0_coarse(p, cells, psi, Mb0)))
    u, G = gen.make_fluid(p.nx, p.ny)
    dt = 0.5 * gen.cfl_dt(p, [(u, G)])
    outs = []
    for cfl in (0.0, 1e6):
        p.motor_cfl = cfl
        o = A.OracleR0(p)
        o.set_state(psi, Mb0)
        o.set_fluid(u, G)
        o.step(3, dt)
        outs.append(o.get_state())
    assert A.motor_substeps(p, dt) == 1
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_substeps_by_anchors():
    """Two micro-steps of 3 motor sub-steps with depletion against the pure-Python step by
    anchors applied to each sub-step: the clamp and the pool of every anchor are re-formed from
    the current sub-state before each sub-step, psi held at its start-of-step value (Alg. 2);
    psi then follows the m0 of the last sub-step."""
    p = ModelParams(nx=7, ny=6, ntheta=6, ns=7, rc=0.75, v0=1.1, k_on=0.9, k_off=0.6)
    cells = A.r0_cells(p)
    psi = gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0)
    Mb0 = gen.make_Mb0_random(len(cells), p.nx, p.ny, p.k_on, p.k_off, seed=4)
    p.m_total = float(np.median(A.r0_coarse(p, cells, psi, Mb0)))
    u, G = gen.make_fluid(p.nx, p.ny)
    dt = 0.5 * gen.cfl_dt(p, [(u, G)])
    rate = p.v0 / (p.L / p.ns) + p.k_off
    p.motor_cfl = dt * rate / 2.5  # n = 3
    n = A.motor_substeps(p, dt)
    assert n == 3
    Mb_of = {}
    for q, (a, b, k, l) in enumerate(cells):
        for i in range(p.nx):
            for j in range(p.ny):
                Mb_of[((i - a) % p.nx, (j - b) % p.ny, i, j, int(k), int(l))] = Mb0[q, i, j]
    ps = psi.copy()
    clamped = []
    for _ in range(2):
        for _ in range(n):
            Mb_of, coarse, m0, m1 = py_r0_step(p, dt / n, ps, Mb_of)
            clamped.append(np.mean(coarse > p.m_total))
        ps = A.psi_step(p, dt, ps, m0, u, G)
    assert 0.2 < clamped[0] < 0.8
    o = A.OracleR0(p)
    o.set_state(psi, Mb0)
    o.set_fluid(u, G)
    o.step(2, dt)
    got = np.zeros_like(Mb0)
    for (i0, j0, i, j, k, l), v in Mb_of.items():
        a, b = (i - i0) % p.nx, (j - j0) % p.ny
        a = a if a <= p.nx // 2 else a - p.nx
        b = b if b <= p.ny // 2 else b - p.ny
        q = np.nonzero((cells == (a, b, k, l)).all(axis=1))[0]
        got[q[0], i, j] = v
    assert np.max(np.abs(o.Mb - got)) <= 1e-13 * np.max(np.abs(got))
    gm0, gm1 = o.marginals()
    assert np.max(np.abs(gm0 - m0)) <= 1e-13 * np.max(np.abs(m0))
    assert np.max(np.abs(gm1 - m1)) <= 1e-13 * np.max(np.abs(m1))
    assert np.max(np.abs(o.psi - ps)) <= 1e-13 * np.max(np.abs(ps))
