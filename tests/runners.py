"""Drives the HIP library and the oracle through the same call sequence (test helper)."""
from __future__ import annotations

import numpy as np

from oracle import oracle_a as A
from paper_1908_04279_amd import inputs as gen


def run_oracle(p, psi0, M0, fluids, K, n, dt):
    """Full FP64 oracle: n steps, fluid e used for steps [eK, (e+1)K)."""
    o = A.OracleA(p)
    o.set_state(psi0, M0)
    done, e = 0, 0
    while done < n:
        o.set_fluid(*fluids[min(e, len(fluids) - 1)])
        k = min(K, n - done)
        o.step(k, dt)
        done += k
        e += 1
    stress, mom = o.get_stress_moments()
    mass, ss = A.global_sums(p, o.psi, stress)
    return dict(psi=o.psi, M=o.M, m0=o.m0, m1=o.m1, stress=stress, mom=mom, mass=mass, sum_sigma=ss)


def run_oracle_uniform_columns(p, psi0, fluids, K, n, dt, col0=None):
    """Oracle for an initial M whose columns are all equal (col0, default 0): every column
    then follows the same trajectory, so one oracle column and the oracle's psi step with
    the broadcast m0 give the full oracle result exactly (checked bitwise on the CPU)."""
    col = np.zeros(p.ns) if col0 is None else np.array(col0, dtype=np.float64)
    psi = np.array(psi0, dtype=np.float64)
    m0c = m1c = 0.0
    for step in range(n):
        col = A.column_step(p, dt, col)
        m0c, m1c = A.column_moments(p, col)
        u, g = fluids[min(step // K, len(fluids) - 1)]
        psi = A.psi_step(p, dt, psi, np.full(psi.shape, m0c), u, g)
    m0 = np.full(psi.shape, m0c)
    m1 = np.full(psi.shape, m1c)
    stress, mom = A.moments(p, psi, m0, m1)
    mass, ss = A.global_sums(p, psi, stress)
    return dict(psi=psi, col=col, m0=m0, m1=m1, stress=stress, mom=mom, mass=mass, sum_sigma=ss)


def run_gpu(p, psi0, M0, fluids, K, n, dt, precision=0, keep_ctx=False, want_M=True, options=None, profile=False):
    import torch
    from paper_1908_04279_amd import mmk
    ctx = mmk.Context(p, precision=precision, options=options)
    if profile:
        ctx.profile(True)
    ctx.set_state(torch.as_tensor(psi0), None if M0 is None else torch.as_tensor(M0))
    done, e = 0, 0
    while done < n:
        u, g = fluids[min(e, len(fluids) - 1)]
        ctx.set_fluid(torch.as_tensor(u), torch.as_tensor(g))
        k = min(K, n - done)
        ctx.step(k, dt)
        done += k
        e += 1
    out = {}
    if want_M:
        psi, M = ctx.get_state()
        out["M"] = M.double().cpu().numpy()
    else:
        psi = ctx.get_psi()
    m0, m1 = ctx.get_motor_moments()
    out.update(psi=psi.double().cpu().numpy(), stress=ctx.get_stress().double().cpu().numpy(),
               mom=ctx.get_moments().double().cpu().numpy(), m0=m0.double().cpu().numpy(),
               m1=m1.double().cpu().numpy())
    out["mass"], out["sum_sigma"] = ctx.get_sums()
    torch.cuda.synchronize()
    if keep_ctx:
        out["ctx"] = ctx
    else:
        ctx.close()
    return out


def seeded_case(p, n_exchanges=1, new_each=True, M0_kind="zero"):
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=0)
    fluids = gen.fluid_schedule(p.nx, p.ny, n_exchanges, p.lx, p.ly, new_each=new_each)
    dt = gen.cfl_dt(p, fluids)
    if M0_kind == "zero":
        M0 = None
    else:
        M0 = gen.make_M0_random(p.nx, p.ny, p.ntheta, p.ns, p.k_on, p.k_off, seed=5)
    return psi0, M0, fluids, dt


def run_r0_oracle(p, psi0, Mb0, fluids, K, n, dt):
    """FP64 oracle of the anchor-resolved model through the same call sequence."""
    o = A.OracleR0(p)
    o.set_state(psi0, Mb0)
    done, e = 0, 0
    while done < n:
        o.set_fluid(*fluids[min(e, len(fluids) - 1)])
        k = min(K, n - done)
        o.step(k, dt)
        done += k
        e += 1
    stress, mom = o.get_stress_moments()
    mass, ss = A.global_sums(p, o.psi, stress)
    m0, m1 = o.marginals()
    coarse = o.coarse()
    free = (p.m_total - np.minimum(coarse, p.m_total)) if p.m_total > 0 else np.ones_like(coarse)
    return dict(psi=o.psi, M=o.Mb, m0=m0, m1=m1, stress=stress, mom=mom, mass=mass, sum_sigma=ss,
                coarse=coarse, free=free)


def run_r0_gpu(p, psi0, Mb0, fluids, K, n, dt, precision=0, options=None):
    """The HIP library on the anchor-resolved model, with the per-anchor outputs and the number of
    motor launches of each kind (launches: one anchor per block, one per sub-step or step)."""
    import torch
    out = run_gpu(p, psi0, Mb0, fluids, K, n, dt, precision=precision, keep_ctx=True, options=options, profile=True)
    ctx = out.pop("ctx")
    out["launches"] = {k: ctx.profile_read(k)[1] for k in ("r0_anchor_step", "r0_motor_step")}
    coarse, free = ctx.get_anchors()
    out["coarse"] = coarse.double().cpu().numpy()
    out["free"] = free.double().cpu().numpy()
    torch.cuda.synchronize()
    ctx.close()
    return out


def run_oracle_window(p, psi0, M0_of_cols, fluids, calls, dt, i, j, R):
    """FP64 oracle at grid point (i, j) after the micro-steps of `calls` (K of each mmk_step
    call; call e uses fluids[e]), from the (2R+1) x (2R+1) patch of the periodic grid centred
    there.  The patch runs as a periodic grid of its own with the full grid's cell sizes.  The
    donor-cell stencil reaches one cell per step and the motor columns of the linear model are
    independent, so for sum(calls) <= R the patch centre sees only its true neighbours and the
    result there is the full-grid oracle's, bit for bit (pinned on the CPU).
    psi0: the full [nx][ny][nth] array; M0_of_cols(cols) -> [len(cols)][ns], the initial motor
    columns by flat column index (i, j, k) -> (i ny + j) nth + k.
    Returns the centre's psi [nth], M [nth][ns], m0, m1 [nth], stress [3], moments [7]."""
    from dataclasses import replace
    n = int(sum(calls))
    assert R >= n
    w = 2 * R + 1
    if w >= min(p.nx, p.ny):
        raise ValueError("window as large as the grid: run the full oracle")
    ii = (i + np.arange(-R, R + 1)) % p.nx
    jj = (j + np.arange(-R, R + 1)) % p.ny
    q = replace(p, nx=w, ny=w, lx=p.lx / p.nx * w, ly=p.ly / p.ny * w)
    psi = np.ascontiguousarray(np.asarray(psi0)[np.ix_(ii, jj)], dtype=np.float64)
    cols = ((ii[:, None, None] * p.ny + jj[None, :, None]) * p.ntheta
            + np.arange(p.ntheta)[None, None, :]).reshape(-1)
    M = np.ascontiguousarray(M0_of_cols(cols), dtype=np.float64).reshape(w, w, p.ntheta, p.ns)
    o = A.OracleA(q)
    o.set_state(psi, M)
    for e, k in enumerate(calls):
        u, g = fluids[e]
        o.set_fluid(np.ascontiguousarray(u[:, ii][:, :, jj]), np.ascontiguousarray(g[:, ii][:, :, jj]))
        o.step(int(k), dt)
    stress, mom = o.get_stress_moments()
    return dict(psi=o.psi[R, R].copy(), M=o.M[R, R].copy(), m0=o.m0[R, R].copy(), m1=o.m1[R, R].copy(),
                stress=stress[:, R, R].copy(), mom=mom[:, R, R].copy())
