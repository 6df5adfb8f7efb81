"""Pins of the oracle's free-motor depletion and over-binding clamp (Eqs. (5)-(6), Alg. 2).

Reading: each micro-step starts from the coarse bound density of the current state,
B(x, y) = sum_th psi m0 dth; where B exceeds the total motor density m_total, every bound-motor
column at (x, y) is scaled by m_total / B and the free pool is 0, elsewhere the pool is
m_total - B; the motor step then attaches at rate k_on * pool.
"""
import math

import numpy as np
import pytest

from oracle import oracle_a as A
from oracle import oracle_torch as B
from paper_1908_04279_amd import inputs as gen
from paper_1908_04279_amd.inputs import ModelParams
from tests.conftest import rel_err


def uniform_case(ns=16, m_total=0.5, nx=2, ny=3, nt=4, limiter=1, **kw):
    """Uniform psi of unit mass on a unit box (2 pi psi_bar = 1), no flow."""
    p = ModelParams(nx=nx, ny=ny, ntheta=nt, ns=ns, lx=1.0, ly=1.0, limiter=limiter, m_total=m_total, **kw)
    psi = np.full((nx, ny, nt), 1.0 / (2.0 * math.pi))
    u = np.zeros((2, nx, ny))
    g = np.zeros((4, nx, ny))
    return p, psi, u, g


def test_depleted_steady_state_closed_form():
    """First-order flux, uniform psi, no flow: the fixed point of the coupled system.  The
    column's fixed point with source k_on F is (k_on F / k_off)(1 - rho^{l+1}),
    rho = v0 / (v0 + k_off ds), so m0 = (k_on F / k_off) S with S = ds sum_l (1 - rho^{l+1}),
    B = 2 pi psi_bar m0, and F = m_total - B gives F = m_total / (1 + 2 pi psi_bar k_on S / k_off)."""
    ns = 16
    p, psi, u, g = uniform_case(ns=ns, m_total=0.5, k_on=1.3, k_off=0.7, v0=0.9)
    ds = p.L / ns
    rho = p.v0 / (p.v0 + p.k_off * ds)
    S = ds * sum(1.0 - rho ** (l + 1) for l in range(ns))
    psibar = psi[0, 0, 0]
    Fstar = p.m_total / (1.0 + 2.0 * math.pi * psibar * p.k_on * S / p.k_off)
    want = (p.k_on * Fstar / p.k_off) * (1.0 - rho ** (np.arange(ns) + 1.0))
    dt = 0.4 / (p.v0 / ds + p.k_off)
    o = A.OracleA(p)
    o.set_state(psi)
    o.set_fluid(u, g)
    o.step(6000, dt)
    _, M = o.get_state()
    assert Fstar > 0 and 2.0 * math.pi * psibar * (p.k_on * Fstar / p.k_off) * S < p.m_total
    for col in M.reshape(-1, ns):
        assert np.max(np.abs(col - want)) <= 1e-12 * np.max(want)


def test_clamp_scales_columns_to_the_total():
    """B of the initial state above m_total: the step equals the plain step without
    attachment (k_on = 0, the pinned linear path) applied to the columns scaled by
    m_total / B, and the scaled state holds exactly m_total bound motors per unit area."""
    ns = 12
    p, psi, u, g = uniform_case(ns=ns, m_total=0.2, limiter=0, k_on=0.9, k_off=0.6, v0=1.1)
    rng = np.random.default_rng(11)
    M0 = rng.uniform(0.5, 2.0, (p.nx, p.ny, p.ntheta, ns))
    ds = p.L / ns
    dt = 0.4 / (p.v0 / ds + p.k_off)
    # coarse bound density by hand: sum over th of psi times sum_s M ds, times dth
    Bhand = (psi * (M0 * ds).sum(-1)).sum(-1) * (2.0 * math.pi / p.ntheta)
    assert np.all(Bhand > p.m_total)
    scale = p.m_total / Bhand
    q = ModelParams(**{**p.as_dict(), "k_on": 0.0, "m_total": 0.0})
    want = np.empty_like(M0)
    for idx in np.ndindex(p.nx, p.ny, p.ntheta):
        want[idx] = A.column_step(q, dt, scale[idx[:2]] * M0[idx])
    o = A.OracleA(p)
    o.set_state(psi, M0)
    o.set_fluid(u, g)
    o.step(1, dt)
    _, M1 = o.get_state()
    assert np.max(np.abs(M1 - want)) <= 1e-15 * np.max(np.abs(want))
    m0 = (M0 * ds).sum(-1)
    Bc = A.coarse_bound(p, psi, m0)
    np.testing.assert_allclose(Bc, Bhand, rtol=1e-14)
    sc, src = A.depletion(p, Bc)
    np.testing.assert_allclose(A.coarse_bound(p, psi, m0 * sc[:, :, None]), p.m_total, rtol=1e-14)
    assert np.all(src == 0.0)


@pytest.mark.parametrize("limiter", [0, 1])
def test_budget_identity_with_attachment_source(limiter):
    """Summing R over the column telescopes with any source: m0(M') - m0(M) =
    dt [src L - k_off m0(M*) - v0 M*_{ns-1}], M* the midpoint stage."""
    rng = np.random.default_rng(5)
    for ns in [3, 16, 33]:
        p = ModelParams(nx=1, ny=1, ntheta=1, ns=ns, limiter=limiter, k_on=0.8, k_off=1.7, v0=1.3)
        ds = p.L / ns
        dt = 0.4 / (p.v0 / ds + p.k_off)
        for src in [0.0, 0.37, 2.5]:
            M = rng.uniform(0, 2, ns)
            Ms = M + 0.5 * dt * A.motor_rhs_src(p, M, src)
            M1 = A.column_step_src(p, dt, M, src)
            m0a, _ = A.column_moments(p, M)
            m0b, _ = A.column_moments(p, M1)
            m0s, _ = A.column_moments(p, Ms)
            want = dt * (src * p.L - p.k_off * m0s - p.v0 * Ms[-1])
            assert (m0b - m0a) == pytest.approx(want, rel=1e-12, abs=1e-15)


def test_free_pool_and_clamp_rule():
    """Per point: B <= m_total keeps the columns and leaves m_total - B free; B > m_total
    scales them to m_total and leaves none; B = m_total is the unclamped branch."""
    p = ModelParams(nx=2, ny=2, ntheta=4, ns=4, k_on=1.5, m_total=0.8)
    Bv = np.array([[0.0, 0.8], [0.81, 3.2]])
    scale, src = A.depletion(p, Bv)
    np.testing.assert_array_equal(scale, [[1.0, 1.0], [0.8 / 0.81, 0.25]])
    np.testing.assert_array_equal(src, [[1.5 * 0.8, 0.0], [0.0, 0.0]])


def test_c_and_torch_oracles_agree_with_depletion():
    """Random non-uniform state and flow on a small grid, m_total between the smallest and
    the largest coarse bound density so both branches occur, 12 steps, both limiters."""
    for limiter in (0, 1):
        p = ModelParams(nx=3, ny=4, ntheta=8, ns=8, limiter=limiter, k_on=0.9, k_off=0.6, v0=1.2, F=0.8)
        psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0)
        M0 = gen.make_M0_random(p.nx, p.ny, p.ntheta, p.ns, seed=5)
        m0 = M0.sum(-1) * (p.L / p.ns)
        Bv = A.coarse_bound(p, psi0, m0)
        p.m_total = float(0.5 * (Bv.min() + Bv.max()))
        assert (Bv > p.m_total).any() and (Bv < p.m_total).any()
        fl = gen.fluid_schedule(p.nx, p.ny, 1)
        dt = gen.cfl_dt(p, fl)
        o = A.OracleA(p)
        o.set_state(psi0, M0)
        o.set_fluid(*fl[0])
        o.step(12, dt)
        psi_a, M_a = o.get_state()
        s_a, mom_a = o.get_stress_moments()
        psi_b, M_b, s_b, mom_b = B.forward(p, psi0, M0, fl, 12, 12, dt)
        for x, y in [(psi_a, psi_b), (M_a, M_b), (s_a, s_b), (mom_a, mom_b)]:
            assert rel_err(x, y.numpy()) <= 1e-13
