"""Pins of the oracle's motor-column step (walk + attach/detach, superbee MUSCL, midpoint RK2)
against values fixed by mathematics rather than by the oracle itself."""
import math
import os

import numpy as np
import pytest

from oracle import oracle_a as A
from paper_1908_04279_amd.inputs import ModelParams

GOLD = os.path.join(os.path.dirname(__file__), "golden", "superbee_values.txt")


def col_params(ns, **kw):
    p = ModelParams(nx=1, ny=1, ntheta=1, ns=ns)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_superbee_textbook_table():
    rows = np.loadtxt(GOLD)
    for a, b, want in rows:
        assert A.superbee(a, b) == want, (a, b)


def test_superbee_matches_ratio_form_and_is_odd():
    rng = np.random.default_rng(11)
    for _ in range(2000):
        a, b = rng.standard_normal(2) * 10.0 ** rng.uniform(-3, 3, 2)
        got = A.superbee(a, b)
        r = a / b
        phi = max(0.0, min(2 * r, 1.0), min(r, 2.0))
        assert got == pytest.approx(phi * b, rel=1e-14, abs=0.0)
        assert A.superbee(-a, -b) == -got
        # TVD region: slope lies between 0 and 2*min-type bounds
        assert abs(got) <= 2 * max(abs(a), abs(b)) + 0.0


def discrete_upwind_steady(p):
    """Exact steady state of the first-order upwind column scheme: from
    0 = -v0 (M_l - M_{l-1})/ds + k_on - k_off M_l with M_{-1} = 0 one gets
    M_l - c = rho (M_{l-1} - c), c = k_on/k_off, rho = v0 / (v0 + k_off ds)."""
    ds = p.L / p.ns
    c = p.k_on / p.k_off
    rho = p.v0 / (p.v0 + p.k_off * ds)
    l = np.arange(p.ns)
    return c * (1.0 - rho ** (l + 1))


@pytest.mark.parametrize("ns", [1, 2, 7, 16, 64])
def test_upwind_exact_discrete_steady_state(ns):
    p = col_params(ns, limiter=1, k_on=1.3, k_off=0.7, v0=0.9)
    Mss = discrete_upwind_steady(p)
    # it is a zero of the right-hand side ...
    R = A.motor_rhs(p, Mss)
    assert np.abs(R).max() <= 1e-13 * (p.v0 * ns / p.L) * Mss.max()
    # ... and the midpoint map converges to it from M = 0
    ds = p.L / ns
    dt = 0.4 / (p.v0 / ds + p.k_off)
    M = np.zeros(ns)
    for _ in range(int(60.0 / dt)):
        M = A.column_step(p, dt, M)
    assert np.abs(M - Mss).max() <= 1e-14 * Mss.max() * 10


def continuum_cell_averages(p):
    """Cell averages of the continuum steady profile M(s) = c (1 - exp(-k_off s / v0))."""
    ds = p.L / p.ns
    c, lam = p.k_on / p.k_off, p.k_off / p.v0
    lo = np.arange(p.ns) * ds
    return c * (1.0 - np.exp(-lam * lo) * (1.0 - np.exp(-lam * ds)) / (lam * ds))


def run_to_steady(p, t_end=40.0):
    ds = p.L / p.ns
    dt = 0.4 / (p.v0 / ds + p.k_off)
    M = np.zeros(p.ns)
    for _ in range(int(t_end / dt)):
        M = A.column_step(p, dt, M)
    return M


def test_superbee_converges_to_continuum_steady_state():
    """Interior: second order (mean error / 4 per refinement).  The plus-end cell uses the
    first-order outflow flux, so the max error (found there) is first order."""
    emax, emean = [], []
    sizes = [16, 32, 64, 128, 256]
    for ns in sizes:
        p = col_params(ns)
        e = np.abs(run_to_steady(p) - continuum_cell_averages(p))
        emax.append(e.max())
        emean.append(e.mean())
    omax = [math.log2(emax[i] / emax[i + 1]) for i in range(len(sizes) - 1)]
    omean = [math.log2(emean[i] / emean[i + 1]) for i in range(len(sizes) - 1)]
    assert min(omax) >= 0.95, (emax, omax)
    assert min(omean) >= 1.8, (emean, omean)
    assert emean[-1] < 1e-5 and emax[-1] < 1.3e-3
    # steady m0 against c [L - (v0/k_off)(1 - exp(-k_off L / v0))]
    p = col_params(256)
    m0, _ = A.column_moments(p, run_to_steady(p))
    c = p.k_on / p.k_off
    m0_ss = c * (p.L - (p.v0 / p.k_off) * (1.0 - math.exp(-p.k_off * p.L / p.v0)))
    assert abs(m0 - m0_ss) < 2e-3 * m0_ss
    assert m0_ss == pytest.approx(0.42612, abs=1e-5)


@pytest.mark.parametrize("limiter", [0, 1])
def test_budget_identity_each_step(limiter):
    """Summing R over the column telescopes: m0(M') - m0(M) = dt [k_on L - k_off m0(M*)
    - v0 M*_{ns-1}], with M* the midpoint stage."""
    rng = np.random.default_rng(3)
    for ns in [3, 16, 33]:
        p = col_params(ns, limiter=limiter, k_on=0.8, k_off=1.7, v0=1.3)
        ds = p.L / ns
        dt = 0.4 / (p.v0 / ds + p.k_off)
        M = rng.uniform(0, 2, ns)
        Ms = M + 0.5 * dt * A.motor_rhs(p, M)
        M1 = A.column_step(p, dt, M)
        m0a, _ = A.column_moments(p, M)
        m0b, _ = A.column_moments(p, M1)
        m0s, _ = A.column_moments(p, Ms)
        want = dt * (p.k_on * p.L - p.k_off * m0s - p.v0 * Ms[-1])
        assert (m0b - m0a) == pytest.approx(want, rel=1e-12, abs=1e-15)


def test_no_walking_is_the_midpoint_rule_closed_form():
    """v0 = 0 decouples cells: M_n = c + (M_0 - c) g^n, g = 1 - h + h^2/2, h = k_off dt
    (explicit midpoint applied to dM/dt = k_on - k_off M)."""
    rng = np.random.default_rng(4)
    p = col_params(9, v0=0.0, k_on=0.6, k_off=1.1)
    dt = 0.05
    M0 = rng.uniform(0, 3, 9)
    M = M0.copy()
    n = 37
    for _ in range(n):
        M = A.column_step(p, dt, M)
    h = p.k_off * dt
    g = 1 - h + 0.5 * h * h
    c = p.k_on / p.k_off
    assert np.abs(M - (c + (M0 - c) * g ** n)).max() <= 1e-14 * 10


def test_linear_upwind_step_is_second_order_taylor_polynomial():
    """With the first-order flux the column step is M' = (I + dt A + dt^2 A^2 / 2) M + (dt + dt^2 A/2) k_on 1
    for the bidiagonal upwind matrix A (independently assembled here)."""
    rng = np.random.default_rng(5)
    ns = 11
    p = col_params(ns, limiter=1, k_on=0.3, k_off=0.9, v0=1.4)
    ds = p.L / ns
    dt = 0.3 / (p.v0 / ds + p.k_off)
    Amat = np.zeros((ns, ns))
    for l in range(ns):
        Amat[l, l] = -p.v0 / ds - p.k_off
        if l > 0:
            Amat[l, l - 1] = p.v0 / ds
    b = np.full(ns, p.k_on)
    M = rng.uniform(0, 2, ns)
    I = np.eye(ns)
    want = (I + dt * Amat + 0.5 * dt * dt * Amat @ Amat) @ M + (dt * I + 0.5 * dt * dt * Amat) @ b
    assert np.abs(A.column_step(p, dt, M) - want).max() <= 1e-14 * 20


def test_degenerate_no_motors_stays_zero():
    p = col_params(16, k_on=0.0, k_off=0.0)
    M = np.zeros(16)
    for _ in range(50):
        M = A.column_step(p, 0.02, M)
    assert np.all(M == 0.0)


def test_superbee_on_linear_data_is_unlimited_slope():
    """On a strictly increasing linear profile the superbee slope equals the difference
    (phi(1) = 1), so interior MUSCL fluxes are v0 (M_l + d/2): the face-centred value."""
    p = col_params(8, k_on=0.0, k_off=0.0, v0=1.0)
    ds = p.L / 8
    M = 1.0 + 0.25 * np.arange(8)
    R = A.motor_rhs(p, M)
    # interior cells l = 2..6: flux difference is v0 * 0.25 -> R = -v0 * 0.25 / ds
    assert np.allclose(R[2:7], -0.25 / ds, rtol=1e-14, atol=0)
    # first cell: Phi_{-1/2} = 0 and sigma_0 = superbee(M_0 - 0, 0.25) = 0.25 * phi(4) = 0.5
    assert R[0] == pytest.approx(-(1.0 + 0.25) / ds, rel=1e-14)
