"""Pins of the oracle's motor force density (Eq. (10), bilinear-hat spreading of the motor
heads at (x, y) + (s - L/2) p, periodic)."""
import math

import numpy as np
import pytest

from oracle import oracle_a as A
from oracle import oracle_torch as B
from paper_1908_04279_amd import inputs as gen
from paper_1908_04279_amd.inputs import ModelParams
from tests.conftest import rel_err


def hat(r):
    return np.maximum(0.0, 1.0 - np.abs(r))


def min_image(d, box):
    return d - box * np.round(d / box)


def test_single_motor_lands_on_the_hat_weights():
    """One filament point, one orientation, one occupied arclength cell: the force is
    F p psi M ds dth times the hat of the (periodic) distance to every cell centre."""
    p = ModelParams(nx=9, ny=7, ntheta=12, ns=10, lx=2.0, ly=1.5, L=1.7, F=1.3)
    rng = np.random.default_rng(1)
    for _ in range(20):
        i, j, k, l = (int(rng.integers(n)) for n in (p.nx, p.ny, p.ntheta, p.ns))
        psi = np.zeros((p.nx, p.ny, p.ntheta))
        M = np.zeros((p.nx, p.ny, p.ntheta, p.ns))
        psi[i, j, k] = 0.8
        M[i, j, k, l] = 1.9
        dx, dy, dth, ds = p.lx / p.nx, p.ly / p.ny, 2 * math.pi / p.ntheta, p.L / p.ns
        th = k * dth
        lever = (l + 0.5) * ds - p.L / 2
        hx, hy = (i + 0.5) * dx + lever * math.cos(th), (j + 0.5) * dy + lever * math.sin(th)
        xc = (np.arange(p.nx) + 0.5) * dx
        yc = (np.arange(p.ny) + 0.5) * dy
        w = hat(min_image(xc - hx, p.lx) / dx)[:, None] * hat(min_image(yc - hy, p.ly) / dy)[None, :]
        v = p.F * 0.8 * 1.9 * ds * dth
        want = np.stack([v * math.cos(th) * w, v * math.sin(th) * w])
        got = A.motor_force(p, psi, M)
        assert np.max(np.abs(got - want)) <= 4e-15 * abs(v)  # a few ulps: two ways to form the weights


def test_total_force_is_conserved():
    """The hat weights sum to one: sum F2 dx dy = F sum p psi m0 dth dx dy."""
    p = ModelParams(nx=11, ny=8, ntheta=16, ns=12, lx=3.0, ly=2.0, L=1.3, F=0.7)
    psi = gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=2)
    M = gen.make_M0_random(p.nx, p.ny, p.ntheta, p.ns, seed=7)
    f = A.motor_force(p, psi, M)
    dx, dy, dth, ds = p.lx / p.nx, p.ly / p.ny, 2 * math.pi / p.ntheta, p.L / p.ns
    th = np.arange(p.ntheta) * dth
    m0 = M.sum(-1) * ds
    want = p.F * np.array([(psi * m0 * np.cos(th)).sum(), (psi * m0 * np.sin(th)).sum()]) * dth * dx * dy
    got = f.sum(axis=(1, 2)) * dx * dy
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-16)


def test_first_moment_is_the_head_position():
    """Away from the periodic wrap the hat reproduces linear functions: sum x F2 dx dy equals the
    sum over motor cells of F p psi M ds dth dx dy times the head's x (and likewise in y)."""
    p = ModelParams(nx=24, ny=20, ntheta=8, ns=6, lx=4.0, ly=4.0, L=0.9, F=1.1)
    rng = np.random.default_rng(4)
    psi = np.zeros((p.nx, p.ny, p.ntheta))
    psi[9:15, 8:12] = rng.uniform(0.1, 1.0, (6, 4, p.ntheta))
    M = rng.uniform(0, 2, (p.nx, p.ny, p.ntheta, p.ns))
    f = A.motor_force(p, psi, M)
    dx, dy, dth, ds = p.lx / p.nx, p.ly / p.ny, 2 * math.pi / p.ntheta, p.L / p.ns
    xc = (np.arange(p.nx) + 0.5) * dx
    yc = (np.arange(p.ny) + 0.5) * dy
    th = np.arange(p.ntheta) * dth
    lever = (np.arange(p.ns) + 0.5) * ds - p.L / 2
    hx = xc[:, None, None, None] + lever * np.cos(th)[None, None, :, None]
    hy = yc[None, :, None, None] + lever * np.sin(th)[None, None, :, None]
    v = p.F * psi[..., None] * M * ds * dth
    for comp, pc in ((0, np.cos(th)), (1, np.sin(th))):
        vv = v * pc[None, None, :, None]
        np.testing.assert_allclose((f[comp] * xc[:, None]).sum() * dx * dy, (vv * hx).sum() * dx * dy, rtol=1e-13)
        np.testing.assert_allclose((f[comp] * yc[None, :]).sum() * dx * dy, (vv * hy).sum() * dx * dy, rtol=1e-13)


def test_isotropic_state_has_no_force():
    """Uniform psi and M over x, y and th: every orientation lands the same amount on every
    cell, and the orientations cancel."""
    p = ModelParams(nx=10, ny=10, ntheta=24, ns=8)
    f = A.motor_force(p, np.full((10, 10, 24), 0.3), np.full((10, 10, 24, 8), 1.7))
    assert np.max(np.abs(f)) <= 1e-15


def test_shift_equivariance():
    p = ModelParams(nx=7, ny=6, ntheta=8, ns=5)
    psi = gen.make_psi0(7, 6, 8, seed=3)
    M = gen.make_M0_random(7, 6, 8, 5, seed=9)
    f = A.motor_force(p, psi, M)
    g = A.motor_force(p, np.roll(psi, (2, -1), (0, 1)), np.roll(M, (2, -1), (0, 1)))
    np.testing.assert_allclose(g, np.roll(f, (2, -1), (1, 2)), rtol=0, atol=1e-15 * np.abs(f).max())


def test_c_and_torch_oracles_agree():
    for shape in [(5, 4, 8, 6), (13, 9, 16, 16)]:
        nx, ny, nt, ns = shape
        p = ModelParams(nx=nx, ny=ny, ntheta=nt, ns=ns, L=1.4, F=0.9)
        psi = gen.make_psi0(nx, ny, nt, seed=0)
        M = gen.make_M0_random(nx, ny, nt, ns, seed=5)
        a = A.motor_force(p, psi, M)
        b = B.motor_force(B.to_t(psi), B.to_t(M), p.F, p.L, p.lx, p.ly).numpy()
        assert rel_err(a, b) <= 1e-13
