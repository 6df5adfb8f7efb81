"""Pins of the oracle's filament-density step (donor-cell transport in x, y, theta) and of
its theta-moments, against conservation laws, textbook closed forms and symmetries."""
import math

import numpy as np
import pytest
from scipy.special import comb

from oracle import oracle_a as A
from paper_1908_04279_amd import inputs as gen
from paper_1908_04279_amd.inputs import ModelParams

TWO_PI = 2 * math.pi


def rand_case(nx, ny, nth, seed, F=1.0):
    rng = np.random.default_rng(seed)
    p = ModelParams(nx=nx, ny=ny, ntheta=nth, ns=4, F=F)
    psi = rng.uniform(0.0, 1.0, (nx, ny, nth))
    m0 = rng.uniform(0.0, p.L * p.k_on / p.k_off, (nx, ny, nth))
    u, g = gen.make_fluid(nx, ny, seed=seed + 1)
    dt = gen.cfl_dt(p, [(u, g)])
    return p, psi, m0, u, g, dt


@pytest.mark.parametrize("shape", [(16, 16, 16), (7, 5, 12), (1, 3, 5), (2, 1, 1)])
def test_mass_is_conserved(shape):
    p, psi, m0, u, g, dt = rand_case(*shape, seed=7)
    mass0, _ = A.global_sums(p, psi, np.zeros((3, p.nx, p.ny)))
    for _ in range(50):
        psi = A.psi_step(p, dt, psi, m0, u, g)
    mass1, _ = A.global_sums(p, psi, np.zeros((3, p.nx, p.ny)))
    assert abs(mass1 - mass0) <= 1e-13 * mass0


def test_positivity_at_cfl_04():
    """Each donor-cell update coefficient is >= 1 - 2 * 0.4 > 0, so psi >= 0 stays >= 0,
    even from rough data with exact zeros."""
    p, psi, m0, u, g, dt = rand_case(12, 10, 16, seed=8)
    rng = np.random.default_rng(9)
    psi = np.where(rng.uniform(size=psi.shape) < 0.3, 0.0, psi)
    for _ in range(100):
        psi = A.psi_step(p, dt, psi, m0, u, g)
        assert psi.min() >= 0.0


def test_uniform_isotropic_state_is_bitwise_steady():
    p = ModelParams(nx=6, ny=5, ntheta=8, ns=16)
    psi = np.full((6, 5, 8), 0.37)
    M = np.full((6, 5, 8, 16), 0.81)
    u = np.zeros((2, 6, 5))
    g = np.zeros((4, 6, 5))
    o = A.OracleA(p)
    o.set_state(psi, M)
    o.set_fluid(u, g)
    o.step(40, 0.01)
    assert np.array_equal(o.psi, psi)
    stress, mom = o.get_stress_moments()
    c = mom[0]
    assert np.allclose(mom[3], 0.5 * c, rtol=1e-15, atol=0)        # D = c I / 2
    assert np.allclose(mom[5], 0.5 * c, rtol=1e-15, atol=0)
    assert np.abs(mom[4]).max() <= 1e-16 * c.max()
    assert np.abs(mom[1:3]).max() <= 1e-16 * c.max()                # no polar order


def binomial_shift(f0, nu, n, axis):
    """n donor-cell steps at constant Courant number nu >= 0 along a periodic axis:
    f_n[i] = sum_r C(n,r) nu^r (1-nu)^(n-r) f_0[i-r] (textbook upwind Green's function)."""
    out = np.zeros_like(f0)
    for r in range(n + 1):
        out += comb(n, r) * nu ** r * (1 - nu) ** (n - r) * np.roll(f0, r, axis=axis)
    return out


def test_donor_cell_binomial_in_x_and_y():
    rng = np.random.default_rng(10)
    p = ModelParams(nx=9, ny=7, ntheta=4, ns=4, F=0.0)
    psi0 = rng.uniform(0, 1, (9, 7, 4))
    m0 = rng.uniform(0, 1, psi0.shape)   # F = 0: motors exert no force
    dx = p.lx / p.nx
    dy = p.ly / p.ny
    for comp, axis, h, vel in [(0, 0, dx, 0.7), (1, 1, dy, -0.45)]:
        u = np.zeros((2, 9, 7))
        u[comp] = vel
        g = np.zeros((4, 9, 7))
        dt = 0.3 * h / abs(vel)
        psi = psi0.copy()
        n = 13
        for _ in range(n):
            psi = A.psi_step(p, dt, psi, m0, u, g)
        nu = abs(vel) * dt / h
        f0 = psi0 if vel > 0 else np.flip(psi0, axis=axis)
        want = binomial_shift(f0, nu, n, axis)
        if vel < 0:
            want = np.flip(want, axis=axis)
        assert np.abs(psi - want).max() <= 1e-14 * psi0.max()


def test_donor_cell_binomial_in_theta_under_solid_rotation():
    """u = Omega (-y, x): G_xy = -Omega, G_yx = Omega gives p_perp . G . p = Omega at every angle."""
    rng = np.random.default_rng(12)
    p = ModelParams(nx=3, ny=4, ntheta=16, ns=4, F=0.0)
    psi0 = rng.uniform(0, 1, (3, 4, 16))
    m0 = np.zeros_like(psi0)
    omega = 0.8
    u = np.zeros((2, 3, 4))
    g = np.zeros((4, 3, 4))
    g[1] = -omega
    g[2] = omega
    dth = TWO_PI / 16
    dt = 0.35 * dth / omega
    psi = psi0.copy()
    n = 11
    for _ in range(n):
        psi = A.psi_step(p, dt, psi, m0, u, g)
    want = binomial_shift(psi0, omega * dt / dth, n, axis=2)
    assert np.abs(psi - want).max() <= 1e-14 * psi0.max()


def test_shift_equivariance_is_bitwise():
    p, psi, m0, u, g, dt = rand_case(6, 5, 8, seed=13)
    out = A.psi_step(p, dt, psi, m0, u, g)
    for ax in (0, 1):
        sh = lambda a, lead=0: np.roll(a, 1, axis=ax + lead)
        out_s = A.psi_step(p, dt, sh(psi), sh(m0), sh(u, 1), sh(g, 1))
        assert np.array_equal(out_s, sh(out))


def rot_field(f):
    """Rotate a scalar field [nx][ny](...) by +90 degrees about the box centre."""
    return np.rot90(f, k=1, axes=(0, 1))


def test_rotation_by_quarter_turn():
    n, nth = 8, 16
    p, psi, m0, u, g, dt = rand_case(n, n, nth, seed=14)
    out = A.psi_step(p, dt, psi, m0, u, g)
    q = nth // 4
    rpsi = np.roll(rot_field(psi), q, axis=2)
    rm0 = np.roll(rot_field(m0), q, axis=2)
    ru = np.stack([-rot_field(u[1]), rot_field(u[0])])
    # G -> R G R^T with R the quarter turn: (Gyy, -Gyx, -Gxy, Gxx)
    rg = np.stack([rot_field(g[3]), -rot_field(g[2]), -rot_field(g[1]), rot_field(g[0])])
    out_r = A.psi_step(p, dt, rpsi, rm0, ru, rg)
    want = np.roll(rot_field(out), q, axis=2)
    assert np.abs(out_r - want).max() <= 1e-14 * psi.max()
    # moments transform as scalar / vector / tensor
    m1 = np.random.default_rng(15).uniform(-0.1, 0.1, m0.shape)
    s, mo = A.moments(p, out, m0, m1)
    s_r, mo_r = A.moments(p, out_r, rm0, np.roll(rot_field(m1), q, axis=2))
    tol = 1e-13
    assert np.allclose(mo_r[0], rot_field(mo[0]), rtol=tol, atol=tol * mo[0].max())
    assert np.allclose(mo_r[1], -rot_field(mo[2]), rtol=tol, atol=tol * mo[0].max())
    assert np.allclose(mo_r[2], rot_field(mo[1]), rtol=tol, atol=tol * mo[0].max())
    assert np.allclose(mo_r[3], rot_field(mo[5]), rtol=tol, atol=tol * mo[0].max())
    assert np.allclose(mo_r[4], -rot_field(mo[4]), rtol=tol, atol=tol * mo[0].max())
    a = np.abs(s).max()
    assert np.allclose(s_r[0], rot_field(s[2]), rtol=tol, atol=tol * a)
    assert np.allclose(s_r[1], -rot_field(s[1]), rtol=tol, atol=tol * a)
    assert np.allclose(s_r[2], rot_field(s[0]), rtol=tol, atol=tol * a)


def test_moments_of_aligned_and_isotropic_densities():
    nth = 32
    p = ModelParams(nx=2, ny=3, ntheta=nth, ns=4, F=1.7, sigma_f=0.9)
    dth = TWO_PI / nth
    # all filaments along theta = 0
    psi = np.zeros((2, 3, nth))
    psi[..., 0] = 2.0 / dth
    m0 = np.full(psi.shape, 0.3)
    m1 = np.zeros(psi.shape)
    s, mo = A.moments(p, psi, m0, m1)
    c = 2.0
    assert np.allclose(mo[0], c, rtol=1e-15)
    assert np.allclose(mo[1], c, rtol=1e-15) and np.abs(mo[2]).max() < 1e-15
    assert np.allclose(mo[3], c, rtol=1e-15) and np.abs(mo[5]).max() < 1e-15
    assert np.allclose(mo[6], 0.3 * c, rtol=1e-15)
    assert np.allclose(s[0], 0.5 * p.sigma_f * c, rtol=1e-15)
    assert np.allclose(s[2], -0.5 * p.sigma_f * c, rtol=1e-15)
    assert np.abs(s[1]).max() < 1e-15
    # isotropic: filament stress vanishes, motor dipole stress is F m1 psi pi I
    psi = np.full((2, 3, nth), 0.25)
    m1 = np.full(psi.shape, 0.07)
    s, mo = A.moments(p, psi, m0, m1)
    want = p.F * 0.07 * 0.25 * math.pi
    assert np.allclose(s[0], want, rtol=1e-14) and np.allclose(s[2], want, rtol=1e-14)
    assert np.abs(s[1]).max() < 1e-16
    assert np.allclose(mo[0], 0.25 * TWO_PI, rtol=1e-15)


def test_motor_gliding_moves_filaments_against_their_orientation():
    """With no fluid, a filament with m0 bound motors glides at speed F m0 along -p
    (motors walk towards the plus end and push the filament the other way): density in
    the theta = 0 bin is a donor-cell shift towards -x, theta = pi/2 towards -y, and
    theta = pi towards +x, each with the binomial closed form."""
    nth = 8
    p = ModelParams(nx=11, ny=11, ntheta=nth, ns=4, F=1.3)
    rng = np.random.default_rng(16)
    f0 = rng.uniform(0, 1, (11, 11))
    psi0 = np.zeros((11, 11, nth))
    for k in (0, 2, 4):
        psi0[:, :, k] = f0
    m = 0.4
    m0 = np.full(psi0.shape, m)
    u = np.zeros((2, 11, 11))
    g = np.zeros((4, 11, 11))
    dx = p.lx / p.nx
    dt = 0.3 * dx / (p.F * m)
    psi = psi0.copy()
    n = 9
    for _ in range(n):
        psi = A.psi_step(p, dt, psi, m0, u, g)
    nu = p.F * m * dt / dx
    minus_x = np.flip(binomial_shift(np.flip(f0, 0), nu, n, 0), 0)
    minus_y = np.flip(binomial_shift(np.flip(f0, 1), nu, n, 1), 1)
    plus_x = binomial_shift(f0, nu, n, 0)
    # cos(pi/2) and sin(pi) are ~1e-16, not 0: allow that leak
    assert np.abs(psi[:, :, 0] - minus_x).max() <= 1e-13
    assert np.abs(psi[:, :, 2] - minus_y).max() <= 1e-13
    assert np.abs(psi[:, :, 4] - plus_x).max() <= 1e-13


def test_global_sums_closed_forms():
    """mass = sum psi dx dy dth and sum_sigma = sum sigma dx dy (the FP64 global sums of the
    extra-stress step), pinned on states whose integrals are known in closed form.  The box is
    not square and dx != dy, so a dx/dy swap, a missing dth or a missing dx dy fails.
      * uniform psi = a: mass = a 2 pi lx ly;
      * all filaments along th = 0 with c = int psi dth: sum sigma_xx = sigma_f c lx ly / 2,
        sum sigma_yy = -sigma_f c lx ly / 2, sum sigma_xy = 0, mass = c lx ly;
      * isotropic psi = a with lever moment m1: the motor dipole stress integrates to
        F m1 a pi lx ly on the diagonal, the filament part to 0;
      * one occupied cell: mass = psi dx dy dth exactly."""
    nth = 16
    lx, ly = 2.0, 3.5
    p = ModelParams(nx=4, ny=5, ntheta=nth, ns=4, lx=lx, ly=ly, F=1.3, sigma_f=0.8)
    dth = TWO_PI / nth
    zero_stress = np.zeros((3, p.nx, p.ny))
    a = 0.37
    mass, _ = A.global_sums(p, np.full((p.nx, p.ny, nth), a), zero_stress)
    assert mass == pytest.approx(a * TWO_PI * lx * ly, rel=1e-14)

    c = 1.9
    psi = np.zeros((p.nx, p.ny, nth))
    psi[..., 0] = c / dth
    s, _ = A.moments(p, psi, np.full(psi.shape, 0.3), np.zeros(psi.shape))
    mass, ss = A.global_sums(p, psi, s)
    assert mass == pytest.approx(c * lx * ly, rel=1e-14)
    assert ss[0] == pytest.approx(0.5 * p.sigma_f * c * lx * ly, rel=1e-14)
    assert ss[2] == pytest.approx(-0.5 * p.sigma_f * c * lx * ly, rel=1e-14)
    assert abs(ss[1]) < 1e-14

    m1 = 0.07
    psi = np.full((p.nx, p.ny, nth), a)
    s, _ = A.moments(p, psi, np.full(psi.shape, 0.3), np.full(psi.shape, m1))
    mass, ss = A.global_sums(p, psi, s)
    want = p.F * m1 * a * math.pi * lx * ly
    assert ss[0] == pytest.approx(want, rel=1e-13) and ss[2] == pytest.approx(want, rel=1e-13)
    assert abs(ss[1]) < 1e-14

    psi = np.zeros((p.nx, p.ny, nth))
    psi[3, 4, 7] = 2.5
    mass, _ = A.global_sums(p, psi, zero_stress)
    assert mass == pytest.approx(2.5 * (lx / p.nx) * (ly / p.ny) * dth, rel=1e-15)
