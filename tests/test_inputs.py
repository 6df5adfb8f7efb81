"""The seeded generators produce what their docstrings promise."""
import math

import numpy as np

from paper_1908_04279_amd import inputs as gen


def test_psi0_unit_mass_positive_and_seeded():
    a = gen.make_psi0(16, 12, 8, seed=0)
    b = gen.make_psi0(16, 12, 8, seed=0)
    assert np.array_equal(a, b)
    vol = (2 * math.pi / 16) * (2 * math.pi / 12) * (2 * math.pi / 8)
    assert abs(a.sum() * vol - 1.0) < 1e-14
    assert a.min() > 0
    assert not np.array_equal(a, gen.make_psi0(16, 12, 8, seed=1))


def test_fluid_is_divergence_free_with_exact_gradient():
    n = 64
    u, g = gen.make_fluid(n, n, seed=1)
    # du_x/dx + du_y/dy = 0 analytically
    assert np.abs(g[0] + g[3]).max() < 1e-15
    # spectral derivative of the sampled velocity reproduces the analytic gradient
    k = np.fft.fftfreq(n, d=2 * math.pi / n) * 2 * math.pi
    dxf = lambda f: np.real(np.fft.ifft(1j * k[:, None] * np.fft.fft(f, axis=0), axis=0))
    dyf = lambda f: np.real(np.fft.ifft(1j * k[None, :] * np.fft.fft(f, axis=1), axis=1))
    assert np.abs(dxf(u[0]) - g[0]).max() < 1e-12
    assert np.abs(dyf(u[0]) - g[1]).max() < 1e-12
    assert np.abs(dxf(u[1]) - g[2]).max() < 1e-12
    assert np.abs(dyf(u[1]) - g[3]).max() < 1e-12
    # three modes of speed 0.1 each
    assert np.hypot(u[0], u[1]).max() <= 0.3 + 1e-12


def test_single_mode_speed_is_the_amplitude():
    u, _ = gen.make_fluid(128, 128, seed=4, n_modes=1, amp=0.1)
    assert abs(np.hypot(u[0], u[1]).max() - 0.1) < 1e-3


def test_cfl_dt_matches_the_stated_limits():
    p = gen.params_for("fp64_16x16x16x16")
    fl = [gen.make_fluid(16, 16, seed=1)]
    dt = gen.cfl_dt(p, fl)
    ds = p.L / p.ns
    assert dt <= 0.4 / (p.v0 / ds + p.k_off) + 1e-18
    assert abs(dt - 0.4 / 16.5) < 1e-15      # motor walk limit binds for this workload


def test_other_generators():
    m = gen.make_M0_random(2, 3, 4, 5, seed=5)
    assert m.shape == (2, 3, 4, 5) and m.min() >= 0 and m.max() <= 2.0
    t = gen.make_target_stress(4, 5)
    assert t.shape == (3, 4, 5) and np.abs(t).max() < 1e-2
    d = gen.make_direction((3, 4, 5), seed=100)
    assert abs(np.abs(d).max() - 1.0) < 1e-15
