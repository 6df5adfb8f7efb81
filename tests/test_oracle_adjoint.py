"""The reference adjoint (autograd through the PyTorch oracle) against central finite
differences of the C oracle's forward, which is itself pinned elsewhere."""
import numpy as np
import pytest

from oracle import oracle_a as A
from oracle import oracle_torch as B
from paper_1908_04279_amd import inputs as gen
from paper_1908_04279_amd.inputs import ModelParams


def stress_after(p, psi0, M0, fluids, K, n, dt):
    o = A.OracleA(p)
    o.set_state(psi0, M0)
    done, e = 0, 0
    while done < n:
        o.set_fluid(*fluids[min(e, len(fluids) - 1)])
        k = min(K, n - done)
        o.step(k, dt)
        done += k
        e += 1
    return o.get_stress_moments()


def l2_loss(stress, target):
    d = stress - target
    return float(np.sqrt((d[0] ** 2 + 2 * d[1] ** 2 + d[2] ** 2).sum()))


def torch_l2(target):
    import torch
    t = torch.as_tensor(target, dtype=torch.float64)

    def f(stress, mom):
        d = stress - t
        return torch.sqrt((d[0] ** 2 + 2 * d[1] ** 2 + d[2] ** 2).sum())
    return f


@pytest.mark.parametrize("M0_kind", ["zero", "random"])
def test_autograd_gradients_match_central_differences(M0_kind):
    p = ModelParams(nx=6, ny=5, ntheta=8, ns=8)
    psi0 = gen.make_psi0(6, 5, 8, seed=0)
    M0 = (np.zeros((6, 5, 8, 8)) if M0_kind == "zero"
          else gen.make_M0_random(6, 5, 8, 8, seed=5))
    fl = [gen.make_fluid(6, 5, seed=1 + e) for e in range(3)]
    dt = gen.cfl_dt(p, fl)
    n, K = 30, 10
    target = gen.make_target_stress(6, 5)
    loss, gpsi, gpar = B.gradients(p, psi0, M0, fl, K, n, dt, loss_fn=torch_l2(target))
    s, _ = stress_after(p, psi0, M0, fl, K, n, dt)
    assert loss == pytest.approx(l2_loss(s, target), rel=1e-13)
    h = 1e-6
    for i, name in enumerate(["k_on", "k_off", "v0"]):
        vals = []
        for sgn in (+1, -1):
            q = ModelParams(**p.as_dict())
            setattr(q, name, getattr(p, name) + sgn * h)
            vals.append(l2_loss(stress_after(q, psi0, M0, fl, K, n, dt)[0], target))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert gpar[i] == pytest.approx(fd, rel=2e-6, abs=1e-10), name
    for seed in (100, 101, 102):
        d = gen.make_direction(psi0.shape, seed)
        lp = l2_loss(stress_after(p, psi0 + h * d, M0, fl, K, n, dt)[0], target)
        lm = l2_loss(stress_after(p, psi0 - h * d, M0, fl, K, n, dt)[0], target)
        fd = (lp - lm) / (2 * h)
        assert float((gpsi * d).sum()) == pytest.approx(fd, rel=2e-6, abs=1e-10)


def test_checkpointed_reverse_pass_is_identical():
    p = ModelParams(nx=4, ny=3, ntheta=8, ns=8)
    psi0 = gen.make_psi0(4, 3, 8, seed=0)
    M0 = gen.make_M0_random(4, 3, 8, 8, seed=5)
    fl = [gen.make_fluid(4, 3, seed=1)]
    dt = gen.cfl_dt(p, fl)
    rng = np.random.default_rng(2)
    gs, gm = rng.standard_normal((3, 4, 3)), rng.standard_normal((7, 4, 3))
    a = B.gradients(p, psi0, M0, fl, 25, 25, dt, gs, gm)
    b = B.gradients(p, psi0, M0, fl, 25, 25, dt, gs, gm, ckpt=7)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1]) and a[2] == b[2]


@pytest.mark.parametrize("M0_kind,m_total", [("zero", 0.05), ("random", None)])
def test_depleted_gradients_are_finite_and_match_central_differences(M0_kind, m_total):
    """The depleted model (Eqs. (5)-(6), the clamp of Alg. 2) differentiated by autograd.
    From M0 = 0 the coarse density starts at B = 0, where a clamp factor m_total / B in the
    discarded branch would make the gradient NaN; from a random M0 with m_total between the
    smallest and the largest B both branches are taken.  The gradients must be finite and
    equal central differences of the C oracle."""
    p = ModelParams(nx=5, ny=4, ntheta=8, ns=8)
    psi0 = gen.make_psi0(5, 4, 8, seed=0)
    if M0_kind == "zero":
        M0 = np.zeros((5, 4, 8, 8))
    else:
        M0 = gen.make_M0_random(5, 4, 8, 8, seed=5)
        m0, _ = A.column_moments(p, M0)
        Bv = A.coarse_bound(p, psi0, m0)
        m_total = float(0.5 * (Bv.min() + Bv.max()))
    p.m_total = m_total
    fl = [gen.make_fluid(5, 4, seed=1 + e) for e in range(2)]
    dt = gen.cfl_dt(p, fl)
    n, K = 20, 10
    target = gen.make_target_stress(5, 4)
    loss, gpsi, gpar = B.gradients(p, psi0, M0, fl, K, n, dt, loss_fn=torch_l2(target))
    assert np.isfinite(gpsi).all() and np.isfinite(gpar).all()
    s, _ = stress_after(p, psi0, M0, fl, K, n, dt)
    assert loss == pytest.approx(l2_loss(s, target), rel=1e-13)
    h = 1e-6
    for i, name in enumerate(["k_on", "k_off", "v0"]):
        vals = []
        for sgn in (+1, -1):
            q = ModelParams(**p.as_dict())
            setattr(q, name, getattr(p, name) + sgn * h)
            vals.append(l2_loss(stress_after(q, psi0, M0, fl, K, n, dt)[0], target))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert gpar[i] == pytest.approx(fd, rel=2e-6, abs=1e-10), name
    for seed in (100, 101):
        d = gen.make_direction(psi0.shape, seed)
        lp = l2_loss(stress_after(p, psi0 + h * d, M0, fl, K, n, dt)[0], target)
        lm = l2_loss(stress_after(p, psi0 - h * d, M0, fl, K, n, dt)[0], target)
        fd = (lp - lm) / (2 * h)
        assert float((gpsi * d).sum()) == pytest.approx(fd, rel=2e-6, abs=1e-10)
