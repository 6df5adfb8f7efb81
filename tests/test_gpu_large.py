"""Largest single-GPU case: 512^2 x 128 x 64 in FP32 (2^31 motor cells, byte offsets past
2^33), in the launch configuration the benchmark uses."""
import numpy as np
import pytest

from oracle import oracle_a as A
from paper_1908_04279_amd import inputs as gen
from tests.conftest import rel_err
from tests.runners import run_oracle_uniform_columns

pytestmark = pytest.mark.gpu


def run(p, psi0, fl, K, n, dt):
    import torch
    from paper_1908_04279_amd import mmk
    ctx = mmk.Context(p, precision=mmk.FP32)
    ctx.set_state(torch.as_tensor(psi0))
    done, e = 0, 0
    while done < n:
        ctx.set_fluid(*map(torch.as_tensor, fl[e]))
        k = min(K, n - done)
        ctx.step(k, dt)
        done += k
        e += 1
    return ctx


def test_fp32_512x512x128x64_largest_case():
    import torch
    p = gen.params_for("fp32_512x512x128x64")
    assert p.nx * p.ny * p.ntheta * p.ns == 2 ** 31
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, seed=0)
    fl = gen.fluid_schedule(p.nx, p.ny, 20)
    dt = gen.cfl_dt(p, fl)
    # 10 steps: every field against the FP64 oracle (column decomposition)
    print("gpu 10 steps", flush=True)
    ctx = run(p, psi0, fl, 10, 10, dt)
    psi, M = ctx.get_state()
    stress = ctx.get_stress().double().cpu().numpy()
    mom = ctx.get_moments().double().cpu().numpy()
    print("oracle 10 steps", flush=True)
    o = run_oracle_uniform_columns(p, psi0, fl, 10, 10, dt)
    col = torch.as_tensor(o["col"], dtype=torch.float32, device=M.device)
    m_err = float((M - col).abs().max() / col.abs().max())
    # the last cells of the field (offsets beyond 2^33 bytes) are checked explicitly
    tail = M.view(-1)[-p.ns:].double().cpu().numpy()
    errs = dict(psi=rel_err(psi.double().cpu().numpy(), o["psi"]), M=m_err,
                M_tail=rel_err(tail, o["col"]), stress=rel_err(stress, o["stress"]),
                mom=rel_err(mom, o["mom"]))
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    del psi, M
    ctx.close()
    for k, v in errs.items():
        assert v <= 1e-5, k
    # 200 steps with a new fluid every 10: conservation, positivity, columns
    print("gpu 200 steps", flush=True)
    ctx = run(p, psi0, fl, 10, 200, dt)
    mass, _ = ctx.get_sums()
    psi, M = ctx.get_state()
    assert abs(mass - 1.0) <= 1e-5, mass
    assert float(psi.min()) >= 0.0
    # every column against the oracle column after 200 steps
    c200 = np.zeros(p.ns)
    for _ in range(200):
        c200 = A.column_step(p, dt, c200)
    col = torch.as_tensor(c200, dtype=torch.float32, device=M.device)
    m_err = float((M - col).abs().max() / col.abs().max())
    print(f"mass {mass!r}, min psi {float(psi.min()):.3e}, M vs oracle column {m_err:.2e}", flush=True)
    assert m_err <= 1e-5
    ctx.close()
