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


def sample_points(nx, ny):
    """Grid points whose columns span the motor field: the first, the last, both sides of the
    middle row boundary (byte offsets around 2^30 in FP64 at 256^2 x 64 x 64 and 2^32 in FP32 at
    512^2 x 128 x 64) and one point inside the upper half."""
    return [(0, 0), (nx // 2 - 1, ny - 1), (nx // 2, 0), (nx // 2 + nx // 12, 17 % ny), (nx - 1, ny - 1)]


@pytest.mark.parametrize("name,precision,tol", [
    ("fp32_512x512x128x64", 1, 1e-5),
    ("fp32_256x256x64x64", 1, 1e-5),
    ("fp32_256x256x64x64", 0, 1e-12),
])
def test_full_size_columns_differ(name, precision, tol):
    """Full grid, every motor column different (a closed-form pattern with period 97 in the
    column index, so a read from another column, or through an offset wrapped at 2^32 bytes,
    gives other values), 12 micro-steps in two calls (one blocked launch of 10, one of 2) with
    their own fluid fields, in the launch configuration the benchmark times.  Sampled points
    (first, last, around the middle, above 2^32 bytes at 512^2 x 128 x 64) are compared with the
    FP64 oracle run on a 25 x 25 window around each: psi, every M column, m0, m1 of the point,
    its stress and moments."""
    import torch
    from paper_1908_04279_amd import mmk
    from tests.runners import run_oracle_window
    p = gen.params_for(name)
    dtype = torch.float32 if precision else torch.float64
    np_dt = np.float32 if precision else np.float64
    calls = [10, 2]
    fl = gen.fluid_schedule(p.nx, p.ny, len(calls), p.lx, p.ly)
    dt = gen.cfl_dt(p, fl)
    psi0 = gen.make_psi0(p.nx, p.ny, p.ntheta, p.lx, p.ly, seed=0).astype(np_dt)
    print(f"{name} {'FP32' if precision else 'FP64'}: gpu {sum(calls)} steps", flush=True)
    ctx = mmk.Context(p, precision=precision)
    M0 = gen.make_M0_columns_device(p.nx, p.ny, p.ntheta, p.ns, dtype, ctx.device, p.k_on, p.k_off)
    ctx.set_state(torch.as_tensor(psi0), M0)
    torch.cuda.synchronize()
    del M0
    for e, k in enumerate(calls):
        ctx.set_fluid(*map(torch.as_tensor, fl[e]))
        ctx.step(k, dt)
    psi, M = ctx.get_state()
    m0, m1 = ctx.get_motor_moments()
    stress, mom = ctx.get_stress(), ctx.get_moments()
    got = {f: [] for f in ("psi", "M", "m0", "m1", "stress", "mom")}
    for i, j in sample_points(p.nx, p.ny):
        got["psi"].append(psi[i, j].double().cpu().numpy())
        got["M"].append(M[i, j].double().cpu().numpy())
        got["m0"].append(m0[i, j].double().cpu().numpy())
        got["m1"].append(m1[i, j].double().cpu().numpy())
        got["stress"].append(stress[:, i, j].double().cpu().numpy())
        got["mom"].append(mom[:, i, j].double().cpu().numpy())
    del psi, M, m0, m1
    ctx.close()
    print("oracle windows", flush=True)
    # the oracle takes the inputs as the GPU holds them (rounded to its precision)
    M0_of = lambda c: gen.M0_columns_values(c, p.ns, p.k_on, p.k_off).astype(np_dt)
    ref = {f: [] for f in got}
    for i, j in sample_points(p.nx, p.ny):
        w = run_oracle_window(p, psi0, M0_of, fl, calls, dt, i, j, R=sum(calls))
        for f in ref:
            ref[f].append(w[f])
    errs = {f: rel_err(np.stack(got[f]), np.stack(ref[f])) for f in got}
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)
