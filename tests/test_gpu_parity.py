"""FP64 HIP path against the FP64 oracle, element by element, through the C-ABI.

Tolerance: 1e-12 norm-wise relative error (max |gpu - oracle| / max |oracle|) per field.
"""
import numpy as np
import pytest

from paper_1908_04279_amd import inputs as gen
from paper_1908_04279_amd.inputs import ModelParams
from tests.conftest import rel_err
from tests.runners import run_gpu, run_oracle, run_oracle_uniform_columns, seeded_case

pytestmark = pytest.mark.gpu
TOL = 1e-12
FIELDS = ["psi", "M", "m0", "m1", "stress", "mom"]


def compare(g, o, fields=FIELDS, tol=TOL):
    errs = {f: rel_err(g[f], o[f]) for f in fields}
    errs["mass"] = abs(g["mass"] - o["mass"]) / abs(o["mass"])
    errs["sum_sigma"] = rel_err(g["sum_sigma"], o["sum_sigma"])
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)


def test_fp64_16x16x16x16_all_fields():
    p = gen.params_for("fp64_16x16x16x16")
    psi0, M0, fl, dt = seeded_case(p)
    g = run_gpu(p, psi0, M0, fl, 100, 100, dt)
    o = run_oracle(p, psi0, np.zeros((16, 16, 16, 16)), fl, 100, 100, dt)
    compare(g, o)


@pytest.mark.parametrize("ns", [8, 16, 32, 64, 128, 256, 1, 2, 3, 5, 20, 33, 100, 300])
def test_random_M0_every_column_length(ns):
    """Exact tilings (8 .. 256) and the masked generic kernel (any other length), with
    columns that differ, an odd grid and three fluid exchanges."""
    p = ModelParams(nx=5, ny=7, ntheta=12, ns=ns, k_on=0.9, k_off=0.6, v0=1.2, F=0.8)
    psi0, M0, fl, dt = seeded_case(p, n_exchanges=3, M0_kind="random")
    g = run_gpu(p, psi0, M0, fl, 4, 12, dt)
    o = run_oracle(p, psi0, M0, fl, 4, 12, dt)
    compare(g, o)


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 3, 2), (2, 1, 5), (3, 3, 64), (9, 17, 33), (1, 1, 128)])
@pytest.mark.parametrize("limiter", [0, 1])
def test_degenerate_and_ragged_grids(shape, limiter):
    nx, ny, nt = shape
    p = ModelParams(nx=nx, ny=ny, ntheta=nt, ns=16, limiter=limiter, lx=3.0, ly=5.0)
    psi0, M0, fl, dt = seeded_case(p, n_exchanges=2, M0_kind="random")
    g = run_gpu(p, psi0, M0, fl, 5, 9, dt)
    o = run_oracle(p, psi0, M0, fl, 5, 9, dt)
    compare(g, o)


def test_tile_tails_span_several_tiles():
    """Grid bigger than one psi tile in both directions with ragged tails, ns = 64."""
    p = ModelParams(nx=21, ny=19, ntheta=64, ns=64)
    psi0, M0, fl, dt = seeded_case(p, n_exchanges=2, M0_kind="random")
    g = run_gpu(p, psi0, M0, fl, 10, 20, dt)
    o = run_oracle(p, psi0, M0, fl, 10, 20, dt)
    compare(g, o)


def test_fp64_128x128x64x32_full_size_against_column_decomposition():
    """128^2 x 64 x 32, 1000 steps, a new fluid field every 10 steps, M0 = 0.  Every GPU
    column is checked against the oracle column; psi, stress and moments in full."""
    p = gen.params_for("fp64_128x128x64x32")
    psi0, _, fl, dt = seeded_case(p, n_exchanges=100)
    print("gpu run", flush=True)
    g = run_gpu(p, psi0, None, fl, 10, 1000, dt)
    print("oracle run", flush=True)
    o = run_oracle_uniform_columns(p, psi0, fl, 10, 1000, dt)
    o["M"] = np.broadcast_to(o["col"], g["M"].shape)
    compare(g, o)


def test_k_zero_is_a_no_op_and_state_round_trips():
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=4, ny=3, ntheta=8, ns=16)
    psi0, M0, fl, dt = seeded_case(p, M0_kind="random")
    ctx = mmk.Context(p)
    ctx.set_state(torch.as_tensor(psi0), torch.as_tensor(M0))
    ctx.set_fluid(*map(torch.as_tensor, fl[0]))
    ctx.step(0, dt)
    psi, M = ctx.get_state()
    assert np.array_equal(psi.cpu().numpy(), psi0) and np.array_equal(M.cpu().numpy(), M0)
    with pytest.raises(mmk.MMKError) as ei:
        ctx.get_stress()
    assert ei.value.status == mmk.MMK_ERR_STATE


def test_repeat_runs_are_bitwise_identical_and_resume_matches():
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=24, ny=20, ntheta=32, ns=32)
    psi0, M0, fl, dt = seeded_case(p, M0_kind="random")
    a = run_gpu(p, psi0, M0, fl, 30, 30, dt)
    b = run_gpu(p, psi0, M0, fl, 30, 30, dt)
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), f
    assert a["mass"] == b["mass"] and a["sum_sigma"] == b["sum_sigma"]
    # 15 steps, copy out, new context, 15 more steps == 30 steps
    c1 = run_gpu(p, psi0, M0, fl, 15, 15, dt, keep_ctx=True)
    psi, M = c1["ctx"].get_state()
    c1["ctx"].close()
    c2 = run_gpu(p, psi.cpu().numpy(), M.cpu().numpy(), fl, 15, 15, dt)
    for f in FIELDS:
        assert np.array_equal(c2[f], a[f]), f


def test_gpu_invariants():
    import torch
    from paper_1908_04279_amd import mmk
    # mass conservation and positivity over 200 steps of the 16x16x16x16 workload with random M0
    p = gen.params_for("fp64_16x16x16x16")
    psi0, M0, fl, dt = seeded_case(p, n_exchanges=4, M0_kind="random")
    g = run_gpu(p, psi0, M0, fl, 50, 200, dt)
    assert abs(g["mass"] - 1.0) <= 1e-13
    assert g["psi"].min() >= 0.0
    # uniform isotropic state with zero flow is bitwise steady
    q = ModelParams(nx=6, ny=5, ntheta=8, ns=16)
    psi = np.full((6, 5, 8), 0.37)
    M = np.full((6, 5, 8, 16), 0.81)
    zero = (np.zeros((2, 6, 5)), np.zeros((4, 6, 5)))
    h = run_gpu(q, psi, M, [zero], 40, 40, 0.01)
    assert np.array_equal(h["psi"], psi)
    assert np.allclose(h["mom"][3], 0.5 * h["mom"][0], rtol=1e-15, atol=0)


def test_error_codes():
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=4, ny=4, ntheta=8, ns=16)
    ctx = mmk.Context(p)
    with pytest.raises(mmk.MMKError) as ei:
        ctx.step(1, 0.01)
    assert ei.value.status == mmk.MMK_ERR_STATE
    psi0, M0, fl, dt = seeded_case(p)
    ctx.set_state(torch.as_tensor(psi0))
    with pytest.raises(mmk.MMKError) as ei:
        ctx.step(1, 0.01)
    assert ei.value.status == mmk.MMK_ERR_STATE and "set_fluid" in str(ei.value)
    ctx.set_fluid(*map(torch.as_tensor, fl[0]))
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(mmk.MMKError) as ei:
            ctx.step(1, bad)
        assert ei.value.status == mmk.MMK_ERR_ARG
    with pytest.raises(mmk.MMKError) as ei:
        ctx.step(-1, dt)
    assert ei.value.status == mmk.MMK_ERR_ARG
    with pytest.raises(mmk.MMKError) as ei:
        ctx.tape_begin(5)
    assert ei.value.status == mmk.MMK_ERR_STATE
    ctx.step(3, dt)
    assert np.isfinite(ctx.get_stress().cpu().numpy()).all()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("shape", [(20, 18, 64, 64), (13, 7, 128, 16), (9, 5, 64, 128), (1, 1, 64, 32),
                                   (17, 3, 128, 64)])
def test_walking_and_lds_psi_kernels_agree(precision, shape):
    """ntheta = 64, 128: the LDS-free walking psi kernel (8 x 4 pencil tiles, one wave per row)
    against the LDS-tiled one, over several calls and fluid exchanges, on grids that are not
    multiples of either tile; the FP64 result also against the oracle."""
    nx, ny, nt, ns = shape
    p = ModelParams(nx=nx, ny=ny, ntheta=nt, ns=ns)
    psi0, M0, fl, dt = seeded_case(p, n_exchanges=4, M0_kind="random")
    runs = {}
    for name, kernel in (("walk", 2), ("lds", 1)):
        runs[name] = run_gpu(p, psi0, M0, fl, 7, 25, dt, precision=precision, options={"psi_kernel": kernel})
    compare(runs["walk"], runs["lds"], tol=1e-12 if precision == 0 else 1e-5)
    if precision == 0:
        compare(runs["walk"], run_oracle(p, psi0, M0, fl, 7, 25, dt))


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("shape", [(16, 18, 64, 64), (8, 7, 64, 32), (24, 5, 128, 16), (40, 3, 128, 32),
                                   (20, 6, 64, 16)])
def test_walking_psi_ring_depths_agree(precision, shape):
    """The walking psi kernel with a ring of 4 and 8 register sets (x extent a multiple of the
    walk length 8; 20 is not, and runs the two-set form) against the two-set form, over several
    calls and fluid exchanges; FP64 also against the oracle; with depletion factors (DEPL) too."""
    nx, ny, nt, ns = shape
    for m_total in (0.0, 0.05):
        p = ModelParams(nx=nx, ny=ny, ntheta=nt, ns=ns, m_total=m_total)
        psi0, M0, fl, dt = seeded_case(p, n_exchanges=4, M0_kind="random")
        runs = {d: run_gpu(p, psi0, M0, fl, 7, 25, dt, precision=precision,
                           options={"psi_kernel": 2, "psi_depth": d}) for d in (2, 4, 8)}
        for d in (4, 8):
            compare(runs[d], runs[2], tol=1e-14 if precision == 0 else 1e-6)
        if precision == 0:
            compare(runs[8], run_oracle(p, psi0, M0, fl, 7, 25, dt))


@pytest.mark.parametrize("precision", [0, 1])
def test_sums_follow_the_outputs_they_belong_to(precision):
    """mmk_get_sums reduces the block partials of the last outputs when first asked: after the
    psi kernel is switched (other block rows) and after a second call, the sums still match a
    context that ran the same steps straight through, and asking twice gives the same bits."""
    import torch
    from paper_1908_04279_amd import mmk
    p = ModelParams(nx=24, ny=20, ntheta=64, ns=16)
    psi0, M0, fl, dt = seeded_case(p, n_exchanges=2, M0_kind="random")
    ref = run_gpu(p, psi0, M0, fl, 6, 12, dt, precision=precision)
    ctx = mmk.Context(p, precision=precision, options={"psi_kernel": 2})
    ctx.set_state(torch.as_tensor(psi0), torch.as_tensor(M0))
    ctx.set_fluid(*map(torch.as_tensor, fl[0]))
    ctx.step(6, dt)
    ctx.set_option("psi_kernel", 1)       # the sums pending are still those of the walking kernel
    first = ctx.get_sums()
    assert first == ctx.get_sums()
    ctx.set_fluid(*map(torch.as_tensor, fl[1]))
    ctx.step(6, dt)                       # LDS-tiled psi kernel: other partial rows
    mass, ss = ctx.get_sums()
    ctx.close()
    tol = 1e-12 if precision == 0 else 1e-5
    assert abs(mass - ref["mass"]) <= tol * abs(ref["mass"])
    assert np.max(np.abs(np.array(ss) - np.array(ref["sum_sigma"]))) <= tol * np.max(np.abs(ref["sum_sigma"]))
    assert first[0] == pytest.approx(ref["mass"], rel=1e-6)
