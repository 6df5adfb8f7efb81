"""Host-side accounting of bench.py (CPU): algorithmic bytes and flops of the launches, the
launch plan of a K-step call, the counter-summary lookup, and the one-GPU guard."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1908_04279_amd import inputs as gen  # noqa: E402


def c3():
    return gen.params_for("fp32_256x256x64x64")


def test_motor_bytes_of_the_benchmark_launches():
    p = c3()
    n_psi, n_m = 256 * 256 * 64, 256 * 256 * 64 * 64
    # one launch per micro-step: read M, write M and m0 (+ m1 on output launches)
    assert bench.motor_bytes(p, 4, False) == 4 * (2 * n_m + n_psi) == 2164260864
    assert bench.motor_bytes(p, 4, True) == 4 * (2 * n_m + 2 * n_psi)
    # blocked over the 10 micro-steps of a call: m0 of every micro-step and m1 of the last
    assert bench.motor_bytes(p, 4, True, 10) == 4 * (2 * n_m + 11 * n_psi) == 2332033024
    assert bench.motor_bytes(p, 8, False) == 2 * bench.motor_bytes(p, 4, False)


def test_psi_bytes_of_the_benchmark_launches():
    p = c3()
    n_psi, nxy = 256 * 256 * 64, 256 * 256
    assert bench.psi_bytes(p, 4, False) == 4 * (3 * n_psi + 6 * nxy) == 51904512
    assert bench.psi_bytes(p, 4, True) == 4 * (4 * n_psi + 16 * nxy) == 71303168


def test_anchor_resolved_bytes():
    p = gen.ModelParams(nx=128, ny=128, ntheta=32, ns=32, rc=0.1)
    nxy, ncell, nrun = 128 * 128, 13216, 3056
    # one launch per micro-step with one anchor per block: read and write M_b, read psi, write the
    # run-total pairs; the marginals read the pairs and write m0, m1
    assert bench.r0_anchor_bytes(p, 4, ncell, nrun) == 4 * (2 * ncell * nxy + nxy * 32 + 2 * nrun * nxy) == 2134900736
    assert bench.r0_marg_bytes(p, 4, nrun) == 4 * (2 * nrun * nxy + 2 * nxy * 32) == 404750336
    # the plain anchor-resolved motor launch: M_b both ways, run totals, marginals, clamp and pool
    assert bench.r0_motor_bytes(p, 4, ncell, nrun, True) == 1936850944
    cells = np.array([[0, 0, 0, 0], [0, 0, 0, 1], [0, 0, 0, 3], [0, 0, 1, 4], [1, 0, 1, 5]])
    assert bench.r0_runs(cells) == 4   # a gap in l, a new k, a new a


def test_motor_flops_scale_with_cells_and_steps():
    p = c3()
    one = bench.motor_flops(p, False, 1)
    assert one > 0
    assert bench.motor_flops(p, False, 10) == pytest.approx(10 * one)
    assert bench.motor_flops(p, True, 10) > bench.motor_flops(p, False, 10)


def test_block_plan():
    p = c3()
    assert bench.block_plan(p, 10) == [10]
    assert bench.block_plan(p, 25) == [16, 9]
    assert bench.block_plan(p, 10, {"motor_block": 0}) == [1] * 10
    assert bench.block_plan(gen.params_for("fp32_256x256x64x64", m_total=0.02), 3) == [1, 1, 1]


def test_counter_summary_lookup(tmp_path):
    files = ["motor.hip", "device_util.h", "kernels.h"]
    path = tmp_path / "summary.txt"
    body = ("# a comment line = not a key\n"
            f"sources_sha256_16={bench.sources_sha(files)}\nmicro_steps_per_launch=10\n"
            "hbm_bytes_per_launch=2.0e9\nhbm_bytes_per_output_launch=3.0e9\n")
    path.write_text(body)
    assert bench.counters_traffic(1, 1, 10, (str(path), files)) == pytest.approx(2.5e9)
    assert bench.counters_traffic(0, 2, 10, (str(path), files)) == pytest.approx(3.0e9)
    # other launches, other sources, no file: no traffic figure
    assert bench.counters_traffic(0, 2, 1, (str(path), files)) is None
    path.write_text(body.replace(bench.sources_sha(files), "0" * 16))
    assert bench.counters_traffic(0, 2, 10, (str(path), files)) is None
    assert bench.counters_traffic(0, 2, 10, (str(tmp_path / "missing.txt"), files)) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
