"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every symbol
the header declares, sizes workspaces and rejects bad arguments before any HIP call."""
import ctypes as C
import os
import re

import pytest

from paper_1908_04279_amd import mmk
from paper_1908_04279_amd.inputs import ModelParams

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mmk.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mmk_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = mmk.lib()
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(mmk.EXPORTS)


def params(**kw):
    p = ModelParams(nx=16, ny=12, ntheta=8, ns=32)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_workspace_bytes_scales_with_fields_and_tape():
    f64 = mmk.workspace_bytes(mmk.make_params(params(), mmk.FP64))
    f32 = mmk.workspace_bytes(mmk.make_params(params(), mmk.FP32))
    nm = 16 * 12 * 8 * 32
    assert f64 >= 2 * nm * 8 and f32 >= 2 * nm * 4
    assert f32 < f64
    tape = mmk.workspace_bytes(mmk.make_params(params(), mmk.FP64), 10, 100)
    # 11 checkpoints + 10 segment slots + 2 adjoint fields of M at least
    assert tape - f64 >= (11 + 10 + 2) * nm * 8


@pytest.mark.parametrize("bad", [dict(nx=0), dict(ny=-1), dict(ntheta=0), dict(ns=0),
                                 dict(lx=0.0), dict(L=-1.0), dict(v0=-0.5), dict(k_on=float("nan")),
                                 dict(limiter=7), dict(m_total=-1.0), dict(m_total=float("inf")),
                                 dict(motor_cfl=-0.5), dict(motor_cfl=float("nan")), dict(rc=-0.1),
                                 dict(rc=float("nan")), dict(rc=2.7)])
def test_invalid_params_are_rejected(bad):
    n = mmk.lib().mmk_workspace_bytes(C.byref(mmk.make_params(params(**bad))), 0, 0)
    assert n == 0
    assert mmk.lib().mmk_last_error(None)
    h = C.c_void_p()
    st = mmk.lib().mmk_create(C.byref(mmk.make_params(params(**bad))), C.c_void_p(256), 1 << 30,
                              None, 0, 0, C.byref(h))
    assert st == mmk.MMK_ERR_ARG and not h.value


def test_unsupported_sizes_and_workspace_checks():
    h = C.c_void_p()
    L = mmk.lib()
    st = L.mmk_create(C.byref(mmk.make_params(params(ntheta=1024))), C.c_void_p(256), 1 << 40, None, 0, 0,
                      C.byref(h))
    assert st == mmk.MMK_ERR_UNSUPPORTED
    assert b"ntheta" in L.mmk_last_error(None)
    p = mmk.make_params(params())
    need = mmk.workspace_bytes(p)
    assert L.mmk_create(C.byref(p), None, need, None, 0, 0, C.byref(h)) == mmk.MMK_ERR_ARG
    assert L.mmk_create(C.byref(p), C.c_void_p(256 + 8), need, None, 0, 0, C.byref(h)) == mmk.MMK_ERR_ARG
    assert L.mmk_create(C.byref(p), C.c_void_p(256), need - 1, None, 0, 0, C.byref(h)) == mmk.MMK_ERR_NOMEM
    assert b"needs" in L.mmk_last_error(None)
    assert L.mmk_create(C.byref(p), C.c_void_p(256), need, None, -1, 0, C.byref(h)) == mmk.MMK_ERR_ARG
    assert L.mmk_create(C.byref(p), C.c_void_p(256), need, None, 0, 0, None) == mmk.MMK_ERR_ARG


def test_null_context_is_an_argument_error():
    L = mmk.lib()
    assert L.mmk_step(None, 1, 0.1) == mmk.MMK_ERR_ARG
    assert L.mmk_destroy(None) == mmk.MMK_ERR_ARG
    assert L.mmk_set_state(None, None, None) == mmk.MMK_ERR_ARG
    assert L.mmk_get_sums(None, None, None) == mmk.MMK_ERR_ARG
    assert L.mmk_tape_backward(None, None, None, None, None) == mmk.MMK_ERR_ARG


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(mmk, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(mmk, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        mmk.lib()


@pytest.mark.parametrize("kw", [dict(nx=12, ny=12, ntheta=8, ns=8, rc=0.45),
                                dict(nx=9, ny=14, ntheta=6, ns=5, rc=0.8, lx=5.0, ly=7.0),
                                dict(nx=128, ny=128, ntheta=32, ns=32, rc=0.1),
                                dict(nx=8, ny=8, ntheta=8, ns=4, rc=0.01)])
def test_r0_cells_match_the_oracle(kw):
    """The library's tracked-cell table (host code) equals the oracle's, entry for entry."""
    import numpy as np
    from oracle import oracle_a as A
    p = ModelParams(**kw)
    assert np.array_equal(mmk.r0_cells(p), A.r0_cells(p))


def test_r0_cells_refusals_and_workspace():
    assert mmk.lib().mmk_r0_cells(C.byref(mmk.make_params(params())), None) == -1          # rc = 0
    assert mmk.lib().mmk_r0_cells(C.byref(mmk.make_params(params(rc=3.0))), None) == -1    # too large
    p = params(nx=32, ny=32, ntheta=16, ns=16, rc=0.3)
    n = mmk.lib().mmk_r0_cells(C.byref(mmk.make_params(p)), None)
    ws = mmk.workspace_bytes(mmk.make_params(p, mmk.FP64))
    assert ws >= 2 * n * 32 * 32 * 8
    for bad, msg in [(dict(ns=64, rc=0.5), "longer than 32")]:
        q = params(**bad)
        assert mmk.lib().mmk_workspace_bytes(C.byref(mmk.make_params(q)), 0, 0) == 0
        assert msg in mmk.lib().mmk_last_error(None).decode()
