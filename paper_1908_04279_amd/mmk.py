"""ctypes binding of libmmk.so (the HIP micro-step library): argument marshalling only.

Every operation of the method runs in the library's HIP kernels; this module turns torch
tensors into device pointers and status codes into exceptions.  If libmmk.so is missing it
raises instead of falling back to anything else.

Names follow include/mmk.h: `Context.step(K, dt)` calls `mmk_step`, and so on.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmmk.so")

MMK_OK, MMK_ERR_ARG, MMK_ERR_NOMEM, MMK_ERR_HIP, MMK_ERR_STATE, MMK_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
FP64, FP32 = 0, 1
SUPERBEE, UPWIND1 = 0, 1
# implementation options (mmk_set_option): name -> id
OPTIONS = {"motor_block": 0, "psi_kernel": 1, "depl_fused": 2, "motor_lanes": 3, "motor_chunks": 4,
           "motor_nt": 5, "psi_depth": 6, "r0_onepass": 7}
KERNEL_IDS = {"motor_step": 0, "psi_step": 1, "global_sums": 2, "psi_step_reverse": 3,
              "motor_step_reverse": 4, "motor_force": 5, "r0_motor_step": 6, "r0_coarse": 7,
              "r0_anchor_step": 8, "r0_marginals": 9}

EXPORTS = ["mmk_workspace_bytes", "mmk_create", "mmk_destroy", "mmk_set_params", "mmk_set_state",
           "mmk_set_fluid", "mmk_step", "mmk_get_state", "mmk_get_stress", "mmk_get_moments",
           "mmk_get_motor_moments", "mmk_get_force", "mmk_get_anchors", "mmk_r0_cells", "mmk_get_sums", "mmk_tape_begin", "mmk_tape_backward",
           "mmk_tape_end", "mmk_profile", "mmk_profile_read", "mmk_profile_every", "mmk_set_option",
           "mmk_step_graph", "mmk_sums_static",
           "mmk_last_error"]


class MMKError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mmk status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("ntheta", C.c_int32), ("ns", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("L", C.c_double),
                ("k_on", C.c_double), ("k_off", C.c_double), ("v0", C.c_double),
                ("F", C.c_double), ("sigma_f", C.c_double),
                ("precision", C.c_int32), ("limiter", C.c_int32), ("m_total", C.c_double),
                ("motor_cfl", C.c_double), ("rc", C.c_double)]


_lib = None


def lib():
    """Loads libmmk.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1908_04279_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        P = C.POINTER(Params)
        sig = {
            "mmk_workspace_bytes": ([P, i32, i32], C.c_size_t),
            "mmk_create": ([P, vp, C.c_size_t, vp, i32, i32, C.POINTER(vp)], C.c_int),
            "mmk_destroy": ([vp], C.c_int),
            "mmk_set_params": ([vp, d, d, d], C.c_int),
            "mmk_set_state": ([vp, vp, vp], C.c_int),
            "mmk_set_fluid": ([vp, vp, vp], C.c_int),
            "mmk_step": ([vp, i32, d], C.c_int),
            "mmk_step_graph": ([vp, i32, d], C.c_int),
            "mmk_get_state": ([vp, vp, vp], C.c_int),
            "mmk_get_stress": ([vp, vp], C.c_int),
            "mmk_get_moments": ([vp, vp], C.c_int),
            "mmk_get_motor_moments": ([vp, vp, vp], C.c_int),
            "mmk_get_force": ([vp, vp], C.c_int),
            "mmk_get_anchors": ([vp, vp, vp], C.c_int),
            "mmk_r0_cells": ([P, vp], i64),
            "mmk_get_sums": ([vp, C.POINTER(d), C.POINTER(d)], C.c_int),
            "mmk_tape_begin": ([vp, i32], C.c_int),
            "mmk_tape_backward": ([vp, vp, vp, vp, C.POINTER(d)], C.c_int),
            "mmk_tape_end": ([vp], C.c_int),
            "mmk_profile": ([vp, i32], C.c_int),
            "mmk_profile_read": ([vp, i32, C.POINTER(d), C.POINTER(i64)], C.c_int),
            "mmk_profile_every": ([vp, i32, i32], C.c_int),
            "mmk_set_option": ([vp, i32, i32], C.c_int),
            "mmk_sums_static": ([P, vp, vp, vp, C.POINTER(d), C.POINTER(d)], C.c_int),
            "mmk_last_error": ([vp], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def make_params(p, precision=FP64) -> Params:
    """From any object with the ModelParams attribute names."""
    return Params(int(p.nx), int(p.ny), int(p.ntheta), int(p.ns), float(p.lx), float(p.ly),
                  float(p.L), float(p.k_on), float(p.k_off), float(p.v0), float(p.F),
                  float(p.sigma_f), int(precision), int(getattr(p, "limiter", 0)),
                  float(getattr(p, "m_total", 0.0)), float(getattr(p, "motor_cfl", 0.0)),
                  float(getattr(p, "rc", 0.0)))


def workspace_bytes(params: Params, ckpt_every=0, max_tape_steps=0) -> int:
    n = lib().mmk_workspace_bytes(C.byref(params), int(ckpt_every), int(max_tape_steps))
    if n == 0:
        raise MMKError(MMK_ERR_ARG, lib().mmk_last_error(None).decode())
    return n


def r0_cells(p):
    """Tracked cells of the anchor-resolved model (p.rc > 0): int32 array [ncell][4] = (a, b, k, l)."""
    import numpy as np
    params = make_params(p)
    n = lib().mmk_r0_cells(C.byref(params), None)
    if n < 0:
        raise MMKError(MMK_ERR_ARG, "rc must be > 0 with rc + L/2 below lx/2 and ly/2")
    cells = np.zeros((n, 4), dtype=np.int32)
    if n > 0:
        lib().mmk_r0_cells(C.byref(params), C.c_void_p(cells.ctypes.data))
    return cells


def sums_static(p, precision, psi, sigma, stream=None):
    """mmk_sums_static: (mass, sum_sigma[3]) of device tensors psi [nx][ny][ntheta] and sigma
    [3][nx][ny] without a context (the library's static scratch; nothing is allocated)."""
    params = make_params(p, precision)
    mass = C.c_double()
    ss = (C.c_double * 3)()
    s = stream if stream is not None else torch.cuda.current_stream(psi.device)
    st = lib().mmk_sums_static(C.byref(params), _ptr(psi), _ptr(sigma), C.c_void_p(s.cuda_stream),
                               C.byref(mass), ss)
    if st != MMK_OK:
        raise MMKError(st, lib().mmk_last_error(None).decode())
    return mass.value, [ss[0], ss[1], ss[2]]


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


class Context:
    """One micro-step problem resident on the current GPU.

    The workspace is a torch uint8 tensor owned by this object; fields are typed torch
    tensors (float64 for FP64, float32 for FP32) on the same device.
    """

    def __init__(self, p, precision=FP64, ckpt_every=0, max_tape_steps=0, device=None,
                 stream=None, options=None):
        self.p = p
        self.params = make_params(p, precision)
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        self.device = torch.device(device if device is not None else "cuda")
        self.ws_bytes = workspace_bytes(self.params, ckpt_every, max_tape_steps)
        # torch's caching allocator returns >= 512-byte aligned blocks
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = lib().mmk_create(C.byref(self.params), _ptr(self.workspace), self.ws_bytes,
                              C.c_void_p(self.stream.cuda_stream), int(ckpt_every),
                              int(max_tape_steps), C.byref(h))
        if st != MMK_OK:
            raise MMKError(st, lib().mmk_last_error(None).decode())
        self.h = h
        nx, ny, nt, ns = p.nx, p.ny, p.ntheta, p.ns
        self.shape_psi = (nx, ny, nt)
        if getattr(p, "rc", 0.0) > 0:   # anchor-resolved: Mb [ncell][nx][ny]
            self.ncell = int(lib().mmk_r0_cells(C.byref(self.params), None))
            self.shape_M = (self.ncell, nx, ny)
        else:
            self.shape_M = (nx, ny, nt, ns)
        for name, value in (options or {}).items():
            self.set_option(name, value)

    # -- helpers ------------------------------------------------------------------------
    def _check(self, st):
        if st != MMK_OK:
            raise MMKError(st, lib().mmk_last_error(self.h).decode())

    def _dev(self, a, shape):
        t = torch.as_tensor(a)
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
        return t.to(device=self.device, dtype=self.dtype).contiguous()

    def empty(self, shape):
        return torch.empty(shape, dtype=self.dtype, device=self.device)

    def close(self):
        if getattr(self, "h", None):
            lib().mmk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C-ABI calls ------------------------------------------------------------------------
    def set_params(self, k_on, k_off, v0):
        self._check(lib().mmk_set_params(self.h, float(k_on), float(k_off), float(v0)))

    def set_option(self, name, value):
        """mmk_set_option by name (OPTIONS): an implementation choice of the same micro-step."""
        self._check(lib().mmk_set_option(self.h, OPTIONS[name], int(value)))

    def set_state(self, psi, M=None):
        psi_t = self._dev(psi, self.shape_psi)
        M_t = None if M is None else self._dev(M, self.shape_M)
        self._check(lib().mmk_set_state(self.h, _ptr(psi_t), _ptr(M_t)))
        self._keep = (psi_t, M_t)   # the copy is stream-ordered; keep sources alive

    def set_fluid(self, u, gradu):
        u_t = self._dev(u, (2, self.p.nx, self.p.ny))
        g_t = self._dev(gradu, (4, self.p.nx, self.p.ny))
        self._check(lib().mmk_set_fluid(self.h, _ptr(u_t), _ptr(g_t)))
        self._keep_fluid = (u_t, g_t)

    def step(self, K, dt):
        self._check(lib().mmk_step(self.h, int(K), float(dt)))

    def step_graph(self, K, dt):
        """mmk_step_graph: the K micro-steps of step(K, dt) as one replayed HIP graph."""
        self._check(lib().mmk_step_graph(self.h, int(K), float(dt)))

    def get_state(self):
        psi, M = self.empty(self.shape_psi), self.empty(self.shape_M)
        self._check(lib().mmk_get_state(self.h, _ptr(psi), _ptr(M)))
        return psi, M

    def get_psi(self):
        psi = self.empty(self.shape_psi)
        self._check(lib().mmk_get_state(self.h, _ptr(psi), None))
        return psi

    def get_stress(self):
        s = self.empty((3, self.p.nx, self.p.ny))
        self._check(lib().mmk_get_stress(self.h, _ptr(s)))
        return s

    def get_moments(self):
        m = self.empty((7, self.p.nx, self.p.ny))
        self._check(lib().mmk_get_moments(self.h, _ptr(m)))
        return m

    def get_motor_moments(self):
        m0, m1 = self.empty(self.shape_psi), self.empty(self.shape_psi)
        self._check(lib().mmk_get_motor_moments(self.h, _ptr(m0), _ptr(m1)))
        return m0, m1

    def get_force(self):
        """Motor force density F2 [2][nx][ny] = (f_x, f_y) of the current state (Eq. (10)):
        F p psi M ds dth of every bound-motor cell spread from its head, (x_i, y_j) +
        (s_l - L/2) p, onto the four surrounding cell centres (bilinear hat, periodic).  With
        rc > 0, M is the anchor marginal of M_b (the r0 integral of Eq. (10))."""
        f = self.empty((2, self.p.nx, self.p.ny))
        self._check(lib().mmk_get_force(self.h, _ptr(f)))
        return f

    def get_anchors(self):
        """Anchor-resolved model: (coarse, free) [nx][ny], the coarse bound-motor density of Eq. (5)
        at every anchor of the current state and its free pool of Eq. (6) before the next clamp."""
        co, fr = self.empty((self.p.nx, self.p.ny)), self.empty((self.p.nx, self.p.ny))
        self._check(lib().mmk_get_anchors(self.h, _ptr(co), _ptr(fr)))
        return co, fr

    def get_sums(self):
        mass = C.c_double()
        ss = (C.c_double * 3)()
        self._check(lib().mmk_get_sums(self.h, C.byref(mass), ss))
        return mass.value, [ss[0], ss[1], ss[2]]

    def tape_begin(self, ckpt_every):
        self._check(lib().mmk_tape_begin(self.h, int(ckpt_every)))

    def tape_backward(self, g_sigma=None, g_moments=None):
        gs = None if g_sigma is None else self._dev(g_sigma, (3, self.p.nx, self.p.ny))
        gm = None if g_moments is None else self._dev(g_moments, (7, self.p.nx, self.p.ny))
        g_psi0 = self.empty(self.shape_psi)
        gp = (C.c_double * 3)()
        self._check(lib().mmk_tape_backward(self.h, _ptr(gs), _ptr(gm), _ptr(g_psi0), gp))
        return g_psi0, [gp[0], gp[1], gp[2]]

    def tape_end(self):
        self._check(lib().mmk_tape_end(self.h))

    def profile(self, enable=True, every=1):
        """Time every `every`-th launch of each kernel with HIP events (enable=False: off)."""
        self._check(lib().mmk_profile(self.h, int(every) if enable else 0))

    def profile_every(self, kernel, every):
        """After profile(): time every `every`-th launch of one kernel (0: none)."""
        kid = KERNEL_IDS[kernel] if isinstance(kernel, str) else int(kernel)
        self._check(lib().mmk_profile_every(self.h, kid, int(every)))

    def profile_read(self, kernel):
        kid = KERNEL_IDS[kernel] if isinstance(kernel, str) else int(kernel)
        ms = C.c_double()
        n = C.c_int64()
        self._check(lib().mmk_profile_read(self.h, kid, C.byref(ms), C.byref(n)))
        return ms.value, n.value
