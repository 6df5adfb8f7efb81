"""ctypes front end of the C oracle (liboracle.so).  TEST INFRASTRUCTURE ONLY.

`OracleA` mirrors the call sequence of the HIP library (set_state, set_fluid, step(K, dt),
get_*) on host numpy float64 arrays so that the tests can drive both the same way.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
TWO_PI = 2.0 * np.pi


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nth", C.c_int), ("ns", C.c_int),
                ("lx", C.c_double), ("ly", C.c_double), ("L", C.c_double),
                ("k_on", C.c_double), ("k_off", C.c_double), ("v0", C.c_double),
                ("F", C.c_double), ("sigma_f", C.c_double), ("limiter", C.c_int),
                ("m_total", C.c_double), ("motor_cfl", C.c_double), ("rc", C.c_double)]


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build
            build.build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(_Params)
        L.oracle_superbee.argtypes = [C.c_double, C.c_double]
        L.oracle_superbee.restype = C.c_double
        L.oracle_motor_rhs.argtypes = [P, _dp, _dp]
        L.oracle_motor_rhs_src.argtypes = [P, _dp, C.c_double, _dp]
        L.oracle_column_step.argtypes = [P, C.c_double, _dp, _dp]
        L.oracle_column_step_src.argtypes = [P, C.c_double, _dp, C.c_double, _dp]
        L.oracle_coarse_bound.argtypes = [P, _dp, _dp, _dp]
        L.oracle_depletion.argtypes = [P, _dp, _dp, _dp]
        L.oracle_motor_force.argtypes = [P, _dp, _dp, _dp]
        L.oracle_column_moments.argtypes = [P, _dp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_motor_step.argtypes = [P, C.c_double, _dp, _dp, C.c_void_p, C.c_void_p]
        L.oracle_motor_substeps.argtypes = [P, C.c_double]
        L.oracle_motor_substeps.restype = C.c_int
        L.oracle_motor_substepped.argtypes = [P, C.c_double, _dp, _dp, C.c_void_p, C.c_void_p]
        L.oracle_psi_step.argtypes = [P, C.c_double, _dp, _dp, _dp, _dp, _dp]
        L.oracle_moments.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        L.oracle_global_sums.argtypes = [P, _dp, _dp, C.POINTER(C.c_double), _dp]
        L.oracle_run.argtypes = [P, C.c_double, C.c_int, _dp, _dp, _dp, _dp, C.c_void_p, C.c_void_p]
        _ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        L.oracle_run_step.argtypes = [P, C.c_int, C.c_double, _dp, C.c_double, _dp]
        L.oracle_r0_cells.argtypes = [P, C.c_void_p]
        L.oracle_r0_cells.restype = C.c_long
        L.oracle_r0_coarse.argtypes = [P, _ip, C.c_long, _dp, _dp, _dp]
        L.oracle_r0_motor_step.argtypes = [P, C.c_double, _ip, C.c_long, _dp, _dp, C.c_void_p, C.c_void_p]
        L.oracle_r0_marginal.argtypes = [P, _ip, C.c_long, _dp, C.c_void_p, C.c_void_p]
        L.oracle_r0_marginal_field.argtypes = [P, _ip, C.c_long, _dp, _dp]
        L.oracle_r0_run.argtypes = [P, C.c_double, C.c_int, _ip, C.c_long, _dp, _dp, _dp, _dp,
                                    C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_max_threads.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def cparams(p) -> _Params:
    """Accepts any object with the ModelParams attribute names."""
    return _Params(p.nx, p.ny, p.ntheta, p.ns, p.lx, p.ly, p.L, p.k_on, p.k_off, p.v0,
                   p.F, p.sigma_f, int(getattr(p, "limiter", 0)), float(getattr(p, "m_total", 0.0)),
                   float(getattr(p, "motor_cfl", 0.0)), float(getattr(p, "rc", 0.0)))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def superbee(a, b):
    return lib().oracle_superbee(float(a), float(b))


def motor_rhs(p, z):
    z = _f64(z)
    R = np.empty_like(z)
    lib().oracle_motor_rhs(C.byref(cparams(p)), z, R)
    return R


def column_step(p, dt, M):
    M = _f64(M)
    out = np.empty_like(M)
    lib().oracle_column_step(C.byref(cparams(p)), float(dt), M, out)
    return out


def motor_rhs_src(p, z, src):
    z = _f64(z)
    R = np.empty_like(z)
    lib().oracle_motor_rhs_src(C.byref(cparams(p)), z, float(src), R)
    return R


def column_step_src(p, dt, M, src):
    M = _f64(M)
    out = np.empty_like(M)
    lib().oracle_column_step_src(C.byref(cparams(p)), float(dt), M, float(src), out)
    return out


def coarse_bound(p, psi, m0):
    B = np.empty((p.nx, p.ny))
    lib().oracle_coarse_bound(C.byref(cparams(p)), _f64(psi), _f64(m0), B)
    return B


def depletion(p, B):
    """(scale, src) per (x, y): the over-binding clamp factor and k_on times the free pool."""
    B = _f64(B)
    scale = np.empty_like(B)
    src = np.empty_like(B)
    lib().oracle_depletion(C.byref(cparams(p)), B, scale, src)
    return scale, src


def motor_force(p, psi, M):
    """Motor force density [2][nx][ny] of (psi, M), Eq. (10) with the bilinear hat spreading."""
    f = np.empty((2, p.nx, p.ny))
    lib().oracle_motor_force(C.byref(cparams(p)), _f64(psi), _f64(M), f)
    return f


def column_moments(p, M):
    a, b = C.c_double(), C.c_double()
    lib().oracle_column_moments(C.byref(cparams(p)), _f64(M), C.byref(a), C.byref(b))
    return a.value, b.value


def motor_step(p, dt, M):
    M = _f64(M)
    out = np.empty_like(M)
    m0 = np.empty(M.shape[:-1])
    m1 = np.empty(M.shape[:-1])
    lib().oracle_motor_step(C.byref(cparams(p)), float(dt), M, out, _ptr(m0), _ptr(m1))
    return out, m0, m1


def motor_substeps(p, dt):
    """Sub-steps of one micro-step (the oracle's local dt* rule, Alg. 2)."""
    return int(lib().oracle_motor_substeps(C.byref(cparams(p)), float(dt)))


def motor_substepped(p, dt, M):
    """motor_substeps(p, dt) midpoint steps of dt / n of every column, and the s-moments."""
    M = _f64(M)
    out = np.empty_like(M)
    m0 = np.empty(M.shape[:-1])
    m1 = np.empty(M.shape[:-1])
    lib().oracle_motor_substepped(C.byref(cparams(p)), float(dt), M, out, _ptr(m0), _ptr(m1))
    return out, m0, m1


def psi_step(p, dt, psi, m0, u, gradu):
    psi = _f64(psi)
    out = np.empty_like(psi)
    lib().oracle_psi_step(C.byref(cparams(p)), float(dt), psi, _f64(m0), _f64(u), _f64(gradu), out)
    return out


def moments(p, psi, m0, m1):
    stress = np.empty((3, p.nx, p.ny))
    mom = np.empty((7, p.nx, p.ny))
    lib().oracle_moments(C.byref(cparams(p)), _f64(psi), _f64(m0), _f64(m1), stress, mom)
    return stress, mom


def global_sums(p, psi, stress):
    mass = C.c_double()
    ss = np.empty(3)
    lib().oracle_global_sums(C.byref(cparams(p)), _f64(psi), _f64(stress), C.byref(mass), ss)
    return mass.value, ss


def run_step(p, dt, M, src):
    """One midpoint step of a run of len(M) cells (minus-end rules first, plus-end rules last)."""
    M = _f64(M)
    out = np.empty_like(M)
    lib().oracle_run_step(C.byref(cparams(p)), len(M), float(dt), M, float(src), out)
    return out


# ---- anchor-resolved bound motors (oracle_r0.c) ----------------------------------------------
def r0_cells(p):
    """Tracked cells [n][4] = (a, b, k, l) in lexicographic order; raises if rc is unusable."""
    n = lib().oracle_r0_cells(C.byref(cparams(p)), None)
    if n < 0:
        raise ValueError("rc must be > 0 with rc + L/2 < lx/2 and ly/2")
    cells = np.empty((n, 4), dtype=np.int32)
    lib().oracle_r0_cells(C.byref(cparams(p)), cells.ctypes.data_as(C.c_void_p))
    return cells


def r0_coarse(p, cells, psi, Mb):
    out = np.empty((p.nx, p.ny))
    lib().oracle_r0_coarse(C.byref(cparams(p)), cells, len(cells), _f64(psi), _f64(Mb), out)
    return out


def r0_motor_step(p, dt, cells, Mb, scale=None, src=None):
    Mb = _f64(Mb)
    out = np.empty_like(Mb)
    scale = None if scale is None else _f64(scale)
    src = None if src is None else _f64(src)
    lib().oracle_r0_motor_step(C.byref(cparams(p)), float(dt), cells, len(cells), Mb, out, _ptr(scale), _ptr(src))
    return out


def r0_marginal(p, cells, Mb):
    m0 = np.empty((p.nx, p.ny, p.ntheta))
    m1 = np.empty((p.nx, p.ny, p.ntheta))
    lib().oracle_r0_marginal(C.byref(cparams(p)), cells, len(cells), _f64(Mb), _ptr(m0), _ptr(m1))
    return m0, m1


def r0_marginal_field(p, cells, Mb):
    """Anchor-marginal bound motors M [nx][ny][nth][ns] = sum over anchors of M_b dx dy."""
    M = np.empty((p.nx, p.ny, p.ntheta, p.ns))
    lib().oracle_r0_marginal_field(C.byref(cparams(p)), cells, len(cells), _f64(Mb), M)
    return M


def r0_motor_force(p, cells, psi, Mb):
    """Motor force density [2][nx][ny] of an anchor-resolved state (Eq. (10) with its r0 integral)."""
    return motor_force(p, psi, r0_marginal_field(p, cells, Mb))


class OracleR0:
    """Host-side stepper of the anchor-resolved model, in the HIP library's call order."""

    def __init__(self, p):
        self.p = p
        self.cells = r0_cells(p)
        self.psi = self.Mb = self.u = self.gradu = None

    def set_state(self, psi, Mb=None):
        p = self.p
        self.psi = _f64(psi).copy()
        self.Mb = np.zeros((len(self.cells), p.nx, p.ny)) if Mb is None else _f64(Mb).copy()

    def set_fluid(self, u, gradu):
        self.u, self.gradu = _f64(u).copy(), _f64(gradu).copy()

    def step(self, K, dt):
        lib().oracle_r0_run(C.byref(cparams(self.p)), float(dt), int(K), self.cells, len(self.cells),
                            self.psi, self.Mb, self.u, self.gradu, None, None, None)

    def get_state(self):
        return self.psi.copy(), self.Mb.copy()

    def marginals(self):
        return r0_marginal(self.p, self.cells, self.Mb)

    def coarse(self):
        return r0_coarse(self.p, self.cells, self.psi, self.Mb)

    def get_stress_moments(self):
        m0, m1 = self.marginals()
        return moments(self.p, self.psi, m0, m1)

    def get_sums(self):
        stress, _ = self.get_stress_moments()
        return global_sums(self.p, self.psi, stress)


def max_threads():
    return lib().oracle_max_threads()


def set_threads(n):
    lib().oracle_set_threads(int(n))


class OracleA:
    """Host-side stepper with the same call order as the HIP library's context."""

    def __init__(self, p):
        self.p = p
        self.psi = None
        self.M = None
        self.u = None
        self.gradu = None
        self.m0 = None
        self.m1 = None

    def set_params(self, k_on, k_off, v0):
        self.p.k_on, self.p.k_off, self.p.v0 = float(k_on), float(k_off), float(v0)

    def set_state(self, psi, M=None):
        p = self.p
        self.psi = _f64(psi).copy()
        self.M = (np.zeros((p.nx, p.ny, p.ntheta, p.ns)) if M is None else _f64(M).copy())
        self.m0 = self.m1 = None

    def set_fluid(self, u, gradu):
        self.u, self.gradu = _f64(u).copy(), _f64(gradu).copy()

    def step(self, K, dt):
        p = self.p
        m0 = np.empty(self.psi.shape)
        m1 = np.empty(self.psi.shape)
        lib().oracle_run(C.byref(cparams(p)), float(dt), int(K), self.psi, self.M, self.u,
                         self.gradu, _ptr(m0), _ptr(m1))
        self.m0, self.m1 = m0, m1

    def get_state(self):
        return self.psi.copy(), self.M.copy()

    def get_stress_moments(self):
        return moments(self.p, self.psi, self.m0, self.m1)

    def get_sums(self):
        stress, _ = self.get_stress_moments()
        return global_sums(self.p, self.psi, stress)
