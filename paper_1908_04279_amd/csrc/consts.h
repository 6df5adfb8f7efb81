// Kernel constants from the model parameters, rounded once to the field precision.
#pragma once
#include "../../include/mmk.h"
#include "kernels.h"

#include <cmath>

namespace mmk {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kMaxSubsteps = 4096;

// Motor sub-steps of one micro-step of length dt (Alg. 2: local dt* from the motor's stability
// limit, v0 / ds + k_off, which is the same at every point): 1 without sub-cycling
// (motor_cfl = 0), else ceil(dt (v0 / ds + k_off) / motor_cfl), at least 1; 0 when that
// exceeds kMaxSubsteps (the caller refuses the step).
inline int motor_substeps(const mmk_params &p, double dt) {
    if (!(p.motor_cfl > 0)) return 1;
    const double q = std::ceil(dt * (p.v0 / (p.L / p.ns) + p.k_off) / p.motor_cfl);
    if (!(q <= kMaxSubsteps)) return 0;
    return q < 1 ? 1 : (int)q;
}

template <typename T>
inline MotorConst<T> motor_const(const mmk_params &p, double dt) {
    const double ds = p.L / p.ns;
    const int n = motor_substeps(p, dt);
    const double h = dt / n;
    MotorConst<T> c;
    c.k_on = (T)p.k_on;
    c.k_off = (T)p.k_off;
    c.v0 = (T)p.v0;
    c.nv_ds = (T)(-p.v0 / ds);
    c.nsub = n;
    c.nstep = 1;
    c.m0_steps = nullptr;
    c.dt = (T)h;
    c.half_dt = (T)(0.5 * h);
    c.ds = (T)ds;
    c.ds2 = (T)(ds * ds);
    c.nth = p.ntheta;
    c.wide = 0;
    c.lanes = 0;
    c.chunks = 0;
    c.nt = -1;
    c.nth_shift = -1;
    for (int k = 0; k < 31; ++k)
        if ((1 << k) == p.ntheta) c.nth_shift = k;
    return c;
}

template <typename T>
inline PsiConst<T> psi_const(const mmk_params &p, double dt) {
    PsiConst<T> c;
    c.nx = p.nx;
    c.ny = p.ny;
    c.nth = p.ntheta;
    c.dt = (T)dt;
    c.inv_dx = (T)(p.nx / p.lx);
    c.inv_dy = (T)(p.ny / p.ly);
    c.inv_dth = (T)(p.ntheta / kTwoPi);
    c.F = (T)p.F;
    c.sigma_f = (T)p.sigma_f;
    c.dth = (T)(kTwoPi / p.ntheta);
    c.m_total = (T)p.m_total;
    return c;
}

}  // namespace mmk
