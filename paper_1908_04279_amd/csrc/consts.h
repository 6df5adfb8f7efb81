// Kernel constants from the model parameters, rounded once to the field precision.
#pragma once
#include "../../include/mmk.h"
#include "kernels.h"

namespace mmk {

constexpr double kTwoPi = 6.283185307179586476925286766559;

template <typename T>
inline MotorConst<T> motor_const(const mmk_params &p, double dt) {
    const double ds = p.L / p.ns;
    MotorConst<T> c;
    c.k_on = (T)p.k_on;
    c.k_off = (T)p.k_off;
    c.v0 = (T)p.v0;
    c.nv_ds = (T)(-p.v0 / ds);
    c.dt = (T)dt;
    c.half_dt = (T)(0.5 * dt);
    c.ds = (T)ds;
    c.ds2 = (T)(ds * ds);
    c.nth = p.ntheta;
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
