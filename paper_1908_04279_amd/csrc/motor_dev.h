// Device code of the motor column step (walk + attach/detach along filament arclength s),
// shared by the motor kernel and the fused micro-step kernel.
//
// Model: Cook & Shinar, Sec. 2 Eq. (4) with linear attachment k_on and detachment k_off M,
// walking speed v0 towards the plus end; superbee-limited upwind flux in s (Sec. 2); the
// two-stage Runge-Kutta of Sec. 3.1 / Alg. 2 as the explicit midpoint rule.  Boundary
// readings: no walking influx at s = 0 (ghost M_{-1} = 0, flux 0), first-order free outflow
// at s = L (ghost M_{ns} = M_{ns-1}, so the last slope is 0 and the last flux is v0 M).
//
// Layout: M[col][s] with s contiguous.  A column of ns = CPL * LPC cells is spread over LPC
// consecutive lanes, CPL cells per lane, loaded with 16-byte vector loads.  Neighbour cells
// across lanes move with DPP shifts; the s-reductions m0, m1 are DPP butterflies inside the
// group.  Both Runge-Kutta stages live in registers: one read and one write of M per step,
// the HBM floor of this update.
#pragma once
#include "device_util.h"
#include "kernels.h"

#include <type_traits>

namespace mmk {

// Superbee slope of the one-sided differences a (left) and b (right): zero unless a and b
// have the same strict sign, else sgn(b) max(min(2|a|,|b|), min(|a|,2|b|)).
template <typename T>
__device__ __forceinline__ T superbee(T a, T b) {
    const T aa = fabs(a), ab = fabs(b);
    const T m = fmax(fmin(aa + aa, ab), fmin(aa, ab + ab));
    return (a * b > T(0)) ? copysign(m, b) : T(0);
}
// FP32: minmod(x, y) = med3(x, y, 0), and superbee = maxmod(minmod(2a, b), minmod(a, 2b)).
// Both minmods carry the sign of b (or are 0), so their maxmod is med3(p, q, sgn(b) inf).
// Every operation is exact (doubling, median, sign copy): the value equals the definition.
template <>
__device__ __forceinline__ float superbee<float>(float a, float b) {
    const float p = __builtin_amdgcn_fmed3f(a + a, b, 0.0f);
    const float q = __builtin_amdgcn_fmed3f(a, b + b, 0.0f);
    return __builtin_amdgcn_fmed3f(p, q, copysignf(__builtin_inff(), b));
}

// R(z) on this lane's CPL cells.  g: lane index inside the column group; l0 = g * CPL.
// With the face value h_l = z_l + sigma_l / 2 (flux v0 h_l; h_{-1} = 0 carries the zero
// influx, and the zero last slope makes h_{ns-1} = z_{ns-1}, the first-order outflow):
//   R_l = -(v0/ds) (h_l - h_{l-1}) + (k_on - k_off z_l).
template <typename T, int CPL, int LPC, int LIM, bool RAGGED>
__device__ __forceinline__ void motor_rhs(const T (&z)[CPL], T (&R)[CPL], const MotorConst<T> &c,
                                          int g, int l0, int ns) {
    const T zl = from_prev<LPC>(z[CPL - 1], T(0), g);        // z_{l0-1}; ghost 0 at s = 0
    const T zr = from_next<LPC>(z[0], z[CPL - 1], g);        // z_{l0+CPL}; ghost at s = L
    T d[CPL + 1];                                             // d[j] = z_{l0+j} - z_{l0+j-1}
    d[0] = z[0] - zl;
#pragma unroll
    for (int j = 1; j < CPL; ++j) d[j] = z[j] - z[j - 1];
    d[CPL] = zr - z[CPL - 1];
    if constexpr (RAGGED) {
        // the cell right of l = ns-1 is the ghost z_{ns} = z_{ns-1}: zero difference
#pragma unroll
        for (int j = 0; j < CPL; ++j)
            if (l0 + j + 1 >= ns) d[j + 1] = T(0);
    }
    T h[CPL];                                                 // face value at l + 1/2
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const T sig = (LIM == 0) ? superbee(d[j], d[j + 1]) : T(0);
        h[j] = z[j] + T(0.5) * sig;
    }
    const T hl = from_prev<LPC>(h[CPL - 1], T(0), g);        // h_{-1} = 0: no influx
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const T left = (j == 0) ? hl : h[j - 1];
        R[j] = c.nv_ds * (h[j] - left) + (c.k_on - c.k_off * z[j]);
    }
}

// One block's share of the motor step: 256 / LPC columns starting at column vblock * 256 / LPC.
template <typename T, int CPL, int LPC, int LIM, bool RAGGED, bool WANT_M1, bool NT>
__device__ __forceinline__ void motor_cols(const T *__restrict__ M_in, T *__restrict__ M_out,
                                           T *__restrict__ m0, T *__restrict__ m1, int64_t ncol, int ns,
                                           const MotorConst<T> &c, int64_t vblock) {
    constexpr int COLS = 256 / LPC;
    const int g = threadIdx.x % LPC;
    const int64_t col = vblock * COLS + threadIdx.x / LPC;
    const bool active = col < ncol;
    const int l0 = g * CPL;
    const int64_t base = col * (int64_t)ns + l0;

    T x[CPL];
    if constexpr (!RAGGED) {
        if (active) {
            load_cells<T, CPL, NT>(M_in + base, x);
        } else {
#pragma unroll
            for (int j = 0; j < CPL; ++j) x[j] = T(0);
        }
    } else {
#pragma unroll
        for (int j = 0; j < CPL; ++j) x[j] = (active && l0 + j < ns) ? M_in[base + j] : T(0);
    }

    T R[CPL], y[CPL];
    motor_rhs<T, CPL, LPC, LIM, RAGGED>(x, R, c, g, l0, ns);
#pragma unroll
    for (int j = 0; j < CPL; ++j) y[j] = x[j] + c.half_dt * R[j];
    motor_rhs<T, CPL, LPC, LIM, RAGGED>(y, R, c, g, l0, ns);
#pragma unroll
    for (int j = 0; j < CPL; ++j) y[j] = x[j] + c.dt * R[j];

    if constexpr (!RAGGED) {
        if (active) store_cells<T, CPL, NT>(M_out + base, y);
    } else {
#pragma unroll
        for (int j = 0; j < CPL; ++j)
            if (active && l0 + j < ns) M_out[base + j] = y[j];
    }

    // s-moments of the new column: m0 = ds sum M, m1 = ds^2 sum (l + 1/2 - ns/2) M, the
    // weights being exact half-integers.  FP32: Kahan inside the lane, TwoSum butterfly.
    if constexpr (std::is_same<T, float>::value) {
        Kahan a0, a1;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            const bool in = !RAGGED || (l0 + j < ns);
            const float v = in ? y[j] : 0.0f;
            a0.add(v);
            if constexpr (WANT_M1) a1.add(v * (0.5f * (float)(2 * (l0 + j) + 1 - ns)));
        }
        const float s0 = group_sum_comp<LPC>(a0.sum, a0.comp);
        if (active && g == 0) m0[col] = s0 * c.ds;
        if constexpr (WANT_M1) {
            const float s1 = group_sum_comp<LPC>(a1.sum, a1.comp);
            if (active && g == 0) m1[col] = s1 * c.ds2;
        }
    } else {
        T a0 = 0, a1 = 0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            const bool in = !RAGGED || (l0 + j < ns);
            const T v = in ? y[j] : T(0);
            a0 += v;
            if constexpr (WANT_M1) a1 += v * (T(0.5) * (T)(2 * (l0 + j) + 1 - ns));
        }
        const T s0 = group_sum<LPC>(a0);
        if (active && g == 0) m0[col] = s0 * c.ds;
        if constexpr (WANT_M1) {
            const T s1 = group_sum<LPC>(a1);
            if (active && g == 0) m1[col] = s1 * c.ds2;
        }
    }
}

}  // namespace mmk
