// Hand-written reverse (adjoint) kernels of the micro-step for gfx950.
//
// Forward step n (see motor.hip and psi.hip): M' = M + dt R(M + dt/2 R(M)), m0' = ds sum M',
// psi' = psi - dt div(f(psi; A(m0', u), w(gradu))).  Given the cotangents of the step's
// outputs these kernels return the cotangents of its inputs and of k_on, k_off, v0:
//   psi reverse:   lam_psi' -> lam_psi (transposed donor-cell fluxes) and lam_m0' (through
//                  the face velocities A = mean(u - F m0 p));
//   motor reverse: lam_M' + lam_m0' ds (+ lam_m1' (s - L/2) ds on the last step) -> lam_M,
//                  recomputing the midpoint stage and the limiter branches in registers;
//                  parameter gradients are summed in FP64 per block.
// Kinks follow one fixed branch rule: a superbee pair with a*b <= 0 is the zero branch, min
// keeps its first argument on <=, max its first on >=, a face velocity of exactly 0 takes
// the left cell.
#include "adjoint.h"
#include "device_util.h"

#include <type_traits>

namespace mmk {

// ---------------------------------------------------------------------------------------
// Motor column reverse step.

// Superbee on its selected branch: sigma = ca a + cb b with (ca, cb) one of (0,0), (2,0),
// (0,1), (1,0), (0,2).  With one coefficient zero the sum is exact, so sigma equals the
// forward slope bit for bit.
template <typename T>
__device__ __forceinline__ void superbee_branch(T a, T b, T &ca, T &cb) {
    const T aa = fabs(a), ab = fabs(b);
    const bool p_first = (aa + aa <= ab);  // p = min(2|a|, |b|): 2|a| on ties
    const bool q_first = (aa <= ab + ab);  // q = min(|a|, 2|b|): |a| on ties
    const T p = p_first ? aa + aa : ab;
    const T q = q_first ? aa : ab + ab;
    const bool take_p = (p >= q);          // max(p, q): p on ties
    T ca_ = take_p ? (p_first ? T(2) : T(0)) : (q_first ? T(1) : T(0));
    T cb_ = take_p ? (p_first ? T(0) : T(1)) : (q_first ? T(0) : T(2));
    const bool same = (a * b > T(0));
    ca = same ? ca_ : T(0);
    cb = same ? cb_ : T(0);
}

struct RevAcc {
    double kon = 0, koff = 0, v0 = 0;
};

// Limiter branches and face values h of a column state z (this lane's CPL cells).
template <typename T, int CPL, int LPC, int LIM, bool RAGGED>
__device__ __forceinline__ void faces(const T (&z)[CPL], T (&ca)[CPL], T (&cb)[CPL], T (&h)[CPL], T &hl,
                                      int g, int l0, int ns) {
    const T zl = from_prev<LPC>(z[CPL - 1], T(0), g);
    const T zr = from_next<LPC>(z[0], z[CPL - 1], g);
    T d[CPL + 1];
    d[0] = z[0] - zl;
#pragma unroll
    for (int j = 1; j < CPL; ++j) d[j] = z[j] - z[j - 1];
    d[CPL] = zr - z[CPL - 1];
    if constexpr (RAGGED) {
#pragma unroll
        for (int j = 0; j < CPL; ++j)
            if (l0 + j + 1 >= ns) d[j + 1] = T(0);
    }
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        if constexpr (LIM == 0) {
            superbee_branch(d[j], d[j + 1], ca[j], cb[j]);
        } else {
            ca[j] = T(0);
            cb[j] = T(0);
        }
        h[j] = z[j] + T(0.5) * (ca[j] * d[j] + cb[j] * d[j + 1]);
    }
    hl = from_prev<LPC>(h[CPL - 1], T(0), g);
}

// out = (dR/dz)^T mu at state z, and the parameter terms of mu . R(z) added to acc:
//   d/dk_on = sum mu, d/dk_off = -sum mu z, d/dv0 = -(1/ds) sum mu (h_l - h_{l-1}).
// With nu_l = (v0/ds)(mu_{l+1} - mu_l) (mu_ns = 0) the cotangent of the face value h_l:
//   out_l = nu_l + (1/2)[(ca_l - cb_l) nu_l + cb_{l-1} nu_{l-1} - ca_{l+1} nu_{l+1}] - k_off mu_l.
template <typename T, int CPL, int LPC, int LIM, bool RAGGED>
__device__ __forceinline__ void rhs_vjp(const T (&z)[CPL], const T (&mu)[CPL], T (&out)[CPL],
                                        const MotorConst<T> &c, T inv_ds, int g, int l0, int ns, T &s_kon,
                                        T &s_koff, T &s_v0) {
    T ca[CPL], cb[CPL], h[CPL], hl;
    faces<T, CPL, LPC, LIM, RAGGED>(z, ca, cb, h, hl, g, l0, ns);
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        s_kon += mu[j];
        s_koff -= mu[j] * z[j];
        s_v0 -= mu[j] * (h[j] - (j == 0 ? hl : h[j - 1]));
    }
    const T mu_next = from_next<LPC>(mu[0], T(0), g);  // mu_{ns} = 0
    const T v0_ds = c.v0 * inv_ds;
    T nu[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) nu[j] = v0_ds * ((j + 1 < CPL ? mu[j + 1] : mu_next) - mu[j]);
    const T cbnu_prev = from_prev<LPC>(cb[CPL - 1] * nu[CPL - 1], T(0), g);
    const T canu_next = from_next<LPC>(ca[0] * nu[0], T(0), g);
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const T left = (j == 0) ? cbnu_prev : cb[j - 1] * nu[j - 1];
        const T right = (j + 1 < CPL) ? ca[j + 1] * nu[j + 1] : canu_next;
        out[j] = nu[j] + T(0.5) * ((ca[j] - cb[j]) * nu[j] + left - right) - c.k_off * mu[j];
    }
}

template <typename T, int CPL, int LPC, int LIM, bool RAGGED>
__global__ __launch_bounds__(256) void k_motor_reverse(const T *__restrict__ M, const T *__restrict__ lam_in,
                                                       const T *__restrict__ lam_m0, const T *__restrict__ lam_m1,
                                                       T *__restrict__ lam_out, double *__restrict__ gpart,
                                                       int64_t ncol, int ns, MotorConst<T> c, T inv_ds) {
    constexpr int COLS = 256 / LPC;
    const int g = threadIdx.x % LPC;
    const int l0 = g * CPL;
    RevAcc acc;
    for (int64_t col0 = (int64_t)blockIdx.x * COLS; col0 < ncol; col0 += (int64_t)gridDim.x * COLS) {
        const int64_t col = col0 + threadIdx.x / LPC;
        const bool active = col < ncol;
        const int64_t base = col * (int64_t)ns + l0;
        T x[CPL], lam[CPL];
        const T a0 = active ? lam_m0[col] * c.ds : T(0);
        const T a1 = (active && lam_m1) ? lam_m1[col] * c.ds2 : T(0);
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            const bool in = active && (!RAGGED || l0 + j < ns);
            x[j] = in ? M[base + j] : T(0);
            const T w = T(0.5) * (T)(2 * (l0 + j) + 1 - ns);  // (s_l - L/2) / ds
            lam[j] = in ? ((lam_in ? lam_in[base + j] : T(0)) + a0 + a1 * w) : T(0);
        }
        // recompute the midpoint stage
        T R[CPL], y[CPL];
        {
            // forward right-hand side at x (same expression as the forward kernel)
            T ca[CPL], cb[CPL], h[CPL], hl;
            faces<T, CPL, LPC, LIM, RAGGED>(x, ca, cb, h, hl, g, l0, ns);
#pragma unroll
            for (int j = 0; j < CPL; ++j)
                R[j] = c.nv_ds * (h[j] - (j == 0 ? hl : h[j - 1])) + (c.k_on - c.k_off * x[j]);
        }
#pragma unroll
        for (int j = 0; j < CPL; ++j) y[j] = x[j] + c.half_dt * R[j];
        // second stage: M' = x + dt R(y)
        T mu[CPL], zeta[CPL], w[CPL];
        T s_kon = 0, s_koff = 0, s_v0 = 0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) mu[j] = c.dt * lam[j];
        rhs_vjp<T, CPL, LPC, LIM, RAGGED>(y, mu, zeta, c, inv_ds, g, l0, ns, s_kon, s_koff, s_v0);
        // first stage: y = x + dt/2 R(x)
#pragma unroll
        for (int j = 0; j < CPL; ++j) mu[j] = c.half_dt * zeta[j];
        rhs_vjp<T, CPL, LPC, LIM, RAGGED>(x, mu, w, c, inv_ds, g, l0, ns, s_kon, s_koff, s_v0);
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            const bool in = active && (!RAGGED || l0 + j < ns);
            if (in) lam_out[base + j] = lam[j] + zeta[j] + w[j];
        }
        acc.kon += (double)s_kon;
        acc.koff += (double)s_koff;
        acc.v0 += (double)s_v0 * (double)inv_ds;
    }
    // fixed-order block sum, added to this block's running FP64 partials
    __shared__ double red[4][3];
    double v[3] = {acc.kon, acc.koff, acc.v0};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        for (int m = 32; m >= 1; m >>= 1) v[a] += __shfl_xor(v[a], m, 64);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0)
        for (int a = 0; a < 3; ++a) red[wave][a] = v[a];
    __syncthreads();
    if (threadIdx.x < 3) {
        const int a = threadIdx.x;
        const double s = (red[0][a] + red[1][a]) + (red[2][a] + red[3][a]);
        gpart[(size_t)blockIdx.x * 4 + a] += s;
    }
}

template <typename T, int CPL, int LPC, bool RAGGED>
static hipError_t rev_cfg(const T *M, const T *lam_in, const T *lam_m0, const T *lam_m1, T *lam_out,
                          double *gpart, int gblocks, int64_t ncol, int ns, int limiter, const MotorConst<T> &c,
                          T inv_ds, hipStream_t s) {
    constexpr int COLS = 256 / LPC;
    int64_t blocks = (ncol + COLS - 1) / COLS;
    if (blocks > gblocks) blocks = gblocks;
    if (blocks < 1) blocks = 1;
    if (limiter == 0)
        hipLaunchKernelGGL((k_motor_reverse<T, CPL, LPC, 0, RAGGED>), dim3((unsigned)blocks), dim3(256), 0, s, M,
                           lam_in, lam_m0, lam_m1, lam_out, gpart, ncol, ns, c, inv_ds);
    else
        hipLaunchKernelGGL((k_motor_reverse<T, CPL, LPC, 1, RAGGED>), dim3((unsigned)blocks), dim3(256), 0, s, M,
                           lam_in, lam_m0, lam_m1, lam_out, gpart, ncol, ns, c, inv_ds);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_motor_reverse(const T *M, const T *lam_in, const T *lam_m0, const T *lam_m1, T *lam_out,
                                double *gpart, int gblocks, int64_t ncol, int ns, int limiter,
                                const MotorConst<T> &c, double inv_ds, hipStream_t s) {
    const T ids = (T)inv_ds;
    switch (ns) {
        case 8: return rev_cfg<T, 4, 2, false>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
        case 16: return rev_cfg<T, 4, 4, false>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
        case 32: return rev_cfg<T, 4, 8, false>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
        case 64: return rev_cfg<T, 4, 16, false>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
        case 128: return rev_cfg<T, 8, 16, false>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
        default: break;
    }
    if (ns <= 16) return rev_cfg<T, 1, 16, true>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
    if (ns <= 32) return rev_cfg<T, 2, 16, true>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
    if (ns <= 64) return rev_cfg<T, 4, 16, true>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
    if (ns <= 128) return rev_cfg<T, 8, 16, true>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
    if (ns <= 256) return rev_cfg<T, 16, 16, true>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
    if (ns <= 512) return rev_cfg<T, 32, 16, true>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
    return hipErrorInvalidValue;
}
template hipError_t launch_motor_reverse<float>(const float *, const float *, const float *, const float *, float *,
                                                double *, int, int64_t, int, int, const MotorConst<float> &, double,
                                                hipStream_t);
template hipError_t launch_motor_reverse<double>(const double *, const double *, const double *, const double *,
                                                 double *, double *, int, int64_t, int, int,
                                                 const MotorConst<double> &, double, hipStream_t);

// ---------------------------------------------------------------------------------------
// Psi reverse step.  LDS tile of lam', psi and m0 with a one-pencil halo (as the forward).
//   mu_face = dt/h (lam'_right - lam'_left)
//   lam_psi_c = lam'_c + sum over the c's faces of  mu * (upwind weight of psi_c)
//   dL/dA = mu * (A >= 0 ? psi_left : psi_right);  A_{i+1/2} = (a_i + a_{i+1}) / 2,
//   a = u - F m0 p  =>  lam_m0_c = -(F/2) [cos th (gAx+ + gAx-) + sin th (gAy+ + gAy-)].
template <typename T>
__global__ __launch_bounds__(256) void k_psi_reverse(const T *__restrict__ lam_in, const T *__restrict__ psi,
                                                     const T *__restrict__ m0, const T *__restrict__ u,
                                                     const T *__restrict__ Gr, const T *__restrict__ tab,
                                                     T *__restrict__ lam_out, T *__restrict__ lam_m0,
                                                     int accumulate_m0, PsiConst<T> c, PsiLaunch pl) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = c.nx, ny = c.ny, nth = c.nth;
    const int TI = pl.ti, TJ = pl.tj, HI = TI + 2, HJ = TJ + 2, NH = HI * HJ;
    T *s_lam = reinterpret_cast<T *>(smem);       // [NH][nth]
    T *s_psi = s_lam + (size_t)NH * nth;           // [NH][nth]
    T *s_m0 = s_psi + (size_t)NH * nth;            // [NH][nth]
    T *s_u = s_m0 + (size_t)NH * nth;              // [2][NH]
    T *s_G = s_u + 2 * NH;                         // [4][TI*TJ]
    T *s_tab = s_G + 4 * TI * TJ;                  // [TAB_N][nth]
    const int tid = threadIdx.x;
    const int per = gridDim.x / 8;
    const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= pl.tiles_i * pl.tiles_j) return;
    const int i0 = (tile / pl.tiles_j) * TI, j0 = (tile % pl.tiles_j) * TJ;
    const int64_t nxy = (int64_t)nx * ny;
    const int G = pl.group, NG = 256 / G;
    const int grp = tid / G, kk = tid % G;
    auto wrap = [](int i, int n) {
        if (i < 0) i += n;
        while (i >= n) i -= n;
        return i;
    };
    for (int q = grp; q < NH; q += NG) {
        const int qi = q / HJ, qj = q - qi * HJ;
        if ((qi == 0 || qi == HI - 1) && (qj == 0 || qj == HJ - 1)) continue;
        const int64_t pen = (int64_t)wrap(i0 + qi - 1, nx) * ny + wrap(j0 + qj - 1, ny);
        for (int k = kk; k < nth; k += G) {
            s_lam[q * nth + k] = lam_in[pen * nth + k];
            s_psi[q * nth + k] = psi[pen * nth + k];
            s_m0[q * nth + k] = m0[pen * nth + k];
        }
        if (kk == 0) {
            s_u[q] = u[pen];
            s_u[NH + q] = u[nxy + pen];
        }
    }
    for (int p = tid; p < TI * TJ; p += 256) {
        const int64_t pen = (int64_t)wrap(i0 + p / TJ, nx) * ny + wrap(j0 + p % TJ, ny);
        for (int a = 0; a < 4; ++a) s_G[a * TI * TJ + p] = Gr[a * nxy + pen];
    }
    for (int k = tid; k < TAB_N * nth; k += 256) s_tab[k] = tab[k];
    __syncthreads();

    const T hx = c.dt * c.inv_dx, hy = c.dt * c.inv_dy, ht = c.dt * c.inv_dth;
    for (int p = grp; p < TI * TJ; p += NG) {
        const int pi = p / TJ, pj = p - pi * TJ;
        const int gi = i0 + pi, gj = j0 + pj;
        if (gi >= nx || gj >= ny) continue;
        const int q = (pi + 1) * HJ + (pj + 1);
        const int qxm = q - HJ, qxp = q + HJ, qym = q - 1, qyp = q + 1;
        const T ux_c = s_u[q], ux_m = s_u[qxm], ux_p = s_u[qxp];
        const T uy_c = s_u[NH + q], uy_m = s_u[NH + qym], uy_p = s_u[NH + qyp];
        const T Gxx = s_G[p], Gxy = s_G[TI * TJ + p], Gyx = s_G[2 * TI * TJ + p], Gyy = s_G[3 * TI * TJ + p];
        const int64_t pen = (int64_t)gi * ny + gj;
        for (int k = kk; k < nth; k += G) {
            const int kp = (k + 1 == nth) ? 0 : k + 1;
            const int km = (k == 0) ? nth - 1 : k - 1;
            const T co = s_tab[TAB_C * nth + k], si = s_tab[TAB_S * nth + k];
            const T chp = s_tab[TAB_CH * nth + k], shp = s_tab[TAB_SH * nth + k];
            const T chm = s_tab[TAB_CH * nth + km], shm = s_tab[TAB_SH * nth + km];
            const T ps = s_psi[q * nth + k], lc = s_lam[q * nth + k], mc = s_m0[q * nth + k];
            // face velocities, as in the forward step
            const T ax_c = ux_c - c.F * mc * co;
            const T ax_m = ux_m - c.F * s_m0[qxm * nth + k] * co;
            const T ax_p = ux_p - c.F * s_m0[qxp * nth + k] * co;
            const T Axp = T(0.5) * (ax_c + ax_p), Axm = T(0.5) * (ax_m + ax_c);
            const T ay_c = uy_c - c.F * mc * si;
            const T ay_m = uy_m - c.F * s_m0[qym * nth + k] * si;
            const T ay_p = uy_p - c.F * s_m0[qyp * nth + k] * si;
            const T Ayp = T(0.5) * (ay_c + ay_p), Aym = T(0.5) * (ay_m + ay_c);
            const T wp = -shp * (Gxx * chp + Gxy * shp) + chp * (Gyx * chp + Gyy * shp);
            const T wm = -shm * (Gxx * chm + Gxy * shm) + chm * (Gyx * chm + Gyy * shm);
            // face cotangents
            const T mxp = hx * (s_lam[qxp * nth + k] - lc), mxm = hx * (lc - s_lam[qxm * nth + k]);
            const T myp = hy * (s_lam[qyp * nth + k] - lc), mym = hy * (lc - s_lam[qym * nth + k]);
            const T mtp = ht * (s_lam[q * nth + kp] - lc), mtm = ht * (lc - s_lam[q * nth + km]);
            T l = lc;
            l += (Axp >= T(0) ? Axp : T(0)) * mxp;
            l += (Axm >= T(0) ? T(0) : Axm) * mxm;
            l += (Ayp >= T(0) ? Ayp : T(0)) * myp;
            l += (Aym >= T(0) ? T(0) : Aym) * mym;
            l += (wp >= T(0) ? wp : T(0)) * mtp;
            l += (wm >= T(0) ? T(0) : wm) * mtm;
            lam_out[pen * nth + k] = l;
            const T gAxp = mxp * (Axp >= T(0) ? ps : s_psi[qxp * nth + k]);
            const T gAxm = mxm * (Axm >= T(0) ? s_psi[qxm * nth + k] : ps);
            const T gAyp = myp * (Ayp >= T(0) ? ps : s_psi[qyp * nth + k]);
            const T gAym = mym * (Aym >= T(0) ? s_psi[qym * nth + k] : ps);
            T lm = -T(0.5) * c.F * (co * (gAxp + gAxm) + si * (gAyp + gAym));
            if (accumulate_m0) lm += lam_m0[pen * nth + k];
            lam_m0[pen * nth + k] = lm;
        }
    }
}

template <typename T>
hipError_t launch_psi_reverse(const T *lam_in, const T *psi, const T *m0, const T *u, const T *G, const T *tab,
                              T *lam_out, T *lam_m0, bool accumulate_m0, const PsiConst<T> &c, const PsiLaunch &pl,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_psi_reverse<T>, dim3(pl.blocks), dim3(256), pl.lds_bytes, s, lam_in, psi, m0, u, G, tab,
                       lam_out, lam_m0, accumulate_m0 ? 1 : 0, c, pl);
    return hipGetLastError();
}
template hipError_t launch_psi_reverse<float>(const float *, const float *, const float *, const float *,
                                              const float *, const float *, float *, float *, bool,
                                              const PsiConst<float> &, const PsiLaunch &, hipStream_t);
template hipError_t launch_psi_reverse<double>(const double *, const double *, const double *, const double *,
                                               const double *, const double *, double *, double *, bool,
                                               const PsiConst<double> &, const PsiLaunch &, hipStream_t);

// ---------------------------------------------------------------------------------------
// Cotangents of the final psi, m0 and m1 from those of the stress and the moments.
//   c = sum psi dth, n = sum psi p dth, D = sum psi pp dth, B = sum psi m0 dth,
//   sigma = sum psi [sigma_f (cos2th/2, sin2th/2, -cos2th/2) + F m1 (cc, cs, ss)] dth
template <typename T>
__global__ __launch_bounds__(256) void k_seed(const T *__restrict__ g_sigma, const T *__restrict__ g_mom,
                                              const T *__restrict__ psi, const T *__restrict__ m0,
                                              const T *__restrict__ m1, const T *__restrict__ tab,
                                              T *__restrict__ lam_psi, T *__restrict__ lam_m0,
                                              T *__restrict__ lam_m1, int64_t npsi, int nth, int64_t nxy, T F,
                                              T sigma_f, T dth) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npsi; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pen = i / nth;
        const int k = (int)(i - pen * nth);
        T gm[7] = {0, 0, 0, 0, 0, 0, 0}, gs[3] = {0, 0, 0};
        if (g_mom)
            for (int a = 0; a < 7; ++a) gm[a] = g_mom[a * nxy + pen];
        if (g_sigma)
            for (int a = 0; a < 3; ++a) gs[a] = g_sigma[a * nxy + pen];
        const T co = tab[TAB_C * nth + k], si = tab[TAB_S * nth + k];
        const T cc = tab[TAB_CC * nth + k], cs = tab[TAB_CS * nth + k], ss = tab[TAB_SS * nth + k];
        const T h1 = tab[TAB_H1 * nth + k], h2 = tab[TAB_H2 * nth + k];
        const T ps = psi[i], mm0 = m0[i], fm1 = F * m1[i];
        const T w = gm[0] + gm[1] * co + gm[2] * si + gm[3] * cc + gm[4] * cs + gm[5] * ss + gm[6] * mm0 +
                    gs[0] * (sigma_f * h1 + fm1 * cc) + gs[1] * (sigma_f * h2 + fm1 * cs) +
                    gs[2] * (-sigma_f * h1 + fm1 * ss);
        lam_psi[i] = w * dth;
        lam_m0[i] = gm[6] * ps * dth;
        lam_m1[i] = F * ps * (gs[0] * cc + gs[1] * cs + gs[2] * ss) * dth;
    }
}

template <typename T>
hipError_t launch_seed(const T *g_sigma, const T *g_mom, const T *psi, const T *m0, const T *m1, const T *tab,
                       T *lam_psi, T *lam_m0, T *lam_m1, int64_t npsi, int nth, int64_t nxy, T F, T sigma_f, T dth,
                       hipStream_t s) {
    int64_t blocks = (npsi + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_seed<T>, dim3((unsigned)blocks), dim3(256), 0, s, g_sigma, g_mom, psi, m0, m1, tab, lam_psi,
                       lam_m0, lam_m1, npsi, nth, nxy, F, sigma_f, dth);
    return hipGetLastError();
}
template hipError_t launch_seed<float>(const float *, const float *, const float *, const float *, const float *,
                                       const float *, float *, float *, float *, int64_t, int, int64_t, float, float,
                                       float, hipStream_t);
template hipError_t launch_seed<double>(const double *, const double *, const double *, const double *,
                                        const double *, const double *, double *, double *, double *, int64_t, int,
                                        int64_t, double, double, double, hipStream_t);

__global__ void k_zero_f64(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_f64, dim3(64), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace mmk
