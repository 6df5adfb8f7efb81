// Anchor-resolved bound motors on the capture ball (Sec. 2; Eqs. (4)-(6); Alg. 2) for gfx950.
//
// Layout: M_b[cell][x] with x = (i, j) the filament cell, contiguous, so the 64 lanes of a wave
// hold 64 consecutive filament cells of one run (a, b, k, lo..lo+len-1) and every load and
// store of the run moves 64 consecutive values.  The run (at most kR0MaxRun cells) lives in
// registers through both Runge-Kutta stages: M_b is read and written once per micro-step.
//
// The two reductions of the model go in opposite directions: the anchor marginal m0(x, th)
// sums over the anchors of a filament cell, the coarse density of Eq. (5) over the filament
// cells of an anchor.  The motor kernel makes the first in a block that owns one orientation
// and 64 filament cells (its four waves take every fourth run of that orientation, then add
// their totals through LDS in a fixed order) and writes each run's total q0 = sum M ds.  The
// coarse kernel makes the second from q0 and psi (a gather of psi from L2), one row of
// partials per wave, and a last kernel adds the rows in a fixed order and forms the clamp and
// the free pool.  No atomics: every result is the same from run to run.
#include "device_util.h"
#include "r0.h"

#include <algorithm>
#include <cmath>

namespace mmk {

// ---- host: tracked cells and runs ------------------------------------------------------------
// The motor point of cell (a, b, k, l) relative to its anchor is (a dx, b dy) + t p_k with
// t = s_l - L/2; the cell is tracked when the squared length is at most rc^2 (evaluated in FP64
// in this order, without contraction, so that the decision is the one the model's definition
// gives in FP64).
static bool tracked(double dx, double dy, double dth, double ds, double L, double rc, int a, int b, int k, int l) {
#pragma clang fp contract(off)
    const double t = (l + 0.5) * ds - 0.5 * L;
    const double th = k * dth;
    const double hx = a * dx + t * std::cos(th);
    const double hy = b * dy + t * std::sin(th);
    return hx * hx + hy * hy <= rc * rc;
}

R0Plan plan_r0(int nx, int ny, int nth, int ns, double lx, double ly, double L, double rc, bool cells_only) {
    R0Plan P;
    if (!(rc > 0) || !(rc + 0.5 * L < 0.5 * lx) || !(rc + 0.5 * L < 0.5 * ly)) return P;
    const double dx = lx / nx, dy = ly / ny, dth = 6.283185307179586476925286766559 / nth, ds = L / ns;
    // every tracked motor point lies within rc + L/2 of its anchor
    const int A = (int)std::ceil((rc + 0.5 * L) / dx) + 1;
    const int B = (int)std::ceil((rc + 0.5 * L) / dy) + 1;
    for (int a = -A; a <= A; ++a)
        for (int b = -B; b <= B; ++b)
            for (int k = 0; k < nth; ++k)
                for (int l = 0; l < ns; ++l)
                    if (tracked(dx, dy, dth, ds, L, rc, a, b, k, l)) {
                        P.cells.insert(P.cells.end(), {a, b, k, l});
                        ++P.ncell;
                    }
    P.ok = true;
    if (cells_only) return P;
    std::vector<std::vector<R0Seg>> byk(nth);
    for (int64_t c0 = 0; c0 < P.ncell;) {
        const int32_t *q = &P.cells[4 * c0];
        int64_t c1 = c0 + 1;
        while (c1 < P.ncell && P.cells[4 * c1] == q[0] && P.cells[4 * c1 + 1] == q[1] &&
               P.cells[4 * c1 + 2] == q[2] && P.cells[4 * c1 + 3] == P.cells[4 * (c1 - 1) + 3] + 1)
            ++c1;
        const int len = (int)(c1 - c0);
        P.lmax = std::max(P.lmax, len);
        byk[q[2]].push_back(R0Seg{(int32_t)c0, q[0], q[1], q[3] | (std::min(len, 1023) << 10) | (q[2] << 20)});
        c0 = c1;
    }
    P.seg_start.assign(nth + 1, 0);
    for (int k = 0; k < nth; ++k) {
        P.seg_start[k] = (int32_t)P.seg.size();
        P.seg.insert(P.seg.end(), byk[k].begin(), byk[k].end());
    }
    P.seg_start[nth] = (int32_t)P.seg.size();
    P.nseg = (int)P.seg.size();
    // enough coarse blocks to cover the chip (about 2048), 4 rows of runs per block
    const int64_t gx = ((int64_t)nx * ny + 63) / 64;
    const int64_t want = (2048 + gx - 1) / gx;
    P.nsplit = (int)std::max<int64_t>(1, std::min<int64_t>({want, 64, (P.nseg + 3) / 4}));
    return P;
}

// ---- device: one run ------------------------------------------------------------------------
// R(y) of a run of len cells (len <= LM, uniform across the wave): with the face value
// h_t = y_t + sigma_t / 2 and h_{-1} = 0 (no influx at the run's first cell; the ghost
// y_len = y_{len-1} makes the last slope 0, so the last flux is the first-order outflow v0 y):
//   R_t = -(v0/ds)(h_t - h_{t-1}) + (src - k_off y_t).
template <typename T, int LM, int LIM>
__device__ __forceinline__ void run_rhs(const T (&y)[LM], T (&R)[LM], int len, T nv_ds, T src, T k_off) {
    T h[LM];
#pragma unroll
    for (int t = 0; t < LM; ++t) {
        const T left = (t == 0) ? T(0) : y[t > 0 ? t - 1 : 0];
        const T right = (t + 1 < len) ? y[t + 1 < LM ? t + 1 : t] : y[t];
        const T sig = (LIM == 0) ? superbee(y[t] - left, right - y[t]) : T(0);
        h[t] = y[t] + T(0.5) * sig;
    }
#pragma unroll
    for (int t = 0; t < LM; ++t) {
        const T hl = (t == 0) ? T(0) : h[t > 0 ? t - 1 : 0];
        R[t] = nv_ds * (h[t] - hl) + (src - k_off * y[t]);
    }
}

template <typename T, int LM, int LIM>
__global__ __launch_bounds__(256) void k_r0_motor(const T *__restrict__ Min, T *__restrict__ Mout, T *__restrict__ q0,
                                                  T *__restrict__ m0, T *__restrict__ m1,
                                                  const R0Seg *__restrict__ seg, const int32_t *__restrict__ seg_start,
                                                  const T *__restrict__ scale, const T *__restrict__ pool,
                                                  R0Const<T> c) {
    __shared__ double red[2][4][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int k = blockIdx.y;
    const int64_t x = (int64_t)blockIdx.x * 64 + lane;
    const bool act = x < c.nxy;
    const int i = act ? (int)(x / c.ny) : 0;
    const int j = act ? (int)(x - (int64_t)i * c.ny) : 0;
    double a0 = 0.0, a1 = 0.0;
    const int s_end = seg_start[k + 1];
    for (int s = seg_start[k] + w; s < s_end; s += 4) {
        const R0Seg r = seg[s];
        const int lo = r.pack & 1023, len = (r.pack >> 10) & 1023;
        // the anchor of this run at filament cell x: r0 = x - (a, b), periodic (|a| < nx/2)
        int ia = i - r.a, ja = j - r.b;
        ia += ia < 0 ? c.nx : 0;
        ia -= ia >= c.nx ? c.nx : 0;
        ja += ja < 0 ? c.ny : 0;
        ja -= ja >= c.ny ? c.ny : 0;
        T sc = T(1), src = c.k_on;
        if (scale != nullptr && act) {
            const int64_t r0 = (int64_t)ia * c.ny + ja;
            sc = scale[r0];
            src = pool[r0];
        }
        const T *pin = Min + (int64_t)r.off * c.nxy + x;
        T z[LM];
#pragma unroll
        for (int t = 0; t < LM; ++t) z[t] = (t < len && act) ? sc * pin[(int64_t)t * c.nxy] : T(0);
        if (c.advance) {
            T R[LM], y[LM];
            run_rhs<T, LM, LIM>(z, R, len, c.nv_ds, src, c.k_off);
#pragma unroll
            for (int t = 0; t < LM; ++t) y[t] = z[t] + c.half_dt * R[t];
            run_rhs<T, LM, LIM>(y, R, len, c.nv_ds, src, c.k_off);
#pragma unroll
            for (int t = 0; t < LM; ++t) z[t] = z[t] + c.dt * R[t];
            T *pout = Mout + (int64_t)r.off * c.nxy + x;
#pragma unroll
            for (int t = 0; t < LM; ++t)
                if (t < len && act) pout[(int64_t)t * c.nxy] = z[t];
        }
        double t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int t = 0; t < LM; ++t)
            if (t < len) {
                t0 += (double)z[t];
                t1 += ((double)(lo + t) + 0.5 - c.half_ns) * (double)z[t];
            }
        if (act) q0[(int64_t)s * c.nxy + x] = (T)(t0 * c.ds);
        a0 += t0;
        a1 += t1;
    }
    red[0][w][lane] = a0;
    red[1][w][lane] = a1;
    __syncthreads();
    if (w == 0 && act) {
        const double s0 = ((red[0][0][lane] + red[0][1][lane]) + red[0][2][lane]) + red[0][3][lane];
        const double s1 = ((red[1][0][lane] + red[1][1][lane]) + red[1][2][lane]) + red[1][3][lane];
        m0[x * c.nth + k] = (T)(s0 * c.ds * c.dA);
        m1[x * c.nth + k] = (T)(s1 * c.ds2 * c.dA);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_r0_coarse(const T *__restrict__ q0, const T *__restrict__ psi,
                                                   const R0Seg *__restrict__ seg, double *__restrict__ part,
                                                   R0Const<T> c, int nseg, int nrow) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.y * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t r0 = (int64_t)blockIdx.x * 64 + lane;
    const bool act = r0 < c.nxy;
    const int i0 = act ? (int)(r0 / c.ny) : 0;
    const int j0 = act ? (int)(r0 - (int64_t)i0 * c.ny) : 0;
    double acc = 0.0;
    for (int s = row; s < nseg; s += nrow) {
        const R0Seg r = seg[s];
        const int k = r.pack >> 20;
        // the filament cell of this run at anchor r0: x = r0 + (a, b), periodic
        int i = i0 + r.a, j = j0 + r.b;
        i += i < 0 ? c.nx : 0;
        i -= i >= c.nx ? c.nx : 0;
        j += j < 0 ? c.ny : 0;
        j -= j >= c.ny ? c.ny : 0;
        const int64_t x = (int64_t)i * c.ny + j;
        if (act) acc += (double)q0[(int64_t)s * c.nxy + x] * (double)psi[x * c.nth + k];
    }
    if (act) part[(int64_t)row * c.nxy + r0] = acc;
}

// coarse = w sum of the rows (fixed order); Alg. 2 / Eq. (6): where coarse > m_total the
// anchor's factor is m_total / coarse and the pool 0, else 1 and m_total - coarse (pool 1 and
// no factor without depletion).
template <typename T>
__global__ __launch_bounds__(256) void k_r0_pool(const double *__restrict__ part, int nrow, T *__restrict__ scale,
                                                 T *__restrict__ pool, T *__restrict__ coarse_out,
                                                 T *__restrict__ free_out, int64_t nxy, double w, double m_total,
                                                 double k_on) {
    const int64_t r0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r0 >= nxy) return;
    double sum = 0.0;
    for (int r = 0; r < nrow; ++r) sum += part[(int64_t)r * nxy + r0];
    const double B = sum * w;
    double f = 1.0;
    if (m_total > 0) {
        const bool over = B > m_total;
        f = over ? 0.0 : m_total - B;
        if (scale != nullptr) {
            scale[r0] = (T)(over ? m_total / B : 1.0);
            pool[r0] = (T)(k_on * f);
        }
    }
    if (coarse_out != nullptr) coarse_out[r0] = (T)B;
    if (free_out != nullptr) free_out[r0] = (T)f;
}

// ---- launchers --------------------------------------------------------------------------------
template <typename T, int LM>
static hipError_t motor_lm(const T *Min, T *Mout, T *q0, T *m0, T *m1, const R0Seg *seg, const int32_t *ss,
                           const T *scale, const T *pool, const R0Const<T> &c, int limiter, hipStream_t s) {
    const dim3 grid((unsigned)((c.nxy + 63) / 64), (unsigned)c.nth);
    if (limiter == 0)
        hipLaunchKernelGGL((k_r0_motor<T, LM, 0>), grid, dim3(256), 0, s, Min, Mout, q0, m0, m1, seg, ss, scale, pool, c);
    else
        hipLaunchKernelGGL((k_r0_motor<T, LM, 1>), grid, dim3(256), 0, s, Min, Mout, q0, m0, m1, seg, ss, scale, pool, c);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_r0_motor(const T *M_in, T *M_out, T *q0, T *m0, T *m1, const R0Seg *seg, const int32_t *seg_start,
                           const T *scale, const T *pool, const R0Const<T> &c, int lmax, int limiter, hipStream_t s) {
    if (c.nxy <= 0 || c.nth <= 0) return hipSuccess;
    if (lmax <= 8) return motor_lm<T, 8>(M_in, M_out, q0, m0, m1, seg, seg_start, scale, pool, c, limiter, s);
    if (lmax <= 16) return motor_lm<T, 16>(M_in, M_out, q0, m0, m1, seg, seg_start, scale, pool, c, limiter, s);
    if (lmax <= kR0MaxRun) return motor_lm<T, 32>(M_in, M_out, q0, m0, m1, seg, seg_start, scale, pool, c, limiter, s);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_r0_coarse(const T *q0, const T *psi, const R0Seg *seg, double *part, T *scale, T *pool,
                            T *coarse_out, T *free_out, const R0Const<T> &c, int nseg, int nsplit, double dth,
                            double m_total, double k_on, hipStream_t s) {
    if (c.nxy <= 0) return hipSuccess;
    const unsigned gx = (unsigned)((c.nxy + 63) / 64);
    hipLaunchKernelGGL(k_r0_coarse<T>, dim3(gx, (unsigned)nsplit), dim3(256), 0, s, q0, psi, seg, part, c, nseg,
                       4 * nsplit);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double w = c.dA * dth;  // dx dy dth (q0 already carries ds)
    hipLaunchKernelGGL(k_r0_pool<T>, dim3((unsigned)((c.nxy + 255) / 256)), dim3(256), 0, s, part, 4 * nsplit, scale,
                       pool, coarse_out, free_out, c.nxy, w, m_total, k_on);
    return hipGetLastError();
}

template hipError_t launch_r0_motor<float>(const float *, float *, float *, float *, float *, const R0Seg *,
                                           const int32_t *, const float *, const float *, const R0Const<float> &, int,
                                           int, hipStream_t);
template hipError_t launch_r0_motor<double>(const double *, double *, double *, double *, double *, const R0Seg *,
                                            const int32_t *, const double *, const double *, const R0Const<double> &,
                                            int, int, hipStream_t);
template hipError_t launch_r0_coarse<float>(const float *, const float *, const R0Seg *, double *, float *, float *,
                                            float *, float *, const R0Const<float> &, int, int, double, double, double,
                                            hipStream_t);
template hipError_t launch_r0_coarse<double>(const double *, const double *, const R0Seg *, double *, double *,
                                             double *, double *, double *, const R0Const<double> &, int, int, double,
                                             double, double, hipStream_t);

}  // namespace mmk
