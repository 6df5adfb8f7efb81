// Filament-density step for gfx950: conservative donor-cell transport of Psi(x, y, th)
// (Cook & Shinar, Sec. 2, Eqs. (1)-(3)) and, on output steps, the theta-moments and the
// extra stress (extra-stress step of Alg. 1).
//
// Velocities: translational a = u - F m0 p (motor gliding along -p plus the fluid),
// face value the mean of the two cells; rotational p_perp . gradu . p at the theta-faces.
// Forward Euler with first-order upwind fluxes, periodic in x, y and th.
//
// Layout: psi/m0 [nx][ny][nth] with th contiguous.  A block owns a TI x TJ tile of (x, y)
// pencils; the tile plus a one-pencil halo of psi and m0 (the stencil is a cross, corner
// pencils are skipped) is staged in LDS, so every value is read from HBM about once.  A
// group of G lanes (16, 32 or 64) walks one pencil over th; the theta-reductions of the
// output step are shuffles inside that group.  Tiles are banded per XCD so the halo
// re-reads of neighbouring tiles hit the same L2.
#include "device_util.h"
#include "kernels.h"

#include <type_traits>

namespace mmk {

PsiLaunch plan_psi(int nx, int ny, int nth, size_t elem) {
    static const int cand[][2] = {{8, 8}, {4, 8}, {4, 4}, {2, 4}, {2, 2}, {1, 2}, {1, 1}};
    PsiLaunch pl{};
    pl.group = nth <= 16 ? 16 : (nth <= 32 ? 32 : 64);
    for (auto &c : cand) {
        const int ti = c[0], tj = c[1];
        const size_t halo = (size_t)(ti + 2) * (tj + 2);
        const size_t lds = elem * (2 * halo * nth + 2 * halo + 4 * (size_t)ti * tj + TAB_N * (size_t)nth)
                           + 16 + 4 * 4 * sizeof(double);
        pl.ti = ti;
        pl.tj = tj;
        pl.lds_bytes = lds;
        if (lds <= 64 * 1024) break;
    }
    pl.tiles_i = (nx + pl.ti - 1) / pl.ti;
    pl.tiles_j = (ny + pl.tj - 1) / pl.tj;
    const int tiles = pl.tiles_i * pl.tiles_j;
    const int per = (tiles + 7) / 8;
    pl.blocks = 8 * per;
    return pl;
}

template <typename T>
__device__ __forceinline__ T donor(T A, T left, T right) {
    return (A >= T(0)) ? A * left : A * right;
}

template <typename T>
__device__ __forceinline__ T shfl_xor_t(T v, int mask, int width) {
    return __shfl_xor(v, mask, width);
}

// sum over the G lanes of a pencil group (G = 16, 32, 64), result in every lane
template <typename T>
__device__ __forceinline__ T group_total(T v, int G) {
    for (int m = G / 2; m >= 1; m >>= 1) v += shfl_xor_t(v, m, G);
    return v;
}
#pragma clang fp contract(off)
template <typename T>
__device__ __forceinline__ T group_total_comp(CSum<T> c, int G) {
    T s = c.hi, e = c.lo;
    for (int m = G / 2; m >= 1; m >>= 1) {
        const T s2 = shfl_xor_t(s, m, G), e2 = shfl_xor_t(e, m, G);
        T t, err;
        two_sum(s, s2, t, err);
        s = t;
        e = e + e2 + err;
    }
    return s + e;
}
#pragma clang fp contract(on)

template <typename T>
struct Acc;  // theta accumulators: plain in FP64, compensated in FP32
template <>
struct Acc<double> {
    double v = 0;
    __device__ void add(double x) { v += x; }
    __device__ double total(int G) const { return group_total(v, G); }
};
template <>
struct Acc<float> {
    CSum<float> c;
    __device__ void add(float x) { c.add(x); }
    __device__ float total(int G) const { return group_total_comp(c, G); }
};

template <typename T>
__global__ __launch_bounds__(256) void k_psi_step(const T *__restrict__ psi_in, T *__restrict__ psi_out,
                                                  const T *__restrict__ m0, const T *__restrict__ m1,
                                                  const T *__restrict__ u, const T *__restrict__ Gr,
                                                  const T *__restrict__ tab, T *__restrict__ stress,
                                                  T *__restrict__ mom, double *__restrict__ partials,
                                                  PsiConst<T> c, PsiLaunch pl) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = c.nx, ny = c.ny, nth = c.nth;
    const int TI = pl.ti, TJ = pl.tj, HI = TI + 2, HJ = TJ + 2, NH = HI * HJ;
    T *s_psi = reinterpret_cast<T *>(smem);          // [NH][nth]
    T *s_m0 = s_psi + (size_t)NH * nth;               // [NH][nth]
    T *s_u = s_m0 + (size_t)NH * nth;                 // [2][NH]
    T *s_G = s_u + 2 * NH;                            // [4][TI*TJ]
    T *s_tab = s_G + 4 * TI * TJ;                     // [TAB_N][nth]
    const size_t red_off = ((reinterpret_cast<uintptr_t>(s_tab + TAB_N * nth) - reinterpret_cast<uintptr_t>(smem)) + 15) & ~(size_t)15;
    double *s_red = reinterpret_cast<double *>(smem + red_off);  // [4 waves][4]
    const bool out = (stress != nullptr);
    const int tid = threadIdx.x;

    // XCD banding: consecutive block ids go to different XCDs; give each XCD a run of tiles.
    const int per = gridDim.x / 8;
    const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
    const int ntiles = pl.tiles_i * pl.tiles_j;
    if (tile >= ntiles) {
        if (out && tid < 4) partials[(size_t)blockIdx.x * 4 + tid] = 0.0;
        return;
    }
    const int i0 = (tile / pl.tiles_j) * TI, j0 = (tile % pl.tiles_j) * TJ;
    const int64_t nxy = (int64_t)nx * ny;

    const int G = pl.group, NG = 256 / G;
    const int grp = tid / G, kk = tid % G;

    for (int q = grp; q < NH; q += NG) {
        const int qi = q / HJ, qj = q - qi * HJ;
        if ((qi == 0 || qi == HI - 1) && (qj == 0 || qj == HJ - 1)) continue;  // corners unused
        const int gi = (i0 + qi - 1 + nx) % nx, gj = (j0 + qj - 1 + ny) % ny;
        const int64_t pen = (int64_t)gi * ny + gj;
        const T *sp = psi_in + pen * nth;
        const T *sm = m0 + pen * nth;
        for (int k = kk; k < nth; k += G) {
            s_psi[q * nth + k] = sp[k];
            s_m0[q * nth + k] = sm[k];
        }
        if (kk == 0) {
            s_u[q] = u[pen];
            s_u[NH + q] = u[nxy + pen];
        }
    }
    for (int p = tid; p < TI * TJ; p += 256) {
        const int gi = (i0 + p / TJ) % nx, gj = (j0 + p % TJ) % ny;
        const int64_t pen = (int64_t)gi * ny + gj;
#pragma unroll
        for (int a = 0; a < 4; ++a) s_G[a * TI * TJ + p] = Gr[a * nxy + pen];
    }
    for (int k = tid; k < TAB_N * nth; k += 256) s_tab[k] = tab[k];
    __syncthreads();

    const T *t_c = s_tab + TAB_C * nth, *t_s = s_tab + TAB_S * nth;
    const T *t_ch = s_tab + TAB_CH * nth, *t_sh = s_tab + TAB_SH * nth;
    double acc_mass = 0, acc_s0 = 0, acc_s1 = 0, acc_s2 = 0;

    for (int p = grp; p < TI * TJ; p += NG) {
        const int pi = p / TJ, pj = p - pi * TJ;
        const int gi = i0 + pi, gj = j0 + pj;
        if (gi >= nx || gj >= ny) continue;  // partial tile (uniform across the group)
        const int q = (pi + 1) * HJ + (pj + 1);
        const int qxm = q - HJ, qxp = q + HJ, qym = q - 1, qyp = q + 1;
        const T ux_c = s_u[q], ux_m = s_u[qxm], ux_p = s_u[qxp];
        const T uy_c = s_u[NH + q], uy_m = s_u[NH + qym], uy_p = s_u[NH + qyp];
        const T Gxx = s_G[p], Gxy = s_G[TI * TJ + p], Gyx = s_G[2 * TI * TJ + p], Gyy = s_G[3 * TI * TJ + p];
        const int64_t pen = (int64_t)gi * ny + gj;
        Acc<T> a_c, a_nx, a_ny, a_dxx, a_dxy, a_dyy, a_b, a_sxx, a_sxy, a_syy;

        for (int k = kk; k < nth; k += G) {
            const int kp = (k + 1 == nth) ? 0 : k + 1;
            const int km = (k == 0) ? nth - 1 : k - 1;
            const T ps = s_psi[q * nth + k];
            const T co = t_c[k], si = t_s[k];
            const T mc = s_m0[q * nth + k];
            // x faces
            const T ax_c = ux_c - c.F * mc * co;
            const T ax_m = ux_m - c.F * s_m0[qxm * nth + k] * co;
            const T ax_p = ux_p - c.F * s_m0[qxp * nth + k] * co;
            const T Axp = T(0.5) * (ax_c + ax_p), Axm = T(0.5) * (ax_m + ax_c);
            const T fxp = donor(Axp, ps, s_psi[qxp * nth + k]);
            const T fxm = donor(Axm, s_psi[qxm * nth + k], ps);
            // y faces
            const T ay_c = uy_c - c.F * mc * si;
            const T ay_m = uy_m - c.F * s_m0[qym * nth + k] * si;
            const T ay_p = uy_p - c.F * s_m0[qyp * nth + k] * si;
            const T Ayp = T(0.5) * (ay_c + ay_p), Aym = T(0.5) * (ay_m + ay_c);
            const T fyp = donor(Ayp, ps, s_psi[qyp * nth + k]);
            const T fym = donor(Aym, s_psi[qym * nth + k], ps);
            // theta faces k+1/2 and k-1/2 (= (k-1)+1/2)
            const T chp = t_ch[k], shp = t_sh[k], chm = t_ch[km], shm = t_sh[km];
            const T wp = -shp * (Gxx * chp + Gxy * shp) + chp * (Gyx * chp + Gyy * shp);
            const T wm = -shm * (Gxx * chm + Gxy * shm) + chm * (Gyx * chm + Gyy * shm);
            const T ftp = donor(wp, ps, s_psi[q * nth + kp]);
            const T ftm = donor(wm, s_psi[q * nth + km], ps);
            const T div = (fxp - fxm) * c.inv_dx + (fyp - fym) * c.inv_dy + (ftp - ftm) * c.inv_dth;
            const T pn = ps - c.dt * div;
            psi_out[pen * nth + k] = pn;
            if (out) {
                const T mm1 = m1[pen * nth + k];
                const T cc = s_tab[TAB_CC * nth + k], cs = s_tab[TAB_CS * nth + k], ss = s_tab[TAB_SS * nth + k];
                const T h1 = s_tab[TAB_H1 * nth + k], h2 = s_tab[TAB_H2 * nth + k];
                a_c.add(pn);
                a_nx.add(pn * co);
                a_ny.add(pn * si);
                a_dxx.add(pn * cc);
                a_dxy.add(pn * cs);
                a_dyy.add(pn * ss);
                a_b.add(pn * mc);
                const T fm = c.F * mm1;
                a_sxx.add(pn * (c.sigma_f * h1 + fm * cc));
                a_sxy.add(pn * (c.sigma_f * h2 + fm * cs));
                a_syy.add(pn * (-c.sigma_f * h1 + fm * ss));
                acc_mass += (double)pn;
            }
        }
        if (out) {
            const T dth = c.dth;
            const T v0 = a_c.total(G) * dth, v1 = a_nx.total(G) * dth, v2 = a_ny.total(G) * dth;
            const T v3 = a_dxx.total(G) * dth, v4 = a_dxy.total(G) * dth, v5 = a_dyy.total(G) * dth;
            const T v6 = a_b.total(G) * dth;
            const T s0 = a_sxx.total(G) * dth, s1 = a_sxy.total(G) * dth, s2 = a_syy.total(G) * dth;
            if (kk == 0) {
                mom[0 * nxy + pen] = v0;
                mom[1 * nxy + pen] = v1;
                mom[2 * nxy + pen] = v2;
                mom[3 * nxy + pen] = v3;
                mom[4 * nxy + pen] = v4;
                mom[5 * nxy + pen] = v5;
                mom[6 * nxy + pen] = v6;
                stress[0 * nxy + pen] = s0;
                stress[1 * nxy + pen] = s1;
                stress[2 * nxy + pen] = s2;
                acc_s0 += (double)s0;
                acc_s1 += (double)s1;
                acc_s2 += (double)s2;
            }
        }
    }

    if (out) {
        // fixed-order block reduction of the FP64 partials: wave butterfly, then wave 0..3
        double v[4] = {acc_mass, acc_s0, acc_s1, acc_s2};
#pragma unroll
        for (int a = 0; a < 4; ++a)
            for (int m = 32; m >= 1; m >>= 1) v[a] += __shfl_xor(v[a], m, 64);
        const int wave = tid / 64, lane = tid % 64;
        if (lane == 0)
            for (int a = 0; a < 4; ++a) s_red[wave * 4 + a] = v[a];
        __syncthreads();
        if (tid < 4) {
            double s = 0;
            for (int w = 0; w < 4; ++w) s += s_red[w * 4 + tid];
            partials[(size_t)blockIdx.x * 4 + tid] = s;
        }
    }
}

template <typename T>
hipError_t launch_psi_step(const T *psi_in, T *psi_out, const T *m0, const T *m1, const T *u,
                           const T *G, const T *tab, T *stress, T *mom, double *partials,
                           const PsiConst<T> &c, const PsiLaunch &pl, hipStream_t s) {
    hipLaunchKernelGGL(k_psi_step<T>, dim3(pl.blocks), dim3(256), pl.lds_bytes, s, psi_in, psi_out, m0, m1,
                       u, G, tab, stress, mom, partials, c, pl);
    return hipGetLastError();
}

template hipError_t launch_psi_step<float>(const float *, float *, const float *, const float *, const float *,
                                           const float *, const float *, float *, float *, double *,
                                           const PsiConst<float> &, const PsiLaunch &, hipStream_t);
template hipError_t launch_psi_step<double>(const double *, double *, const double *, const double *,
                                            const double *, const double *, const double *, double *, double *,
                                            double *, const PsiConst<double> &, const PsiLaunch &, hipStream_t);

// ---------------------------------------------------------------------------------------
// Deterministic FP64 totals of per-block partials: each thread runs a Neumaier sum over a
// fixed stride, then a fixed pairwise tree with TwoSum error terms.
#pragma clang fp contract(off)
__global__ __launch_bounds__(256) void k_reduce_partials(const double *__restrict__ partials, int n,
                                                          double *__restrict__ out, double s0, double s1) {
    __shared__ double sh[4][256], se[4][256];
    const int t = threadIdx.x;
    for (int a = 0; a < 4; ++a) {
        double s = 0, e = 0;
        for (int i = t; i < n; i += 256) {
            double x = partials[(size_t)i * 4 + a], hi, lo;
            two_sum(s, x, hi, lo);
            s = hi;
            e += lo;
        }
        sh[a][t] = s;
        se[a][t] = e;
    }
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w)
            for (int a = 0; a < 4; ++a) {
                double hi, lo;
                two_sum(sh[a][t], sh[a][t + w], hi, lo);
                sh[a][t] = hi;
                se[a][t] = se[a][t] + se[a][t + w] + lo;
            }
        __syncthreads();
    }
    if (t < 4) out[t] = (sh[t][0] + se[t][0]) * (t == 0 ? s0 : s1);
}
#pragma clang fp contract(on)

hipError_t launch_reduce_partials(const double *partials, int n, double *out, double s0, double s1,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partials, n, out, s0, s1);
    return hipGetLastError();
}

template <typename T>
__global__ void k_zero(T *out, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = T(0);
}

template <typename T>
hipError_t launch_zero(T *out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)blocks), dim3(256), 0, s, out, n);
    return hipGetLastError();
}
template hipError_t launch_zero<float>(float *, int64_t, hipStream_t);
template hipError_t launch_zero<double>(double *, int64_t, hipStream_t);

}  // namespace mmk
