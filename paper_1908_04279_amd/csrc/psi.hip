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
#include "adjoint.h"
#include "psi_dev.h"

#include <cstdio>
#include <type_traits>

namespace mmk {

static size_t psi_lds(int ti, int tj, int nth, size_t elem, int nf) {
    const size_t halo = (size_t)(ti + 2) * (tj + 2);
    return elem * (nf * halo * nth + 2 * halo + 4 * (size_t)ti * tj + TAB_N * (size_t)nth) + 16 + 4 * 4 * sizeof(double);
}

// Tile choice: the largest of the candidate tiles whose LDS footprint stays <= 40 KB (so
// several blocks share a CU), else <= 64 KB, that still gives at least kMinTiles blocks; a grid
// too small for that takes the fitting compiled tile with the most blocks (latency, not
// bandwidth, bounds such grids).
static constexpr int kMinTiles = 1024;
PsiLaunch plan_psi(int nx, int ny, int nth, size_t elem, int nf) {
    static const int cand[][2] = {{8, 8}, {4, 8}, {4, 4}, {2, 4}, {2, 2}, {1, 2}, {1, 1}};
    static const int ncompiled = 4;  // the first four have compile-time kernels
    PsiLaunch pl{};
    pl.group = nth <= 16 ? 16 : (nth <= 32 ? 32 : 64);
    bool chosen = false;
    auto ntiles = [&](int ti, int tj) { return (long)((nx + ti - 1) / ti) * ((ny + tj - 1) / tj); };
    for (size_t limit : {(size_t)40 * 1024, (size_t)64 * 1024}) {
        if (chosen) break;
        int small = -1;  // fitting compiled tile with the most blocks
        for (int i = 0; i < ncompiled; ++i) {
            if (psi_lds(cand[i][0], cand[i][1], nth, elem, nf) > limit) continue;
            if (ntiles(cand[i][0], cand[i][1]) >= kMinTiles) {
                pl.ti = cand[i][0];
                pl.tj = cand[i][1];
                chosen = true;
                break;
            }
            small = i;
        }
        if (!chosen && small >= 0) {
            pl.ti = cand[small][0];
            pl.tj = cand[small][1];
            chosen = true;
        }
        for (auto &c : cand) {
            if (chosen) break;
            if (psi_lds(c[0], c[1], nth, elem, nf) <= limit) {
                pl.ti = c[0];
                pl.tj = c[1];
                chosen = true;
            }
        }
    }
    if (!chosen) {
        pl.ti = 1;
        pl.tj = 1;
    }
    pl.lds_bytes = psi_lds(pl.ti, pl.tj, nth, elem, nf);
    pl.tiles_i = (nx + pl.ti - 1) / pl.ti;
    pl.tiles_j = (ny + pl.tj - 1) / pl.tj;
    const int tiles = pl.tiles_i * pl.tiles_j;
    const int per = (tiles + 7) / 8;
    pl.blocks = 8 * per;
    return pl;
}

// Per-lane constants of one orientation k: p, the two theta faces and the moment weights.
template <typename T>
struct AngleK {
    T co, si, chp, shp, chm, shm, h1, h2, cc, cs, ss;
    int k, kp, km;
};

template <typename T>
__device__ __forceinline__ AngleK<T> angle_k(const T *s_tab, int nth, int k) {
    AngleK<T> a;
    a.k = k;
    a.kp = (k + 1 == nth) ? 0 : k + 1;
    a.km = (k == 0) ? nth - 1 : k - 1;
    a.co = s_tab[TAB_C * nth + k];
    a.si = s_tab[TAB_S * nth + k];
    a.chp = s_tab[TAB_CH * nth + k];
    a.shp = s_tab[TAB_SH * nth + k];
    a.chm = s_tab[TAB_CH * nth + a.km];
    a.shm = s_tab[TAB_SH * nth + a.km];
    a.h1 = s_tab[TAB_H1 * nth + k];
    a.h2 = s_tab[TAB_H2 * nth + k];
    a.cc = s_tab[TAB_CC * nth + k];
    a.cs = s_tab[TAB_CS * nth + k];
    a.ss = s_tab[TAB_SS * nth + k];
    return a;
}

// Stages NF fields of a TI x TJ tile plus its one-pencil halo (cross stencil: corner pencils
// skipped) into LDS (field f at s_f + f * NH * nth), with u of the halo, gradu of the tile and
// the angle tables.  NTH_C, TI_C, TJ_C > 0 fix ntheta and the tile at compile time: then every
// global load of the phase is issued before the first LDS write, so the in-order vmcnt waits
// never serialise them; 0 takes them from the launch arguments (any ntheta).
template <typename T, int NTH_C, int TI_C, int TJ_C, int NF>
__device__ __forceinline__ void stage_tile(const T *const (&src)[NF], T *s_f, T *s_u, T *s_G, T *s_tab,
                                           const T *__restrict__ u, const T *__restrict__ Gr,
                                           const T *__restrict__ tab, int i0, int j0, int nx, int ny, int nth,
                                           int TI, int TJ, int G, int grp, int kk, int tid) {
    constexpr bool FIXED = NTH_C > 0 && TI_C > 0 && TJ_C > 0;
    const int HI = TI + 2, HJ = TJ + 2, NH = HI * HJ, NG = 256 / G;
    const int64_t nxy = (int64_t)nx * ny;
    if constexpr (FIXED) {
        constexpr int G_ = NTH_C <= 16 ? 16 : (NTH_C <= 32 ? 32 : 64);
        constexpr int NG_ = 256 / G_, KPL = (NTH_C + G_ - 1) / G_;
        constexpr int HJ_ = TJ_C + 2, NH_ = (TI_C + 2) * HJ_, NP_ = TI_C * TJ_C;
        constexpr int NQ = (NH_ + NG_ - 1) / NG_;
        constexpr int NT = (TAB_N * NTH_C + 255) / 256;
        static_assert(NH_ <= 256 && NP_ <= 256, "tile too large for one pass");
        if constexpr (G_ == 64) {
            // one wave per pencil: wave grp takes halo rows grp, grp+4, ...; the wrapped column
            // index of each pencil of a row is computed once per wave (uniform, scalar)
            constexpr int HI_ = TI_C + 2, NR = (HI_ + 3) / 4;
            int gj[HJ_];
#pragma unroll
            for (int qj = 0; qj < HJ_; ++qj) gj[qj] = wrap(j0 + qj - 1, ny);
            T r[NF][NR][HJ_][KPL];
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                const int qi = grp + 4 * rr;
                const int64_t row = (int64_t)wrap(i0 + qi - 1, nx) * ny;
#pragma unroll
                for (int qj = 0; qj < HJ_; ++qj) {
                    const bool ok = qi < HI_ && !((qi == 0 || qi == HI_ - 1) && (qj == 0 || qj == HJ_ - 1));
                    const int64_t pen = row + gj[qj];
#pragma unroll
                    for (int j = 0; j < KPL; ++j) {
                        const int k = kk + j * 64;
                        if (ok && k < NTH_C)
#pragma unroll
                            for (int f = 0; f < NF; ++f) r[f][rr][qj][j] = src[f][pen * NTH_C + k];
                    }
                }
            }
            T ru0 = 0, ru1 = 0, rg[4] = {0, 0, 0, 0}, rt[NT];
            if (tid < NH_) {
                const int qi = tid / HJ_, qj = tid - qi * HJ_;
                const int64_t pen = (int64_t)wrap(i0 + qi - 1, nx) * ny + wrap(j0 + qj - 1, ny);
                ru0 = u[pen];
                ru1 = u[nxy + pen];
            }
            if (tid < NP_) {
                const int64_t pen = (int64_t)wrap(i0 + tid / TJ_C, nx) * ny + wrap(j0 + tid % TJ_C, ny);
#pragma unroll
                for (int a = 0; a < 4; ++a) rg[a] = Gr[a * nxy + pen];
            }
#pragma unroll
            for (int v = 0; v < NT; ++v)
                if (tid + 256 * v < TAB_N * NTH_C) rt[v] = tab[tid + 256 * v];
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                const int qi = grp + 4 * rr;
#pragma unroll
                for (int qj = 0; qj < HJ_; ++qj) {
                    const bool ok = qi < HI_ && !((qi == 0 || qi == HI_ - 1) && (qj == 0 || qj == HJ_ - 1));
                    const int q = qi * HJ_ + qj;
#pragma unroll
                    for (int j = 0; j < KPL; ++j) {
                        const int k = kk + j * 64;
                        if (ok && k < NTH_C)
#pragma unroll
                            for (int f = 0; f < NF; ++f) s_f[(size_t)f * NH_ * NTH_C + q * NTH_C + k] = r[f][rr][qj][j];
                    }
                }
            }
            if (tid < NH_) {
                s_u[tid] = ru0;
                s_u[NH_ + tid] = ru1;
            }
            if (tid < NP_)
#pragma unroll
                for (int a = 0; a < 4; ++a) s_G[a * NP_ + tid] = rg[a];
#pragma unroll
            for (int v = 0; v < NT; ++v)
                if (tid + 256 * v < TAB_N * NTH_C) s_tab[tid + 256 * v] = rt[v];
            return;
        }
        T r[NF][NQ][KPL];
        int dst[NQ];
#pragma unroll
        for (int v = 0; v < NQ; ++v) {
            const int q = grp + v * NG_;
            const int qi = q / HJ_, qj = q - qi * HJ_;
            const bool ok = q < NH_ && !((qi == 0 || qi == TI_C + 1) && (qj == 0 || qj == TJ_C + 1));
            dst[v] = ok ? q : -1;
            const int64_t pen = (int64_t)wrap(i0 + qi - 1, nx) * ny + wrap(j0 + qj - 1, ny);
#pragma unroll
            for (int j = 0; j < KPL; ++j) {
                const int k = kk + j * G_;
                if (ok && k < NTH_C)
#pragma unroll
                    for (int f = 0; f < NF; ++f) r[f][v][j] = src[f][pen * NTH_C + k];
            }
        }
        T ru0 = 0, ru1 = 0, rg[4] = {0, 0, 0, 0}, rt[NT];
        if (tid < NH_) {
            const int qi = tid / HJ_, qj = tid - qi * HJ_;
            const int64_t pen = (int64_t)wrap(i0 + qi - 1, nx) * ny + wrap(j0 + qj - 1, ny);
            ru0 = u[pen];
            ru1 = u[nxy + pen];
        }
        if (tid < NP_) {
            const int64_t pen = (int64_t)wrap(i0 + tid / TJ_C, nx) * ny + wrap(j0 + tid % TJ_C, ny);
#pragma unroll
            for (int a = 0; a < 4; ++a) rg[a] = Gr[a * nxy + pen];
        }
#pragma unroll
        for (int v = 0; v < NT; ++v)
            if (tid + 256 * v < TAB_N * NTH_C) rt[v] = tab[tid + 256 * v];
#pragma unroll
        for (int v = 0; v < NQ; ++v) {
#pragma unroll
            for (int j = 0; j < KPL; ++j) {
                const int k = kk + j * G_;
                if (dst[v] >= 0 && k < NTH_C)
#pragma unroll
                    for (int f = 0; f < NF; ++f) s_f[(size_t)f * NH_ * NTH_C + dst[v] * NTH_C + k] = r[f][v][j];
            }
        }
        if (tid < NH_) {
            s_u[tid] = ru0;
            s_u[NH_ + tid] = ru1;
        }
        if (tid < NP_)
#pragma unroll
            for (int a = 0; a < 4; ++a) s_G[a * NP_ + tid] = rg[a];
#pragma unroll
        for (int v = 0; v < NT; ++v)
            if (tid + 256 * v < TAB_N * NTH_C) s_tab[tid + 256 * v] = rt[v];
    } else {
        for (int q = grp; q < NH; q += NG) {
            const int qi = q / HJ, qj = q - qi * HJ;
            if ((qi == 0 || qi == HI - 1) && (qj == 0 || qj == HJ - 1)) continue;
            const int64_t pen = (int64_t)wrap(i0 + qi - 1, nx) * ny + wrap(j0 + qj - 1, ny);
            for (int k = kk; k < nth; k += G)
                for (int f = 0; f < NF; ++f) s_f[(size_t)f * NH * nth + q * nth + k] = src[f][pen * nth + k];
            if (kk == 0) {
                s_u[q] = u[pen];
                s_u[NH + q] = u[nxy + pen];
            }
        }
        for (int p = tid; p < TI * TJ; p += 256) {
            const int64_t pen = (int64_t)wrap(i0 + p / TJ, nx) * ny + wrap(j0 + p % TJ, ny);
#pragma unroll
            for (int a = 0; a < 4; ++a) s_G[a * TI * TJ + p] = Gr[a * nxy + pen];
        }
        for (int k = tid; k < TAB_N * nth; k += 256) s_tab[k] = tab[k];
    }
}

template <typename T, int NTH_C, int TI_C, int TJ_C>
__global__ __launch_bounds__(256) void k_psi_step(const T *__restrict__ psi_in, T *__restrict__ psi_out,
                                                  const T *__restrict__ m0, const T *__restrict__ m1,
                                                  const T *__restrict__ u, const T *__restrict__ Gr,
                                                  const T *__restrict__ tab, T *__restrict__ stress,
                                                  T *__restrict__ mom, double *__restrict__ partials,
                                                  T *__restrict__ Dxy, PsiConst<T> c, PsiLaunch pl) {
    constexpr bool FIXED = NTH_C > 0 && TI_C > 0 && TJ_C > 0;
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = c.nx, ny = c.ny;
    const int nth = NTH_C ? NTH_C : c.nth;
    const int TI = TI_C ? TI_C : pl.ti, TJ = TJ_C ? TJ_C : pl.tj;
    const int HJ = TJ + 2, NH = (TI + 2) * HJ;
    const int G = NTH_C ? (NTH_C <= 16 ? 16 : (NTH_C <= 32 ? 32 : 64)) : pl.group;
    const int NG = 256 / G;
    T *s_psi = reinterpret_cast<T *>(smem);          // [NH][nth]
    T *s_m0 = s_psi + (size_t)NH * nth;               // [NH][nth]
    T *s_u = s_m0 + (size_t)NH * nth;                 // [2][NH]
    T *s_G = s_u + 2 * NH;                            // [4][TI*TJ]
    T *s_tab = s_G + 4 * TI * TJ;                     // [TAB_N][nth]
    const size_t red_off =
        ((reinterpret_cast<uintptr_t>(s_tab + TAB_N * nth) - reinterpret_cast<uintptr_t>(smem)) + 15) & ~(size_t)15;
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
    // With G = 64 a pencil group is exactly one wave: its pencil index is wave-uniform, so it
    // goes to a scalar register and the per-pencil address arithmetic runs on the SALU.
    const int grp = (G == 64) ? __builtin_amdgcn_readfirstlane(tid / 64) : tid / G;
    const int kk = tid % G;

    const T *const srcs[2] = {psi_in, m0};
    stage_tile<T, NTH_C, TI_C, TJ_C, 2>(srcs, s_psi, s_u, s_G, s_tab, u, Gr, tab, i0, j0, nx, ny, nth, TI, TJ, G,
                                        grp, kk, tid);
    __syncthreads();

    // ---- donor-cell update, one pencil per lane group, th over the group's lanes ----
    constexpr int KMAX = NTH_C ? (NTH_C + 63) / 64 : 0;  // k slots per lane when fixed
    AngleK<T> ak[KMAX > 0 ? KMAX : 1];
    if constexpr (FIXED) {
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
            const int k = kk + j * G;
            if (k < nth) ak[j] = angle_k(s_tab, nth, k);
        }
    }
    // FP64 block partials: mass on every lane; each stress component on the lanes that hold it
    double acc_mass = 0, acc_sig = 0;
    int lane_q = -1;
    constexpr bool COMP = std::is_same<T, float>::value;
    const int lane = tid % 64;

    // WALK (one wave per pencil): wave grp takes TJ/4 tile columns and walks each along x, so
    // the flux through a pencil's upper x-face is carried into the next pencil as its lower
    // x-face flux (the same value the next pencil would compute: the face velocity is the
    // symmetric mean of the two cells).  With 64 orientations the lower theta-face flux of
    // lane k is lane k-1's upper one, taken with a wave rotate.
    constexpr bool WALK = FIXED && NTH_C >= 64 && (TJ_C % 4 == 0);
    constexpr bool THROT = WALK && NTH_C == 64;
    T fx_carry[KMAX > 0 ? KMAX : 1];
    const int n_iter = WALK ? (TI * TJ) / 4 : (TI * TJ + NG - 1) / NG;
    for (int it = 0; it < n_iter; ++it) {
        int pi, pj;
        if constexpr (WALK) {
            pi = it % TI_C;
            pj = grp * (TJ_C / 4) + it / TI_C;
        } else {
            const int p = grp + it * NG;
            if (p >= TI * TJ) break;
            pi = p / TJ;
            pj = p - pi * TJ;
        }
        const int p = pi * TJ + pj;
        const int gi = i0 + pi, gj = j0 + pj;
        if (gi >= nx || gj >= ny) continue;  // partial tile (uniform across the group)
        const bool carried = WALK && pi > 0;
        const int q = (pi + 1) * HJ + (pj + 1);
        const int qxm = q - HJ, qxp = q + HJ, qym = q - 1, qyp = q + 1;
        const T ux_c = s_u[q], ux_m = s_u[qxm], ux_p = s_u[qxp];
        const T uy_c = s_u[NH + q], uy_m = s_u[NH + qym], uy_p = s_u[NH + qyp];
        const T Gxx = s_G[p], Gxy = s_G[TI * TJ + p], Gyx = s_G[2 * TI * TJ + p], Gyy = s_G[3 * TI * TJ + p];
        const int64_t pen = (int64_t)gi * ny + gj;
        T ms[NMOM], me[NMOM];  // this lane's theta partial sums of the moments (output steps)
#pragma unroll
        for (int m = 0; m < NMOM; ++m) ms[m] = me[m] = T(0);
        T bs = T(0), bc = T(0);  // coarse bound density: sum psi_out m0 over this lane

        auto cell = [&](const AngleK<T> &a, int slot, bool first) {
            const int k = a.k;
            const T ps = s_psi[q * nth + k];
            const T mc = s_m0[q * nth + k];
            // x faces: cell velocity u_x - F m0 cos th, face value the mean of the two cells
            const T ax_c = ux_c - c.F * mc * a.co;
            const T ax_p = ux_p - c.F * s_m0[qxp * nth + k] * a.co;
            const T Axp = T(0.5) * (ax_c + ax_p);
            const T fxp = donor(Axp, ps, s_psi[qxp * nth + k]);
            T fxm;
            if (carried) {
                fxm = fx_carry[slot];
            } else {
                const T ax_m = ux_m - c.F * s_m0[qxm * nth + k] * a.co;
                const T Axm = T(0.5) * (ax_m + ax_c);
                fxm = donor(Axm, s_psi[qxm * nth + k], ps);
            }
            if constexpr (WALK) fx_carry[slot] = fxp;
            // y faces
            const T ay_c = uy_c - c.F * mc * a.si;
            const T ay_m = uy_m - c.F * s_m0[qym * nth + k] * a.si;
            const T ay_p = uy_p - c.F * s_m0[qyp * nth + k] * a.si;
            const T Ayp = T(0.5) * (ay_c + ay_p), Aym = T(0.5) * (ay_m + ay_c);
            const T fyp = donor(Ayp, ps, s_psi[qyp * nth + k]);
            const T fym = donor(Aym, s_psi[qym * nth + k], ps);
            // theta faces k+1/2 and k-1/2: rotation rate p_perp . gradu . p
            const T wp = -a.shp * (Gxx * a.chp + Gxy * a.shp) + a.chp * (Gyx * a.chp + Gyy * a.shp);
            const T ftp = donor(wp, ps, s_psi[q * nth + a.kp]);
            T ftm;
            if constexpr (THROT) {
                ftm = dpp_any<DPP_WAVE_ROR1>(ftp);  // lane k-1 (lane 63 for k = 0)
            } else {
                const T wm = -a.shm * (Gxx * a.chm + Gxy * a.shm) + a.chm * (Gyx * a.chm + Gyy * a.shm);
                ftm = donor(wm, s_psi[q * nth + a.km], ps);
            }
            const T div = (fxp - fxm) * c.inv_dx + (fyp - fym) * c.inv_dy + (ftp - ftm) * c.inv_dth;
            const T pn = ps - c.dt * div;
            psi_out[pen * nth + k] = pn;
            if (Dxy) {
                if (first) bs = pn * mc;
                else kahan_add(bs, bc, pn * mc);
            }
            if (out) {
                const T fm = c.F * m1[pen * nth + k];
                const T terms[NMOM] = {pn,
                                       pn * a.co,
                                       pn * a.si,
                                       pn * a.cc,
                                       pn * a.cs,
                                       pn * a.ss,
                                       pn * mc,
                                       pn * (c.sigma_f * a.h1 + fm * a.cc),
                                       pn * (c.sigma_f * a.h2 + fm * a.cs),
                                       pn * (-c.sigma_f * a.h1 + fm * a.ss)};
#pragma unroll
                for (int m = 0; m < NMOM; ++m) mom_add<COMP>(ms[m], me[m], terms[m], first);
                acc_mass += (double)pn;
            }
        };
        if constexpr (FIXED) {
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (kk + j * G < nth) cell(ak[j], j, j == 0);
        } else {
            for (int k = kk; k < nth; k += G) cell(angle_k(s_tab, nth, k), 0, k == kk);
        }
        if (Dxy) {
            T tb;
            if constexpr (FIXED) {
                tb = pencil_total<(NTH_C <= 16 ? 16 : (NTH_C <= 32 ? 32 : 64))>(bs, bc);
            } else if (G == 64) {
                tb = pencil_total<64>(bs, bc);
            } else if (G == 32) {
                tb = pencil_total<32>(bs, bc);
            } else {
                tb = pencil_total<16>(bs, bc);
            }
            if (kk == 0) {
                T sc, pool;
                depletion_of(tb * c.dth, c.m_total, sc, pool);
                Dxy[2 * pen] = sc;
                Dxy[2 * pen + 1] = pool;
            }
        }
        if (out) {
            // one lane per quantity stores its total (moments 0..6, stress 7..9)
            int qm;
            T tot;
            if constexpr (FIXED) {
                tot = group_moments<(NTH_C <= 16 ? 16 : (NTH_C <= 32 ? 32 : 64)), COMP, KMAX == 1>(ms, me, lane, qm);
            } else if (G == 64) {
                tot = group_moments<64, COMP, false>(ms, me, lane, qm);
            } else if (G == 32) {
                tot = group_moments<32, COMP, false>(ms, me, lane, qm);
            } else {
                tot = group_moments<16, COMP, false>(ms, me, lane, qm);
            }
            if (qm >= 0) {
                const T v = tot * c.dth;
                if (qm < 7) {
                    mom[qm * nxy + pen] = v;
                } else {
                    stress[(qm - 7) * nxy + pen] = v;
                    acc_sig += (double)v;
                }
                lane_q = qm;
            }
        }
    }

    if (out) {
        // fixed-order block reduction of the FP64 partials: wave butterfly, then waves 0..3
        double v[4] = {acc_mass, lane_q == 7 ? acc_sig : 0.0, lane_q == 8 ? acc_sig : 0.0,
                       lane_q == 9 ? acc_sig : 0.0};
#pragma unroll
        for (int a = 0; a < 4; ++a)
            for (int m = 32; m >= 1; m >>= 1) v[a] += __shfl_xor(v[a], m, 64);
        const int wave = tid / 64, lane = tid % 64;
        if (lane == 0)
            for (int a = 0; a < 4; ++a) s_red[wave * 4 + a] = v[a];
        __syncthreads();
        if (tid < 4) {
            double sum = 0;
            for (int w = 0; w < 4; ++w) sum += s_red[w * 4 + tid];
            partials[(size_t)blockIdx.x * 4 + tid] = sum;
        }
    }
}

template <typename T, int NTH, int TI, int TJ>
static void launch_fixed(const T *psi_in, T *psi_out, const T *m0, const T *m1, const T *u, const T *G,
                         const T *tab, T *stress, T *mom, double *partials, T *Dxy, const PsiConst<T> &c,
                         const PsiLaunch &pl, hipStream_t s) {
    hipLaunchKernelGGL((k_psi_step<T, NTH, TI, TJ>), dim3(pl.blocks), dim3(256), pl.lds_bytes, s, psi_in,
                       psi_out, m0, m1, u, G, tab, stress, mom, partials, Dxy, c, pl);
}

template <typename T>
hipError_t launch_psi_step(const T *psi_in, T *psi_out, const T *m0, const T *m1, const T *u,
                           const T *G, const T *tab, T *stress, T *mom, double *partials, T *Dxy,
                           const PsiConst<T> &c, const PsiLaunch &pl, hipStream_t s) {
#define MMK_PSI_CASE(N, A, B)                                                                             \
    if (c.nth == N && pl.ti == A && pl.tj == B) {                                                         \
        launch_fixed<T, N, A, B>(psi_in, psi_out, m0, m1, u, G, tab, stress, mom, partials, Dxy, c, pl, s); \
        return hipGetLastError();                                                                    \
    }
#define MMK_PSI_TILES(N) MMK_PSI_CASE(N, 8, 8) MMK_PSI_CASE(N, 4, 8) MMK_PSI_CASE(N, 4, 4) MMK_PSI_CASE(N, 2, 4)
    MMK_PSI_TILES(16)
    MMK_PSI_TILES(32)
    MMK_PSI_TILES(64)
    MMK_PSI_TILES(128)
#undef MMK_PSI_TILES
#undef MMK_PSI_CASE
    hipLaunchKernelGGL((k_psi_step<T, 0, 0, 0>), dim3(pl.blocks), dim3(256), pl.lds_bytes, s, psi_in, psi_out,
                       m0, m1, u, G, tab, stress, mom, partials, Dxy, c, pl);
    return hipGetLastError();
}

template hipError_t launch_psi_step<float>(const float *, float *, const float *, const float *, const float *,
                                           const float *, const float *, float *, float *, double *, float *,
                                           const PsiConst<float> &, const PsiLaunch &, hipStream_t);
template hipError_t launch_psi_step<double>(const double *, double *, const double *, const double *,
                                            const double *, const double *, const double *, double *, double *,
                                            double *, double *, const PsiConst<double> &, const PsiLaunch &,
                                            hipStream_t);

// ---------------------------------------------------------------------------------------
// Reverse of the donor-cell step.  LDS tile of lam', psi and m0 with the same halo.
//   mu_face = dt/h (lam'_right - lam'_left)
//   lam_psi_c = lam'_c + sum over c's faces of mu * (upwind weight of psi_c)
//   dL/dA = mu * (A >= 0 ? psi_left : psi_right);  A_{i+1/2} = (a_i + a_{i+1}) / 2,
//   a = u - F m0 p  =>  lam_m0_c = -(F/2) [cos th (gAx+ + gAx-) + sin th (gAy+ + gAy-)].
template <typename T, int NTH_C, int TI_C, int TJ_C>
__global__ __launch_bounds__(256) void k_psi_reverse(const T *__restrict__ lam_in, const T *__restrict__ psi,
                                                     const T *__restrict__ m0, const T *__restrict__ u,
                                                     const T *__restrict__ Gr, const T *__restrict__ tab,
                                                     T *__restrict__ lam_out, T *__restrict__ lam_m0,
                                                     int accumulate_m0, PsiConst<T> c, PsiLaunch pl) {
    constexpr bool FIXED = NTH_C > 0 && TI_C > 0 && TJ_C > 0;
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = c.nx, ny = c.ny;
    const int nth = NTH_C ? NTH_C : c.nth;
    const int TI = TI_C ? TI_C : pl.ti, TJ = TJ_C ? TJ_C : pl.tj;
    const int HJ = TJ + 2, NH = (TI + 2) * HJ;
    const int G = NTH_C ? (NTH_C <= 16 ? 16 : (NTH_C <= 32 ? 32 : 64)) : pl.group;
    const int NG = 256 / G;
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
    const int grp = (G == 64) ? __builtin_amdgcn_readfirstlane(tid / 64) : tid / G;
    const int kk = tid % G;
    const T *const srcs[3] = {lam_in, psi, m0};
    stage_tile<T, NTH_C, TI_C, TJ_C, 3>(srcs, s_lam, s_u, s_G, s_tab, u, Gr, tab, i0, j0, nx, ny, nth, TI, TJ, G,
                                        grp, kk, tid);
    __syncthreads();

    constexpr int KMAX = NTH_C ? (NTH_C + 63) / 64 : 0;
    AngleK<T> ak[KMAX > 0 ? KMAX : 1];
    if constexpr (FIXED) {
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
            const int k = kk + j * G;
            if (k < nth) ak[j] = angle_k(s_tab, nth, k);
        }
    }
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
        auto cell = [&](const AngleK<T> &a) {
            const int k = a.k;
            const T ps = s_psi[q * nth + k], lc = s_lam[q * nth + k], mc = s_m0[q * nth + k];
            // face velocities, as in the forward step
            const T ax_c = ux_c - c.F * mc * a.co;
            const T ax_m = ux_m - c.F * s_m0[qxm * nth + k] * a.co;
            const T ax_p = ux_p - c.F * s_m0[qxp * nth + k] * a.co;
            const T Axp = T(0.5) * (ax_c + ax_p), Axm = T(0.5) * (ax_m + ax_c);
            const T ay_c = uy_c - c.F * mc * a.si;
            const T ay_m = uy_m - c.F * s_m0[qym * nth + k] * a.si;
            const T ay_p = uy_p - c.F * s_m0[qyp * nth + k] * a.si;
            const T Ayp = T(0.5) * (ay_c + ay_p), Aym = T(0.5) * (ay_m + ay_c);
            const T wp = -a.shp * (Gxx * a.chp + Gxy * a.shp) + a.chp * (Gyx * a.chp + Gyy * a.shp);
            const T wm = -a.shm * (Gxx * a.chm + Gxy * a.shm) + a.chm * (Gyx * a.chm + Gyy * a.shm);
            // face cotangents
            const T mxp = hx * (s_lam[qxp * nth + k] - lc), mxm = hx * (lc - s_lam[qxm * nth + k]);
            const T myp = hy * (s_lam[qyp * nth + k] - lc), mym = hy * (lc - s_lam[qym * nth + k]);
            const T mtp = ht * (s_lam[q * nth + a.kp] - lc), mtm = ht * (lc - s_lam[q * nth + a.km]);
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
            T lm = -T(0.5) * c.F * (a.co * (gAxp + gAxm) + a.si * (gAyp + gAym));
            if (accumulate_m0) lm += lam_m0[pen * nth + k];
            lam_m0[pen * nth + k] = lm;
        };
        if constexpr (FIXED) {
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (kk + j * G < nth) cell(ak[j]);
        } else {
            for (int k = kk; k < nth; k += G) cell(angle_k(s_tab, nth, k));
        }
    }
}

template <typename T>
hipError_t launch_psi_reverse(const T *lam_in, const T *psi, const T *m0, const T *u, const T *G, const T *tab,
                              T *lam_out, T *lam_m0, bool accumulate_m0, const PsiConst<T> &c, const PsiLaunch &pl,
                              hipStream_t s) {
    const int acc = accumulate_m0 ? 1 : 0;
#define MMK_REVPSI_CASE(N, A, B)                                                                           \
    if (c.nth == N && pl.ti == A && pl.tj == B) {                                                          \
        hipLaunchKernelGGL((k_psi_reverse<T, N, A, B>), dim3(pl.blocks), dim3(256), pl.lds_bytes, s, lam_in, \
                           psi, m0, u, G, tab, lam_out, lam_m0, acc, c, pl);                               \
        return hipGetLastError();                                                                          \
    }
#define MMK_REVPSI_TILES(N) MMK_REVPSI_CASE(N, 8, 8) MMK_REVPSI_CASE(N, 4, 8) MMK_REVPSI_CASE(N, 4, 4) MMK_REVPSI_CASE(N, 2, 4)
    MMK_REVPSI_TILES(16)
    MMK_REVPSI_TILES(32)
    MMK_REVPSI_TILES(64)
    MMK_REVPSI_TILES(128)
#undef MMK_REVPSI_TILES
#undef MMK_REVPSI_CASE
    hipLaunchKernelGGL((k_psi_reverse<T, 0, 0, 0>), dim3(pl.blocks), dim3(256), pl.lds_bytes, s, lam_in, psi, m0, u,
                       G, tab, lam_out, lam_m0, acc, c, pl);
    return hipGetLastError();
}
template hipError_t launch_psi_reverse<float>(const float *, const float *, const float *, const float *,
                                              const float *, const float *, float *, float *, bool,
                                              const PsiConst<float> &, const PsiLaunch &, hipStream_t);
template hipError_t launch_psi_reverse<double>(const double *, const double *, const double *, const double *,
                                               const double *, const double *, double *, double *, bool,
                                               const PsiConst<double> &, const PsiLaunch &, hipStream_t);

// ---------------------------------------------------------------------------------------
// Deterministic FP64 totals of per-block partials: each thread runs a Neumaier sum over a
// fixed stride, then a fixed pairwise tree with TwoSum error terms.
#pragma clang fp contract(off)
__global__ __launch_bounds__(256) void k_reduce_partials(const double *__restrict__ partials, int n,
                                                          double *__restrict__ out, double s0, double s1) {
    // thread t takes rows t, t + 256, ... (four independent compensated chains per thread),
    // then a fixed-order TwoSum tree over the threads: the same bits on every run
    __shared__ double sh[4][256], se[4][256];
    const int t = threadIdx.x;
    double s[4] = {0, 0, 0, 0}, e[4] = {0, 0, 0, 0};
    for (int i = t; i < n; i += 256) {
        const double2 x01 = reinterpret_cast<const double2 *>(partials)[(size_t)i * 2];
        const double2 x23 = reinterpret_cast<const double2 *>(partials)[(size_t)i * 2 + 1];
        const double x[4] = {x01.x, x01.y, x23.x, x23.y};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            double hi, lo;
            two_sum(s[a], x[a], hi, lo);
            s[a] = hi;
            e[a] += lo;
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        sh[a][t] = s[a];
        se[a][t] = e[a];
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

// Coarse bound density of a state (start of a depleted run): one block per (x, y) point sums
// psi[th] M[th][s] over the point's nth * ns cells, Kahan per thread and a TwoSum tree over
// the block, times ds dth; stores depletion_of() of it.
#pragma clang fp contract(off)
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_bound(const T *__restrict__ M, const T *__restrict__ psi,
                                                      T *__restrict__ Dxy, int64_t nxy, int nth, int ns, T ds,
                                                      T dth, T m_total) {
    __shared__ T sh[256], se[256];
    const int t = threadIdx.x;
    const int64_t n = (int64_t)nth * ns;
    for (int64_t xy = blockIdx.x; xy < nxy; xy += gridDim.x) {
        T s = 0, cmp = 0;
        if (M)
            for (int64_t i = t; i < n; i += 256) kahan_add(s, cmp, psi[xy * nth + i / ns] * M[xy * n + i]);
        sh[t] = s;
        se[t] = -cmp;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (t < w) {
                T hi, lo;
                two_sum(sh[t], sh[t + w], hi, lo);
                sh[t] = hi;
                se[t] = se[t] + se[t + w] + lo;
            }
            __syncthreads();
        }
        if (t == 0) {
            T sc, pool;
            depletion_of((sh[0] + se[0]) * ds * dth, m_total, sc, pool);
            Dxy[2 * xy] = sc;
            Dxy[2 * xy + 1] = pool;
        }
        __syncthreads();
    }
}
#pragma clang fp contract(on)

template <typename T>
hipError_t launch_coarse_bound(const T *M, const T *psi, T *Dxy, int64_t nxy, int nth, int ns, T ds, T dth,
                               T m_total, hipStream_t s) {
    if (nxy <= 0) return hipSuccess;
    const int64_t blocks = nxy < 65536 ? nxy : 65536;
    hipLaunchKernelGGL(k_coarse_bound<T>, dim3((unsigned)blocks), dim3(256), 0, s, M, psi, Dxy, nxy, nth, ns, ds,
                       dth, m_total);
    return hipGetLastError();
}
template hipError_t launch_coarse_bound<float>(const float *, const float *, float *, int64_t, int, int, float,
                                               float, float, hipStream_t);
template hipError_t launch_coarse_bound<double>(const double *, const double *, double *, int64_t, int, int,
                                                double, double, double, hipStream_t);

// Depletion factors (clamp factor, free pool) per (x, y) from psi and the s-moment m0 of the
// current motor state: B = dth sum_th psi m0 (Eq. (5) in the anchor-marginal reading), one wave
// per point, compensated in FP32.  Used between the sub-steps of a depleted micro-step.
template <typename T>
__global__ __launch_bounds__(256) void k_depletion_m0(const T *__restrict__ psi, const T *__restrict__ m0,
                                                      T *__restrict__ Dxy, int64_t nxy, int nth, T dth, T m_total) {
    const int lane = threadIdx.x & 63;
    const int64_t xy = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (xy >= nxy) return;  // the whole wave
    T s = T(0), cmp = T(0);
    for (int k = lane; k < nth; k += 64) {
        const T v = psi[xy * nth + k] * m0[xy * nth + k];
        if (k == lane) s = v;
        else kahan_add(s, cmp, v);
    }
    const T tot = pencil_total<64>(s, cmp);
    if (lane == 0) {
        T sc, pool;
        depletion_of(tot * dth, m_total, sc, pool);
        Dxy[2 * xy] = sc;
        Dxy[2 * xy + 1] = pool;
    }
}

template <typename T>
hipError_t launch_depletion_m0(const T *psi, const T *m0, T *Dxy, int64_t nxy, int nth, T dth, T m_total,
                               hipStream_t s) {
    if (nxy <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_depletion_m0<T>, dim3((unsigned)((nxy + 3) / 4)), dim3(256), 0, s, psi, m0, Dxy, nxy, nth,
                       dth, m_total);
    return hipGetLastError();
}
template hipError_t launch_depletion_m0<float>(const float *, const float *, float *, int64_t, int, float, float,
                                               hipStream_t);
template hipError_t launch_depletion_m0<double>(const double *, const double *, double *, int64_t, int, double,
                                                double, hipStream_t);

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
