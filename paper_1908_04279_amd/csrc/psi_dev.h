// Device code of the filament-density (psi) step shared by the LDS-tiled psi kernels and the
// LDS-free walking psi kernel: the donor-cell flux, the split butterfly for the
// theta-moments, and the walking tile.
#pragma once
#include "device_util.h"
#include "kernels.h"

#include <type_traits>

namespace mmk {

// first-order upwind (donor-cell) flux through a face with velocity A; A = 0 takes the left cell
template <typename T>
__device__ __forceinline__ T donor(T A, T left, T right) {
    return (A >= T(0)) ? A * left : A * right;
}

// ---- theta-moments of a pencil: NMOM per-lane partial sums reduced over the G lanes ----
// Quantities: c, n_x, n_y, D_xx, D_xy, D_yy, B (moments 0..6) and sigma_xx, sigma_xy,
// sigma_yy (7..9).
constexpr int NMOM = 10;

// Value of the partner lane across lane bit B (the butterfly partner of level B; the mirror
// forms inside a row pair lanes that differ in bit B, which is all the reduction needs).
template <int B, typename T>
__device__ __forceinline__ T xchg(T v) {
    if constexpr (B == 0) return dpp_any<DPP_QUAD_XOR1>(v);
    else if constexpr (B == 1) return dpp_any<DPP_QUAD_XOR2>(v);
    else if constexpr (B == 2) return dpp_any<DPP_ROW_HALF_MIRROR>(v);
    else if constexpr (B == 3) return dpp_any<DPP_ROW_MIRROR>(v);
    else return __shfl_xor(v, 1 << B, 64);
}

// One level of the split butterfly over lane bit B with N quantities still open in s[0..N)
// (FP32: e carries the compensation).  A lane with bit B clear keeps the lower H = ceil(N/2)
// quantities, a lane with the bit set the upper ones (padded with a zero), and each adds its
// partner's copy of what it keeps, so the work halves at every level.  Once one quantity is
// left the remaining levels are a plain butterfly.  [off, end) tracks which quantities the
// lane's slots hold; the summation order is fixed by the lane index (reproducible).
#pragma clang fp contract(off)
template <int B, int N, bool COMP, bool E0, typename T>
__device__ __forceinline__ void split_level(T (&s)[NMOM], T (&e)[NMOM], int lane, int &off, int &end) {
    if constexpr (B >= 0) {
        constexpr int H = (N + 1) / 2;
        const bool up = N >= 2 && ((lane >> B) & 1);
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const T ls = s[j], hs = (N >= 2 && j + H < N) ? s[j + H] : T(0);
            const T ks = up ? hs : ls, ss = up ? ls : hs;
            const T rs = xchg<B>(N >= 2 ? ss : ls);
            if constexpr (COMP) {
                T ke = T(0), re = T(0);
                if constexpr (!E0) {
                    const T le = e[j], he = (N >= 2 && j + H < N) ? e[j + H] : T(0);
                    ke = up ? he : le;
                    re = xchg<B>(N >= 2 ? (up ? le : he) : le);
                }
                T t, err;
                two_sum(ks, rs, t, err);
                s[j] = t;
                e[j] = E0 ? err : (ke + re) + err;
            } else {
                s[j] = ks + rs;
            }
        }
        if constexpr (N >= 2) {
            if (up) off += H;
            else end = min(end, off + H);
        }
        split_level<B - 1, H, COMP, false>(s, e, lane, off, end);
    }
}

// Totals of the NMOM quantities over a group of G lanes.  Returns the total held by this lane
// and sets q to its quantity, or -1 for a lane that holds none or a duplicate.
template <int G, bool COMP, bool E0, typename T>
__device__ __forceinline__ T group_moments(T (&s)[NMOM], T (&e)[NMOM], int lane, int &q) {
    constexpr int LB = G == 64 ? 5 : (G == 32 ? 4 : 3);  // top lane bit of the group
    int off = 0, end = NMOM;
    split_level<LB, NMOM, COMP, E0>(s, e, lane, off, end);
    // the split levels are the top four bits; below them every lane of a sub-group holds the
    // same total, the one with those low bits clear stores it
    constexpr int LOW = (1 << (LB - 3)) - 1;
    q = (off < end && (lane & LOW) == 0) ? off : -1;
    if constexpr (COMP) return s[0] + e[0];
    else return s[0];
}
#pragma clang fp contract(on)

// Total over the G lanes of a pencil group of a per-lane Kahan pair (FP32: compensated
// butterfly) or plain sum (FP64); every lane of the group gets it.
template <int G, typename T>
__device__ __forceinline__ T pencil_total(T s, T comp) {
    if constexpr (std::is_same<T, float>::value) return group_sum_comp<G>(s, comp);
    else return group_sum<G>(s);
}

// per-lane partial sum of one quantity: the first term sets it, later terms add (compensated
// in FP32)
#pragma clang fp contract(off)
template <bool COMP, typename T>
__device__ __forceinline__ void mom_add(T &s, T &e, T v, bool first) {
    if (first) {
        s = v;
        e = T(0);
    } else if constexpr (COMP) {
        T t, err;
        two_sum(s, v, t, err);
        s = t;
        e += err;
    } else {
        s += v;
    }
}
#pragma clang fp contract(on)

// periodic index for i in [-1, n + 16): a halo index is off by at most one tile
__device__ __forceinline__ int wrap(int i, int n) {
    if (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
}


// value of lane l (wave-uniform l) on every lane
template <typename T>
__device__ __forceinline__ T lane_value(T v, int l) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    } else {
        const long long b = __builtin_bit_cast(long long, v);
        const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
        return __builtin_bit_cast(T, ((long long)hi << 32) | (unsigned int)lo);
    }
}

// ---- LDS-free psi step: one wave walks a row of pencils along x ----------------------------
// For ntheta = 64 KPL a pencil is one wave (lane k holds orientations k, k + 64, ...).  A block
// of four waves owns a tile of TI x 4 pencils; wave w walks the pencils (i0 .. i0+TI-1, j0+w)
// in x order.  The upper x-face flux of a pencil is the lower one of the next (the face
// velocity is the symmetric mean of its two cells, so the carried value equals the one the
// next pencil would compute), the theta neighbours are wave rotations, and the x-, y-halo
// pencils are plain loads that the neighbouring waves of the block and of the XCD-banded
// neighbouring tiles also read, so they hit in the caches.  u and gradu are wave-uniform per
// pencil.
//
// Same flux and update expressions as the LDS-tiled kernel; OUT adds the theta-moments, the
// stress and the FP64 block partials (mass, sum sigma) of the new state; DEPL adds the
// depletion factors of the new state (Dxy).
template <typename T, int KPL, int TI, bool OUT, bool DEPL, int D>
__device__ __forceinline__ void psi_walk_tile(const T *__restrict__ psi_in, T *__restrict__ psi_out,
                                              const T *__restrict__ m0, const T *__restrict__ m1,
                                              const T *__restrict__ u, const T *__restrict__ Gr,
                                              const T *__restrict__ tab, T *__restrict__ stress,
                                              T *__restrict__ mom, double *__restrict__ partials,
                                              T *__restrict__ Dxy, const PsiConst<T> &c, int tiles_i,
                                              int tiles_j, int per, int vblock) {
    constexpr int NTH = 64 * KPL;
    constexpr bool COMP = std::is_same<T, float>::value;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nx = c.nx, ny = c.ny;
    const int64_t nxy = (int64_t)nx * ny;
    // XCD banding as in the LDS-tiled kernel: virtual block v runs on XCD v % 8
    const int tile = (vblock & 7) * per + (vblock >> 3);
    double acc_mass = 0, acc_sig = 0;
    int lane_q = -1;
    const int j = (tile % tiles_j) * 4 + w;
    if (tile < tiles_i * tiles_j && j < ny) {
        const int i0 = (tile / tiles_j) * TI;
        const int jm = (j == 0) ? ny - 1 : j - 1, jp = (j + 1 == ny) ? 0 : j + 1;
        T co[KPL], si[KPL], chp[KPL], shp[KPL];
#pragma unroll
        for (int s = 0; s < KPL; ++s) {
            const int k = lane + 64 * s;
            co[s] = tab[TAB_C * NTH + k];
            si[s] = tab[TAB_S * NTH + k];
            chp[s] = tab[TAB_CH * NTH + k];
            shp[s] = tab[TAB_SH * NTH + k];
        }
        // output steps: the theta tables of the moments and stress
        T tcc[KPL], tcs[KPL], tss[KPL], th1[KPL], th2[KPL];
        if constexpr (OUT) {
#pragma unroll
            for (int s = 0; s < KPL; ++s) {
                const int k = lane + 64 * s;
                tcc[s] = tab[TAB_CC * NTH + k];
                tcs[s] = tab[TAB_CS * NTH + k];
                tss[s] = tab[TAB_SS * NTH + k];
                th1[s] = tab[TAB_H1 * NTH + k];
                th2[s] = tab[TAB_H2 * NTH + k];
            }
        }
        // The wave-uniform u and grad u go through the vector memory path (an offset the compiler
        // cannot prove uniform): all loads then retire in order, and no wait on the scalar cache
        // holds a pipeline of loads.
        const int64_t vz = (int64_t)__builtin_amdgcn_mbcnt_lo(0u, 0u);  // 0 on every lane
        // the neighbour cells of one pencil (per lane) and its face velocities and velocity
        // gradient (wave-uniform)
        struct Nv {
            T Pxp[KPL], Mxp[KPL], Pym[KPL], Mym[KPL], Pyp[KPL], Myp[KPL];
            T M1[OUT ? KPL : 1];  // output steps: m1 of the pencil itself
        };
        struct Nu {
            T ux_p, uy_c, uy_m, uy_p, Gxx, Gxy, Gyx, Gyy;
        };
        auto fetch_v = [&](Nv &X, int i) {
            const int ip = (i + 1 == nx) ? 0 : i + 1;
            const int64_t pxp = (int64_t)ip * ny + j;
            const int64_t pym = (int64_t)i * ny + jm, pyp = (int64_t)i * ny + jp;
#pragma unroll
            for (int s = 0; s < KPL; ++s) {
                const int k = lane + 64 * s;
                X.Pxp[s] = psi_in[pxp * NTH + k];
                X.Mxp[s] = m0[pxp * NTH + k];
                X.Pym[s] = psi_in[pym * NTH + k];
                X.Mym[s] = m0[pym * NTH + k];
                X.Pyp[s] = psi_in[pyp * NTH + k];
                X.Myp[s] = m0[pyp * NTH + k];
                if constexpr (OUT) X.M1[s] = m1[((int64_t)i * ny + j) * NTH + k];
            }
        };
        // field f of Nu for pencil i: its address in u (f < 4) or grad u (f >= 4)
        auto u_offset = [&](int i, int f) -> int64_t {
            const int ip = (i + 1 == nx) ? 0 : i + 1;
            const int64_t pc = (int64_t)i * ny + j;
            switch (f) {
                case 0: return (int64_t)ip * ny + j;
                case 1: return nxy + pc;
                case 2: return nxy + (int64_t)i * ny + jm;
                case 3: return nxy + (int64_t)i * ny + jp;
                default: return (int64_t)(f - 4) * nxy + pc;
            }
        };
        auto fetch_u = [&](Nu &X, int i) {
            X.ux_p = u[u_offset(i, 0) + vz];
            X.uy_c = u[u_offset(i, 1) + vz];
            X.uy_m = u[u_offset(i, 2) + vz];
            X.uy_p = u[u_offset(i, 3) + vz];
            X.Gxx = Gr[u_offset(i, 4) + vz];
            X.Gxy = Gr[u_offset(i, 5) + vz];
            X.Gyx = Gr[u_offset(i, 6) + vz];
            X.Gyy = Gr[u_offset(i, 7) + vz];
        };
        // centre cells of the first pencil and the flux through its lower x-face: loads, then
        // the flux
        T Pc[KPL], Mc[KPL], fxc[KPL], Pm[KPL], Mm[KPL];
        const int64_t pc0 = (int64_t)i0 * ny + j;
        const int im0 = (i0 == 0) ? nx - 1 : i0 - 1;
        const int64_t pm0 = (int64_t)im0 * ny + j;
        const int64_t uz = D > 0 ? vz : 0;
        T ux_c = u[pc0 + uz];
        const T ux_m = u[pm0 + uz];
#pragma unroll
        for (int s = 0; s < KPL; ++s) {
            const int k = lane + 64 * s;
            Pm[s] = psi_in[pm0 * NTH + k];
            Mm[s] = m0[pm0 * NTH + k];
            Pc[s] = psi_in[pc0 * NTH + k];
            Mc[s] = m0[pc0 * NTH + k];
        }
        if constexpr (D > 0) __builtin_amdgcn_sched_barrier(0);
        auto first_flux = [&]() {
#pragma unroll
            for (int s = 0; s < KPL; ++s) {
                const T ax_m = ux_m - c.F * Mm[s] * co[s];
                const T ax_c = ux_c - c.F * Mc[s] * co[s];
                const T Axm = T(0.5) * (ax_m + ax_c);
                fxc[s] = donor(Axm, Pm[s], Pc[s]);
            }
        };
        auto pencil = [&](const Nv &X, const Nu &U, int i) {
            const int64_t pc = (int64_t)i * ny + j;
            const T(&Pxp)[KPL] = X.Pxp;
            const T(&Mxp)[KPL] = X.Mxp;
            const T(&Pym)[KPL] = X.Pym;
            const T(&Mym)[KPL] = X.Mym;
            const T(&Pyp)[KPL] = X.Pyp;
            const T(&Myp)[KPL] = X.Myp;
            const T ux_p = U.ux_p;
            const T uy_c = U.uy_c, uy_m = U.uy_m, uy_p = U.uy_p;
            const T Gxx = U.Gxx, Gxy = U.Gxy, Gyx = U.Gyx, Gyy = U.Gyy;
            // psi at orientation k+1: lane k+1, or lane 0 of the next slot for lane 63
            T rp[KPL];
#pragma unroll
            for (int s = 0; s < KPL; ++s) rp[s] = dpp_any<DPP_WAVE_ROL1>(Pc[s]);
            T fxp[KPL], fxm[KPL], fyp[KPL], fym[KPL], ftp[KPL];
#pragma unroll
            for (int s = 0; s < KPL; ++s) {
                const T Pkp = (KPL == 1 || lane != 63) ? rp[s] : rp[(s + 1) % KPL];
                const T ax_c = ux_c - c.F * Mc[s] * co[s];
                const T ax_p = ux_p - c.F * Mxp[s] * co[s];
                const T Axp = T(0.5) * (ax_c + ax_p);
                fxp[s] = donor(Axp, Pc[s], Pxp[s]);
                fxm[s] = fxc[s];
                fxc[s] = fxp[s];
                const T ay_c = uy_c - c.F * Mc[s] * si[s];
                const T ay_m = uy_m - c.F * Mym[s] * si[s];
                const T ay_p = uy_p - c.F * Myp[s] * si[s];
                const T Ayp = T(0.5) * (ay_c + ay_p), Aym = T(0.5) * (ay_m + ay_c);
                fyp[s] = donor(Ayp, Pc[s], Pyp[s]);
                fym[s] = donor(Aym, Pym[s], Pc[s]);
                const T wp = -shp[s] * (Gxx * chp[s] + Gxy * shp[s]) + chp[s] * (Gyx * chp[s] + Gyy * shp[s]);
                ftp[s] = donor(wp, Pc[s], Pkp);
            }
            // flux through the lower theta face: lane k-1's upper one (lane 63 of the previous
            // slot for lane 0)
            T rm[KPL];
#pragma unroll
            for (int s = 0; s < KPL; ++s) rm[s] = dpp_any<DPP_WAVE_ROR1>(ftp[s]);
            T ms[NMOM], me[NMOM];
#pragma unroll
            for (int m = 0; m < NMOM; ++m) ms[m] = me[m] = T(0);
            T bs = T(0), bc = T(0);  // coarse bound density: sum psi_out m0 over this lane
#pragma unroll
            for (int s = 0; s < KPL; ++s) {
                const int k = lane + 64 * s;
                const T ftm = (KPL == 1 || lane != 0) ? rm[s] : rm[(s + KPL - 1) % KPL];
                const T div = (fxp[s] - fxm[s]) * c.inv_dx + (fyp[s] - fym[s]) * c.inv_dy + (ftp[s] - ftm) * c.inv_dth;
                const T pn = Pc[s] - c.dt * div;
                psi_out[pc * NTH + k] = pn;
                if constexpr (DEPL) {
                    if (s == 0) bs = pn * Mc[s];
                    else kahan_add(bs, bc, pn * Mc[s]);
                }
                if constexpr (OUT) {
                    const T fm = c.F * X.M1[s];
                    const T cc = tcc[s], cs = tcs[s], ss = tss[s], h1 = th1[s], h2 = th2[s];
                    const T terms[NMOM] = {pn,
                                           pn * co[s],
                                           pn * si[s],
                                           pn * cc,
                                           pn * cs,
                                           pn * ss,
                                           pn * Mc[s],
                                           pn * (c.sigma_f * h1 + fm * cc),
                                           pn * (c.sigma_f * h2 + fm * cs),
                                           pn * (-c.sigma_f * h1 + fm * ss)};
#pragma unroll
                    for (int m = 0; m < NMOM; ++m) mom_add<COMP>(ms[m], me[m], terms[m], s == 0);
                    acc_mass += (double)pn;
                }
            }
            if constexpr (DEPL) {
                const T tb = pencil_total<64>(bs, bc);
                if (lane == 0) {
                    T sc, pool;
                    depletion_of(tb * c.dth, c.m_total, sc, pool);
                    Dxy[2 * pc] = sc;
                    Dxy[2 * pc + 1] = pool;
                }
            }
            if constexpr (OUT) {
                int qm;
                const T tot = group_moments<64, COMP, KPL == 1>(ms, me, lane, qm);
                if (qm >= 0) {
                    const T v = tot * c.dth;
                    if (qm < 7) {
                        mom[qm * nxy + pc] = v;
                    } else {
                        stress[(qm - 7) * nxy + pc] = v;
                        acc_sig += (double)v;
                    }
                    lane_q = qm;
                }
            }
#pragma unroll
            for (int s = 0; s < KPL; ++s) {
                Pc[s] = Pxp[s];
                Mc[s] = Mxp[s];
            }
            ux_c = ux_p;
        };
        if constexpr (D == 0) {
            // Two sets of neighbour registers: the loads of pencil t + 1 go into one set before
            // the arithmetic of pencil t reads the other (software pipelining without register
            // copies, so each wait counts only the older set's loads).  Every fetch is issued
            // (the last ones reload a pencil already in range), so that each path leaves the
            // same loads in flight and the waits stay exact.  Any x extent.
            first_flux();
            Nv A, B;
            Nu UA, UB;
            fetch_v(A, i0);
            fetch_u(UA, i0);
#pragma unroll 1
            for (int t = 0; t < TI; t += 2) {
                const int i = i0 + t;
                if (i >= nx) break;
                const bool more = t + 1 < TI && i + 1 < nx;
                fetch_v(B, more ? i + 1 : i);
                fetch_u(UB, more ? i + 1 : i);
                pencil(A, UA, i);
                if (!more) break;
                const int in = (t + 2 < TI && i + 2 < nx) ? i + 2 : i + 1;
                fetch_v(A, in);
                fetch_u(UA, in);
                pencil(B, UB, i + 1);
            }
        } else {
            // A ring of D register sets (x extent a multiple of TI, no ragged walk): the first D
            // pencils' cells are loaded at once, and pencil t + D's into the set that pencil t
            // has just used; the schedule barriers keep that order, so D pencils are in flight.
            // The uniform values of all TI pencils come in one load, field f of pencil t in lane
            // 8 t + f, and are broadcast from there (lane_value).
            static_assert(TI * 8 <= 64, "one lane per uniform value of the walk");
            const int lt = lane >> 3, lf = lane & 7;
            const int64_t lo = u_offset(i0 + (lt < TI ? lt : 0), lf);
            const T uvec = lf < 4 ? u[lo] : Gr[lo];
            Nv S[D];
#pragma unroll
            for (int t = 0; t < D; ++t) fetch_v(S[t], i0 + t);
            __builtin_amdgcn_sched_barrier(0);
            first_flux();
#pragma unroll
            for (int t = 0; t < TI; ++t) {
                Nu U;
                U.ux_p = lane_value(uvec, 8 * t + 0);
                U.uy_c = lane_value(uvec, 8 * t + 1);
                U.uy_m = lane_value(uvec, 8 * t + 2);
                U.uy_p = lane_value(uvec, 8 * t + 3);
                U.Gxx = lane_value(uvec, 8 * t + 4);
                U.Gxy = lane_value(uvec, 8 * t + 5);
                U.Gyx = lane_value(uvec, 8 * t + 6);
                U.Gyy = lane_value(uvec, 8 * t + 7);
                pencil(S[t % D], U, i0 + t);
                if (t + D < TI) fetch_v(S[t % D], i0 + t + D);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    if constexpr (OUT) {
        // fixed-order block sum of the FP64 partials: wave butterfly, then waves 0..3
        __shared__ double red[4][4];
        double v[4] = {acc_mass, lane_q == 7 ? acc_sig : 0.0, lane_q == 8 ? acc_sig : 0.0,
                       lane_q == 9 ? acc_sig : 0.0};
#pragma unroll
        for (int a = 0; a < 4; ++a)
            for (int m = 32; m >= 1; m >>= 1) v[a] += __shfl_xor(v[a], m, 64);
        if (lane == 0)
            for (int a = 0; a < 4; ++a) red[w][a] = v[a];
        __syncthreads();
        if (tid < 4) {
            double sum = 0;
            for (int q = 0; q < 4; ++q) sum += red[q][tid];
            partials[(size_t)vblock * 4 + tid] = sum;
        }
    }
}

}  // namespace mmk
