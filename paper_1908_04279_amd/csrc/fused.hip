// The LDS-free walking psi kernel and the fused micro-step kernel for gfx950.
//
// Within a micro-step the psi step needs m0 of the new motor state, so the motor step and the
// psi step of one micro-step are ordered.  The motor step of micro-step n+1 does not read psi
// (attachment is linear, the motor field is independent of the filament density), so it can
// run in the same launch as the psi step of micro-step n: a K-step run becomes one motor
// launch, K-1 fused launches and one psi launch, instead of 2K launches.  The psi blocks are
// spread through the grid in octets (one block per XCD), so their latency-bound work runs in
// the shadow of the bandwidth-bound motor stream; the motor blocks take the remaining
// indices in order.  m0 is double-buffered by the caller: the motor part writes the buffer
// of micro-step n+2 while the psi part reads the one of n+1.
#include "motor_dev.h"
#include "psi_dev.h"

#include <cstdlib>

namespace mmk {

WalkPlan plan_walk(int nx, int ny, int nth) {
    WalkPlan w{};
    if (nth != 64 && nth != 128) return w;
    w.ok = 1;
    w.kpl = nth / 64;
    w.ti = 8;
    w.tiles_i = (nx + w.ti - 1) / w.ti;
    w.tiles_j = (ny + 3) / 4;
    w.per = (w.tiles_i * w.tiles_j + 7) / 8;
    w.blocks = 8 * w.per;
    return w;
}

template <typename T, int KPL, int TI, bool OUT>
__global__ __launch_bounds__(256) void k_psi_walk(const T *__restrict__ psi_in, T *__restrict__ psi_out,
                                                  const T *__restrict__ m0, const T *__restrict__ m1,
                                                  const T *__restrict__ u, const T *__restrict__ G,
                                                  const T *__restrict__ tab, T *__restrict__ stress,
                                                  T *__restrict__ mom, double *__restrict__ partials,
                                                  PsiConst<T> c, int tiles_i, int tiles_j, int per) {
    psi_walk_tile<T, KPL, TI, OUT>(psi_in, psi_out, m0, m1, u, G, tab, stress, mom, partials, c, tiles_i, tiles_j,
                                   per, (int)blockIdx.x);
}

template <typename T>
hipError_t launch_psi_walk(const T *psi_in, T *psi_out, const T *m0, const T *m1, const T *u, const T *G,
                           const T *tab, T *stress, T *mom, double *partials, const PsiConst<T> &c,
                           const WalkPlan &wp, hipStream_t s) {
    if (!wp.ok || wp.ti != 8) return hipErrorInvalidValue;
    const bool out = stress != nullptr;
#define MMK_WALK(KPL, OUT)                                                                                  \
    hipLaunchKernelGGL((k_psi_walk<T, KPL, 8, OUT>), dim3(wp.blocks), dim3(256), 0, s, psi_in, psi_out, m0, m1, u, \
                       G, tab, stress, mom, partials, c, wp.tiles_i, wp.tiles_j, wp.per)
    if (wp.kpl == 1) {
        if (out) MMK_WALK(1, true); else MMK_WALK(1, false);
    } else {
        if (out) MMK_WALK(2, true); else MMK_WALK(2, false);
    }
#undef MMK_WALK
    return hipGetLastError();
}
template hipError_t launch_psi_walk<float>(const float *, float *, const float *, const float *, const float *,
                                           const float *, const float *, float *, float *, double *,
                                           const PsiConst<float> &, const WalkPlan &, hipStream_t);
template hipError_t launch_psi_walk<double>(const double *, double *, const double *, const double *,
                                            const double *, const double *, const double *, double *, double *,
                                            double *, const PsiConst<double> &, const WalkPlan &, hipStream_t);

// Block roles of a fused grid.  Octet o = blockIdx / 8 holds psi blocks if o = o0 + r R with
// 0 <= r < per (psi virtual block r * 8 + blockIdx % 8, so psi tile bands stay per XCD); every
// other block is motor block b - 8 (number of psi octets before o), idle past motor_blocks.
struct FuseMap {
    int per, R, o0;
    int tiles_i, tiles_j;
    int64_t motor_blocks;
};

template <typename T, int CPL, int LPC, bool WANT_M1, bool NT, int KPL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_step_fused(const T *__restrict__ M_in, T *__restrict__ M_out,
                                                    T *__restrict__ m0_new, T *__restrict__ m1, int64_t ncol,
                                                    int ns, MotorConst<T> mc, const T *__restrict__ psi_in,
                                                    T *__restrict__ psi_out, const T *__restrict__ m0_cur,
                                                    const T *__restrict__ u, const T *__restrict__ G,
                                                    const T *__restrict__ tab, PsiConst<T> pc, FuseMap fm) {
    const int b = blockIdx.x, o = b >> 3;
    const int rel = o - fm.o0;
    const int r = rel >= 0 ? rel / fm.R : -1;
    if (rel >= 0 && rel == r * fm.R && r < fm.per) {
        psi_walk_tile<T, KPL, 8, false>(psi_in, psi_out, m0_cur, nullptr, u, G, tab, nullptr, nullptr, nullptr, pc,
                                        fm.tiles_i, fm.tiles_j, fm.per, r * 8 + (b & 7));
        return;
    }
    const int before = rel <= 0 ? 0 : min(fm.per, (rel + fm.R - 1) / fm.R);
    const int64_t mb = (int64_t)b - 8 * (int64_t)before;
    if (mb >= fm.motor_blocks) return;
    motor_cols<T, CPL, LPC, 0, false, WANT_M1, NT>(M_in, M_out, m0_new, m1, ncol, ns, mc, mb);
}

// fused kernels exist for the default plain tilings (16 bytes of a column per lane) of these
// column lengths, the default nontemporal choice, superbee, ntheta = 64 or 128
static bool fused_tiling(int ns, int elem, int limiter, int nth, int *lpc_out) {
    bool nt = false;
    const int lpc = motor_plain_lpc(ns, elem, &nt);
    *lpc_out = lpc;
    if (limiter != 0 || (nth != 64 && nth != 128) || lpc == 0) return false;
    if (nt != (elem == 4)) return false;
    if (lpc * (16 / elem) != ns) return false;
    return ns == 16 || ns == 32 || ns == 64 || ns == 128;
}

bool fused_supported(int ns, int elem, int limiter, int nth) {
    int lpc;
    return fused_tiling(ns, elem, limiter, nth, &lpc);
}

template <typename T, int CPL, int LPC, int KPL>
static hipError_t launch_fused_cfg(const T *M_in, T *M_out, T *m0_new, T *m1, int64_t ncol, int ns,
                                   const MotorConst<T> &mc, const T *psi_in, T *psi_out, const T *m0_cur,
                                   const T *u, const T *G, const T *tab, const PsiConst<T> &pc,
                                   const WalkPlan &wp, hipStream_t s) {
    constexpr int COLS = 256 / LPC;
    constexpr bool NT = sizeof(T) == 4;
    FuseMap fm{};
    fm.per = wp.per;
    fm.tiles_i = wp.tiles_i;
    fm.tiles_j = wp.tiles_j;
    fm.motor_blocks = (ncol + COLS - 1) / COLS;
    const int64_t octets = (fm.motor_blocks + 8 * (int64_t)wp.per + 7) / 8;
    // placement of the psi octets: spread over the grid (default), first, or last
    static const int place = [] {
        const char *e = getenv("MMK_FUSE_PLACE");
        return e ? atoi(e) : 0;
    }();
    int64_t R = octets / (wp.per > 0 ? wp.per : 1), o0 = 0;
    if (place == 1) R = 1;
    if (place == 2) {
        R = 1;
        o0 = octets - wp.per;
    }
    if (wp.per <= 0 || R < 1 || R > 0x7fffffff || octets * 8 > 0x7fffffff) return hipErrorInvalidConfiguration;
    fm.R = (int)R;
    fm.o0 = (int)o0;
    const dim3 grid((unsigned)(octets * 8));
    if (m1)
        hipLaunchKernelGGL((k_step_fused<T, CPL, LPC, true, NT, KPL>), grid, dim3(256), 0, s, M_in, M_out, m0_new, m1,
                           ncol, ns, mc, psi_in, psi_out, m0_cur, u, G, tab, pc, fm);
    else
        hipLaunchKernelGGL((k_step_fused<T, CPL, LPC, false, NT, KPL>), grid, dim3(256), 0, s, M_in, M_out, m0_new,
                           m1, ncol, ns, mc, psi_in, psi_out, m0_cur, u, G, tab, pc, fm);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step_fused(const T *M_in, T *M_out, T *m0_new, T *m1, int64_t ncol, int ns, int limiter,
                             const MotorConst<T> &mc, const T *psi_in, T *psi_out, const T *m0_cur, const T *u,
                             const T *G, const T *tab, const PsiConst<T> &pc, const WalkPlan &wp, hipStream_t s) {
    int lpc;
    if (!wp.ok || !fused_tiling(ns, (int)sizeof(T), limiter, pc.nth, &lpc)) return hipErrorInvalidValue;
    constexpr int CPL = 16 / sizeof(T);
#define MMK_FUSED_CASE(NS)                                                                                         \
    if (ns == NS) {                                                                                                \
        if (wp.kpl == 1)                                                                                           \
            return launch_fused_cfg<T, CPL, NS / CPL, 1>(M_in, M_out, m0_new, m1, ncol, ns, mc, psi_in, psi_out,   \
                                                         m0_cur, u, G, tab, pc, wp, s);                            \
        return launch_fused_cfg<T, CPL, NS / CPL, 2>(M_in, M_out, m0_new, m1, ncol, ns, mc, psi_in, psi_out,       \
                                                     m0_cur, u, G, tab, pc, wp, s);                                \
    }
    MMK_FUSED_CASE(16)
    MMK_FUSED_CASE(32)
    MMK_FUSED_CASE(64)
    MMK_FUSED_CASE(128)
#undef MMK_FUSED_CASE
    return hipErrorInvalidValue;
}
template hipError_t launch_step_fused<float>(const float *, float *, float *, float *, int64_t, int, int,
                                             const MotorConst<float> &, const float *, float *, const float *,
                                             const float *, const float *, const float *, const PsiConst<float> &,
                                             const WalkPlan &, hipStream_t);
template hipError_t launch_step_fused<double>(const double *, double *, double *, double *, int64_t, int, int,
                                              const MotorConst<double> &, const double *, double *, const double *,
                                              const double *, const double *, const double *,
                                              const PsiConst<double> &, const WalkPlan &, hipStream_t);

}  // namespace mmk
