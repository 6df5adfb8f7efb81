// The LDS-free walking psi kernel for gfx950 (the tile walk itself is psi_walk_tile in
// psi_dev.h): tiles of 8 x 4 pencils, one wave per row of 8 pencils, XCD-banded blocks.
#include "psi_dev.h"

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

template <typename T, int KPL, int TI, bool OUT, bool DEPL, int D>
__global__ __launch_bounds__(256) void k_psi_walk(const T *__restrict__ psi_in, T *__restrict__ psi_out,
                                                  const T *__restrict__ m0, const T *__restrict__ m1,
                                                  const T *__restrict__ u, const T *__restrict__ G,
                                                  const T *__restrict__ tab, T *__restrict__ stress,
                                                  T *__restrict__ mom, double *__restrict__ partials,
                                                  T *__restrict__ Dxy, PsiConst<T> c, int tiles_i, int tiles_j,
                                                  int per) {
    psi_walk_tile<T, KPL, TI, OUT, DEPL, D>(psi_in, psi_out, m0, m1, u, G, tab, stress, mom, partials, Dxy, c, tiles_i,
                                   tiles_j, per, (int)blockIdx.x);
}

template <typename T>
hipError_t launch_psi_walk(const T *psi_in, T *psi_out, const T *m0, const T *m1, const T *u, const T *G,
                           const T *tab, T *stress, T *mom, double *partials, T *Dxy, const PsiConst<T> &c,
                           const WalkPlan &wp, hipStream_t s) {
    if (!wp.ok || wp.ti != 8) return hipErrorInvalidValue;
    const bool out = stress != nullptr;
#define MMK_WALK(KPL, OUT, DEPL, D)                                                                        \
    hipLaunchKernelGGL((k_psi_walk<T, KPL, 8, OUT, DEPL, D>), dim3(wp.blocks), dim3(256), 0, s, psi_in, psi_out,   \
                       m0, m1, u, G, tab, stress, mom, partials, Dxy, c, wp.tiles_i, wp.tiles_j, wp.per)
#define MMK_WALK_O(KPL, D)                                                    \
    if (out) {                                                                \
        if (Dxy) MMK_WALK(KPL, true, true, D); else MMK_WALK(KPL, true, false, D);   \
    } else {                                                                  \
        if (Dxy) MMK_WALK(KPL, false, true, D); else MMK_WALK(KPL, false, false, D); \
    }
    const int d = (c.nx % wp.ti == 0) ? wp.depth : 0;
    if (wp.kpl == 1) {
        if (d == 8) { MMK_WALK_O(1, 8) }
        else if (d == 4) { MMK_WALK_O(1, 4) }
        else { MMK_WALK_O(1, 0) }
    } else {
        if (d == 4 || d == 8) { MMK_WALK_O(2, 4) }
        else { MMK_WALK_O(2, 0) }
    }
#undef MMK_WALK_O
#undef MMK_WALK
    return hipGetLastError();
}
template hipError_t launch_psi_walk<float>(const float *, float *, const float *, const float *, const float *,
                                           const float *, const float *, float *, float *, double *, float *,
                                           const PsiConst<float> &, const WalkPlan &, hipStream_t);
template hipError_t launch_psi_walk<double>(const double *, double *, const double *, const double *,
                                            const double *, const double *, const double *, double *, double *,
                                            double *, double *, const PsiConst<double> &, const WalkPlan &,
                                            hipStream_t);

}  // namespace mmk
