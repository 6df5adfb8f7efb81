// Launch interface of the reverse (adjoint) kernels.
#pragma once
#include "kernels.h"

namespace mmk {

// lam_out = (dM'/dM)^T lam', lam' = lam_in (NULL = 0) + lam_m0 ds + lam_m1 (s - L/2) ds
// (lam_m1 may be NULL); adds this step's k_on, k_off, v0 gradient terms to gpart[block][0..2].
// The grid is the device's resident block count, at most gblocks (rows of gpart) and at most
// one block per chunk of columns; motor_reverse_blocks() bounds it for sizing gpart.
template <typename T>
hipError_t launch_motor_reverse(const T *M, const T *lam_in, const T *lam_m0, const T *lam_m1, T *lam_out,
                                double *gpart, int gblocks, int64_t ncol, int ns, int limiter,
                                const MotorConst<T> &c, double inv_ds, hipStream_t s);

// lam_out = (dpsi'/dpsi)^T lam_in; lam_m0 = (dpsi'/dm0')^T lam_in (+ previous lam_m0 if accumulate).
template <typename T>
hipError_t launch_psi_reverse(const T *lam_in, const T *psi, const T *m0, const T *u, const T *G, const T *tab,
                              T *lam_out, T *lam_m0, bool accumulate_m0, const PsiConst<T> &c, const PsiLaunch &pl,
                              hipStream_t s);

// cotangents of the final psi, m0 and m1 from those of stress [3][nx][ny] and moments [7][nx][ny]
template <typename T>
hipError_t launch_seed(const T *g_sigma, const T *g_mom, const T *psi, const T *m0, const T *m1, const T *tab,
                       T *lam_psi, T *lam_m0, T *lam_m1, int64_t npsi, int nth, int64_t nxy, T F, T sigma_f, T dth,
                       hipStream_t s);

hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s);

// upper bound of the grid of launch_motor_reverse (rows of gpart it may touch)
int64_t motor_reverse_blocks(int64_t ncol, int ns, int elem);

}  // namespace mmk
