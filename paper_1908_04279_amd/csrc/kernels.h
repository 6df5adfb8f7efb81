// Internal launch interface between the C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mmk {

// Constants of the motor column step, already in the field precision.
template <typename T>
struct MotorConst {
    T k_on, k_off, v0;
    T nv_ds;       // -v0 / ds
    T dt, half_dt; // sub-step and its midpoint stage
    int nsub;      // sub-steps per micro-step (>= 1)
    int nstep;     // micro-steps per launch (>= 1): M stays in registers between them
    T *m0_steps;   // [nstep - 1][ncol]: m0 after micro-steps 0 .. nstep-2 (nstep > 1)
    T ds, ds2;     // m0 = ds * sum M,  m1 = ds^2 * sum (l + 1/2 - ns/2) M
    int nth;       // columns per (x, y) point, and log2 of it when a power of two (else -1)
    int nth_shift;
    int wide;      // 1: 32 bytes of the column per lane (launches doing several micro-steps or
                   // sub-steps of arithmetic per load), 0: 16 bytes (one step per load)
    int lanes;     // lanes per column asked for (0: from ns, the precision and `wide`)
    int chunks;    // 16-byte chunks per lane of the chunked tiling (0 or 1: plain tiling)
    int nt;        // nontemporal M accesses: -1 the default, 0 none, 1 loads and stores, 2 loads
};

// Forward motor step over `ncol` independent columns of `ns` cells, in registers: c.nstep
// micro-steps of c.nsub sub-steps each,
//   M <- M + dt R(M + dt/2 R(M)),
// with m0 after micro-step t < nstep-1 in c.m0_steps[t]; M_out = M after the last,
// m0 = sum M_out ds, m1 (if non-null) likewise.
// Dxy (non-null: depletion) holds [nx][ny][2] = (clamp factor, free-motor pool) of the
// current state (depletion_of() of its coarse bound density); the columns of point
// xy = col / nth are first scaled by the factor, and the attachment source is k_on times the
// pool instead of k_on.
template <typename T>
hipError_t launch_motor_step(const T *M_in, T *M_out, T *m0, T *m1, int64_t ncol, int ns,
                             int limiter, const MotorConst<T> &c, const T *Dxy, hipStream_t s);

// Geometry and constants of the filament-density step.
template <typename T>
struct PsiConst {
    int nx, ny, nth;
    T dt, inv_dx, inv_dy, inv_dth, F, sigma_f, dth;
    T m_total;  // depletion: total motors per unit area
};

// Free-motor pool (Eq. (6)) and over-binding clamp factor (Alg. 2) of one (x, y) point from
// its coarse bound density B: B > m_total scales the point's motor columns by m_total / B and
// leaves no free motors; otherwise factor 1 and pool m_total - B.
template <typename T>
__host__ __device__ inline void depletion_of(T B, T m_total, T &scale, T &pool) {
    if (B > m_total) {
        scale = m_total / B;
        pool = T(0);
    } else {
        scale = T(1);
        pool = m_total - B;
    }
}

// Precomputed angle tables: [9][nth] = cos th_k, sin th_k, cos th_{k+1/2}, sin th_{k+1/2},
// cos(2 th_k)/2, sin(2 th_k)/2, cos^2, cos sin, sin^2.
enum { TAB_C = 0, TAB_S, TAB_CH, TAB_SH, TAB_H1, TAB_H2, TAB_CC, TAB_CS, TAB_SS, TAB_N };

struct PsiLaunch {
    int ti, tj;          // tile of pencils per block
    int tiles_i, tiles_j;
    int blocks;          // grid size (XCD-banded, >= tiles)
    int group;           // lanes per pencil group (16, 32 or 64)
    size_t lds_bytes;
};
// nfields: staged fields per halo pencil (2 forward: psi, m0; 3 reverse: lam, psi, m0)
PsiLaunch plan_psi(int nx, int ny, int nth, size_t elem, int nfields);

// Donor-cell update psi_out = psi_in - dt div(flux).  If `stress` is non-null, also writes
// stress[3][nx][ny], mom[7][nx][ny] of (psi_out, m0, m1) and per-block FP64 partials
// partials[blocks][4] = (sum psi_out, sum sxx, sum sxy, sum syy).
// Dxy (non-null) receives depletion_of(B) per (x, y) of the new state on every step, with the
// coarse bound density B = sum_th psi_out m0 dth (one fixed-order reduction, the same on
// output and plain steps).
template <typename T>
hipError_t launch_psi_step(const T *psi_in, T *psi_out, const T *m0, const T *m1, const T *u,
                           const T *G, const T *tab, T *stress, T *mom, double *partials,
                           T *Dxy, const PsiConst<T> &c, const PsiLaunch &pl, hipStream_t s);

// LDS-free psi step for ntheta = 64 or 128: tiles of ti x 4 pencils, one wave walking each
// row of ti pencils along x; XCD-banded blocks (8 * per).
struct WalkPlan {
    int ok;              // 0: ntheta not supported by the walking kernel
    int kpl;             // orientations per lane (ntheta / 64)
    int ti, tiles_i, tiles_j, per, blocks;
    int depth;           // 0: two alternating register sets; 4, 8: a ring of that many (nx % ti == 0)
};
WalkPlan plan_walk(int nx, int ny, int nth);

// Same update and outputs as launch_psi_step, with the walking kernel.
template <typename T>
hipError_t launch_psi_walk(const T *psi_in, T *psi_out, const T *m0, const T *m1, const T *u, const T *G,
                           const T *tab, T *stress, T *mom, double *partials, T *Dxy, const PsiConst<T> &c,
                           const WalkPlan &wp, hipStream_t s);

// Depleted micro-step with c.nsub sub-steps of c.dt in one launch: one block per (x, y) point
// holding its nth columns; the clamp and the free pool of the current sub-state before each
// sub-step.  hipErrorNotSupported where depl_sub_supported() is false: ns of 32 bytes per lane
// (64 for FP32 ns = 64) times a power of two up to 16 lanes, nth * lanes a multiple of 64 and
// at most 1024 (the caller then launches one sub-step at a time).
bool depl_sub_supported(size_t esz, int nth, int ns, int64_t nxy);
template <typename T>
hipError_t launch_motor_depl_sub(const T *M_in, T *M_out, T *m0, T *m1, const T *psi, int64_t nxy, int nth, int ns,
                                 int limiter, const MotorConst<T> &c, double dth, double m_total, hipStream_t s);
// depletion_of() of B[x][y] = dth sum_th psi[x][y][th] m0[x][y][th] into Dxy[x][y][2] (between
// the sub-steps of a depleted micro-step).  Compensated sums in FP32.
template <typename T>
hipError_t launch_depletion_m0(const T *psi, const T *m0, T *Dxy, int64_t nxy, int nth, T dth, T m_total,
                               hipStream_t s);
// depletion_of() of the coarse bound density of a state,
// B[x][y] = dth ds sum_{th, s} psi[x][y][th] M[x][y][th][s] (M NULL: zero), into Dxy[x][y][2].
// Compensated sums in FP32.
template <typename T>
hipError_t launch_coarse_bound(const T *M, const T *psi, T *Dxy, int64_t nxy, int nth, int ns, T ds, T dth,
                               T m_total, hipStream_t s);

// Fixed-order compensated FP64 sum of partials[n][4] -> out[4] * scale[4].
hipError_t launch_reduce_partials(const double *partials, int n, double *out, double s0,
                                  double s1, hipStream_t s);

// out[i] = 0, i < n (typed fill so graph capture never records a memset node)
template <typename T>
hipError_t launch_zero(T *out, int64_t n, hipStream_t s);

}  // namespace mmk
