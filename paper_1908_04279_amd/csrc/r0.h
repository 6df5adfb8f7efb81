// Anchor-resolved bound motors M_b(r0, x, th, s) on the capture ball B_rc(r0) (Sec. 2; Eqs. (4)-(6);
// Alg. 2): the tracked cells, their runs along s, and the three kernels of a micro-step.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace mmk {

// Tracked cells and their runs.  A cell (a, b, k, l) is the filament centred at x = r0 + (a dx, b dy)
// with angle th_k and arclength cell l whose motor point x + (s_l - L/2) p_k lies within rc of
// the anchor r0 (anchors on the cell centres).  cells lists them in lexicographic (a, b, k, l)
// order; M_b is stored [cell][nx][ny], indexed by the filament cell x.  A run is a maximal set
// of consecutive l with the same (a, b, k); runs are grouped by k (seg_start[k] .. seg_start[k+1])
// keeping their cell order inside a group.
struct R0Seg {
    int32_t off;   // first cell of the run
    int32_t a, b;  // anchor offset: r0 = x - (a, b)
    int32_t pack;  // lo | len << 10 | k << 20
};
struct R0Plan {
    bool ok = false;           // rc usable (rc > 0, rc + L/2 below half of lx and of ly)
    int64_t ncell = 0;
    int nseg = 0, lmax = 0;
    std::vector<int32_t> cells;    // [ncell][4]
    std::vector<R0Seg> seg;        // [nseg], grouped by k
    std::vector<int32_t> seg_start;  // [nth + 1]
    int nsplit = 1;                // coarse blocks per anchor tile (4 partial rows each), r0_coarse_split
};
// cells_only: fill ncell (and cells) but no runs.
R0Plan plan_r0(int nx, int ny, int nth, int ns, double lx, double ly, double L, double rc, bool cells_only);
constexpr int kR0MaxRun = 32;  // longest run the motor kernel holds in registers

template <typename T>
struct R0Const {
    T k_on, k_off, nv_ds, dt, half_dt;  // as in the full-column step
    double ds, ds2, dA;                 // m0 = ds dA sum M, m1 = ds^2 dA sum (l + 1/2 - ns/2) M
    double half_ns;
    int nx, ny, nth;
    int64_t nxy, ncell;
    int vx;       // filament cells per lane (r0_vx); the tile is 64 vx cells
    int advance;  // 0: moments and run totals of the given state only (no update, no store)
    int nsub;     // midpoint steps of dt per launch (> 1 only without the clamp: scale == nullptr)
};

// Filament cells per lane of the motor kernel for runs of at most lmax cells: 2 for runs <= 8,
// 8 bytes for runs <= 16, one value for longer runs (register budget).
int r0_vx(size_t esz, int lmax);
// Blocks per anchor tile of the coarse kernel (each makes 4 rows of partials).
int r0_coarse_split(int64_t nxy, int nseg, size_t esz);
// Elements of the tiled state M[tile][cell][64 vx] (the last tile padded).
int64_t r0_tiled_elems(int64_t ncell, int64_t nxy, int vx);

// c.nsub motor steps of c.dt of every run (M_in -> M_out, tiled layout), each run a column with the no-influx
// and free-outflow ends; the anchor's clamp factor scale[r0] multiplies the run first and pool[r0]
// (k_on times the free pool) is its source (scale == nullptr: factor 1, source k_on).  Writes the
// run totals by anchor, q0[run][r0] = sum M ds, and the anchor marginals m0, m1 [nx][ny][nth] of
// the new state.
template <typename T>
hipError_t launch_r0_motor(const T *M_in, T *M_out, T *q0, T *m0, T *m1, const R0Seg *seg, const int32_t *seg_start,
                           const T *scale, const T *pool, const R0Const<T> &c, int lmax, int limiter, hipStream_t s);

// Coarse density of Eq. (5) at every anchor from the run totals and psi (psiT [nth][nx][ny]:
// scratch for psi by orientation): coarse = dx dy dth sum over runs of q0 psi(x, th_k), then the
// clamp factor and the source of Alg. 2 / Eq. (6) (m_total > 0), and optionally coarse and the
// free pool in the field precision.
template <typename T>
hipError_t launch_r0_coarse(const T *q0, const T *psi, T *psiT, const R0Seg *seg, double *part, T *scale, T *pool,
                            T *coarse_out, T *free_out, const R0Const<T> &c, int nseg, int nsplit, double dth,
                            double m_total, double k_on, hipStream_t s);

// The anchor-marginal field M[nx][ny][nth][ns] = dx dy sum over anchors of M_b (tiled Mb), the
// input of the motor force; LDS bytes per block r0_field_lds (hipErrorInvalidValue above 160 KB).
size_t r0_field_lds(int ns, size_t esz);
template <typename T>
hipError_t launch_r0_field(const T *Mb, T *M, const R0Seg *seg, const int32_t *seg_start, const R0Const<T> &c, int ns,
                           hipStream_t s);

// Caller layout Mb[cell][nx][ny] -> tiled (to_tiled), or back.
template <typename T>
hipError_t launch_r0_layout(const T *src, T *dst, int64_t ncell, int64_t nxy, int vx, bool to_tiled, hipStream_t s);

}  // namespace mmk
