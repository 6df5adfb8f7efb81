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
// (q0: the motor kernel's run totals q0[run][r0], or with pairs the one-pass kernel's
// q01[r0 / 16][run][r0 % 16][2])
template <typename T>
hipError_t launch_r0_coarse(const T *q0, bool pairs, const T *psi, T *psiT, const R0Seg *seg, double *part, T *scale,
                            T *pool, T *coarse_out, T *free_out, const R0Const<T> &c, int nseg, int nsplit,
                            double dth, double m_total, double k_on, hipStream_t s);

// The anchor-marginal field M[nx][ny][nth][ns] = dx dy sum over anchors of M_b (tiled Mb), the
// input of the motor force; LDS bytes per block r0_field_lds (hipErrorInvalidValue above 160 KB).
size_t r0_field_lds(int ns, size_t esz);
template <typename T>
hipError_t launch_r0_field(const T *Mb, T *M, const R0Seg *seg, const int32_t *seg_start, const R0Const<T> &c, int ns,
                           hipStream_t s);

// ---- one anchor per block: depleted sub-cycling in one pass (Alg. 2's inner loop) ----------
// With the clamp, every sub-step needs the coarse density of each anchor over all its tracked
// cells.  In the anchor layout a block holds the tracked cells of one anchor at a time in
// registers (nthr threads of C slots, whole runs per thread, the rest padding) and runs the n
// sub-steps there, re-forming the clamp by a block-wide sum before each: M_b is read and written
// once per micro-step.  The state is M[r0][C/4][nthr][4]: slot j of thread t (slot id j nthr + t) at
// ((j / 4) nthr + t) 4 + j % 4, so that a thread's slots come in 16-byte groups.
struct R0Slots {
    bool ok = false;
    int C = 0, nthr = 0;               // slots per thread, threads per anchor
    std::vector<int32_t> slot_run;     // [C][nthr]: run of the slot, -1 for padding
    // [C][nthr][2]: the slot's run and its first arclength cell, run | lo << 20 (-1 for padding),
    // and the run's offset and orientation, (a + 1024) | (b + 1024) << 11 | k << 22
    std::vector<int32_t> slot_tab;
    // [ncell][3]: slot (j nthr + t), a, b of every tracked cell; then [C nthr]: the cell at each
    // position ((j / 4) nthr + t) 4 + j % 4 of an anchor's state, -1 for padding
    std::vector<int32_t> cell_pos;
    int64_t per_anchor() const { return (int64_t)C * nthr; }
};
// Dynamic LDS of the one-pass kernel: its decoded slot table, 8 C nthr bytes (at most 160 KB).
size_t r0_anchor_lds(int C, int nthr);
// Packs the runs of P into threads (best fit by decreasing length); ok = false when the tracked
// set does not fit 1024 threads of the largest slot count compiled for the precision (24 in FP32,
// 16 in FP64), a run is longer than it, or the slot table's fields overflow (2^20 runs, offsets
// beyond 1023 cells).
R0Slots plan_r0_slots(const R0Plan &P, size_t esz);

// nsub steps of dt of one micro-step with the clamp re-formed before each (Alg. 2; Eqs. (5)-(6)):
// coarse = w sum over the anchor's cells of psi(x, th_k) M (w = dx dy dth ds; psi of the step's
// start), the factor m_total / coarse and pool 0 where coarse > m_total, else 1 and
// k_on (m_total - coarse).  Anchor layout in and out (in place allowed).  Writes the run totals
// of the final state side by side in tiles of 16 anchors, q01[r0 / 16][run][r0 % 16] = (sum M
// ds, sum (l + 1/2 - ns/2) M ds^2), which k_r0_marg turns into m0, m1 (and the coarse kernel
// reads as pairs).
template <typename T>
hipError_t launch_r0_anchor(const T *M_in, T *M_out, T *q01, const int32_t *slot_tab, const T *psi,
                            const R0Const<T> &c, int nrun, int C, int nthr, int nsub, double m_total, double k_on,
                            double dth, int limiter, hipStream_t s);
// m0 = dA sum over the runs of orientation th of q0 of the run at anchor x - (a, b), m1 likewise
// from q1, in run order (FP64 sums).
template <typename T>
hipError_t launch_r0_marg(const T *q01, int nrun, const R0Seg *seg, const int32_t *seg_start, T *m0, T *m1,
                          const R0Const<T> &c, hipStream_t s);
// Between the anchor layout and the tiled one (vx > 0: M[tile][cell][64 vx]) or the caller's
// (vx = 0: Mb[cell][x]); to_anchor = 1 writes the anchor layout (its padding slots untouched: the
// kernel loads them with their group and drops them), else the other one (the tiled padding set
// to 0).
template <typename T>
hipError_t launch_r0_anchor_layout(const T *src, T *dst, const int32_t *cell_pos, const R0Const<T> &c, int vx,
                                   int64_t per_anchor, int nthr, bool to_anchor, hipStream_t s);

// Caller layout Mb[cell][nx][ny] -> tiled (to_tiled), or back.
template <typename T>
hipError_t launch_r0_layout(const T *src, T *dst, int64_t ncell, int64_t nxy, int vx, bool to_tiled, hipStream_t s);

}  // namespace mmk
