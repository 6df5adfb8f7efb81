// Launch interface of the motor-force spreading kernels.
#pragma once
#include "kernels.h"

#include <vector>

namespace mmk {

// Window geometry of the spreading: tiles of 8 x 8 filament points; each tile's window covers
// the corners of its points' heads, [wx][wy] cells from (tile origin - (rx, ry)); the partial
// array holds one window of FP64 (fx, fy) pairs per tile.  Orientations k and k + nth/2 (nth
// even) are spread together, see force.hip.
struct ForcePlan {
    int rx, ry, wx, wy;
    int tiles_i, tiles_j;
    int nt;             // window cells per lane held in registers (0: the window is too large)
    int nslice;         // launches, each folding 64 nt consecutive window cells (one M read each)
    int chunk;          // arclength cells staged at a time (32 for FP32, 16 for FP64)
    int npass;          // orientation passes: nth / 2 (paired) or nth
    bool paired;
    size_t lds_bytes;   // per block (one wave): the pass's window and the staging rows
    size_t part_elems;  // FP64 elements of the partial-window array
};
ForcePlan plan_force(int nx, int ny, int nth, int ns, double lx, double ly, double L, size_t elem);

// Spreading records, built on the host in FP64.  For orientation k the head of arclength cell
// l sits at offset (a + ax, b + ay) cells from its filament point (a, b integers), and moves
// monotonically along sx = sign(cos th_k), sy = sign(sin th_k) as l grows.  Of the two corner
// columns x in {a, a + 1} the "trailing" one is the one a later head can no longer reach
// (a for sx > 0, a + 1 for sx < 0), the other "leading"; likewise in y.  Per pass k < npass
// and cell l < lpad (l padded to a multiple of the chunk with zero weights):
//   rec:    8 cell + code; code, how the corners moved from cell l - 1 (0 none, 1 one step
//           along x, 2 one step along y, 3 one step along both, 7 anything else; 0 at
//           l = 0), and cell, the window cell (x_t + rx) wy + (y_t + ry) of the
//           trailing-trailing corner for the tile's first point,
//   w[4]:   the bilinear weights of the corners (tt, lt, tl, ll), first letter x.
// exy[k] = (sx wy, sy): steps from a trailing to the leading corner cell; cs = [cos], [sin].
struct ForceRecords {
    int lpad = 0;
    std::vector<int> rec, exy;
    std::vector<double> w, cs;
};
// false if some corner would fall outside the window (not expected for any geometry).
bool force_records(int nth, int ns, double lx, double ly, double L, int nx, int ny, const ForcePlan &fp,
                   ForceRecords *out);

// Device image of the records: one block of 256 dwords per (pass, chunk), record j of the
// chunk at dwords [j * 256 / chunk, ...): rec, then the four weights in the field precision
// (FP32 at dwords 1..4; FP64 at dwords 2..9).
constexpr int kForceBlock = 256;
void force_record_blocks(const ForceRecords &r, const ForcePlan &fp, size_t elem, std::vector<uint32_t> *out);

// force[2][nx][ny] (fx, fy) of the state (M, psi): Eq. (10) with the bilinear hat, periodic.
// blk: force_record_blocks() on the device; exy, cs: the records' steps and angle table;
// part: scratch of plan.part_elems FP64 elements.
// hipErrorInvalidValue (nothing launched) if the window does not fit the device's LDS per
// block.
template <typename T>
hipError_t launch_motor_force(const T *M, const T *psi, const uint32_t *blk, const int *exy, const double *cs,
                              double *part, T *force, int nx, int ny, int nth, int ns, double F, double L,
                              const ForcePlan &fp, hipStream_t s);

}  // namespace mmk
