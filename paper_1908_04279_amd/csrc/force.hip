// Motor force density for gfx950 (Cook & Shinar, Eq. (10)): every bound-motor cell l of a
// filament centred at (x_i, y_j) with orientation p_k pushes with F p_k psi M_l ds dth at its
// head (x_i, y_j) + (s_l - L/2) p_k; the delta function is the two-point hat (bilinear) in x
// and y, periodic.
//
// For a fixed orientation k the push is along p_k for every term, so the spreading first
// builds the scalar density G_k = sum over points and cells of F psi M ds dth hat, then adds
// cos(th_k) G_k and sin(th_k) G_k to the force.  The head offset (s_l - L/2) p_k is the same
// for every point and moves monotonically with l, so the bilinear corners of consecutive
// cells l are mostly shared: a lane keeps the four corners of its current head in registers,
// adds each cell's weighted motors to them, and spreads a corner only when the head has moved
// past it.  Spreading is a scatter, done in a fixed order so that the result has the same
// bits on every run:
//   k_motor_force: one wave per 8 x 8 tile of filament points.  The wave owns a private LDS
//     window of G_k around its tile (the tile plus the filament's reach) in FP64, and keeps
//     the window's running (fx, fy) in FP64 registers, NT cells per lane: the x and y sums
//     cancel strongly over the orientations (by a factor ~150 on a near-isotropic state),
//     and FP32 sums lost ~1e-4 relative there.  For each orientation it stages the tile's 64
//     motor columns in LDS (coalesced row loads, the next chunk prefetched) and reads its own
//     column back into registers, then walks the cells with the host-built records (corner
//     move code, corner cell, four weights; wave-uniform scalar loads).  A spread corner goes
//     to window cell point + corner with one LDS atomic add: for a fixed corner the lanes'
//     cells are distinct, no other wave touches the window and the LDS applies one wave's
//     operations in issue order, so each cell's terms are summed in the fixed order.  After
//     the orientation the window is folded into the registers and cleared; at the end the
//     (fx, fy) window goes to a partial array.
//   k_force_merge: each grid cell sums, in tile order, the window cells of every tile whose
//     window covers it (periodic).
#include "force.h"
#include "device_util.h"

#include <cmath>
#include <type_traits>

namespace mmk {

namespace {
constexpr int kNt[] = {4, 8, 16, 24, 32, 40, 44, 48};  // compiled register-window sizes, cells per lane
}  // namespace

ForcePlan plan_force(int nx, int ny, int ns, double lx, double ly, double L, size_t elem) {
    ForcePlan f{};
    const double reach_x = 0.5 * L / (lx / nx), reach_y = 0.5 * L / (ly / ny);
    f.rx = (int)std::ceil(reach_x) + 1;
    f.ry = (int)std::ceil(reach_y) + 1;
    f.wx = 8 + 2 * f.rx + 1;
    f.wy = 8 + 2 * f.ry + 1;
    f.tiles_i = (nx + 7) / 8;
    f.tiles_j = (ny + 7) / 8;
    (void)ns;
    const double cells = (double)f.wx * f.wy;
    f.nt = 0;
    for (int nt : kNt)
        if (cells <= 64.0 * nt) {
            f.nt = nt;
            break;
        }
    const int ch = force_chunk(elem);
    f.lds_bytes = f.nt ? sizeof(double) * ((size_t)f.wx * f.wy + 1) / 2 * 2 + elem * 64 * (ch + 4) : 0;
    f.part_elems = f.nt ? (size_t)f.tiles_i * f.tiles_j * 2 * f.wx * f.wy : 0;
    return f;
}

bool force_records(int nth, int ns, double lx, double ly, double L, int nx, int ny, const ForcePlan &fp, int chunk,
                   ForceRecords *out) {
    const double dx = lx / nx, dy = ly / ny, ds = L / ns, dth = 6.283185307179586476925286766559 / nth;
    ForceRecords &r = *out;
    r.chunk = chunk;
    r.nchunk = (ns + chunk - 1) / chunk;
    r.lpad = r.nchunk * chunk;
    r.rec.assign((size_t)nth * r.lpad * 2, 0);
    r.w.assign((size_t)nth * r.lpad * 4, 0.0);
    r.exy.resize(2 * (size_t)nth);
    r.cs.resize(2 * (size_t)nth);
    bool ok = fp.nt > 0;
    for (int k = 0; k < nth; ++k) {
        const double co = std::cos(k * dth), si = std::sin(k * dth);
        r.cs[k] = co;
        r.cs[nth + k] = si;
        const int sx = co < 0.0 ? -1 : 1, sy = si < 0.0 ? -1 : 1;
        r.exy[2 * k] = sx * fp.wy;
        r.exy[2 * k + 1] = sy;
        int pa = 0, pb = 0, cell = 0;
        for (int l = 0; l < ns; ++l) {
            const double lever = (l + 0.5) * ds - 0.5 * L;
            const double ox = lever * co / dx, oy = lever * si / dy;
            const double fa = std::floor(ox), fb = std::floor(oy), ax = ox - fa, ay = oy - fb;
            const int a = (int)fa, b = (int)fb;
            // trailing corner coordinates and the weights in (trailing, leading) order
            const int xt = sx > 0 ? a : a + 1, yt = sy > 0 ? b : b + 1;
            const double wxt = sx > 0 ? 1.0 - ax : ax, wxl = 1.0 - wxt;
            const double wyt = sy > 0 ? 1.0 - ay : ay, wyl = 1.0 - wyt;
            int code = 0;
            if (l > 0) {
                const int mx = (a - pa) * sx, my = (b - pb) * sy;
                code = (mx == 0 && my == 0) ? 0 : (mx == 1 && my == 0) ? 1 : (mx == 0 && my == 1) ? 2
                                               : (mx == 1 && my == 1) ? 3 : 7;
            }
            pa = a;
            pb = b;
            // every lane's corners (li + x + rx, lj + y + ry), x in {xt, xt + sx}, must lie in the window
            for (int x : {xt, xt + sx})
                if (x + fp.rx < 0 || x + fp.rx + 7 >= fp.wx) ok = false;
            for (int y : {yt, yt + sy})
                if (y + fp.ry < 0 || y + fp.ry + 7 >= fp.wy) ok = false;
            cell = (xt + fp.rx) * fp.wy + yt + fp.ry;
            const size_t q = (size_t)k * r.lpad + l;
            r.rec[2 * q] = code;
            r.rec[2 * q + 1] = cell;
            r.w[4 * q + 0] = wxt * wyt;
            r.w[4 * q + 1] = wxl * wyt;
            r.w[4 * q + 2] = wxt * wyl;
            r.w[4 * q + 3] = wxl * wyl;
        }
        for (int l = ns; l < r.lpad; ++l) r.rec[2 * ((size_t)k * r.lpad + l) + 1] = cell;  // padding: no move
    }
    return ok;
}

template <typename T, int NT, int CH>
__global__ __launch_bounds__(64) void k_motor_force(const T *__restrict__ M, const T *__restrict__ psi,
                                                    const int *__restrict__ rec, const int *__restrict__ exy,
                                                    const T *__restrict__ wts, const double *__restrict__ cs,
                                                    double *__restrict__ part, int nx, int ny, int nth, int ns,
                                                    T cF, ForcePlan fp) {
    constexpr int SR = CH + 4;        // staging row: one point's CH cells, 16-byte aligned
    constexpr int PPL = 64 / CH;      // points per row load
    constexpr int LB = 32 / sizeof(T);  // records per batch of scalar loads
    using V = typename std::conditional<std::is_same<T, float>::value, float4, double2>::type;
    constexpr int VW = sizeof(V) / sizeof(T);
    extern __shared__ __align__(16) unsigned char smem[];
    const int ncells = fp.wx * fp.wy;
    double *G = reinterpret_cast<double *>(smem);              // [wx][wy] density of the current orientation
    T *stg = reinterpret_cast<T *>(G + (ncells + 1) / 2 * 2);  // [64 points][SR], 16-byte aligned
    const int lane = threadIdx.x;
    const int ti = blockIdx.x / fp.tiles_j, tj = blockIdx.x % fp.tiles_j;
    const int li = lane >> 3, lj = lane & 7;
    const int gi = ti * 8 + li, gj = tj * 8 + lj;
    const bool mine = gi < nx && gj < ny;
    const int lcell = li * fp.wy + lj;
    for (int q = lane; q < ncells; q += 64) G[q] = 0.0;
    double tx[NT], ty[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) tx[q] = ty[q] = 0.0;
    // staging: cells s0 .. s0+CH-1 of the tile's 64 columns of one orientation; a row load
    // covers PPL points, lane % CH = cell.  Points past the grid edge and cells past ns load
    // clamped (finite) values: the former spread with psi = 0, the latter have zero weights.
    const int nchunk = (ns + CH - 1) / CH;
    const int64_t pstride = (int64_t)nth * ns;
    const int lc = lane % CH;
    T rows[CH];
    auto load_rows = [&](int k, int s0) {
        const T *Mk = M + (int64_t)k * ns + (s0 + lc < ns ? s0 + lc : ns - 1);
#pragma unroll
        for (int r = 0; r < CH; ++r) {
            const int q = r * PPL + lane / CH;
            const int pi = min(ti * 8 + (q >> 3), nx - 1), pj = min(tj * 8 + (q & 7), ny - 1);
            rows[r] = Mk[((int64_t)pi * ny + pj) * pstride];
        }
    };
    load_rows(0, 0);
    const double *csk = cs;
    for (int k = 0; k < nth; ++k) {
        const T cps = mine ? cF * psi[((int64_t)gi * ny + gj) * nth + k] : T(0);
        const int ex = exy[2 * k], ey = exy[2 * k + 1];
        T att = T(0), alt = T(0), atl = T(0), all = T(0);  // corners of the current head
        int pc = 0;
        auto spread = [&](T v, int c) { atomicAdd(G + c + lcell, (double)(v * cps)); };
        for (int ch = 0; ch < nchunk; ++ch) {
            __syncthreads();  // the previous chunk's reads of the staging rows (and the fold) are done
#pragma unroll
            for (int r = 0; r < CH; ++r) stg[(r * PPL + lane / CH) * SR + lc] = rows[r];
            __syncthreads();  // staging rows (and the cleared window) visible to every lane
            {
                const int nx_it = k * nchunk + ch + 1;
                if (nx_it < nth * nchunk) load_rows(nx_it / nchunk, (nx_it % nchunk) * CH);
            }
            T u[CH];
#pragma unroll
            for (int v = 0; v < CH / VW; ++v) {
                const V x = *reinterpret_cast<const V *>(stg + lane * SR + v * VW);
                if constexpr (VW == 4) {
                    u[4 * v] = x.x;
                    u[4 * v + 1] = x.y;
                    u[4 * v + 2] = x.z;
                    u[4 * v + 3] = x.w;
                } else {
                    u[2 * v] = x.x;
                    u[2 * v + 1] = x.y;
                }
            }
            const size_t r0 = (size_t)k * nchunk * CH + (size_t)ch * CH;
            const int *rk = rec + 2 * r0;
            const T *wk = wts + 4 * r0;
#pragma unroll
            for (int b = 0; b < CH; b += LB) {
                // one batch of wave-uniform records, all loaded before its first atomic
                int code[LB], cell[LB];
                T w[LB][4];
#pragma unroll
                for (int q = 0; q < LB; ++q) {
                    code[q] = rk[2 * (b + q)];
                    cell[q] = rk[2 * (b + q) + 1];
#pragma unroll
                    for (int c = 0; c < 4; ++c) w[q][c] = wk[4 * (b + q) + c];
                }
#pragma unroll
                for (int q = 0; q < LB; ++q) {
                    switch (code[q]) {
                    case 0: break;
                    case 1:  // one step along x: the trailing x column is done
                        spread(att, pc);
                        spread(atl, pc + ey);
                        att = alt;
                        atl = all;
                        alt = all = T(0);
                        break;
                    case 2:  // one step along y: the trailing y row is done
                        spread(att, pc);
                        spread(alt, pc + ex);
                        att = atl;
                        alt = all;
                        atl = all = T(0);
                        break;
                    case 3:  // one step along both: only the leading-leading corner stays
                        spread(att, pc);
                        spread(alt, pc + ex);
                        spread(atl, pc + ey);
                        att = all;
                        alt = atl = all = T(0);
                        break;
                    default:  // a jump: no corner stays
                        spread(att, pc);
                        spread(alt, pc + ex);
                        spread(atl, pc + ey);
                        spread(all, pc + ex + ey);
                        att = alt = atl = all = T(0);
                        break;
                    }
                    pc = cell[q];
                    const T m = u[b + q];
                    att += w[q][0] * m;
                    alt += w[q][1] * m;
                    atl += w[q][2] * m;
                    all += w[q][3] * m;
                }
            }
        }
        spread(att, pc);
        spread(alt, pc + ex);
        spread(atl, pc + ey);
        spread(all, pc + ex + ey);
        __syncthreads();  // the orientation's window is complete
        const double co = csk[k], si = csk[nth + k];
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int c = lane + 64 * q;
            if (c < ncells) {
                const double g = G[c];
                G[c] = 0.0;
                tx[q] += co * g;
                ty[q] += si * g;
            }
        }
    }
    double *dst = part + (size_t)blockIdx.x * 2 * ncells;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int c = lane + 64 * q;
        if (c < ncells) {
            dst[2 * c] = tx[q];
            dst[2 * c + 1] = ty[q];
        }
    }
}

// force[c][x][y] = sum over tiles t (in order) and window cells w of t that land on (x, y)
template <typename T>
__global__ __launch_bounds__(256) void k_force_merge(const double *__restrict__ part, T *__restrict__ force, int nx,
                                                     int ny, ForcePlan fp) {
    const int64_t nxy = (int64_t)nx * ny;
    const int nwin = 2 * fp.wx * fp.wy;
    for (int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cell < nxy;
         cell += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(cell / ny), y = (int)(cell % ny);
        double fx = 0.0, fy = 0.0;
        for (int ti = 0; ti < fp.tiles_i; ++ti) {
            // window x-offset of this cell in tile ti's window (origin ti*8 - rx), periodic
            int wx0 = (x - (ti * 8 - fp.rx)) % nx;
            if (wx0 < 0) wx0 += nx;
            if (wx0 >= fp.wx) continue;
            for (int tj = 0; tj < fp.tiles_j; ++tj) {
                int wy0 = (y - (tj * 8 - fp.ry)) % ny;
                if (wy0 < 0) wy0 += ny;
                if (wy0 >= fp.wy) continue;
                const double *w = part + ((size_t)ti * fp.tiles_j + tj) * nwin;
                for (int wx = wx0; wx < fp.wx; wx += nx)
                    for (int wy = wy0; wy < fp.wy; wy += ny) {
                        fx += w[2 * (wx * fp.wy + wy)];
                        fy += w[2 * (wx * fp.wy + wy) + 1];
                    }
            }
        }
        force[cell] = (T)fx;
        force[nxy + cell] = (T)fy;
    }
}

template <typename T>
hipError_t launch_motor_force(const T *M, const T *psi, const int *rec, const int *exy, const T *w, const double *cs,
                              double *part, T *force, int nx, int ny, int nth, int ns, double F, double L,
                              const ForcePlan &fp, hipStream_t s) {
    int dev = 0, max_lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    if (fp.nt == 0 || fp.lds_bytes > (size_t)max_lds) return hipErrorInvalidValue;
    const int tiles = fp.tiles_i * fp.tiles_j;
    const T cF = (T)(F * (L / ns) * (6.283185307179586476925286766559 / nth));
    constexpr int CH = std::is_same<T, float>::value ? 64 : 32;
#define MMK_FORCE_LAUNCH(NT_)                                                                                    \
    hipLaunchKernelGGL((k_motor_force<T, NT_, CH>), dim3(tiles), dim3(64), fp.lds_bytes, s, M, psi, rec, exy, w, \
                       cs, part, nx, ny, nth, ns, cF, fp)
    switch (fp.nt) {
    case 4: MMK_FORCE_LAUNCH(4); break;
    case 8: MMK_FORCE_LAUNCH(8); break;
    case 16: MMK_FORCE_LAUNCH(16); break;
    case 24: MMK_FORCE_LAUNCH(24); break;
    case 32: MMK_FORCE_LAUNCH(32); break;
    case 40: MMK_FORCE_LAUNCH(40); break;
    case 44: MMK_FORCE_LAUNCH(44); break;
    case 48: MMK_FORCE_LAUNCH(48); break;
    default: return hipErrorInvalidValue;
    }
#undef MMK_FORCE_LAUNCH
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nxy = (int64_t)nx * ny;
    int64_t blocks = (nxy + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_force_merge<T>, dim3((unsigned)blocks), dim3(256), 0, s, part, force, nx, ny, fp);
    return hipGetLastError();
}
template hipError_t launch_motor_force<float>(const float *, const float *, const int *, const int *, const float *,
                                              const double *, double *, float *, int, int, int, int, double, double,
                                              const ForcePlan &, hipStream_t);
template hipError_t launch_motor_force<double>(const double *, const double *, const int *, const int *,
                                               const double *, const double *, double *, double *, int, int, int,
                                               int, double, double, const ForcePlan &, hipStream_t);

}  // namespace mmk
