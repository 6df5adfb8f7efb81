// Motor force density for gfx950 (Cook & Shinar, Eq. (10)): every bound-motor cell l of a
// filament centred at (x_i, y_j) with orientation p_k pushes with F p_k psi M_l ds dth at its
// head (x_i, y_j) + (s_l - L/2) p_k; the delta function is the two-point hat (bilinear) in x
// and y, periodic.
//
// For a fixed orientation k the push is along p_k for every term, so the spreading builds the
// scalar density G_k = sum over points and cells of F psi M ds dth hat and adds cos(th_k) G_k,
// sin(th_k) G_k to the force.  Orientation k + nth/2 pushes along -p_k, and its cell
// ns - 1 - l sits where cell l of orientation k does (s_{ns-1-l} - L/2 = -(s_l - L/2)), so for
// even nth one pass spreads u = F ds dth (psi_k M_k[l] - psi_k' M_k'[ns-1-l]), k' = k + nth/2,
// with orientation k's stencil and adds cos(th_k), sin(th_k) times the result: half the
// spreading of one pass per orientation.  The head offset is the same for every point and
// moves monotonically with l, so the bilinear corners of consecutive cells are mostly shared:
// a lane keeps the four corners of its current head in registers, adds each cell's weighted
// u to them, and spreads a corner only when the head has moved past it.  Spreading is a
// scatter, done in a fixed order so that the result has the same bits on every run:
//   k_motor_force: one wave per 8 x 8 tile of filament points.  The wave owns a private LDS
//     window of the pass's density around its tile (the corners its heads reach) in FP64,
//     and keeps the window's running (fx, fy) in registers in the field precision, NT cells
//     per lane.  (Unpaired, the sums over orientations cancel by a factor ~150 on a
//     near-isotropic state and FP32 sums lost ~1e-4 relative; the paired differences cancel
//     by a factor 1-4 on the same states, where FP32 sums cost ~2e-7.)  For each pass it
//     stages the tile's 64 motor columns of both orientations in LDS (coalesced row loads,
//     the next chunk prefetched) and reads its own u back into registers, then walks the
//     cells with the host-built records (corner move code, corner cell, four weights;
//     wave-uniform scalar loads).  A spread corner goes to window cell point + corner with one LDS atomic add:
//     for a fixed corner the lanes' cells are distinct, no other wave touches the window and
//     the LDS applies one wave's operations in issue order, so each cell's terms are summed
//     in the fixed order.  After the pass the window is folded into the registers and
//     cleared; at the end the (fx, fy) window goes to a partial array.
//   k_force_merge: each grid cell sums, in a fixed order, the window cells of every tile
//     whose window covers it (periodic).
#include "force.h"
#include "device_util.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

namespace mmk {

namespace {
constexpr int kNt[] = {4, 8, 16, 24, 32, 40, 44, 48};  // compiled register-window sizes, cells per lane
constexpr double kTwoPi = 6.283185307179586476925286766559;

// head of arclength cell l of orientation k, in cells from its point: integer and fraction
struct Head {
    int a, b;
    double ax, ay;
};
Head head(int k, int l, int nth, int ns, double lx, double ly, double L, int nx, int ny) {
    const double dx = lx / nx, dy = ly / ny, ds = L / ns, dth = kTwoPi / nth;
    const double lever = (l + 0.5) * ds - 0.5 * L;
    const double ox = lever * std::cos(k * dth) / dx, oy = lever * std::sin(k * dth) / dy;
    const double fa = std::floor(ox), fb = std::floor(oy);
    return {(int)fa, (int)fb, ox - fa, oy - fb};
}
}  // namespace

ForcePlan plan_force(int nx, int ny, int nth, int ns, double lx, double ly, double L, size_t elem) {
    ForcePlan f{};
    f.tiles_i = (nx + 7) / 8;
    f.tiles_j = (ny + 7) / 8;
    f.paired = nth % 2 == 0;
    f.npass = f.paired ? nth / 2 : nth;
    f.chunk = elem == 4 ? 32 : 16;
    // the corners a, a + 1 (b, b + 1) of every head, over all orientations and cells
    int xmin = 0, xmax = 0, ymin = 0, ymax = 0;
    const double reach_x = 0.5 * L / (lx / nx), reach_y = 0.5 * L / (ly / ny);
    if (reach_x > 4096.0 || reach_y > 4096.0) return f;  // far beyond any window: nt = 0
    for (int k = 0; k < nth; ++k)
        for (int l = 0; l < ns; ++l) {
            const Head h = head(k, l, nth, ns, lx, ly, L, nx, ny);
            xmin = std::min(xmin, h.a);
            xmax = std::max(xmax, h.a + 1);
            ymin = std::min(ymin, h.b);
            ymax = std::max(ymax, h.b + 1);
        }
    f.rx = -xmin;
    f.ry = -ymin;
    f.wx = xmax - xmin + 8;
    f.wy = ymax - ymin + 8;
    // the window's (fx, fy) sit in registers, at most 48 cells a lane: larger windows are
    // folded in slices, one launch (and one read of M) per slice
    const double cells = (double)f.wx * f.wy;
    f.nt = 0;
    f.nslice = (int)std::ceil(cells / (64.0 * 48));
    const double per = std::ceil(cells / f.nslice);
    for (int nt : kNt)
        if (per <= 64.0 * nt) {
            f.nt = nt;
            break;
        }
    f.lds_bytes = f.nt ? sizeof(double) * ((size_t)f.wx * f.wy + 1) / 2 * 2 + elem * 2 * 64 * (f.chunk + 4) : 0;
    f.part_elems = f.nt ? (size_t)f.tiles_i * f.tiles_j * 2 * f.wx * f.wy : 0;
    return f;
}

bool force_records(int nth, int ns, double lx, double ly, double L, int nx, int ny, const ForcePlan &fp,
                   ForceRecords *out) {
    ForceRecords &r = *out;
    if (fp.nt == 0) return false;
    const int npass = fp.npass;
    r.lpad = (ns + fp.chunk - 1) / fp.chunk * fp.chunk;
    r.rec.assign((size_t)npass * r.lpad, 0);
    r.w.assign((size_t)npass * r.lpad * 4, 0.0);
    r.exy.resize(2 * (size_t)npass);
    r.cs.resize(2 * (size_t)npass);
    bool ok = true;
    for (int k = 0; k < npass; ++k) {
        const double co = std::cos(k * kTwoPi / nth), si = std::sin(k * kTwoPi / nth);
        r.cs[k] = co;
        r.cs[npass + k] = si;
        const int sx = co < 0.0 ? -1 : 1, sy = si < 0.0 ? -1 : 1;
        r.exy[2 * k] = sx * fp.wy;
        r.exy[2 * k + 1] = sy;
        int pa = 0, pb = 0, cell = 0;
        for (int l = 0; l < ns; ++l) {
            const Head h = head(k, l, nth, ns, lx, ly, L, nx, ny);
            // trailing corner coordinates and the weights in (trailing, leading) order
            const int xt = sx > 0 ? h.a : h.a + 1, yt = sy > 0 ? h.b : h.b + 1;
            const double wxt = sx > 0 ? 1.0 - h.ax : h.ax, wxl = 1.0 - wxt;
            const double wyt = sy > 0 ? 1.0 - h.ay : h.ay, wyl = 1.0 - wyt;
            int code = 0;
            if (l > 0) {
                const int mx = (h.a - pa) * sx, my = (h.b - pb) * sy;
                code = (mx == 0 && my == 0) ? 0 : (mx == 1 && my == 0) ? 1 : (mx == 0 && my == 1) ? 2
                                               : (mx == 1 && my == 1) ? 3 : 7;
            }
            pa = h.a;
            pb = h.b;
            // every lane's corners (li + x + rx, lj + y + ry), x in {xt, xt + sx}, must lie in the window
            for (int x : {xt, xt + sx})
                if (x + fp.rx < 0 || x + fp.rx + 7 >= fp.wx) ok = false;
            for (int y : {yt, yt + sy})
                if (y + fp.ry < 0 || y + fp.ry + 7 >= fp.wy) ok = false;
            cell = (xt + fp.rx) * fp.wy + yt + fp.ry;
            const size_t q = (size_t)k * r.lpad + l;
            r.rec[q] = cell * 8 + code;
            r.w[4 * q + 0] = wxt * wyt;
            r.w[4 * q + 1] = wxl * wyt;
            r.w[4 * q + 2] = wxt * wyl;
            r.w[4 * q + 3] = wxl * wyl;
        }
        for (int l = ns; l < r.lpad; ++l) r.rec[(size_t)k * r.lpad + l] = cell * 8;  // padding: no move
    }
    return ok;
}

void force_record_blocks(const ForceRecords &r, const ForcePlan &fp, size_t elem, std::vector<uint32_t> *out) {
    const int nchunk = r.lpad / fp.chunk, stride = kForceBlock / fp.chunk;
    out->assign((size_t)fp.npass * nchunk * kForceBlock, 0u);
    for (int k = 0; k < fp.npass; ++k)
        for (int l = 0; l < r.lpad; ++l) {
            const size_t q = (size_t)k * r.lpad + l;
            uint32_t *d = out->data() + ((size_t)k * nchunk + l / fp.chunk) * kForceBlock + (l % fp.chunk) * stride;
            d[0] = (uint32_t)r.rec[q];
            for (int c = 0; c < 4; ++c) {
                if (elem == 4) {
                    const float v = (float)r.w[4 * q + c];
                    std::memcpy(d + 1 + c, &v, 4);
                } else {
                    std::memcpy(d + 2 + 2 * c, &r.w[4 * q + c], 8);
                }
            }
        }
}

template <typename T, int NT, int CH, bool VEC>
__global__ __launch_bounds__(64) void k_motor_force(const T *__restrict__ M, const T *__restrict__ psi,
                                                    const uint32_t *__restrict__ blk, const int *__restrict__ exy,
                                                    const double *__restrict__ cs,
                                                    double *__restrict__ part, int nx, int ny, int nth, int ns,
                                                    T cF, int cbase, ForcePlan fp) {
    using V = typename std::conditional<std::is_same<T, float>::value, float4, double2>::type;
    constexpr int VW = sizeof(V) / sizeof(T);
    constexpr int SR = CH + 4;                 // staging row: one point's CH cells, 16-byte aligned
    constexpr int PPL = VEC ? 64 * VW / CH : 64 / CH;  // points per row load
    constexpr int NR = 64 / PPL;               // row loads per orientation and chunk
    constexpr int RS = kForceBlock / CH;       // dwords per record
    extern __shared__ __align__(16) unsigned char smem[];
    const int ncells = fp.wx * fp.wy;
    double *G = reinterpret_cast<double *>(smem);              // [wx][wy] density of the current pass
    T *stg = reinterpret_cast<T *>(G + (ncells + 1) / 2 * 2);  // [2 orientations][64 points][SR]
    const int lane = threadIdx.x;
    const int ti = blockIdx.x / fp.tiles_j, tj = blockIdx.x % fp.tiles_j;
    const int li = lane >> 3, lj = lane & 7;
    const int gi = ti * 8 + li, gj = tj * 8 + lj;
    const bool mine = gi < nx && gj < ny;
    const int lcell = li * fp.wy + lj;
    for (int q = lane; q < ncells; q += 64) G[q] = 0.0;
    T tx[NT], ty[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) tx[q] = ty[q] = T(0);
    // staging of one chunk: cells s0 .. s0+CH-1 of orientation k and cells ns-s0-CH ..
    // ns-s0-1 of its partner k2, for the tile's 64 points; a row load covers PPL points, each
    // lane one cell (or, with VEC, a 16-byte vector of VW cells; ns is then a multiple of VW
    // and every vector lies wholly inside or wholly outside [0, ns)).  Points past the grid
    // edge and cells outside [0, ns) load clamped (finite) values: the former spread with
    // psi = 0, the latter have zero weights.  The chunk's records come with it, 4 dwords a
    // lane.
    const int nchunk = (ns + CH - 1) / CH;
    const int64_t pstride = (int64_t)nth * ns;
    constexpr int LPP = 64 / PPL;  // lanes per point in a row load
    const int lq = lane / LPP, lc = (lane % LPP) * (VEC ? VW : 1);
    typedef T TV __attribute__((ext_vector_type(VW)));  // native vector: stays in registers
    using R = typename std::conditional<VEC, TV, T>::type;
    R rows[2][NR];
    uint32_t rnext[4];
    auto load_rows = [&](int k, int ch) {
        const int s0 = ch * CH;
        const int k2 = fp.paired ? k + nth / 2 : k;
        const int la = min(s0 + lc, ns - (VEC ? VW : 1)), lb = max(ns - s0 - CH + lc, 0);
        const T *Ma = M + (int64_t)k * ns + la, *Mb = M + (int64_t)k2 * ns + lb;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int q = r * PPL + lq;
            const int pi = min(ti * 8 + (q >> 3), nx - 1), pj = min(tj * 8 + (q & 7), ny - 1);
            const int64_t po = ((int64_t)pi * ny + pj) * pstride;
            // M is streamed once: nontemporal, so that it does not push the pass's psi
            // lines and the records out of L2 (with plain loads they were fetched again on
            // most passes, 1.27x the algorithmic bytes)
            rows[0][r] = __builtin_nontemporal_load(reinterpret_cast<const R *>(Ma + po));
            rows[1][r] = __builtin_nontemporal_load(reinterpret_cast<const R *>(Mb + po));
        }
        const uint32_t *b = blk + ((size_t)k * nchunk + ch) * kForceBlock + lane;
#pragma unroll
        for (int j = 0; j < 4; ++j) rnext[j] = b[64 * j];
    };
    load_rows(0, 0);
    // psi of this lane's point at the pass's two orientations, loaded one pass ahead (used at
    // once, its load would cost a memory round trip per pass)
    const T *psi_p = psi + ((int64_t)min(gi, nx - 1) * ny + min(gj, ny - 1)) * nth;
    T pa_next = psi_p[0], pb_next = psi_p[fp.paired ? nth / 2 : 0];
    for (int k = 0; k < fp.npass; ++k) {
        const T pa = pa_next, pb = pb_next;
        if (k + 1 < fp.npass) {
            pa_next = psi_p[k + 1];
            pb_next = psi_p[fp.paired ? k + 1 + nth / 2 : k + 1];
        }
        const T ca = mine ? cF * pa : T(0);
        const T cb = mine && fp.paired ? cF * pb : T(0);
        const int ex = exy[2 * k], ey = exy[2 * k + 1];
        T att = T(0), alt = T(0), atl = T(0), all = T(0);  // corners of the current head
        int pc = 0;
        auto spread = [&](T v, int c) { atomicAdd(G + c + lcell, (double)v); };
        for (int ch = 0; ch < nchunk; ++ch) {
            __syncthreads();  // the previous chunk's reads of the staging rows (and the fold) are done
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                *reinterpret_cast<R *>(stg + (r * PPL + lq) * SR + lc) = rows[0][r];
                *reinterpret_cast<R *>(stg + (64 + r * PPL + lq) * SR + lc) = rows[1][r];
            }
            uint32_t rv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) rv[j] = rnext[j];
            __syncthreads();  // staging rows (and the cleared window) visible to every lane
            {
                const int nit = k * nchunk + ch + 1;
                if (nit < fp.npass * nchunk) load_rows(nit / nchunk, nit % nchunk);
            }
            // u of cell s0 + j: this orientation's cell and the partner's mirror cell
            T u[CH];
#pragma unroll
            for (int v = 0; v < CH / VW; ++v) {
                const V a = *reinterpret_cast<const V *>(stg + lane * SR + v * VW);
                const V b = *reinterpret_cast<const V *>(stg + (64 + lane) * SR + CH - VW - v * VW);
                if constexpr (VW == 4) {
                    u[4 * v] = ca * a.x - cb * b.w;
                    u[4 * v + 1] = ca * a.y - cb * b.z;
                    u[4 * v + 2] = ca * a.z - cb * b.y;
                    u[4 * v + 3] = ca * a.w - cb * b.x;
                } else {
                    u[2 * v] = ca * a.x - cb * b.y;
                    u[2 * v + 1] = ca * a.y - cb * b.x;
                }
            }
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                {
                    // Corners the head has moved past are spread before the move: tt on any
                    // move, tl on a step along x, lt on a step along y, lt and ll as well on
                    // the rare diagonal step or jump.
                    // record j: wave-uniform, read out of the lanes that hold it
                    const int d = j * RS;
                    const int rc = (int)__builtin_amdgcn_readlane(rv[d >> 6], d & 63);
                    T w[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if constexpr (sizeof(T) == 4) {
                            const int e = d + 1 + c;
                            w[c] = __uint_as_float(__builtin_amdgcn_readlane(rv[e >> 6], e & 63));
                        } else {
                            const int e = d + 2 + 2 * c;
                            const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane(rv[e >> 6], e & 63);
                            const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane(rv[(e + 1) >> 6], (e + 1) & 63);
                            w[c] = __longlong_as_double((long long)(lo | hi << 32));
                        }
                    }
                    const int code = rc & 7;
                    const bool sx = code & 1, sy = code & 2;
                    // the move code is wave-uniform: heads that stay in their corner cell (code
                    // 0, about a third of the cells) spread nothing, with no divergence
                    if (code) {
                        spread(att, pc);
                        spread(sx ? atl : alt, sx ? pc + ey : pc + ex);
                        if (sx && sy) {
                            spread(alt, pc + ex);
                            if (code == 7) spread(all, pc + ex + ey);
                        }
                    }
                    // the survivors move to their new roles, the rest restart from 0 (selects)
                    const bool jump = code == 7;
                    const T x1 = sy ? all : alt, x0 = sy ? atl : att;
                    const T ntt = jump ? T(0) : sx ? x1 : x0;
                    const T nlt = sx ? T(0) : x1;
                    const T ntl = sy ? T(0) : sx ? all : atl;
                    const T nll = code ? T(0) : all;
                    att = ntt;
                    alt = nlt;
                    atl = ntl;
                    all = nll;
                    pc = rc >> 3;
                    const T m = u[j];
                    att += w[0] * m;
                    alt += w[1] * m;
                    atl += w[2] * m;
                    all += w[3] * m;
                }
            }
        }
        spread(att, pc);
        spread(alt, pc + ex);
        spread(atl, pc + ey);
        spread(all, pc + ex + ey);
        __syncthreads();  // the pass's window is complete
        const T co = (T)cs[k], si = (T)cs[fp.npass + k];
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int c = cbase + lane + 64 * q;
            if (c < ncells) {
                const T g = (T)G[c];
                G[c] = 0.0;
                tx[q] += co * g;
                ty[q] += si * g;
            }
        }
    }
    double *dst = part + (size_t)blockIdx.x * 2 * ncells;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int c = cbase + lane + 64 * q;
        if (c < ncells) {
            dst[2 * c] = (double)tx[q];
            dst[2 * c + 1] = (double)ty[q];
        }
    }
}

__device__ __forceinline__ int floor_div8(int a) { return a >= 0 ? a / 8 : -((-a + 7) / 8); }
__device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// force[c][x][y] = sum of window cell (x - o_t, y - o_t') of every tile (t, t') whose window
// covers (x, y) modulo the grid, o the window origin 8 t - rx.  For an image X = x + m nx, the
// tiles whose window [8t - rx, 8t - rx + wx) holds X are t in [ceil((X + rx - wx + 1) / 8),
// floor((X + rx) / 8)].  A block: 64 grid cells (one per lane) and 4 waves; wave q takes the
// tiles t with t = q mod 4, in the order (image of x, t, image of y, t'), and the 4 waves' sums
// meet in LDS in a fixed order: the same bits on every run.
template <typename T>
__global__ __launch_bounds__(256) void k_force_merge(const double *__restrict__ part, T *__restrict__ force, int nx,
                                                     int ny, ForcePlan fp) {
    __shared__ double red[2][4][64];
    const int64_t nxy = (int64_t)nx * ny;
    const int nwin = 2 * fp.wx * fp.wy;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t cell = (int64_t)blockIdx.x * 64 + lane;
    const bool ok = cell < nxy;
    const int64_t cz = ok ? cell : 0;
    const int x = (int)(cz / ny), y = (int)(cz % ny);
    double fx = 0.0, fy = 0.0;
    // images X of x that some window can hold: -rx <= X <= 8 (tiles_i - 1) - rx + wx - 1
    const int mx0 = -floor_div(x + fp.rx, nx), mx1 = floor_div(8 * (fp.tiles_i - 1) - fp.rx + fp.wx - 1 - x, nx);
    const int my0 = -floor_div(y + fp.ry, ny), my1 = floor_div(8 * (fp.tiles_j - 1) - fp.ry + fp.wy - 1 - y, ny);
    for (int mx = mx0; mx <= mx1; ++mx) {
        const int X = x + mx * nx;
        const int t0 = max(floor_div8(X + fp.rx - fp.wx + 8), 0), t1 = min(floor_div8(X + fp.rx), fp.tiles_i - 1);
        for (int ti = t0 + ((q - t0) % 4 + 4) % 4; ti <= t1; ti += 4) {
            const int wxc = X - (8 * ti - fp.rx);
            for (int my = my0; my <= my1; ++my) {
                const int Y = y + my * ny;
                const int u0 = max(floor_div8(Y + fp.ry - fp.wy + 8), 0);
                const int u1 = min(floor_div8(Y + fp.ry), fp.tiles_j - 1);
                for (int tj = u0; tj <= u1; ++tj) {
                    const int wyc = Y - (8 * tj - fp.ry);
                    const double *w = part + ((size_t)ti * fp.tiles_j + tj) * nwin + 2 * (wxc * fp.wy + wyc);
                    fx += w[0];
                    fy += w[1];
                }
            }
        }
    }
    red[0][q][lane] = fx;
    red[1][q][lane] = fy;
    __syncthreads();
    if (q == 0 && ok) {
        force[cell] = (T)(((red[0][0][lane] + red[0][1][lane]) + red[0][2][lane]) + red[0][3][lane]);
        force[nxy + cell] = (T)(((red[1][0][lane] + red[1][1][lane]) + red[1][2][lane]) + red[1][3][lane]);
    }
}

template <typename T, bool VEC>
hipError_t launch_spread(const T *M, const T *psi, const uint32_t *blk, const int *exy, const double *cs,
                         double *part, int nx, int ny, int nth, int ns, T cF, int cbase, const ForcePlan &fp,
                         hipStream_t s) {
    constexpr int CH = std::is_same<T, float>::value ? 32 : 16;
    const int tiles = fp.tiles_i * fp.tiles_j;
#define MMK_FORCE_LAUNCH(NT_)                                                                                      \
    hipLaunchKernelGGL((k_motor_force<T, NT_, CH, VEC>), dim3(tiles), dim3(64), fp.lds_bytes, s, M, psi, blk, exy, \
                       cs, part, nx, ny, nth, ns, cF, cbase, fp)
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
    return hipGetLastError();
}

template <typename T>
hipError_t launch_motor_force(const T *M, const T *psi, const uint32_t *blk, const int *exy, const double *cs,
                              double *part, T *force, int nx, int ny, int nth, int ns, double F, double L,
                              const ForcePlan &fp, hipStream_t s) {
    int dev = 0, max_lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    constexpr int CH = std::is_same<T, float>::value ? 32 : 16;
    if (fp.nt == 0 || fp.chunk != CH || fp.lds_bytes > (size_t)max_lds) return hipErrorInvalidValue;
    const T cF = (T)(F * (L / ns) * (kTwoPi / nth));
    // 16-byte row loads when every column starts on a 16-byte boundary
    const bool vec = ns % (16 / sizeof(T)) == 0 && reinterpret_cast<uintptr_t>(M) % 16 == 0;
    for (int sl = 0; sl < fp.nslice && e == hipSuccess; ++sl) {
        const int cbase = sl * 64 * fp.nt;
        e = vec ? launch_spread<T, true>(M, psi, blk, exy, cs, part, nx, ny, nth, ns, cF, cbase, fp, s)
                : launch_spread<T, false>(M, psi, blk, exy, cs, part, nx, ny, nth, ns, cF, cbase, fp, s);
    }
    if (e != hipSuccess) return e;
    const int64_t nxy = (int64_t)nx * ny;
    hipLaunchKernelGGL(k_force_merge<T>, dim3((unsigned)((nxy + 63) / 64)), dim3(256), 0, s, part, force, nx, ny, fp);
    return hipGetLastError();
}
template hipError_t launch_motor_force<float>(const float *, const float *, const uint32_t *, const int *,
                                              const double *, double *, float *, int, int, int, int, double, double,
                                              const ForcePlan &, hipStream_t);
template hipError_t launch_motor_force<double>(const double *, const double *, const uint32_t *, const int *,
                                               const double *, double *, double *, int, int, int, int, double,
                                               double, const ForcePlan &, hipStream_t);

}  // namespace mmk
