// Anchor-resolved bound motors on the capture ball (Sec. 2; Eqs. (4)-(6); Alg. 2) for gfx950.
//
// Layout: the state is tiled over the filament cells x, M[tile][cell][64 vx]: a lane holds vx
// consecutive filament cells (one 16-byte load for short runs), a wave 64 vx of them, and the
// cells of a run (a, b, k, lo..lo+len-1) are consecutive rows of a tile, so one run of one wave
// is len * 64 vx values in one contiguous piece.  The run lives in registers through both
// Runge-Kutta stages: M_b is read and written once per micro-step.  The caller's layout
// Mb[cell][x] is converted at set_state / get_state.
//
// The two reductions of the model go in opposite directions: the anchor marginal m0(x, th)
// sums over the anchors of a filament cell, the coarse density of Eq. (5) over the filament
// cells of an anchor.  The motor kernel makes the first in a block that owns one orientation
// and one tile (its four waves take every fourth run of that orientation, then add their totals
// through LDS in a fixed order) and writes each run's total q0 = sum M ds at its anchor.  The
// coarse kernel makes the second from q0 (read in anchor order) and psi by orientation, one row
// of partials per wave, and a last kernel adds the rows in a fixed order and forms the clamp and
// the free pool.  No atomics: every result is the same from run to run.
#include "device_util.h"
#include "r0.h"

#include <algorithm>
#include <cmath>

namespace mmk {

// ---- host: tracked cells and runs ------------------------------------------------------------
// The motor point of cell (a, b, k, l) relative to its anchor is (a dx, b dy) + t p_k with
// t = s_l - L/2; the cell is tracked when the squared length is at most rc^2 (evaluated in FP64
// in this order, without contraction, so that the decision is the one the model's definition
// gives in FP64).  co, si: cos and sin of k dth.
static bool tracked(double dx, double dy, double co, double si, double ds, double L, double rc, int a, int b, int l) {
#pragma clang fp contract(off)
    const double t = (l + 0.5) * ds - 0.5 * L;
    const double hx = a * dx + t * co;
    const double hy = b * dy + t * si;
    return hx * hx + hy * hy <= rc * rc;
}

R0Plan plan_r0(int nx, int ny, int nth, int ns, double lx, double ly, double L, double rc, bool cells_only) {
    R0Plan P;
    if (!(rc > 0) || !(rc + 0.5 * L < 0.5 * lx) || !(rc + 0.5 * L < 0.5 * ly)) return P;
    const double dx = lx / nx, dy = ly / ny, dth = 6.283185307179586476925286766559 / nth, ds = L / ns;
    std::vector<double> co(nth), si(nth);
    for (int k = 0; k < nth; ++k) {
        co[k] = std::cos(k * dth);
        si[k] = std::sin(k * dth);
    }
    // every tracked motor point lies within rc + L/2 of its anchor
    const double reach = rc + 0.5 * L;
    const int A = (int)std::ceil(reach / dx) + 1;
    const int B = (int)std::ceil(reach / dy) + 1;
    for (int a = -A; a <= A; ++a)
        for (int b = -B; b <= B; ++b) {
            // offsets whose filament centre is farther than rc + L/2 (with a cell of margin)
            // from the anchor hold no tracked cell
            const double ca = std::fabs(a * dx) - dx, cb = std::fabs(b * dy) - dy;
            if (ca > 0 && cb > 0 && ca * ca + cb * cb > reach * reach) continue;
            for (int k = 0; k < nth; ++k)
                for (int l = 0; l < ns; ++l)
                    if (tracked(dx, dy, co[k], si[k], ds, L, rc, a, b, l)) {
                        P.cells.insert(P.cells.end(), {a, b, k, l});
                        ++P.ncell;
                    }
        }
    P.ok = true;
    if (cells_only) return P;
    std::vector<std::vector<R0Seg>> byk(nth);
    for (int64_t c0 = 0; c0 < P.ncell;) {
        const int32_t *q = &P.cells[4 * c0];
        int64_t c1 = c0 + 1;
        while (c1 < P.ncell && P.cells[4 * c1] == q[0] && P.cells[4 * c1 + 1] == q[1] &&
               P.cells[4 * c1 + 2] == q[2] && P.cells[4 * c1 + 3] == P.cells[4 * (c1 - 1) + 3] + 1)
            ++c1;
        const int len = (int)(c1 - c0);
        P.lmax = std::max(P.lmax, len);
        byk[q[2]].push_back(R0Seg{(int32_t)c0, q[0], q[1], q[3] | (std::min(len, 1023) << 10) | (q[2] << 20)});
        c0 = c1;
    }
    P.seg_start.assign(nth + 1, 0);
    for (int k = 0; k < nth; ++k) {
        P.seg_start[k] = (int32_t)P.seg.size();
        P.seg.insert(P.seg.end(), byk[k].begin(), byk[k].end());
    }
    P.seg_start[nth] = (int32_t)P.seg.size();
    P.nseg = (int)P.seg.size();
    return P;
}

// Runs into threads for the one-pass kernel: for each compiled slot count C (at least the longest
// run), the fewest threads (a multiple of 64, at most 1024) into which best fit by decreasing
// length packs every run; each thread's runs take consecutive slots.
static constexpr int kR0SlotC[] = {4, 8, 16, 24};
R0Slots plan_r0_slots(const R0Plan &P, size_t esz) {
    R0Slots S;
    if (!P.ok || P.ncell == 0 || P.nseg == 0) return S;
    std::vector<int> order(P.nseg);
    for (int i = 0; i < P.nseg; ++i) order[i] = i;
    auto len_of = [&](int r) { return (P.seg[r].pack >> 10) & 1023; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return len_of(x) > len_of(y); });
    for (int C : kR0SlotC) {
        // 24 slots of FP64 do not fit the 128 registers of a 1024-thread block
        if (C < P.lmax || (esz == 8 && C > 16)) continue;
        const int64_t tmax = std::min<int64_t>(1024, (160 * 1024 - 512) / (8 * C) / 64 * 64);  // decoded table in LDS
        const int64_t t0 = 64 * ((P.ncell + 64 * C - 1) / (64 * C));
        for (int64_t T = t0; T <= tmax; T += 64) {
            // bins by free capacity; a run goes to a bin with the least free room that holds it
            std::vector<std::vector<int>> byfree(C + 1);
            for (int t = (int)T - 1; t >= 0; --t) byfree[C].push_back(t);
            std::vector<int> fill(T, 0);
            std::vector<int32_t> slot_run((size_t)C * T, -1);
            bool ok = true;
            for (int r : order) {
                const int len = len_of(r);
                int f = len;
                while (f <= C && byfree[f].empty()) ++f;
                if (f > C) {
                    ok = false;
                    break;
                }
                const int t = byfree[f].back();
                byfree[f].pop_back();
                for (int q = 0; q < len; ++q) slot_run[(size_t)(fill[t] + q) * T + t] = r;
                fill[t] += len;
                byfree[f - len].push_back(t);
            }
            if (!ok) continue;
            S.ok = true;
            S.C = C;
            S.nthr = (int)T;
            S.slot_run = std::move(slot_run);
            S.slot_tab.assign((size_t)2 * C * T, -1);
            for (size_t q = 0; q < S.slot_run.size(); ++q) {
                const int r = S.slot_run[q];
                if (r < 0) continue;
                const R0Seg &g = P.seg[r];
                const int lo = g.pack & 1023, k = g.pack >> 20;
                if (r >= (1 << 20) || std::abs(g.a) > 1023 || std::abs(g.b) > 1023 || k >= 512) return R0Slots{};
                S.slot_tab[2 * q] = r | lo << 20;
                S.slot_tab[2 * q + 1] = (g.a + 1024) | (g.b + 1024) << 11 | k << 22;
            }
            // [ncell][3] (slot, a, b), then [C nthr]: the cell at each position of the anchor
            // layout, -1 for padding
            S.cell_pos.assign((size_t)3 * P.ncell + (size_t)C * T, -1);
            for (int t = 0; t < T; ++t)
                for (int j = 0; j < C; ++j) {
                    const int r = S.slot_run[(size_t)j * T + t];
                    if (r < 0) continue;
                    // position in its run: slots of the run above this one in the thread
                    int q = 0;
                    while (j - q - 1 >= 0 && S.slot_run[(size_t)(j - q - 1) * T + t] == r) ++q;
                    const int64_t cell = P.seg[r].off + q;
                    S.cell_pos[3 * cell] = j * (int)T + t;
                    S.cell_pos[3 * cell + 1] = P.seg[r].a;
                    S.cell_pos[3 * cell + 2] = P.seg[r].b;
                    S.cell_pos[3 * P.ncell + ((size_t)(j >> 2) * T + t) * 4 + (j & 3)] = (int32_t)cell;
                }
            return S;
        }
    }
    return S;
}

// ---- device: one run ------------------------------------------------------------------------
// R(y) of a run of len cells (len <= LM, uniform across the wave): with the face value
// h_t = y_t + sigma_t / 2 and h_{-1} = 0 (no influx at the run's first cell; the ghost
// y_len = y_{len-1} makes the last slope 0, so the last flux is the first-order outflow v0 y):
//   R_t = -(v0/ds)(h_t - h_{t-1}) + (src - k_off y_t).
template <typename T, int LM, int LIM>
__device__ __forceinline__ void run_rhs(const T (&y)[LM], T (&R)[LM], int len, T nv_ds, T src, T k_off) {
    T h[LM];
#pragma unroll
    for (int t = 0; t < LM; ++t) {
        const T left = (t == 0) ? T(0) : y[t > 0 ? t - 1 : 0];
        const T right = (t + 1 < len) ? y[t + 1 < LM ? t + 1 : t] : y[t];
        const T sig = (LIM == 0) ? superbee(y[t] - left, right - y[t]) : T(0);
        h[t] = y[t] + T(0.5) * sig;
    }
#pragma unroll
    for (int t = 0; t < LM; ++t) {
        const T hl = (t == 0) ? T(0) : h[t > 0 ? t - 1 : 0];
        R[t] = nv_ds * (h[t] - hl) + (src - k_off * y[t]);
    }
}

// Both Runge-Kutta stages of VX runs of exactly N cells held in the first N slots of z.
template <typename T, int N, int LM, int LIM, int VX>
__device__ __forceinline__ void rk2_exact(T (&z)[VX][LM], const T (&src)[VX], T nv_ds, T k_off, T half_dt, T dt) {
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        T a[N], R[N], y[N];
#pragma unroll
        for (int t = 0; t < N; ++t) a[t] = z[v][t];
        run_rhs<T, N, LIM>(a, R, N, nv_ds, src[v], k_off);
#pragma unroll
        for (int t = 0; t < N; ++t) y[t] = a[t] + half_dt * R[t];
        run_rhs<T, N, LIM>(y, R, N, nv_ds, src[v], k_off);
#pragma unroll
        for (int t = 0; t < N; ++t) z[v][t] = a[t] + dt * R[t];
    }
}

template <typename T, int VX>
__device__ __forceinline__ void ldv(const T *p, T (&o)[VX]) {
    if constexpr (VX == 1) {
        o[0] = *p;
    } else {
        typedef T TV __attribute__((ext_vector_type(VX)));  // one 16-byte load, kept in registers
        const TV v = *reinterpret_cast<const TV *>(p);
#pragma unroll
        for (int i = 0; i < VX; ++i) o[i] = v[i];
    }
}
template <typename T, int VX>
__device__ __forceinline__ void stv(T *p, const T (&o)[VX]) {
    if constexpr (VX == 1) {
        *p = o[0];
    } else {
        typedef T TV __attribute__((ext_vector_type(VX)));
        TV v;
#pragma unroll
        for (int i = 0; i < VX; ++i) v[i] = o[i];
        *reinterpret_cast<TV *>(p) = v;
    }
}

// Wrap an index that is at most one period out of [0, n).
__device__ __forceinline__ int wrap1(int v, int n) {
    v += v < 0 ? n : 0;
    return v - (v >= n ? n : 0);
}

// One block: one orientation k and one x-tile of TT = 64 VX filament cells (lane: VX consecutive
// cells); its four waves take every fourth run of orientation k.  Tiled layout
// M[tile][cell][TT]: the cells of a run are consecutive rows of TT values, so a run's load is
// len * TT * sizeof(T) contiguous bytes.
template <typename T, int LM, int LIM, int VX, bool MULTI>
__global__ __launch_bounds__(256) void k_r0_motor(const T *__restrict__ Min, T *__restrict__ Mout, T *__restrict__ q0,
                                                  T *__restrict__ m0, T *__restrict__ m1,
                                                  const R0Seg *__restrict__ seg, const int32_t *__restrict__ seg_start,
                                                  const T *__restrict__ scale, const T *__restrict__ pool,
                                                  R0Const<T> c) {
    constexpr int TT = 64 * VX;
    __shared__ double red[2][4][TT];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int k = blockIdx.y;
    const int64_t tile = blockIdx.x;
    const int64_t x0 = tile * TT + lane * VX;
    int iv[VX], jv[VX];
    bool ok[VX];
    double a0[VX], a1[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        const int64_t x = x0 + v;
        ok[v] = x < c.nxy;
        iv[v] = ok[v] ? (int)(x / c.ny) : 0;
        jv[v] = ok[v] ? (int)(x - (int64_t)iv[v] * c.ny) : 0;
        a0[v] = a1[v] = 0.0;
    }
    const int64_t base = tile * c.ncell * TT + lane * VX;
    const int s_end = seg_start[k + 1];
    for (int s = seg_start[k] + w; s < s_end; s += 4) {
        const R0Seg r = seg[s];
        const int lo = r.pack & 1023, len = (r.pack >> 10) & 1023;
        // the anchor of this run at filament cell x: r0 = x - (a, b), periodic (|a| < nx/2)
        int32_t r0v[VX];  // nx ny < 2^31
        T sc[VX], src[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            r0v[v] = wrap1(iv[v] - r.a, c.nx) * c.ny + wrap1(jv[v] - r.b, c.ny);
            sc[v] = T(1);
            src[v] = c.k_on;
            if (scale != nullptr) {
                sc[v] = ok[v] ? scale[r0v[v]] : T(1);
                src[v] = ok[v] ? pool[r0v[v]] : T(0);
            }
        }
        const T *pin = Min + base + (int64_t)r.off * TT;
        T z[VX][LM];
#pragma unroll
        for (int t = 0; t < LM; ++t) {
            T q[VX];
            if (t < len) {
                ldv<T, VX>(pin + (int64_t)t * TT, q);
            } else {
#pragma unroll
                for (int v = 0; v < VX; ++v) q[v] = T(0);
            }
#pragma unroll
            for (int v = 0; v < VX; ++v) z[v][t] = sc[v] * q[v];
        }
        // c.nsub midpoint steps of c.dt in registers (sub-cycling without a clamp between them);
        // the one-step instantiation keeps the registers of a single step
        const int nsub = MULTI ? c.nsub : 1;
        for (int sub = 0; c.advance && sub < nsub; ++sub) {
            if constexpr (LM == 8) {
                // the run length is the same on every lane: the step for exactly that length
                switch (len) {
                    case 1: rk2_exact<T, 1, LM, LIM, VX>(z, src, c.nv_ds, c.k_off, c.half_dt, c.dt); break;
                    case 2: rk2_exact<T, 2, LM, LIM, VX>(z, src, c.nv_ds, c.k_off, c.half_dt, c.dt); break;
                    case 3: rk2_exact<T, 3, LM, LIM, VX>(z, src, c.nv_ds, c.k_off, c.half_dt, c.dt); break;
                    case 4: rk2_exact<T, 4, LM, LIM, VX>(z, src, c.nv_ds, c.k_off, c.half_dt, c.dt); break;
                    case 5: rk2_exact<T, 5, LM, LIM, VX>(z, src, c.nv_ds, c.k_off, c.half_dt, c.dt); break;
                    case 6: rk2_exact<T, 6, LM, LIM, VX>(z, src, c.nv_ds, c.k_off, c.half_dt, c.dt); break;
                    case 7: rk2_exact<T, 7, LM, LIM, VX>(z, src, c.nv_ds, c.k_off, c.half_dt, c.dt); break;
                    default: rk2_exact<T, 8, LM, LIM, VX>(z, src, c.nv_ds, c.k_off, c.half_dt, c.dt); break;
                }
            } else {
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    T R[LM], y[LM];
                    run_rhs<T, LM, LIM>(z[v], R, len, c.nv_ds, src[v], c.k_off);
#pragma unroll
                    for (int t = 0; t < LM; ++t) y[t] = z[v][t] + c.half_dt * R[t];
                    run_rhs<T, LM, LIM>(y, R, len, c.nv_ds, src[v], c.k_off);
#pragma unroll
                    for (int t = 0; t < LM; ++t) z[v][t] = z[v][t] + c.dt * R[t];
                }
            }
        }
        if (c.advance) {
            T *pout = Mout + base + (int64_t)r.off * TT;
#pragma unroll
            for (int t = 0; t < LM; ++t)
                if (t < len) {
                    T q[VX];
#pragma unroll
                    for (int v = 0; v < VX; ++v) q[v] = z[v][t];
                    stv<T, VX>(pout + (int64_t)t * TT, q);
                }
        }
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            double t0 = 0.0, t1 = 0.0;
#pragma unroll
            for (int t = 0; t < LM; ++t)
                if (t < len) {
                    t0 += (double)z[v][t];
                    t1 += ((double)(lo + t) + 0.5 - c.half_ns) * (double)z[v][t];
                }
            // run totals by anchor: q0[run][r0], read in anchor order by the coarse kernel
            if (ok[v]) q0[(int64_t)s * c.nxy + r0v[v]] = (T)(t0 * c.ds);
            a0[v] += t0;
            a1[v] += t1;
        }
    }
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        red[0][w][lane * VX + v] = a0[v];
        red[1][w][lane * VX + v] = a1[v];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int v = 0; v < VX; ++v)
            if (ok[v]) {
                const int q = lane * VX + v;
                const double s0 = ((red[0][0][q] + red[0][1][q]) + red[0][2][q]) + red[0][3][q];
                const double s1 = ((red[1][0][q] + red[1][1][q]) + red[1][2][q]) + red[1][3][q];
                m0[(x0 + v) * c.nth + k] = (T)(s0 * c.ds * c.dA);
                m1[(x0 + v) * c.nth + k] = (T)(s1 * c.ds2 * c.dA);
            }
    }
}

// ---- device: one anchor per block (depleted sub-cycling in one pass) -------------------------
// Pair (q0, q1) of run s at anchor r in the one-pass kernel's run totals: tiles of 16 anchors,
// q01[r / 16][s][r % 16] (times 2 values).
__host__ __device__ __forceinline__ int64_t r0_pair_index(int64_t r, int64_t s, int64_t nrun) {
    return ((r >> 4) * nrun + s) * 16 + (r & 15);
}

// The slots of a thread in registers: y (the state) and wg (psi of the slot's run at the anchor);
// bit j of cont is set where slot j continues the run of slot j - 1 (clear at a run's first slot
// and at slot 0).  The run's ends are bit masks (an AND with 0 or all ones, exact): the left
// difference y_j - [cont_j] y_{j-1} is y_j at a run's first cell (no influx), the right one
// [cont_{j+1}] (y_{j+1} - y_j) is 0 at its last (zero slope, first-order outflow), and the face
// value to the left [cont_j] h_{j-1} is 0 at its first; the rest is run_rhs.  The padding slots
// (after a thread's runs) form a run of their own that no sum reads and no store writes.
template <typename T>
__device__ __forceinline__ T keep_if(T v, int mk) {  // mk: 0 (-> +0) or -1 (-> v)
    if constexpr (sizeof(T) == 4)
        return __int_as_float(__float_as_int(v) & mk);
    else
        return __longlong_as_double(__double_as_longlong(v) & (long long)mk);
}
__device__ __forceinline__ int cont_mask(uint32_t cont, int j) {  // bit j as 0 or -1
    return (int)__builtin_amdgcn_sbfe(cont, j, 1);
}

template <typename T, int LIM>
__device__ __forceinline__ T anchor_rate(T yl, T yc, T yr, int ml, int mr, T &hprev, T nv_ds, T src, T k_off) {
    const T sig = (LIM == 0) ? superbee(yc - keep_if(yl, ml), keep_if(yr - yc, mr)) : T(0);
    const T h = yc + T(0.5) * sig;
    const T R = nv_ds * (h - keep_if(hprev, ml)) + (src - k_off * yc);
    hprev = h;
    return R;
}

// One midpoint step of all slots: y1 = y + dt/2 R(y), y <- y + dt R(y1), the two stages
// interleaved slot by slot (stage 2 at slot j needs stage 1 at j + 1), so that only three stage-1
// values are live.
template <typename T, int C, int LIM>
__device__ __forceinline__ void anchor_rk2(T (&y)[C], uint32_t cont, T half_dt, T dt, T nv_ds, T src, T k_off) {
    T h1 = T(0), h2 = T(0);
    T y1l = T(0), y1c, y1r = T(0);
    {
        const int m1 = C > 1 ? cont_mask(cont, 1) : 0;
        y1c = y[0] + half_dt * anchor_rate<T, LIM>(T(0), y[0], y[C > 1 ? 1 : 0], 0, m1, h1, nv_ds, src, k_off);
    }
#pragma unroll
    for (int j = 0; j < C; ++j) {
        const int mc = j > 0 ? cont_mask(cont, j) : 0;
        const int mr = j + 1 < C ? cont_mask(cont, j + 1 < C ? j + 1 : j) : 0;
        if (j + 1 < C) {
            const int n = j + 1 < C ? j + 1 : j;
            const int mrr = n + 1 < C ? cont_mask(cont, n + 1 < C ? n + 1 : n) : 0;
            y1r = y[n] + half_dt * anchor_rate<T, LIM>(y[j], y[n], y[n + 1 < C ? n + 1 : n], mr, mrr, h1, nv_ds, src,
                                                       k_off);
        }
        y[j] = y[j] + dt * anchor_rate<T, LIM>(y1l, y1c, y1r, mc, mr, h2, nv_ds, src, k_off);
        y1l = y1c;
        y1c = y1r;
    }
}

// One anchor at a time per block: all its tracked cells, nthr threads of C slots
// (M[r0][C/4][nthr][4]).  The blocks are persistent: the slot table is the same for every anchor,
// so each thread decodes its part once (the run boundaries and the padding into two registers;
// the run, first cell, offset and orientation of each run's first slot into LDS, where each
// thread reads back only its own entries), so that per anchor there is one round of loads (the
// state and the psi gathers, all issued before any is used).  The blocks on one XCD
// (the dispatcher deals blocks to the 8 XCDs in turn) take the anchors of one contiguous range in
// turn.  Per sub-step: the anchor's coarse density (a wave butterfly,
// then the waves' sums in a fixed order: the same bits on every thread), its clamp factor and
// pool, then both RK2 stages in registers.  (Issuing the next anchor's loads before the current
// anchor's steps, with barriers that fence LDS only, measured no faster at the benchmark workload:
// 1053 against 1031 us per launch; nor did two blocks per CU: 1167.)
template <typename T, int C, int LIM>
__global__ __launch_bounds__(1024) void k_r0_anchor(const T *__restrict__ Min, T *__restrict__ Mout,
                                                    T *__restrict__ q01, const int2 *__restrict__ tab,
                                                    const T *__restrict__ psi, R0Const<T> c, int nrun, int nsub,
                                                    double w, double m_total, double k_on) {
    static_assert(C % 4 == 0, "slots come in groups of 4");
    typedef T TV4 __attribute__((ext_vector_type(4)));
    typedef T T2 __attribute__((ext_vector_type(2)));
    __shared__ double red[2][16];
    extern __shared__ int lds_tab[];  // [2][C][nthr]: run | lo << 20, packed (a, b, k) (-1: none)
    const int nthr = blockDim.x;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = nthr >> 6;
    int *exl = lds_tab, *eyl = lds_tab + C * nthr;
    uint32_t cont = 0;  // bit j: slot j continues the run of slot j - 1
    int nfill = 0;      // slots before the padding
    {
        int2 e[C];
#pragma unroll
        for (int j = 0; j < C; ++j) e[j] = tab[j * nthr + t];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const bool first = j == 0 || e[j].x != e[j > 0 ? j - 1 : 0].x;
            cont |= first ? 0u : 1u << j;
            nfill += e[j].x >= 0;
            exl[j * nthr + t] = e[j].x;
            eyl[j * nthr + t] = first && e[j].x >= 0 ? e[j].y : -1;
        }
    }
    const int xcd = blockIdx.x & 7, bx = blockIdx.x >> 3, nbx = gridDim.x >> 3;
    const int64_t per = (c.nxy + 7) / 8, r_end = min(c.nxy, (int64_t)(xcd + 1) * per);
    // loads of anchor r: the state (nontemporal: M_b is streamed once and must not push the run
    // totals out of L2; a thread's 4 slots of a group are one 16-byte (FP64: 32-byte) load,
    // padding included) and psi(x, th_k) of each run at the anchor, x = r + (a, b), gathered at
    // its first slot (32-bit offsets: nx ny nth < 2^31 for this kernel)
    TV4 v[C / 4];
    T g[C];
    auto issue = [&](int64_t r) {
        const TV4 *src = reinterpret_cast<const TV4 *>(Min + r * (int64_t)(C * nthr));
#pragma unroll
        for (int q = 0; q < C / 4; ++q) v[q] = __builtin_nontemporal_load(src + q * nthr + t);
        const int i0 = (int)(r / c.ny), j0 = (int)(r - (int64_t)i0 * c.ny);
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int f = eyl[j * nthr + t];
            g[j] = T(0);
            if (f >= 0) {
                const int a = (f & 2047) - 1024, b = ((f >> 11) & 2047) - 1024, k = f >> 22;
                g[j] = psi[(wrap1(i0 + a, c.nx) * c.ny + wrap1(j0 + b, c.ny)) * c.nth + k];
            }
        }
    };
    int ph = 0;  // sub-steps so far: which half of red
    // The final state of an anchor and its run totals are stored after the next anchor's loads
    // are issued, so that the stores drain while that anchor is stepped (all blocks leave an
    // anchor at about the same time; stored at once, the state and run totals of 256 blocks
    // queue behind each other): 991-994 against 1080-1104 us per launch at the benchmark
    // workload.  It needs a second copy of the state in registers: FP32 up to 16 slots, FP64 up
    // to 8; otherwise each anchor is stored at its end.
    constexpr bool LATE = sizeof(T) == 4 ? C <= 16 : C <= 8;
    T yp[C];
    int64_t rp = -1;  // the anchor whose final state yp holds
    auto store = [&](int64_t r) {
        TV4 *dst = reinterpret_cast<TV4 *>(Mout + r * (int64_t)(C * nthr));
#pragma unroll
        for (int q = 0; q < C / 4; ++q) {  // (padding slots are stored too: never used)
            TV4 o;
#pragma unroll
            for (int u = 0; u < 4; ++u) o[u] = yp[4 * q + u];
            __builtin_nontemporal_store(o, dst + q * nthr + t);
        }
        // run totals of the final state by anchor
        double t0 = 0.0, t1 = 0.0, lw = 0.0;
        int run = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            if (!((cont >> j) & 1u)) {
                const int ex = exl[j * nthr + t];
                run = ex & 0xFFFFF;
                t0 = t1 = 0.0;
                lw = (double)(ex >> 20) + 0.5 - c.half_ns;
            }
            t0 += (double)yp[j];
            t1 += lw * (double)yp[j];
            lw += 1.0;
            if (j < nfill && (j + 1 == nfill || !((cont >> (j + 1 < C ? j + 1 : j)) & 1u))) {
                // (q0, q1) side by side, in tiles of 16 anchors: q01[r0 / 16][run][r0 % 16].
                // The tile's 16 anchors are in flight at the same time on one XCD, so each line
                // of 16 pairs forms whole in its L2, and a block's stores stay inside one tile
                T2 q;
                q.x = (T)(t0 * c.ds);
                q.y = (T)(t1 * c.ds2);
                *reinterpret_cast<T2 *>(q01 + 2 * r0_pair_index(r, run, nrun)) = q;
            }
        }
    };
    for (int64_t r0 = (int64_t)xcd * per + bx; r0 < r_end; r0 += nbx) {
        issue(r0);
        if (LATE && rp >= 0) store(rp);
        T y[C], wg[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            y[j] = j < nfill ? v[j >> 2][j & 3] : T(0);
            wg[j] = ((cont >> j) & 1u) ? wg[j > 0 ? j - 1 : 0] : g[j];
        }
        for (int sub = 0; sub < nsub; ++sub, ++ph) {
            // the thread's part of the coarse density in the field precision (at most 24 terms),
            // the threads' parts in FP64
            T pt = T(0);
#pragma unroll
            for (int j = 0; j < C; ++j) pt += wg[j] * y[j];
            const double part = group_sum<64>((double)pt);
            if (lane == 0) red[ph & 1][wv] = part;
            __syncthreads();  // (the other half's reads of the sub-step before were done before it)
            double tot = 0.0;
            for (int q = 0; q < nw; ++q) tot += red[ph & 1][q];
            const double B = tot * w;
            const bool over = B > m_total;
            const T sc = (T)(over ? m_total / B : 1.0);
            const T src = (T)(k_on * (over ? 0.0 : m_total - B));
#pragma unroll
            for (int j = 0; j < C; ++j) y[j] = sc * y[j];
            // the run-end masks are taken from cont inside the step (made opaque here, so that
            // the compiler does not hoist one mask register per slot out of the loop)
            uint32_t cs = cont;
            asm volatile("" : "+v"(cs));
            anchor_rk2<T, C, LIM>(y, cs, c.half_dt, c.dt, c.nv_ds, src, c.k_off);
        }
#pragma unroll
        for (int j = 0; j < C; ++j) yp[j] = y[j];
        if (LATE)
            rp = r0;
        else
            store(r0);
    }
    if (LATE && rp >= 0) store(rp);
}

// m0(x, th) = dA sum over the runs s of orientation th of q0 of run s at anchor x - (a_s, b_s)
// (and m1 from q1; the pairs (q0, q1) side by side in tiles of 16 anchors), in run order.  A
// wave: 64 consecutive filament cells, so a run's loads are 64 consecutive anchors: 4 or 5 lines.
template <typename T>
__global__ __launch_bounds__(256) void k_r0_marg(const T *__restrict__ q01, int nrun,
                                                 const R0Seg *__restrict__ seg, const int32_t *__restrict__ seg_start,
                                                 T *__restrict__ m0, T *__restrict__ m1, R0Const<T> c) {
    typedef T T2 __attribute__((ext_vector_type(2)));
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int k = blockIdx.y;
    const bool okx = x < c.nxy;
    const int64_t xz = okx ? x : 0;
    const int iv = (int)(xz / c.ny), jv = (int)(xz - (int64_t)iv * c.ny);
    double s0 = 0.0, s1 = 0.0;
    const int s_end = seg_start[k + 1];
#pragma unroll 4
    for (int s = seg_start[k]; s < s_end; ++s) {
        const R0Seg r = seg[s];
        const int64_t a = r0_pair_index((int64_t)wrap1(iv - r.a, c.nx) * c.ny + wrap1(jv - r.b, c.ny), s, nrun);
        const T2 q = *reinterpret_cast<const T2 *>(q01 + 2 * a);
        s0 += (double)q.x;
        s1 += (double)q.y;
    }
    if (okx) {
        m0[x * c.nth + k] = (T)(s0 * c.dA);
        m1[x * c.nth + k] = (T)(s1 * c.dA);
    }
}

// Anchor layout <-> tiled (tt = 64 vx > 0) or caller (tt = 0) layout, through LDS: a block takes
// 64 consecutive anchors and 64 consecutive positions of the anchor layout.  The anchor side
// moves as 64 rows of 64 consecutive values; on the other side, the cell at one position of 64
// consecutive anchors sits at 64 consecutive filament cells x = r0 + (a, b) (within one row of
// the grid), i.e. consecutive elements.  Padding positions (cell -1) are neither read nor written.
template <typename T>
__global__ __launch_bounds__(256) void k_r0_anchor_layout(const T *__restrict__ src, T *__restrict__ dst,
                                                          const int32_t *__restrict__ cell_pos, R0Const<T> c,
                                                          int tt, int64_t per_anchor, int to_anchor) {
    __shared__ T tile[64][65];
    const int32_t *pos_cell = cell_pos + 3 * c.ncell;
    const int64_t r_base = (int64_t)blockIdx.x * 64, p_base = (int64_t)blockIdx.y * 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // (cell, x) in the other layout
    auto other = [&](int64_t cell, int64_t x) -> int64_t {
        if (tt > 0) {
            const int64_t tl = x / tt;
            return (tl * c.ncell + cell) * tt + (x - tl * tt);
        }
        return cell * c.nxy + x;
    };
    const int64_t ra = r_base + lane;  // this lane's anchor on the other side
    const int ia = (int)(min(ra, c.nxy - 1) / c.ny), ja = (int)(min(ra, c.nxy - 1) - (int64_t)ia * c.ny);
    // the cell and offset of position p_base + lane, read once and broadcast by lane
    const int cell = pos_cell[p_base + lane];
    const int oa = cell >= 0 ? cell_pos[3 * cell + 1] : 0, ob = cell >= 0 ? cell_pos[3 * cell + 2] : 0;
    const int wu = __builtin_amdgcn_readfirstlane(w);
    if (!to_anchor) {
        for (int ai = w; ai < 64; ai += 4) {
            const int64_t r = r_base + ai;
            if (r < c.nxy) tile[ai][lane] = src[r * per_anchor + p_base + lane];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int pi = wu + 4 * q;
            const int cp = __builtin_amdgcn_readlane(cell, pi);
            if (cp < 0 || ra >= c.nxy) continue;
            const int64_t x = (int64_t)wrap1(ia + __builtin_amdgcn_readlane(oa, pi), c.nx) * c.ny +
                              wrap1(ja + __builtin_amdgcn_readlane(ob, pi), c.ny);
            dst[other(cp, x)] = tile[lane][pi];
        }
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int pi = wu + 4 * q;
            const int cp = __builtin_amdgcn_readlane(cell, pi);
            if (cp < 0 || ra >= c.nxy) continue;
            const int64_t x = (int64_t)wrap1(ia + __builtin_amdgcn_readlane(oa, pi), c.nx) * c.ny +
                              wrap1(ja + __builtin_amdgcn_readlane(ob, pi), c.ny);
            tile[lane][pi] = src[other(cp, x)];
        }
        __syncthreads();
        for (int ai = w; ai < 64; ai += 4) {
            const int64_t r = r_base + ai;
            if (r < c.nxy && cell >= 0) dst[r * per_anchor + p_base + lane] = tile[ai][lane];
        }
    }
}

// The tiled layout's padding (filament cells x >= nxy of the last tile) set to 0.
template <typename T>
__global__ __launch_bounds__(256) void k_r0_tiled_pad(T *__restrict__ dst, int64_t ncell, int64_t nxy, int tt) {
    const int64_t last = nxy / tt, rem = nxy - last * tt, pad = tt - rem;
    const int64_t n = ncell * pad;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t cell = e / pad;
        dst[(last * ncell + cell) * tt + rem + (e - cell * pad)] = T(0);
    }
}

// psi [x][th] -> psiT [th][x] (the coarse kernel reads psi at the filament cells of 64 consecutive
// anchors: consecutive x for one orientation).
template <typename T>
__global__ __launch_bounds__(256) void k_r0_psiT(const T *__restrict__ psi, T *__restrict__ psiT, int64_t nxy, int nth) {
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= nxy * nth) return;
    const int64_t k = o / nxy, x = o - k * nxy;
    psiT[o] = psi[x * nth + k];
}

// One lane: one anchor; one wave: one row of partials over every nrow-th run, added in run order.
// The wave's run records come 64 at a time, one per lane (no scalar loads to wait for), and are
// broadcast from there; the run totals and the psi values of four runs are loaded into one of
// two register sets while the other set's four runs are added, so eight runs' loads are in
// flight with no copy of a loaded register (a copy would wait for every load).
template <typename T>
__global__ __launch_bounds__(256) void k_r0_coarse(const T *__restrict__ q0, const T *__restrict__ psiT,
                                                   const R0Seg *__restrict__ seg, double *__restrict__ part,
                                                   R0Const<T> c, int nseg, int nrow, int pairs) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.y * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t r0 = (int64_t)blockIdx.x * 64 + lane;
    const bool ok = r0 < c.nxy;
    const int64_t rz = ok ? r0 : 0;  // lanes past the last anchor load anchor 0 and add nothing
    const int iv = (int)(rz / c.ny), jv = (int)(rz - (int64_t)iv * c.ny);
    double acc = 0.0;
    const int nw = row < nseg ? (nseg - row + nrow - 1) / nrow : 0;
    for (int base = 0; base < nw; base += 64) {
        const int cnt = min(64, nw - base);
        // record of run row + (base + l) nrow in lane l (the last one again past cnt)
        const R0Seg rec = seg[row + (int64_t)(base + min(lane, cnt - 1)) * nrow];
        T qa[4], pa[4], qb[4], pb[4];
        // runs n0 .. n0 + 3 of this batch (clamped to the last, whose repeats are not added)
        auto fetch = [&](T (&q)[4], T (&pv)[4], int n0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int n = min(n0 + u, cnt - 1);
                const int ra = __builtin_amdgcn_readlane(rec.a, n), rb = __builtin_amdgcn_readlane(rec.b, n);
                const int k = __builtin_amdgcn_readlane(rec.pack, n) >> 20;
                const int64_t srun = row + (int64_t)(base + n) * nrow;
                q[u] = pairs ? q0[2 * r0_pair_index(rz, srun, nseg)] : q0[srun * c.nxy + rz];
                // the filament cell of this run at anchor r0: x = r0 + (a, b), periodic
                const int64_t x = (int64_t)wrap1(iv + ra, c.nx) * c.ny + wrap1(jv + rb, c.ny);
                pv[u] = psiT[(int64_t)k * c.nxy + x];
            }
        };
        auto add = [&](const T (&q)[4], const T (&pv)[4], int n0) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (ok && n0 + u < cnt) acc += (double)q[u] * (double)pv[u];
        };
        fetch(qa, pa, 0);
        for (int n0 = 0; n0 < cnt; n0 += 8) {
            fetch(qb, pb, n0 + 4);
            add(qa, pa, n0);
            if (n0 + 4 >= cnt) break;
            fetch(qa, pa, n0 + 8);
            add(qb, pb, n0 + 4);
        }
    }
    if (ok) part[(int64_t)row * c.nxy + r0] = acc;
}

// coarse = w sum of the rows (fixed order); Alg. 2 / Eq. (6): where coarse > m_total the
// anchor's factor is m_total / coarse and the pool 0, else 1 and m_total - coarse (pool 1 and
// no factor without depletion).
// One block: 64 anchors; its four waves add a quarter of the rows each, combined in LDS in a
// fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_r0_pool(const double *__restrict__ part, int nrow, T *__restrict__ scale,
                                                 T *__restrict__ pool, T *__restrict__ coarse_out,
                                                 T *__restrict__ free_out, int64_t nxy, double w, double m_total,
                                                 double k_on) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, qw = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 64 + lane;
    const int per = (nrow + 3) / 4, rb = qw * per, re = min(nrow, rb + per);
    double part_sum = 0.0;
    if (r0 < nxy)
        for (int r = rb; r < re; ++r) part_sum += part[(int64_t)r * nxy + r0];
    red[qw][lane] = part_sum;
    __syncthreads();
    if (qw != 0 || r0 >= nxy) return;
    const double sum = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    const double B = sum * w;
    double f = 1.0;
    if (m_total > 0) {
        const bool over = B > m_total;
        f = over ? 0.0 : m_total - B;
        if (scale != nullptr) {
            scale[r0] = (T)(over ? m_total / B : 1.0);
            pool[r0] = (T)(k_on * f);
        }
    }
    if (coarse_out != nullptr) coarse_out[r0] = (T)B;
    if (free_out != nullptr) free_out[r0] = (T)f;
}

// Between the caller's layout Mb[cell][x] and the tiled one M[tile][cell][tt] (to_tiled = 1: the
// padding of the last tile is set to 0).
template <typename T>
__global__ __launch_bounds__(256) void k_r0_layout(const T *__restrict__ src, T *__restrict__ dst, int64_t ncell,
                                                   int64_t nxy, int tt, int64_t n, int to_tiled) {
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < n; d += (int64_t)gridDim.x * 256) {
        const int64_t per = ncell * tt, tl = d / per, rem = d - tl * per, cell = rem / tt, xi = rem - cell * tt;
        const int64_t x = tl * tt + xi;
        if (to_tiled)
            dst[d] = x < nxy ? src[cell * nxy + x] : T(0);
        else if (x < nxy)
            dst[cell * nxy + x] = src[d];
    }
}

// The anchor-marginal field M[x][k][l] = dx dy sum over anchors of M_b (the r0 integral of
// Eq. (10)), which the motor force spreads.  One wave per block: 64 filament cells and one
// orientation; each lane adds its runs' cells into its own LDS column acc[l][lane] in run order
// (deterministic, no atomics), then the wave writes the block's (x, k) rows of ns contiguous
// values.  acc rows are padded to 65 so that the row-wise reads spread over the banks.
template <typename T>
__global__ __launch_bounds__(64) void k_r0_field(const T *__restrict__ Mb, T *__restrict__ M,
                                                 const R0Seg *__restrict__ seg, const int32_t *__restrict__ seg_start,
                                                 R0Const<T> c, int ns, int tt) {
    extern __shared__ unsigned char smem_raw[];
    T *acc = reinterpret_cast<T *>(smem_raw);  // [ns][65]
    const int lane = threadIdx.x, k = blockIdx.y;
    const int64_t x = (int64_t)blockIdx.x * 64 + lane;
    const bool ok = x < c.nxy;
    for (int l = 0; l < ns; ++l) acc[l * 65 + lane] = T(0);
    const int64_t base = ok ? (x / tt) * c.ncell * tt + (x % tt) : 0;
    const int s_end = seg_start[k + 1];
    for (int s = seg_start[k]; s < s_end; ++s) {
        const R0Seg r = seg[s];
        const int lo = r.pack & 1023, len = (r.pack >> 10) & 1023;
        if (ok)
            for (int t = 0; t < len; ++t) acc[(lo + t) * 65 + lane] += Mb[base + (int64_t)(r.off + t) * tt];
    }
    __syncthreads();
    const T dA = (T)c.dA;
    for (int q = 0; q < 64; ++q) {
        const int64_t x2 = (int64_t)blockIdx.x * 64 + q;
        if (x2 >= c.nxy) break;
        for (int l = lane; l < ns; l += 64) M[(x2 * c.nth + k) * ns + l] = acc[l * 65 + q] * dA;
    }
}

// ---- launchers --------------------------------------------------------------------------------
int r0_vx(size_t esz, int lmax) {
    // runs of at most 8 cells: 2 filament cells a lane (8 bytes in FP32, 16 in FP64; measured
    // at the benchmark workload in FP32: 422 us a launch against 440 with 4 cells and 455 with 1)
    int v = 1;
    if (lmax <= 8) v = 2;
    else if (lmax <= 16) v = (int)(8 / esz);
    return v;
}


int r0_coarse_split(int64_t nxy, int nseg, size_t esz) {
    // about 4096 blocks of 4 waves over the chip, 4 rows of partials per block
    const int64_t target = 4096;
    (void)esz;
    const int64_t gx = (nxy + 63) / 64;
    const int64_t want = (target + gx - 1) / std::max<int64_t>(gx, 1);
    return (int)std::max<int64_t>(1, std::min<int64_t>({want, 64, ((int64_t)nseg + 3) / 4}));
}

int64_t r0_tiled_elems(int64_t ncell, int64_t nxy, int vx) {
    const int64_t tt = 64 * (int64_t)vx;
    return ((nxy + tt - 1) / tt) * ncell * tt;
}

template <typename T, int LM, int VX>
static hipError_t motor_lm(const T *Min, T *Mout, T *q0, T *m0, T *m1, const R0Seg *seg, const int32_t *ss,
                           const T *scale, const T *pool, const R0Const<T> &c, int limiter, hipStream_t s) {
    const dim3 grid((unsigned)((c.nxy + 64 * VX - 1) / (64 * VX)), (unsigned)c.nth);
#define MMK_R0M(LIM, MULTI)                                                                                    \
    hipLaunchKernelGGL((k_r0_motor<T, LM, LIM, VX, MULTI>), grid, dim3(256), 0, s, Min, Mout, q0, m0, m1, seg, ss, \
                       scale, pool, c)
    if (c.nsub > 1) {
        if (limiter == 0) MMK_R0M(0, true); else MMK_R0M(1, true);
    } else {
        if (limiter == 0) MMK_R0M(0, false); else MMK_R0M(1, false);
    }
#undef MMK_R0M
    return hipGetLastError();
}

template <typename T>
hipError_t launch_r0_motor(const T *M_in, T *M_out, T *q0, T *m0, T *m1, const R0Seg *seg, const int32_t *seg_start,
                           const T *scale, const T *pool, const R0Const<T> &c, int lmax, int limiter, hipStream_t s) {
    if (c.nxy <= 0 || c.nth <= 0) return hipSuccess;
    constexpr int V16 = 16 / sizeof(T), V8 = 8 / sizeof(T) > 0 ? 8 / sizeof(T) : 1;
    if (c.vx != r0_vx(sizeof(T), lmax)) return hipErrorInvalidValue;
    if (c.nsub < 1 || (c.nsub > 1 && scale != nullptr)) return hipErrorInvalidValue;  // the clamp is per step
    if (lmax <= 8 && c.vx == 1) return motor_lm<T, 8, 1>(M_in, M_out, q0, m0, m1, seg, seg_start, scale, pool, c, limiter, s);
    if (lmax <= 8 && c.vx == 2) return motor_lm<T, 8, 2>(M_in, M_out, q0, m0, m1, seg, seg_start, scale, pool, c, limiter, s);
    if (lmax <= 8) return motor_lm<T, 8, V16>(M_in, M_out, q0, m0, m1, seg, seg_start, scale, pool, c, limiter, s);
    if (lmax <= 16) return motor_lm<T, 16, V8>(M_in, M_out, q0, m0, m1, seg, seg_start, scale, pool, c, limiter, s);
    if (lmax <= kR0MaxRun) return motor_lm<T, 32, 1>(M_in, M_out, q0, m0, m1, seg, seg_start, scale, pool, c, limiter, s);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_r0_coarse(const T *q0, bool pairs, const T *psi, T *psiT, const R0Seg *seg, double *part, T *scale,
                            T *pool, T *coarse_out, T *free_out, const R0Const<T> &c, int nseg, int nsplit,
                            double dth, double m_total, double k_on, hipStream_t s) {
    if (c.nxy <= 0) return hipSuccess;
    const int64_t np = c.nxy * c.nth;
    hipLaunchKernelGGL(k_r0_psiT<T>, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, psi, psiT, c.nxy, c.nth);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // one anchor per lane (measured at the benchmark workload with the earlier form of the
    // kernel: 98.6 us per coarse pass in FP32 against 109 with 16-byte loads of the run totals)
    hipLaunchKernelGGL((k_r0_coarse<T>), dim3((unsigned)((c.nxy + 63) / 64), (unsigned)nsplit), dim3(256), 0, s,
                       q0, psiT, seg, part, c, nseg, 4 * nsplit, pairs ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double w = c.dA * dth;  // dx dy dth (q0 already carries ds)
    hipLaunchKernelGGL(k_r0_pool<T>, dim3((unsigned)((c.nxy + 63) / 64)), dim3(256), 0, s, part, 4 * nsplit, scale,
                       pool, coarse_out, free_out, c.nxy, w, m_total, k_on);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_r0_layout(const T *src, T *dst, int64_t ncell, int64_t nxy, int vx, bool to_tiled, hipStream_t s) {
    const int64_t n = r0_tiled_elems(ncell, nxy, vx);
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_r0_layout<T>, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, ncell, nxy, 64 * vx, n,
                       to_tiled ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_r0_anchor(const T *M_in, T *M_out, T *q01, const int32_t *slot_tab, const T *psi,
                            const R0Const<T> &c, int nrun, int C, int nthr, int nsub, double m_total, double k_on,
                            double dth, int limiter, hipStream_t s) {
    if (c.nxy <= 0) return hipSuccess;
    if (nthr < 64 || nthr > 1024 || nthr % 64 != 0 || nsub < 1) return hipErrorInvalidValue;
    // persistent blocks: as many as fit the device at once (a multiple of 8, one share per XCD),
    // at most one per anchor
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int per_cu = 1;  // registers and LDS: one block per CU
    const int64_t per = (c.nxy + 7) / 8;
    const int64_t nbx = std::max<int64_t>(1, std::min<int64_t>(per, (int64_t)ncu * per_cu / 8));
    const dim3 grid((unsigned)(8 * nbx)), block((unsigned)nthr);
    const size_t lds = r0_anchor_lds(C, nthr);
    const double w = c.dA * dth * c.ds;  // dx dy dth ds
    const int2 *tab = reinterpret_cast<const int2 *>(slot_tab);
    // (24 slots are FP32 only: the FP64 case instantiates nothing new)
    constexpr int C24 = sizeof(T) == 4 ? 24 : 16;
#define MMK_R0A(C_, CT_)                                                                                          \
    case C_:                                                                                                     \
        if (limiter == 0)                                                                                        \
            hipLaunchKernelGGL((k_r0_anchor<T, CT_, 0>), grid, block, lds, s, M_in, M_out, q01, tab, psi,            \
                               c, nrun, nsub, w, m_total, k_on);                                                 \
        else                                                                                                     \
            hipLaunchKernelGGL((k_r0_anchor<T, CT_, 1>), grid, block, lds, s, M_in, M_out, q01, tab, psi,            \
                               c, nrun, nsub, w, m_total, k_on);                                                 \
        break;
    if (sizeof(T) == 8 && C > 16) return hipErrorInvalidValue;
    switch (C) {
        MMK_R0A(4, 4)
        MMK_R0A(8, 8)
        MMK_R0A(16, 16)
        MMK_R0A(24, C24)
        default: return hipErrorInvalidValue;
    }
#undef MMK_R0A
    return hipGetLastError();
}

template <typename T>
hipError_t launch_r0_marg(const T *q01, int nrun, const R0Seg *seg, const int32_t *seg_start, T *m0, T *m1,
                          const R0Const<T> &c, hipStream_t s) {
    if (c.nxy <= 0 || c.nth <= 0) return hipSuccess;
    const dim3 grid((unsigned)((c.nxy + 255) / 256), (unsigned)c.nth);
    hipLaunchKernelGGL(k_r0_marg<T>, grid, dim3(256), 0, s, q01, nrun, seg, seg_start, m0, m1, c);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_r0_anchor_layout(const T *src, T *dst, const int32_t *cell_pos, const R0Const<T> &c, int vx,
                                   int64_t per_anchor, int nthr, bool to_anchor, hipStream_t s) {
    (void)nthr;  // (the positions of the anchor layout carry their cells: cell_pos after its 3 ncell values)
    if (c.ncell <= 0 || c.nxy <= 0) return hipSuccess;
    if (per_anchor <= 0 || per_anchor % 64 != 0 || per_anchor / 64 > 65535) return hipErrorInvalidValue;
    const int tt = 64 * vx;
    if (!to_anchor && vx > 0 && c.nxy % tt != 0) {
        const int64_t n = c.ncell * (tt - c.nxy % tt);
        hipLaunchKernelGGL(k_r0_tiled_pad<T>, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65536)), dim3(256), 0,
                           s, dst, c.ncell, c.nxy, tt);
    }
    hipLaunchKernelGGL(k_r0_anchor_layout<T>, dim3((unsigned)((c.nxy + 63) / 64), (unsigned)(per_anchor / 64)),
                       dim3(256), 0, s, src, dst, cell_pos, c, tt, per_anchor, to_anchor ? 1 : 0);
    return hipGetLastError();
}

size_t r0_anchor_lds(int C, int nthr) { return (size_t)2 * C * nthr * sizeof(int); }

size_t r0_field_lds(int ns, size_t esz) { return (size_t)ns * 65 * esz; }

template <typename T>
hipError_t launch_r0_field(const T *Mb, T *M, const R0Seg *seg, const int32_t *seg_start, const R0Const<T> &c, int ns,
                           hipStream_t s) {
    if (c.nxy <= 0 || c.nth <= 0) return hipSuccess;
    const size_t lds = r0_field_lds(ns, sizeof(T));
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((c.nxy + 63) / 64), (unsigned)c.nth);
    hipLaunchKernelGGL(k_r0_field<T>, grid, dim3(64), lds, s, Mb, M, seg, seg_start, c, ns, 64 * c.vx);
    return hipGetLastError();
}

#define MMK_R0_INST(T)                                                                                              \
    template hipError_t launch_r0_motor<T>(const T *, T *, T *, T *, T *, const R0Seg *, const int32_t *, const T *, \
                                           const T *, const R0Const<T> &, int, int, hipStream_t);                   \
    template hipError_t launch_r0_coarse<T>(const T *, bool, const T *, T *, const R0Seg *, double *, T *, T *, T *, \
                                            T *, const R0Const<T> &, int, int, double, double, double, hipStream_t); \
    template hipError_t launch_r0_layout<T>(const T *, T *, int64_t, int64_t, int, bool, hipStream_t);            \
    template hipError_t launch_r0_anchor<T>(const T *, T *, T *, const int32_t *, const T *, const R0Const<T> &,     \
                                            int, int, int, int, double, double, double, int, hipStream_t);         \
    template hipError_t launch_r0_marg<T>(const T *, int, const R0Seg *, const int32_t *, T *, T *,                  \
                                          const R0Const<T> &, hipStream_t);                                        \
    template hipError_t launch_r0_anchor_layout<T>(const T *, T *, const int32_t *, const R0Const<T> &, int, int64_t, \
                                                   int, bool, hipStream_t);                                         \
    template hipError_t launch_r0_field<T>(const T *, T *, const R0Seg *, const int32_t *, const R0Const<T> &, int, \
                                           hipStream_t);
MMK_R0_INST(float)
MMK_R0_INST(double)

}  // namespace mmk
