// Motor column step (walk + attach/detach along filament arclength s) for gfx950.
//
// Model: Cook & Shinar, Sec. 2 Eq. (4) with linear attachment k_on and detachment k_off M,
// walking speed v0 towards the plus end; superbee-limited upwind flux in s (Sec. 2); the
// two-stage Runge-Kutta of Sec. 3.1 / Alg. 2 as the explicit midpoint rule.  Boundary
// readings: no walking influx at s = 0 (ghost M_{-1} = 0, flux 0), first-order free outflow
// at s = L (ghost M_{ns} = M_{ns-1}, so the last slope is 0 and the last flux is v0 M).
//
// Layout: M[col][s] with s contiguous.  A column of ns = CPL * LPC cells is spread over LPC
// consecutive lanes (one 16-lane DPP row or a part of it), CPL cells per lane, loaded with
// 16-byte vector loads.  Neighbour cells across lanes move with DPP row shifts; the
// s-reductions m0, m1 are DPP butterflies inside the group.  Both Runge-Kutta stages live
// in registers: one read and one write of M per step, the HBM floor of this update.
#include "device_util.h"
#include "kernels.h"

#include <type_traits>

namespace mmk {

// Face differences dh_l = h_l - h_{l-1} on this lane's CPL cells, with the face value
// h_l = z_l + sigma_l / 2 (flux v0 h_l; h_{-1} = 0 carries the zero influx, and the zero last
// slope makes h_{ns-1} = z_{ns-1}, the first-order outflow), so that
//   R_l = -(v0/ds) dh_l + (src - k_off z_l),  src = k_on times the free pool.
// g: lane index inside the column group; l0 = g * CPL.
template <typename T, int CPL, int LPC, int LIM, bool RAGGED>
__device__ __forceinline__ void motor_dh(const T (&z)[CPL], T (&R)[CPL], int g, int l0, int ns) {
    const T zl = from_prev0<LPC>(z[CPL - 1], g);             // z_{l0-1}; ghost 0 at s = 0
    const T zr = from_next<LPC>(z[0], z[CPL - 1], g);        // z_{l0+CPL}; ghost at s = L
    T d[CPL + 1];                                             // d[j] = z_{l0+j} - z_{l0+j-1}
    d[0] = z[0] - zl;
#pragma unroll
    for (int j = 1; j < CPL; ++j) d[j] = z[j] - z[j - 1];
    d[CPL] = zr - z[CPL - 1];
    if constexpr (RAGGED) {
        // the cell right of l = ns-1 is the ghost z_{ns} = z_{ns-1}: zero difference
#pragma unroll
        for (int j = 0; j < CPL; ++j)
            if (l0 + j + 1 >= ns) d[j + 1] = T(0);
    }
    T h[CPL];                                                 // face value at l + 1/2
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const T sig = (LIM == 0) ? superbee(d[j], d[j + 1]) : T(0);
        h[j] = z[j] + T(0.5) * sig;
    }
    const T hl = from_prev0<LPC>(h[CPL - 1], g);             // h_{-1} = 0: no influx
#pragma unroll
    for (int j = 0; j < CPL; ++j) R[j] = h[j] - ((j == 0) ? hl : h[j - 1]);
}

// The lane's part of m0 = ds sum M: its CPL cells added pairwise in the cell precision (log2 CPL
// roundings on any path, at most 4 units of 2^-24 relative for 16 FP32 cells of one sign), then
// widened once.  The lanes' parts are added in FP64 (column_total) and the total rounded once:
// measured as accurate as Kahan-compensated FP32 sums and 10% faster in the blocked FP32 launch,
// where the sum is taken every micro-step.
template <typename T, int CPL, bool RAGGED>
__device__ __forceinline__ double lane_m0(const T (&y)[CPL], int l0, int ns) {
    T t[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) t[j] = (!RAGGED || l0 + j < ns) ? y[j] : T(0);
#pragma unroll
    for (int w = CPL; w > 1; w >>= 1)
#pragma unroll
        for (int i = 0; i < w / 2; ++i) t[i] = t[2 * i] + t[2 * i + 1];
    return (double)t[0];
}

// The lane's part of m1 = ds^2 sum (l + 1/2 - ns/2) M (the weights are exact half-integers; wb
// is the weight of the lane's first cell): products and sums in FP64, in order (output steps).
template <typename T, int CPL, bool RAGGED>
__device__ __forceinline__ double lane_m1(const T (&y)[CPL], int l0, int ns, T wb) {
    double a1 = 0.0;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const T v = (!RAGGED || l0 + j < ns) ? y[j] : T(0);
        a1 = (j == 0) ? (double)v * (double)wb : a1 + (double)v * (double)(wb + T(j));
    }
    return a1;
}

// Column total of the lane partials in FP64 (every lane of the group; with PAIR, the m0 total in
// the lower half of the group and the m1 total in the upper half), rounded once by the caller.
template <int LPC, bool PAIR>
__device__ __forceinline__ double column_total(double v0, double v1, int g) {
    return group_sum_pair<LPC, false, PAIR, double>(v0, 0.0, v1, 0.0, g);
}

// Occupancy target of k_motor_step: FP32 columns of 16 cells a lane (the blocked launch) are
// held to 64 VGPRs, 8 waves per SIMD (measured 4% faster than the compiler's choice of 78 VGPRs
// and 6 waves: the extra waves cover the dependent limiter and reduction chains); the other
// tilings keep the compiler's allocation (forced down, the larger ones spill).
template <typename T, int CPL, bool RAGGED>
constexpr int motor_waves_per_eu() {
    return (sizeof(T) == 4 && CPL == 16 && !RAGGED) ? 8 : 1;
}

// NT: bit 0 nontemporal loads of M, bit 1 nontemporal stores.
template <typename T, int CPL, int LPC, int LIM, bool RAGGED, bool WANT_M1, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(motor_waves_per_eu<T, CPL, RAGGED>())))
void k_motor_step(const T *__restrict__ M_in, T *__restrict__ M_out,
                                                    T *__restrict__ m0, T *__restrict__ m1,
                                                    int64_t ncol, int ns, MotorConst<T> c,
                                                    const T *__restrict__ Dxy) {
    constexpr int COLS = 256 / LPC;
    const int g = threadIdx.x % LPC;
    const int64_t col = (int64_t)blockIdx.x * COLS + threadIdx.x / LPC;
    const bool active = col < ncol;
    const int l0 = g * CPL;
    const int64_t base = col * (int64_t)ns + l0;

    // free-motor depletion (Eq. (6)) with the over-binding clamp of Alg. 2: the clamp factor
    // and the free pool of this column's (x, y), loaded beside the column
    T scale = T(1), pool = T(0);
    if (Dxy) {
        const int64_t cc = active ? col : 0;
        const int64_t xy = c.nth_shift >= 0 ? (cc >> c.nth_shift) : cc / c.nth;
        scale = Dxy[2 * xy];
        pool = Dxy[2 * xy + 1];
    }

    T x[CPL];
    if constexpr (!RAGGED) {
        if (active) {
            load_cells<T, CPL, (NT & 1) != 0>(M_in + base, x);
        } else {
#pragma unroll
            for (int j = 0; j < CPL; ++j) x[j] = T(0);
        }
    } else {
#pragma unroll
        for (int j = 0; j < CPL; ++j) x[j] = (active && l0 + j < ns) ? M_in[base + j] : T(0);
    }

    T src = c.k_on;
    if (Dxy) {
#pragma unroll
        for (int j = 0; j < CPL; ++j) x[j] *= scale;
        src = c.k_on * pool;
    }

    // One micro-step: c.nsub explicit-midpoint steps of c.dt in registers (sub-cycling:
    // the local dt* of Alg. 2); the first is outside the loop so that one step compiles as
    // straight code.  x: the state before, y: after.  The half step
    //   y = x + (dt/2) R(x) = (1 - (dt/2) k_off) x + (dt/2) src + (dt/2)(-v0/ds) dh
    // takes its constants folded (two multiply-adds per cell); the full step is
    //   y = x + dt (-(v0/ds) dh + (src - k_off y)).
    const T fa = T(1) - c.half_dt * c.k_off, fb = c.half_dt * src, fg = c.half_dt * c.nv_ds;
    T R[CPL], y[CPL];
    auto rk2 = [&]() {
        motor_dh<T, CPL, LPC, LIM, RAGGED>(x, R, g, l0, ns);
#pragma unroll
        for (int j = 0; j < CPL; ++j) y[j] = fg * R[j] + (fa * x[j] + fb);
        motor_dh<T, CPL, LPC, LIM, RAGGED>(y, R, g, l0, ns);
#pragma unroll
        for (int j = 0; j < CPL; ++j) y[j] = x[j] + c.dt * (c.nv_ds * R[j] + (src - c.k_off * y[j]));
    };
    auto micro = [&]() {
        rk2();
        for (int q = 1; q < c.nsub; ++q) {
#pragma unroll
            for (int j = 0; j < CPL; ++j) x[j] = y[j];
            rk2();
        }
    };
    // Temporal blocking (c.nstep > 1): the column stays in registers for nstep micro-steps;
    // each but the last leaves its m0 for the psi step (the same bits as an unblocked step),
    // and only the last is stored.
    for (int t = 0; t + 1 < c.nstep; ++t) {
        micro();
        const double tot = column_total<LPC, false>(lane_m0<T, CPL, RAGGED>(y, l0, ns), 0.0, g);
        if (active && g == 0) c.m0_steps[(int64_t)t * ncol + col] = (T)(tot * (double)c.ds);
#pragma unroll
        for (int j = 0; j < CPL; ++j) x[j] = y[j];
    }
    micro();

    if constexpr (!RAGGED) {
        if (active) store_cells<T, CPL, (NT & 2) != 0>(M_out + base, y);
    } else {
#pragma unroll
        for (int j = 0; j < CPL; ++j)
            if (active && l0 + j < ns) M_out[base + j] = y[j];
    }

    // s-moments of the new column: m0 = ds sum M, m1 = ds^2 sum (l + 1/2 - ns/2) M, the
    // weights being exact half-integers; lane partials (lane_m0, lane_m1), then the column
    // total in FP64 (column_total), rounded once.  On output steps one paired butterfly serves
    // both: lane 0 of the group ends with m0, lane LPC/2 with m1; m0 has the same bits on every
    // step.
    const double a1 = WANT_M1 ? lane_m1<T, CPL, RAGGED>(y, l0, ns, T(0.5) * (T)(2 * l0 + 1 - ns)) : 0.0;
    const double tot = column_total<LPC, WANT_M1>(lane_m0<T, CPL, RAGGED>(y, l0, ns), a1, g);
    if (active && g == 0) m0[col] = (T)(tot * (double)c.ds);
    if constexpr (WANT_M1)
        if (active && g == LPC / 2) m1[col] = (T)(tot * (double)c.ds2);
}

// ---------------------------------------------------------------------------------------
// Chunked tiling: lane g of a group of LPC lanes (2 .. 16, inside one DPP row) holds NCH
// chunks of W = 16 / sizeof(T) consecutive cells, chunk c covering cells [(c LPC + g) W, +W).
// Every wave instruction then loads or stores whole 16-byte spans of one chunk row, the column
// spans fewer lanes, and the s-reduction butterfly is shorter.  Cell order is chunk-major, so
// the neighbour of a chunk's first (last) cell is in lane g-1 (g+1) of the same chunk, or at
// the group edge in lane LPC-1 of the previous chunk (lane 0 of the next chunk).
template <int LPC, typename T>
__device__ __forceinline__ T chunk_left(const T &same_src, const T &wrap_src, bool has_wrap, T edge, int g) {
    const T s = dpp_any<DPP_ROW_SHR1>(same_src);                      // lane g-1
    T w = edge;
    if (has_wrap) w = dpp_any<0x100 + (LPC - 1)>(wrap_src);           // lane g+LPC-1
    return (g == 0) ? w : s;
}
template <int LPC, typename T>
__device__ __forceinline__ T chunk_right(const T &same_src, const T &wrap_src, bool has_wrap, T edge, int g) {
    const T s = dpp_any<DPP_ROW_SHL1>(same_src);                      // lane g+1
    T w = edge;
    if (has_wrap) w = dpp_any<0x110 + (LPC - 1)>(wrap_src);           // lane g-LPC+1
    return (g == LPC - 1) ? w : s;
}

template <typename T, int NCH, int LPC, int LIM>
__device__ __forceinline__ void motor_rhs_chunked(const T (&z)[NCH][16 / sizeof(T)], T (&R)[NCH][16 / sizeof(T)],
                                                  const MotorConst<T> &c, int g) {
    constexpr int W = 16 / sizeof(T);
    T h[NCH][W];
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
        const T zl = chunk_left<LPC>(z[q][W - 1], z[q > 0 ? q - 1 : 0][W - 1], q > 0, T(0), g);
        const T zr = chunk_right<LPC>(z[q][0], z[q + 1 < NCH ? q + 1 : q][0], q + 1 < NCH, z[q][W - 1], g);
        T d[W + 1];
        d[0] = z[q][0] - zl;
#pragma unroll
        for (int j = 1; j < W; ++j) d[j] = z[q][j] - z[q][j - 1];
        d[W] = zr - z[q][W - 1];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const T sig = (LIM == 0) ? superbee(d[j], d[j + 1]) : T(0);
            h[q][j] = z[q][j] + T(0.5) * sig;
        }
    }
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
        const T hl = chunk_left<LPC>(h[q][W - 1], h[q > 0 ? q - 1 : 0][W - 1], q > 0, T(0), g);
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const T left = (j == 0) ? hl : h[q][j - 1];
            R[q][j] = c.nv_ds * (h[q][j] - left) + (c.k_on - c.k_off * z[q][j]);
        }
    }
}

template <typename T, int NCH, int LPC, int LIM, bool WANT_M1, bool NT>
__global__ __launch_bounds__(256) void k_motor_step_chunked(const T *__restrict__ M_in, T *__restrict__ M_out,
                                                            T *__restrict__ m0, T *__restrict__ m1, int64_t ncol,
                                                            int ns, MotorConst<T> c) {
    constexpr int W = 16 / sizeof(T);
    constexpr int COLS = 256 / LPC;
    const int g = threadIdx.x % LPC;
    const int64_t col = (int64_t)blockIdx.x * COLS + threadIdx.x / LPC;
    const bool active = col < ncol;
    const int64_t cbase = col * (int64_t)ns;
    T x[NCH][W], R[NCH][W], y[NCH][W];
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
        if (active) {
            load_cells<T, W, NT>(M_in + cbase + (q * LPC + g) * W, x[q]);
        } else {
#pragma unroll
            for (int j = 0; j < W; ++j) x[q][j] = T(0);
        }
    }
    // one micro-step of c.nsub midpoint steps (x before, y after), as in k_motor_step
    auto rk2 = [&]() {
        motor_rhs_chunked<T, NCH, LPC, LIM>(x, R, c, g);
#pragma unroll
        for (int q = 0; q < NCH; ++q)
#pragma unroll
            for (int j = 0; j < W; ++j) y[q][j] = x[q][j] + c.half_dt * R[q][j];
        motor_rhs_chunked<T, NCH, LPC, LIM>(y, R, c, g);
#pragma unroll
        for (int q = 0; q < NCH; ++q)
#pragma unroll
            for (int j = 0; j < W; ++j) y[q][j] = x[q][j] + c.dt * R[q][j];
    };
    auto keep = [&]() {
#pragma unroll
        for (int q = 0; q < NCH; ++q)
#pragma unroll
            for (int j = 0; j < W; ++j) x[q][j] = y[q][j];
    };
    auto micro = [&]() {
        rk2();
        for (int s = 1; s < c.nsub; ++s) {
            keep();
            rk2();
        }
    };
    // temporal blocking: m0 of every micro-step but the last into c.m0_steps
    for (int t = 0; t + 1 < c.nstep; ++t) {
        micro();
        if constexpr (std::is_same<T, float>::value) {
            Kahan a0;
#pragma unroll
            for (int q = 0; q < NCH; ++q)
#pragma unroll
                for (int j = 0; j < W; ++j) a0.add(y[q][j]);
            const float s0 = group_sum_comp<LPC>(a0.sum, a0.comp);
            if (active && g == 0) c.m0_steps[(int64_t)t * ncol + col] = s0 * c.ds;
        } else {
            T a0 = 0;
#pragma unroll
            for (int q = 0; q < NCH; ++q)
#pragma unroll
                for (int j = 0; j < W; ++j) a0 += y[q][j];
            const T s0 = group_sum<LPC>(a0);
            if (active && g == 0) c.m0_steps[(int64_t)t * ncol + col] = s0 * c.ds;
        }
        keep();
    }
    micro();
    if (active)
#pragma unroll
        for (int q = 0; q < NCH; ++q) store_cells<T, W, NT>(M_out + cbase + (q * LPC + g) * W, y[q]);

    // s-moments; cell index l = (q LPC + g) W + j, m1 weight (l + 1/2 - ns/2) exact
    if constexpr (std::is_same<T, float>::value) {
        Kahan a0, a1;
#pragma unroll
        for (int q = 0; q < NCH; ++q)
#pragma unroll
            for (int j = 0; j < W; ++j) {
                a0.add(y[q][j]);
                if constexpr (WANT_M1) a1.add(y[q][j] * (0.5f * (float)(2 * ((q * LPC + g) * W + j) + 1 - ns)));
            }
        const float s0 = group_sum_comp<LPC>(a0.sum, a0.comp);
        if (active && g == 0) m0[col] = s0 * c.ds;
        if constexpr (WANT_M1) {
            const float s1 = group_sum_comp<LPC>(a1.sum, a1.comp);
            if (active && g == 0) m1[col] = s1 * c.ds2;
        }
    } else {
        T a0 = 0, a1 = 0;
#pragma unroll
        for (int q = 0; q < NCH; ++q)
#pragma unroll
            for (int j = 0; j < W; ++j) {
                a0 += y[q][j];
                if constexpr (WANT_M1) a1 += y[q][j] * (T(0.5) * (T)(2 * ((q * LPC + g) * W + j) + 1 - ns));
            }
        const T s0 = group_sum<LPC>(a0);
        if (active && g == 0) m0[col] = s0 * c.ds;
        if constexpr (WANT_M1) {
            const T s1 = group_sum<LPC>(a1);
            if (active && g == 0) m1[col] = s1 * c.ds2;
        }
    }
}

template <typename T, int NCH, int LPC>
static hipError_t launch_chunked(const T *M_in, T *M_out, T *m0, T *m1, int64_t ncol, int ns, int limiter,
                                 const MotorConst<T> &c, hipStream_t s, bool nt) {
    constexpr int COLS = 256 / LPC;
    const int64_t blocks = (ncol + COLS - 1) / COLS;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)blocks);
#define MMK_CH(LIM, M1, NTV)                                                                                   \
    hipLaunchKernelGGL((k_motor_step_chunked<T, NCH, LPC, LIM, M1, NTV>), grid, dim3(256), 0, s, M_in, M_out, m0, \
                       m1, ncol, ns, c)
    if (limiter == 0) {
        if (m1) { if (nt) MMK_CH(0, true, true); else MMK_CH(0, true, false); }
        else { if (nt) MMK_CH(0, false, true); else MMK_CH(0, false, false); }
    } else {
        if (m1) { if (nt) MMK_CH(1, true, true); else MMK_CH(1, true, false); }
        else { if (nt) MMK_CH(1, false, true); else MMK_CH(1, false, false); }
    }
#undef MMK_CH
    return hipGetLastError();
}

template <typename T, int CPL, int LPC, bool RAGGED, int LIM, int NT>
static hipError_t launch_nt(const T *M_in, T *M_out, T *m0, T *m1, int64_t ncol, int ns,
                            const MotorConst<T> &c, const T *Dxy, hipStream_t s, unsigned blocks) {
    if (m1)
        hipLaunchKernelGGL((k_motor_step<T, CPL, LPC, LIM, RAGGED, true, NT>), dim3(blocks), dim3(256), 0, s,
                           M_in, M_out, m0, m1, ncol, ns, c, Dxy);
    else
        hipLaunchKernelGGL((k_motor_step<T, CPL, LPC, LIM, RAGGED, false, NT>), dim3(blocks), dim3(256), 0, s,
                           M_in, M_out, m0, m1, ncol, ns, c, Dxy);
    return hipGetLastError();
}

// Streaming (nontemporal) accesses of M, as a mask (bit 0 loads, bit 1 stores).  opt -1 (the
// default): in FP32 a launch of one step per load streams both (keeps psi and m0 of the next psi
// step in the caches: measured faster); a launch of several micro-steps or sub-steps per load
// streams neither (its nontemporal 16-byte stores each cover a quarter of a lane's 64-byte span
// and wrote 1.22x the bytes, plain stores merge in the L2 to 1.00x; measured 1256 against
// 1272 us per 10-micro-step launch at 256x256x64x64, 1265 with nontemporal loads only); FP64
// plain (streams measured slower there).  opt 0: plain, 1: loads and stores, 2: loads only.
static int motor_nontemporal(int elem, int opt, bool multi) {
    if (opt == 0) return 0;
    if (opt == 1) return 3;
    if (opt == 2) return 1;
    return (elem == 4 && !multi) ? 3 : 0;
}

template <typename T, int CPL, int LPC, bool RAGGED, int LIM>
static hipError_t launch_lim(const T *M_in, T *M_out, T *m0, T *m1, int64_t ncol, int ns,
                             const MotorConst<T> &c, const T *Dxy, hipStream_t s, unsigned blocks) {
    const int nt = RAGGED ? 0 : motor_nontemporal((int)sizeof(T), c.nt, c.nstep > 1 || c.nsub > 1);
    if (nt == 3) return launch_nt<T, CPL, LPC, RAGGED, LIM, 3>(M_in, M_out, m0, m1, ncol, ns, c, Dxy, s, blocks);
    if (nt == 1) return launch_nt<T, CPL, LPC, RAGGED, LIM, 1>(M_in, M_out, m0, m1, ncol, ns, c, Dxy, s, blocks);
    return launch_nt<T, CPL, LPC, RAGGED, LIM, 0>(M_in, M_out, m0, m1, ncol, ns, c, Dxy, s, blocks);
}

template <typename T, int CPL, int LPC, bool RAGGED>
static hipError_t launch_cfg(const T *M_in, T *M_out, T *m0, T *m1, int64_t ncol, int ns,
                             int limiter, const MotorConst<T> &c, const T *Dxy, hipStream_t s) {
    constexpr int COLS = 256 / LPC;
    const int64_t blocks = (ncol + COLS - 1) / COLS;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (limiter == 0)
        return launch_lim<T, CPL, LPC, RAGGED, 0>(M_in, M_out, m0, m1, ncol, ns, c, Dxy, s, (unsigned)blocks);
    return launch_lim<T, CPL, LPC, RAGGED, 1>(M_in, M_out, m0, m1, ncol, ns, c, Dxy, s, (unsigned)blocks);
}

// Lanes per column for the exact tilings (0: use the masked generic kernel).  Default: 16
// bytes of the column per lane (4 FP32 or 2 FP64 cells), so every vector load and store of a
// wave covers one contiguous span.  Wide launches (several micro-steps or sub-steps per load,
// where the arithmetic bounds the launch) take 32 bytes per lane: fewer neighbour exchanges
// and a shorter s-reduction per cell (measured at 64 cells: FP32 +11%, FP64 +29%; one step per
// load is faster with 16); FP32 columns of 64 cells take 64 bytes (16 cells) per lane, another
// 10% (1302 -> 1168 us per 10-micro-step launch at 256x256x64).  want > 0 (the lanes option)
// replaces the default when it leaves 16 to 64 bytes per lane.
static int lanes_per_column(int ns, int elem, bool wide, int want) {
    const int cpl = 16 / elem;
    if (ns < 2 * cpl || ns % cpl != 0) return 0;
    int lpc = ns / cpl;
    if (lpc > 64 || (lpc & (lpc - 1)) != 0) return 0;
    if (wide && elem == 4 && ns == 64) lpc = 4;
    else if (wide && lpc >= 4) lpc /= 2;
    if (want >= 2 && want <= 64 && (want & (want - 1)) == 0 && ns % want == 0) {
        const int c = ns / want;
        if (c * elem >= 16 && c <= 16) lpc = want;
    }
    return lpc;
}

// Chunks of 16 bytes per lane for the chunked tiling (1: plain tiling): `want` (the chunks
// option) where ns allows it.
static int chunks_per_lane(int ns, int elem, int want) {
    const int w = 16 / elem;
    if (want < 2 || ns % (want * w) != 0) return 1;
    const int lpc = ns / (want * w);
    if (lpc < 2 || lpc > 16 || (lpc & (lpc - 1)) != 0) return 1;
    return want;
}

// Depleted micro-step with sub-cycling in one launch (Alg. 2's inner loop with the clamp inside
// it).  One block per (x, y) point holds all nth of its columns, LPC lanes each.  Before each of
// the c.nsub sub-steps of c.dt the block forms the coarse density B = dth sum_k psi_k m0_k of its
// current columns (each column's m0 as in k_motor_step, the sum over k of psi_k m0_k in LDS in a
// fixed order, Kahan and TwoSum in FP32), the clamp factor and the free pool (Eq. (6)); every
// column is scaled and stepped in registers.  M is read and written once per micro-step.
template <typename T, int CPL, int LPC, int LIM, bool WANT_M1>
__global__ __launch_bounds__(1024) void k_motor_depl_sub(const T *__restrict__ M_in, T *__restrict__ M_out,
                                                         T *__restrict__ m0, T *__restrict__ m1,
                                                         const T *__restrict__ psi, int nth, int ns,
                                                         MotorConst<T> c, double dth, double m_total) {
    // column terms psi_k m0_k of sub-step q in part[q & 1]: one barrier per sub-step (the
    // buffer written at q + 2 was read by every wave before it passed the barrier of q + 1)
    __shared__ T part[2][1024 / LPC];
    const int g = threadIdx.x % LPC, k = threadIdx.x / LPC;
    const int lane = threadIdx.x & 63;
    const int64_t col = (int64_t)blockIdx.x * nth + k;
    const int l0 = g * CPL;
    const int64_t base = col * (int64_t)ns + l0;
    T x[CPL], R[CPL], y[CPL];
    load_cells<T, CPL, false>(M_in + base, x);
    const T ps = psi[col];
    for (int q = 0; q < c.nsub; ++q) {
        const double tot = column_total<LPC, false>(lane_m0<T, CPL, false>(x, l0, ns), 0.0, g);
        if (g == 0) part[q & 1][k] = ps * (T)(tot * (double)c.ds);
        __syncthreads();
        // every wave forms B itself in the same fixed order: lane i adds columns i, i + 64, ...
        // in order (Kahan in FP32), then a butterfly over the wave (compensated in FP32)
        T v = T(0), vc = T(0);
        for (int kk = lane; kk < nth; kk += 64) {
            if constexpr (std::is_same<T, float>::value) kahan_add(v, vc, part[q & 1][kk]);
            else v += part[q & 1][kk];
        }
        const T B = group_sum_pair<64, std::is_same<T, float>::value, false, T>(v, vc, T(0), T(0), 0);
        T sc, pool;
        depletion_of(B * (T)dth, (T)m_total, sc, pool);
        const T src = c.k_on * pool;
#pragma unroll
        for (int j = 0; j < CPL; ++j) x[j] *= sc;
        // the midpoint step of k_motor_step, half step with folded constants
        const T fa = T(1) - c.half_dt * c.k_off, fb = c.half_dt * src, fg = c.half_dt * c.nv_ds;
        motor_dh<T, CPL, LPC, LIM, false>(x, R, g, l0, ns);
#pragma unroll
        for (int j = 0; j < CPL; ++j) y[j] = fg * R[j] + (fa * x[j] + fb);
        motor_dh<T, CPL, LPC, LIM, false>(y, R, g, l0, ns);
#pragma unroll
        for (int j = 0; j < CPL; ++j) y[j] = x[j] + c.dt * (c.nv_ds * R[j] + (src - c.k_off * y[j]));
#pragma unroll
        for (int j = 0; j < CPL; ++j) x[j] = y[j];
    }
    store_cells<T, CPL, false>(M_out + base, x);
    const double a1 = WANT_M1 ? lane_m1<T, CPL, false>(x, l0, ns, T(0.5) * (T)(2 * l0 + 1 - ns)) : 0.0;
    const double tot = column_total<LPC, WANT_M1>(lane_m0<T, CPL, false>(x, l0, ns), a1, g);
    if (g == 0) m0[col] = (T)(tot * (double)c.ds);
    if constexpr (WANT_M1)
        if (g == LPC / 2) m1[col] = (T)(tot * (double)c.ds2);
}

template <typename T, int CPL, int LPC>
static hipError_t launch_depl_sub_cfg(const T *M_in, T *M_out, T *m0, T *m1, const T *psi, int64_t nxy, int nth,
                                      int ns, int limiter, const MotorConst<T> &c, double dth, double m_total,
                                      hipStream_t s) {
    const int threads = nth * LPC;
#define MMK_DS(LIM, M1)                                                                                        \
    hipLaunchKernelGGL((k_motor_depl_sub<T, CPL, LPC, LIM, M1>), dim3((unsigned)nxy), dim3(threads), 0, s, M_in, \
                       M_out, m0, m1, psi, nth, ns, c, dth, m_total)
    if (limiter == 0) {
        if (m1) MMK_DS(0, true); else MMK_DS(0, false);
    } else {
        if (m1) MMK_DS(1, true); else MMK_DS(1, false);
    }
#undef MMK_DS
    return hipGetLastError();
}

// Lanes per column of the single-launch depleted kernel (32 bytes of the column per lane; 64 for
// FP32 columns of 64 cells, measured 8% faster there), 0 where
// it has no tiling for ns.
static int depl_sub_lpc(size_t esz, int ns) {
    if (esz == 4) return ns == 32 ? 4 : ns == 64 ? 4 : ns == 128 ? 16 : 0;
    return ns == 16 ? 4 : ns == 32 ? 8 : ns == 64 ? 16 : 0;
}

bool depl_sub_supported(size_t esz, int nth, int ns, int64_t nxy) {
    const int lpc = depl_sub_lpc(esz, ns);
    return lpc > 0 && nth >= 1 && (int64_t)nth * lpc <= 1024 && (nth * lpc) % 64 == 0 && nxy <= 0x7fffffff;
}

template <typename T>
hipError_t launch_motor_depl_sub(const T *M_in, T *M_out, T *m0, T *m1, const T *psi, int64_t nxy, int nth, int ns,
                                 int limiter, const MotorConst<T> &c, double dth, double m_total, hipStream_t s) {
    if (!depl_sub_supported(sizeof(T), nth, ns, nxy)) return hipErrorNotSupported;
    if (nxy <= 0) return hipSuccess;
    // 32 or 64 bytes of each column per lane (several sub-steps of arithmetic per load)
    if constexpr (sizeof(T) == 4) {
        if (ns == 64) return launch_depl_sub_cfg<T, 16, 4>(M_in, M_out, m0, m1, psi, nxy, nth, ns, limiter, c, dth, m_total, s);
        if (ns == 32) return launch_depl_sub_cfg<T, 8, 4>(M_in, M_out, m0, m1, psi, nxy, nth, ns, limiter, c, dth, m_total, s);
        if (ns == 128) return launch_depl_sub_cfg<T, 8, 16>(M_in, M_out, m0, m1, psi, nxy, nth, ns, limiter, c, dth, m_total, s);
    } else {
        if (ns == 64) return launch_depl_sub_cfg<T, 4, 16>(M_in, M_out, m0, m1, psi, nxy, nth, ns, limiter, c, dth, m_total, s);
        if (ns == 32) return launch_depl_sub_cfg<T, 4, 8>(M_in, M_out, m0, m1, psi, nxy, nth, ns, limiter, c, dth, m_total, s);
        if (ns == 16) return launch_depl_sub_cfg<T, 4, 4>(M_in, M_out, m0, m1, psi, nxy, nth, ns, limiter, c, dth, m_total, s);
    }
    return hipErrorNotSupported;
}
template hipError_t launch_motor_depl_sub<float>(const float *, float *, float *, float *, const float *, int64_t, int,
                                                 int, int, const MotorConst<float> &, double, double, hipStream_t);
template hipError_t launch_motor_depl_sub<double>(const double *, double *, double *, double *, const double *,
                                                  int64_t, int, int, int, const MotorConst<double> &, double, double,
                                                  hipStream_t);

template <typename T>
hipError_t launch_motor_step(const T *M_in, T *M_out, T *m0, T *m1, int64_t ncol, int ns,
                             int limiter, const MotorConst<T> &c, const T *Dxy, hipStream_t s) {
    // the chunked tiling has no depletion
    const int nch = Dxy ? 1 : chunks_per_lane(ns, (int)sizeof(T), c.chunks);
    if (nch > 1) {
        const bool nt = motor_nontemporal((int)sizeof(T), c.nt, c.nstep > 1 || c.nsub > 1) != 0;
        const int lpc = ns / (nch * (16 / (int)sizeof(T)));
#define MMK_CHUNK_CASE(NCH, LPC)                                                              \
        if (nch == NCH && lpc == LPC) return launch_chunked<T, NCH, LPC>(M_in, M_out, m0, m1, ncol, ns, limiter, c, s, nt);
        MMK_CHUNK_CASE(2, 8) MMK_CHUNK_CASE(4, 4) MMK_CHUNK_CASE(2, 16) MMK_CHUNK_CASE(4, 8) MMK_CHUNK_CASE(2, 4)
        MMK_CHUNK_CASE(4, 2) MMK_CHUNK_CASE(2, 2)
#undef MMK_CHUNK_CASE
    }
    const int lpc = lanes_per_column(ns, (int)sizeof(T), c.wide != 0, c.lanes);
#define MMK_MOTOR_CASE(NS, LPC)                                                                   \
    if (ns == NS && lpc == LPC)                                                                   \
        return launch_cfg<T, NS / LPC, LPC, false>(M_in, M_out, m0, m1, ncol, ns, limiter, c, Dxy, s);
    if constexpr (sizeof(T) == 4) {
        MMK_MOTOR_CASE(8, 2) MMK_MOTOR_CASE(16, 4) MMK_MOTOR_CASE(16, 2) MMK_MOTOR_CASE(32, 8)
        MMK_MOTOR_CASE(32, 4) MMK_MOTOR_CASE(64, 16) MMK_MOTOR_CASE(64, 8) MMK_MOTOR_CASE(64, 4) MMK_MOTOR_CASE(128, 32)
        MMK_MOTOR_CASE(128, 16) MMK_MOTOR_CASE(256, 64) MMK_MOTOR_CASE(256, 32)
    } else {
        MMK_MOTOR_CASE(4, 2) MMK_MOTOR_CASE(8, 4) MMK_MOTOR_CASE(8, 2) MMK_MOTOR_CASE(16, 8)
        MMK_MOTOR_CASE(16, 4) MMK_MOTOR_CASE(32, 16) MMK_MOTOR_CASE(32, 8) MMK_MOTOR_CASE(64, 32)
        MMK_MOTOR_CASE(64, 16) MMK_MOTOR_CASE(128, 64) MMK_MOTOR_CASE(128, 32) MMK_MOTOR_CASE(256, 64)
    }
#undef MMK_MOTOR_CASE
    // any other length: 16 lanes per column, masked tail cells, scalar loads
    if (ns <= 16) return launch_cfg<T, 1, 16, true>(M_in, M_out, m0, m1, ncol, ns, limiter, c, Dxy, s);
    if (ns <= 32) return launch_cfg<T, 2, 16, true>(M_in, M_out, m0, m1, ncol, ns, limiter, c, Dxy, s);
    if (ns <= 64) return launch_cfg<T, 4, 16, true>(M_in, M_out, m0, m1, ncol, ns, limiter, c, Dxy, s);
    if (ns <= 128) return launch_cfg<T, 8, 16, true>(M_in, M_out, m0, m1, ncol, ns, limiter, c, Dxy, s);
    if (ns <= 256) return launch_cfg<T, 16, 16, true>(M_in, M_out, m0, m1, ncol, ns, limiter, c, Dxy, s);
    if (ns <= 512) return launch_cfg<T, 32, 16, true>(M_in, M_out, m0, m1, ncol, ns, limiter, c, Dxy, s);
    return hipErrorInvalidValue;
}

template hipError_t launch_motor_step<float>(const float *, float *, float *, float *, int64_t, int, int,
                                             const MotorConst<float> &, const float *, hipStream_t);
template hipError_t launch_motor_step<double>(const double *, double *, double *, double *, int64_t, int,
                                              int, const MotorConst<double> &, const double *, hipStream_t);

}  // namespace mmk
