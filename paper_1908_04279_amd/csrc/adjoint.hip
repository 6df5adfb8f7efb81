// Hand-written reverse (adjoint) kernels of the micro-step for gfx950.
//
// Forward step n (see motor.hip and psi.hip): M' = M + dt R(M + dt/2 R(M)), m0' = ds sum M',
// psi' = psi - dt div(f(psi; A(m0', u), w(gradu))).  Given the cotangents of the step's
// outputs these kernels return the cotangents of its inputs and of k_on, k_off, v0:
//   psi reverse:   lam_psi' -> lam_psi (transposed donor-cell fluxes) and lam_m0' (through
//                  the face velocities A = mean(u - F m0 p));
//   motor reverse: lam_M' + lam_m0' ds (+ lam_m1' (s - L/2) ds on the last step) -> lam_M,
//                  recomputing the midpoint stage and the limiter branches in registers;
//                  parameter gradients are summed in FP64 per block.
// Kinks follow one fixed branch rule: a superbee pair with a*b <= 0 is the zero branch, min
// keeps its first argument on <=, max its first on >=, a face velocity of exactly 0 takes
// the left cell.
#include "adjoint.h"
#include "device_util.h"

#include <mutex>
#include <type_traits>

namespace mmk {

// ---------------------------------------------------------------------------------------
// Motor column reverse step.

// Superbee on its selected branch: sigma = ca a + cb b with (ca, cb) one of (0,0), (2,0),
// (0,1), (1,0), (0,2).  With one coefficient zero the sum is exact, so sigma equals the
// forward slope bit for bit.  The selection follows the forward definition
// sgn(b) max(min(2|a|,|b|), min(|a|,2|b|)) with min keeping its first argument on <= and max
// its first on >=, which for A = |a|, B = |b| (same strict sign) reduces to:
//   2A <= B -> (2,0);  else A > 2B -> (0,2);  else B >= A -> (0,1);  else (1,0).
template <typename T>
__device__ __forceinline__ void superbee_branch(T a, T b, T &ca, T &cb) {
    const T A = fabs(a), B = fabs(b);
    const bool c1 = (A + A <= B);
    const bool c2 = (A > B + B);
    const bool c3 = (B >= A);
    const bool same = (a * b > T(0));
    ca = (same && c1) ? T(2) : ((same && !c2 && !c3) ? T(1) : T(0));
    cb = (!same || c1) ? T(0) : (c2 ? T(2) : (c3 ? T(1) : T(0)));
}

struct RevAcc {
    double kon = 0, koff = 0, v0 = 0;
};

// Face data of a column state: limiter branches ca, cb and face values h (left neighbour hl).
template <typename T, int CPL>
struct Faces {
    T ca[CPL], cb[CPL], h[CPL], hl;
};

// Limiter branches and face values h of a column state z (this lane's CPL cells).
template <typename T, int CPL, int LPC, int LIM, bool RAGGED>
__device__ __forceinline__ void faces(const T (&z)[CPL], Faces<T, CPL> &f, int g, int l0, int ns) {
    const T zl = from_prev0<LPC>(z[CPL - 1], g);
    const T zr = from_next<LPC>(z[0], z[CPL - 1], g);
    T d[CPL + 1];
    d[0] = z[0] - zl;
#pragma unroll
    for (int j = 1; j < CPL; ++j) d[j] = z[j] - z[j - 1];
    d[CPL] = zr - z[CPL - 1];
    if constexpr (RAGGED) {
#pragma unroll
        for (int j = 0; j < CPL; ++j)
            if (l0 + j + 1 >= ns) d[j + 1] = T(0);
    }
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        if constexpr (LIM == 0) {
            superbee_branch(d[j], d[j + 1], f.ca[j], f.cb[j]);
        } else {
            f.ca[j] = T(0);
            f.cb[j] = T(0);
        }
        f.h[j] = z[j] + T(0.5) * (f.ca[j] * d[j] + f.cb[j] * d[j + 1]);
    }
    f.hl = from_prev0<LPC>(f.h[CPL - 1], g);
}

// out = (dR/dz)^T mu at the state with faces f, and the parameter terms of mu . R(z):
//   d/dk_on = sum mu, d/dk_off = -sum mu z, d/dv0 = -(1/ds) sum mu (h_l - h_{l-1}).
// With nu_l = (v0/ds)(mu_{l+1} - mu_l) (mu_ns = 0) the cotangent of the face value h_l:
//   out_l = nu_l + (1/2)[(ca_l - cb_l) nu_l + cb_{l-1} nu_{l-1} - ca_{l+1} nu_{l+1}] - k_off mu_l.
template <typename T, int CPL, int LPC>
__device__ __forceinline__ void rhs_vjp(const T (&z)[CPL], const Faces<T, CPL> &f, const T (&mu)[CPL],
                                        T (&out)[CPL], const MotorConst<T> &c, T v0_ds, int g, T &s_kon,
                                        T &s_koff, T &s_v0) {
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        s_kon += mu[j];
        s_koff -= mu[j] * z[j];
        s_v0 -= mu[j] * (f.h[j] - (j == 0 ? f.hl : f.h[j - 1]));
    }
    const T mu_next = from_next0<LPC>(mu[0], g);  // mu_{ns} = 0
    T nu[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) nu[j] = v0_ds * ((j + 1 < CPL ? mu[j + 1] : mu_next) - mu[j]);
    const T cbnu_prev = from_prev0<LPC>(f.cb[CPL - 1] * nu[CPL - 1], g);
    const T canu_next = from_next0<LPC>(f.ca[0] * nu[0], g);
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const T left = (j == 0) ? cbnu_prev : f.cb[j - 1] * nu[j - 1];
        const T right = (j + 1 < CPL) ? f.ca[j + 1] * nu[j + 1] : canu_next;
        out[j] = nu[j] + T(0.5) * ((f.ca[j] - f.cb[j]) * nu[j] + left - right) - c.k_off * mu[j];
    }
}

template <typename T, int CPL, int LPC, int LIM, bool RAGGED>
__global__ __launch_bounds__(256) void k_motor_reverse(const T *__restrict__ M, const T *__restrict__ lam_in,
                                                       const T *__restrict__ lam_m0, const T *__restrict__ lam_m1,
                                                       T *__restrict__ lam_out, double *__restrict__ gpart,
                                                       int64_t ncol, int ns, MotorConst<T> c, T inv_ds) {
    constexpr int COLS = 256 / LPC;
    const int g = threadIdx.x % LPC;
    const int l0 = g * CPL;
    RevAcc acc;
    // inputs of one chunk of COLS columns: M, lam' (NULL = 0) and the column cotangents
    struct Chunk {
        T x[CPL], lam[CPL], a0, a1;
    };
    auto load_chunk = [&](int64_t col0, Chunk &ch) {
        const int64_t col = col0 + threadIdx.x / LPC;
        const bool active = col < ncol;
        const int64_t base = col * (int64_t)ns + l0;
        ch.a0 = active ? lam_m0[col] * c.ds : T(0);
        ch.a1 = (active && lam_m1) ? lam_m1[col] * c.ds2 : T(0);
        if constexpr (!RAGGED) {
            if (active) {
                load_cells<T, CPL, false>(M + base, ch.x);
                if (lam_in) {
                    load_cells<T, CPL, false>(lam_in + base, ch.lam);
                } else {
#pragma unroll
                    for (int j = 0; j < CPL; ++j) ch.lam[j] = T(0);
                }
            } else {
#pragma unroll
                for (int j = 0; j < CPL; ++j) ch.x[j] = ch.lam[j] = T(0);
            }
        } else {
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                const bool in = active && l0 + j < ns;
                ch.x[j] = in ? M[base + j] : T(0);
                ch.lam[j] = (in && lam_in) ? lam_in[base + j] : T(0);
            }
        }
    };
    // one chunk: recompute the midpoint stage and both stages' limiter branches, then the
    // transposed stages; parameter terms go to this thread's FP64 accumulators
    auto process = [&](const Chunk &cur, int64_t col0) {
        const int64_t col = col0 + threadIdx.x / LPC;
        const bool active = col < ncol;
        const int64_t base = col * (int64_t)ns + l0;
        T lam[CPL];
        const T(&x)[CPL] = cur.x;
        const T a0 = cur.a0, a1 = cur.a1;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            const bool in = active && (!RAGGED || l0 + j < ns);
            const T w = T(0.5) * (T)(2 * (l0 + j) + 1 - ns);  // (s_l - L/2) / ds
            lam[j] = in ? cur.lam[j] + a0 + a1 * w : T(0);
        }
        // recompute the midpoint stage; the faces of x serve the recompute and the first stage
        Faces<T, CPL> fx, fy;
        faces<T, CPL, LPC, LIM, RAGGED>(x, fx, g, l0, ns);
        T y[CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j)
            y[j] = x[j] + c.half_dt * (c.nv_ds * (fx.h[j] - (j == 0 ? fx.hl : fx.h[j - 1])) +
                                       (c.k_on - c.k_off * x[j]));
        faces<T, CPL, LPC, LIM, RAGGED>(y, fy, g, l0, ns);
        const T v0_ds = c.v0 * inv_ds;
        // second stage: M' = x + dt R(y)
        T mu[CPL], zeta[CPL], w[CPL];
        T s_kon = 0, s_koff = 0, s_v0 = 0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) mu[j] = c.dt * lam[j];
        rhs_vjp<T, CPL, LPC>(y, fy, mu, zeta, c, v0_ds, g, s_kon, s_koff, s_v0);
        // first stage: y = x + dt/2 R(x)
#pragma unroll
        for (int j = 0; j < CPL; ++j) mu[j] = c.half_dt * zeta[j];
        rhs_vjp<T, CPL, LPC>(x, fx, mu, w, c, v0_ds, g, s_kon, s_koff, s_v0);
#pragma unroll
        for (int j = 0; j < CPL; ++j) w[j] = lam[j] + zeta[j] + w[j];
        if constexpr (!RAGGED) {
            if (active) store_cells<T, CPL, false>(lam_out + base, w);
        } else {
#pragma unroll
            for (int j = 0; j < CPL; ++j)
                if (active && l0 + j < ns) lam_out[base + j] = w[j];
        }
        acc.kon += (double)s_kon;
        acc.koff += (double)s_koff;
        acc.v0 += (double)s_v0 * (double)inv_ds;
    };
    // grid-stride over chunks, two register sets: the next chunk's loads are in flight while
    // this chunk computes
    const int64_t stride = (int64_t)gridDim.x * COLS;
    Chunk A, B;
    int64_t col0 = (int64_t)blockIdx.x * COLS;
    load_chunk(col0, A);
    while (col0 < ncol) {
        if (col0 + stride < ncol) load_chunk(col0 + stride, B);
        process(A, col0);
        col0 += stride;
        if (col0 >= ncol) break;
        if (col0 + stride < ncol) load_chunk(col0 + stride, A);
        process(B, col0);
        col0 += stride;
    }
    // fixed-order block sum, added to this block's running FP64 partials
    __shared__ double red[4][3];
    double v[3] = {acc.kon, acc.koff, acc.v0};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        for (int m = 32; m >= 1; m >>= 1) v[a] += __shfl_xor(v[a], m, 64);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0)
        for (int a = 0; a < 3; ++a) red[wave][a] = v[a];
    __syncthreads();
    if (threadIdx.x < 3) {
        const int a = threadIdx.x;
        const double s = (red[0][a] + red[1][a]) + (red[2][a] + red[3][a]);
        gpart[(size_t)blockIdx.x * 4 + a] += s;
    }
}

// Blocks of 256 threads of `kern` the current device runs at once (occupancy x CUs), cached
// per device and kernel.
static hipError_t resident_blocks(const void *kern, int *out) {
    struct Entry {
        int dev;
        const void *kern;
        int blocks;
    };
    static Entry cache[64];
    static int n = 0;
    static std::mutex mu;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < n; ++i)
        if (cache[i].dev == dev && cache[i].kern == kern) {
            *out = cache[i].blocks;
            return hipSuccess;
        }
    int cus = 0, per = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, 256, 0);
    if (e != hipSuccess) return e;
    *out = per * cus > 0 ? per * cus : 1;
    if (n < 64) cache[n++] = Entry{dev, kern, *out};
    return hipSuccess;
}

template <typename T, int CPL, int LPC, bool RAGGED>
static hipError_t rev_cfg(const T *M, const T *lam_in, const T *lam_m0, const T *lam_m1, T *lam_out,
                          double *gpart, int gblocks, int64_t ncol, int ns, int limiter, const MotorConst<T> &c,
                          T inv_ds, hipStream_t s) {
    constexpr int COLS = 256 / LPC;
    // persistent grid: as many blocks as the device holds at once (at most gblocks), each
    // owning its row of gpart, so the FP64 accumulation across steps is race-free
    const int64_t chunks = (ncol + COLS - 1) / COLS;
    if (chunks < 1) return hipSuccess;
    const void *kern = limiter == 0 ? reinterpret_cast<const void *>(&k_motor_reverse<T, CPL, LPC, 0, RAGGED>)
                                    : reinterpret_cast<const void *>(&k_motor_reverse<T, CPL, LPC, 1, RAGGED>);
    int res = 0;
    hipError_t e = resident_blocks(kern, &res);
    if (e != hipSuccess) return e;
    int64_t blocks = chunks < res ? chunks : res;
    if (blocks > gblocks) blocks = gblocks;
    if (limiter == 0)
        hipLaunchKernelGGL((k_motor_reverse<T, CPL, LPC, 0, RAGGED>), dim3((unsigned)blocks), dim3(256), 0, s, M,
                           lam_in, lam_m0, lam_m1, lam_out, gpart, ncol, ns, c, inv_ds);
    else
        hipLaunchKernelGGL((k_motor_reverse<T, CPL, LPC, 1, RAGGED>), dim3((unsigned)blocks), dim3(256), 0, s, M,
                           lam_in, lam_m0, lam_m1, lam_out, gpart, ncol, ns, c, inv_ds);
    return hipGetLastError();
}

// Upper bound of the persistent reverse grid (a device holds at most 8 blocks of 256 threads
// per CU; MI355X has 256 CUs).
static constexpr int64_t kRevMaxBlocks = 2048;

// Lanes per column of the reverse tiling: 16 bytes of the column per lane as in the forward
// kernel, or 0 for the masked 16-lane kernel of other lengths.
static int rev_lpc(int ns, int elem) {
    const int cpl = 16 / elem;
    const int lpc = (ns >= 2 * cpl && ns % cpl == 0) ? ns / cpl : 0;
    return (lpc >= 2 && lpc <= 64 && (lpc & (lpc - 1)) == 0) ? lpc : 0;
}

int64_t motor_reverse_blocks(int64_t ncol, int ns, int elem) {
    const int lpc = rev_lpc(ns, elem);
    const int cols = 256 / (lpc ? lpc : 16);
    const int64_t chunks = (ncol + cols - 1) / cols;
    return chunks < kRevMaxBlocks ? chunks : kRevMaxBlocks;
}

template <typename T>
hipError_t launch_motor_reverse(const T *M, const T *lam_in, const T *lam_m0, const T *lam_m1, T *lam_out,
                                double *gpart, int gblocks, int64_t ncol, int ns, int limiter,
                                const MotorConst<T> &c, double inv_ds, hipStream_t s) {
    const T ids = (T)inv_ds;
    // 16 bytes of the column per lane, as in the forward kernel
    constexpr int CPL = 16 / sizeof(T);
    const int lpc = rev_lpc(ns, (int)sizeof(T));
#define MMK_REV_CASE(LPC)                                                                                      \
    if (lpc == LPC)                                                                                            \
        return rev_cfg<T, CPL, LPC, false>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, \
                                           c, ids, s);
    MMK_REV_CASE(2) MMK_REV_CASE(4) MMK_REV_CASE(8) MMK_REV_CASE(16) MMK_REV_CASE(32) MMK_REV_CASE(64)
#undef MMK_REV_CASE
    if (ns <= 16) return rev_cfg<T, 1, 16, true>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
    if (ns <= 32) return rev_cfg<T, 2, 16, true>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
    if (ns <= 64) return rev_cfg<T, 4, 16, true>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
    if (ns <= 128) return rev_cfg<T, 8, 16, true>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
    if (ns <= 256) return rev_cfg<T, 16, 16, true>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
    if (ns <= 512) return rev_cfg<T, 32, 16, true>(M, lam_in, lam_m0, lam_m1, lam_out, gpart, gblocks, ncol, ns, limiter, c, ids, s);
    return hipErrorInvalidValue;
}
template hipError_t launch_motor_reverse<float>(const float *, const float *, const float *, const float *, float *,
                                                double *, int, int64_t, int, int, const MotorConst<float> &, double,
                                                hipStream_t);
template hipError_t launch_motor_reverse<double>(const double *, const double *, const double *, const double *,
                                                 double *, double *, int, int64_t, int, int,
                                                 const MotorConst<double> &, double, hipStream_t);

// ---------------------------------------------------------------------------------------
// Cotangents of the final psi, m0 and m1 from those of the stress and the moments.
//   c = sum psi dth, n = sum psi p dth, D = sum psi pp dth, B = sum psi m0 dth,
//   sigma = sum psi [sigma_f (cos2th/2, sin2th/2, -cos2th/2) + F m1 (cc, cs, ss)] dth
template <typename T>
__global__ __launch_bounds__(256) void k_seed(const T *__restrict__ g_sigma, const T *__restrict__ g_mom,
                                              const T *__restrict__ psi, const T *__restrict__ m0,
                                              const T *__restrict__ m1, const T *__restrict__ tab,
                                              T *__restrict__ lam_psi, T *__restrict__ lam_m0,
                                              T *__restrict__ lam_m1, int64_t npsi, int nth, int64_t nxy, T F,
                                              T sigma_f, T dth) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npsi; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pen = i / nth;
        const int k = (int)(i - pen * nth);
        T gm[7] = {0, 0, 0, 0, 0, 0, 0}, gs[3] = {0, 0, 0};
        if (g_mom)
            for (int a = 0; a < 7; ++a) gm[a] = g_mom[a * nxy + pen];
        if (g_sigma)
            for (int a = 0; a < 3; ++a) gs[a] = g_sigma[a * nxy + pen];
        const T co = tab[TAB_C * nth + k], si = tab[TAB_S * nth + k];
        const T cc = tab[TAB_CC * nth + k], cs = tab[TAB_CS * nth + k], ss = tab[TAB_SS * nth + k];
        const T h1 = tab[TAB_H1 * nth + k], h2 = tab[TAB_H2 * nth + k];
        const T ps = psi[i], mm0 = m0[i], fm1 = F * m1[i];
        const T w = gm[0] + gm[1] * co + gm[2] * si + gm[3] * cc + gm[4] * cs + gm[5] * ss + gm[6] * mm0 +
                    gs[0] * (sigma_f * h1 + fm1 * cc) + gs[1] * (sigma_f * h2 + fm1 * cs) +
                    gs[2] * (-sigma_f * h1 + fm1 * ss);
        lam_psi[i] = w * dth;
        lam_m0[i] = gm[6] * ps * dth;
        lam_m1[i] = F * ps * (gs[0] * cc + gs[1] * cs + gs[2] * ss) * dth;
    }
}

template <typename T>
hipError_t launch_seed(const T *g_sigma, const T *g_mom, const T *psi, const T *m0, const T *m1, const T *tab,
                       T *lam_psi, T *lam_m0, T *lam_m1, int64_t npsi, int nth, int64_t nxy, T F, T sigma_f, T dth,
                       hipStream_t s) {
    int64_t blocks = (npsi + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_seed<T>, dim3((unsigned)blocks), dim3(256), 0, s, g_sigma, g_mom, psi, m0, m1, tab, lam_psi,
                       lam_m0, lam_m1, npsi, nth, nxy, F, sigma_f, dth);
    return hipGetLastError();
}
template hipError_t launch_seed<float>(const float *, const float *, const float *, const float *, const float *,
                                       const float *, float *, float *, float *, int64_t, int, int64_t, float, float,
                                       float, hipStream_t);
template hipError_t launch_seed<double>(const double *, const double *, const double *, const double *,
                                        const double *, const double *, double *, double *, double *, int64_t, int,
                                        int64_t, double, double, double, hipStream_t);

__global__ void k_zero_f64(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_f64, dim3(64), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace mmk
