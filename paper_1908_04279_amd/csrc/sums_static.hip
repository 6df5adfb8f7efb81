// Context-free global sums with no allocation: mass = sum psi dx dy dth and
// sum_sigma[c] = sum sigma_c dx dy of caller-given fields (the extra-stress step of Alg. 1),
// for callers that cannot allocate device memory.  The block partials live in a file-scope
// device array of fixed size, one copy per device, found through hipGetSymbolAddress once per
// device; every call on a device shares it, so calls that overlap on one device race.
#include "../../include/mmk.h"
#include "consts.h"
#include "device_util.h"
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

namespace mmk {
void set_create_error(const char *msg);
}

namespace {

using mmk::two_sum;

constexpr int kStaticBlocks = 4096;  // block partials the scratch holds (4 doubles each)
constexpr int kMaxDevices = 64;

// [kStaticBlocks][4] block partials, then the 4 scaled totals: 131104 bytes per device.
static __device__ __align__(256) double scratch[kStaticBlocks * 4 + 4];

std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (the array's name is only a host-side stand-in).
hipError_t scratch_of_device(int dev, double **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Block b sums the fixed ranges [b chunk_p, (b + 1) chunk_p) of psi and [b chunk_s, ...) of
// the three stress components, each thread with FP64 TwoSum chains, then a fixed-order TwoSum
// tree over the block: the same bits on every run.
#pragma clang fp contract(off)
template <typename T>
__global__ __launch_bounds__(256) void k_static_partials(const T *__restrict__ psi, const T *__restrict__ sigma,
                                                         int64_t n_psi, int64_t nxy, int64_t chunk_p,
                                                         int64_t chunk_s, double *__restrict__ partials) {
    __shared__ double sh[4][256], se[4][256];
    const int t = threadIdx.x;
    double s[4] = {0, 0, 0, 0}, e[4] = {0, 0, 0, 0};
    auto add = [&](int a, double x) {
        double hi, lo;
        two_sum(s[a], x, hi, lo);
        s[a] = hi;
        e[a] += lo;
    };
    const int64_t p0 = (int64_t)blockIdx.x * chunk_p, p1 = p0 + chunk_p < n_psi ? p0 + chunk_p : n_psi;
    for (int64_t i = p0 + t; i < p1; i += 256) add(0, (double)psi[i]);
    const int64_t s0 = (int64_t)blockIdx.x * chunk_s, s1 = s0 + chunk_s < nxy ? s0 + chunk_s : nxy;
    for (int64_t i = s0 + t; i < s1; i += 256) {
        add(1, (double)sigma[i]);
        add(2, (double)sigma[nxy + i]);
        add(3, (double)sigma[2 * nxy + i]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        sh[a][t] = s[a];
        se[a][t] = e[a];
    }
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w)
            for (int a = 0; a < 4; ++a) {
                double hi, lo;
                two_sum(sh[a][t], sh[a][t + w], hi, lo);
                sh[a][t] = hi;
                se[a][t] = se[a][t] + se[a][t + w] + lo;
            }
        __syncthreads();
    }
    if (t < 4) partials[(size_t)blockIdx.x * 4 + t] = sh[t][0] + se[t][0];
}
#pragma clang fp contract(on)

mmk_status fail_static(mmk_status st, const char *msg) {
    mmk::set_create_error(msg);
    return st;
}

}  // namespace

extern "C" mmk_status mmk_sums_static(const mmk_params *p, const void *psi, const void *sigma, void *hip_stream,
                                      double *mass, double sum_sigma[3]) {
    if (!p) return fail_static(MMK_ERR_ARG, "params is NULL");
    if (!psi || !sigma) return fail_static(MMK_ERR_ARG, "psi or sigma is NULL");
    if (!mass || !sum_sigma) return fail_static(MMK_ERR_ARG, "NULL output");
    if (p->nx < 1 || p->ny < 1 || p->ntheta < 1) return fail_static(MMK_ERR_ARG, "nx, ny and ntheta must be >= 1");
    if (p->precision != MMK_FP32 && p->precision != MMK_FP64)
        return fail_static(MMK_ERR_ARG, "precision must be MMK_FP64 or MMK_FP32");
    if (!(p->lx > 0) || !(p->ly > 0) || !std::isfinite(p->lx) || !std::isfinite(p->ly))
        return fail_static(MMK_ERR_ARG, "lx and ly must be finite and > 0");
    const int64_t nxy = (int64_t)p->nx * p->ny, n_psi = nxy * p->ntheta;
    // each of the kStaticBlocks partial rows covers at most 2^24 psi cells: larger fields than
    // 2^36 cells would need more rows than the scratch holds
    constexpr int64_t kMaxChunk = (int64_t)1 << 24;
    if (n_psi > (int64_t)kStaticBlocks * kMaxChunk)
        return fail_static(MMK_ERR_UNSUPPORTED, "more than 2^36 psi cells: beyond the static scratch");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_static(MMK_ERR_HIP, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail_static(MMK_ERR_UNSUPPORTED, "device index beyond 64");
    double *scr = nullptr;
    e = scratch_of_device(dev, &scr);
    if (e != hipSuccess) return fail_static(MMK_ERR_HIP, hipGetErrorString(e));
    // about 4 cells per thread of 256-thread blocks, at most kStaticBlocks blocks; every row
    // a kernel reads is written first in the same call (no clearing needed)
    int64_t nb = (n_psi + 1023) / 1024;
    if (nb > kStaticBlocks) nb = kStaticBlocks;
    if (nb < 1) nb = 1;
    const int64_t chunk_p = (n_psi + nb - 1) / nb, chunk_s = (nxy + nb - 1) / nb;
    hipStream_t s = (hipStream_t)hip_stream;
    if (p->precision == MMK_FP32)
        hipLaunchKernelGGL(k_static_partials<float>, dim3((unsigned)nb), dim3(256), 0, s, (const float *)psi,
                           (const float *)sigma, n_psi, nxy, chunk_p, chunk_s, scr);
    else
        hipLaunchKernelGGL(k_static_partials<double>, dim3((unsigned)nb), dim3(256), 0, s, (const double *)psi,
                           (const double *)sigma, n_psi, nxy, chunk_p, chunk_s, scr);
    e = hipGetLastError();
    if (e != hipSuccess) return fail_static(MMK_ERR_HIP, hipGetErrorString(e));
    const double dx = p->lx / p->nx, dy = p->ly / p->ny, dth = mmk::kTwoPi / p->ntheta;
    double *tot = scr + (size_t)kStaticBlocks * 4;
    e = mmk::launch_reduce_partials(scr, (int)nb, tot, dx * dy * dth, dx * dy, s);
    if (e != hipSuccess) return fail_static(MMK_ERR_HIP, hipGetErrorString(e));
    double h[4];
    e = hipMemcpyAsync(h, tot, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_static(MMK_ERR_HIP, hipGetErrorString(e));
    *mass = h[0];
    sum_sigma[0] = h[1];
    sum_sigma[1] = h[2];
    sum_sigma[2] = h[3];
    return MMK_OK;
}
