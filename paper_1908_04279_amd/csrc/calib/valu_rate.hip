// VALU issue-rate calibration for gfx950 (measurement only; not part of the micro-step).
//
// Every thread runs `iters` rounds of 64 instructions of one kind: 8 independent dependency
// chains, 8 instructions each, written as inline assembly so that the count and the kind are
// exact (no packing, no fusion, no dead-code removal).  Timed with HIP events on the given
// stream; the caller divides the known instruction count by the time.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

enum Kind {
    FMA_F32 = 0, ADD_F32 = 1, MAX_F32 = 2, MED3_F32 = 3, FMA_F64 = 4, MOV_DPP = 5, CNDMASK = 6,
    FMAC_F32 = 7,      // VOP2 form: a += b c
    MUL_F32 = 8,
    SUB_F32 = 9,
    SEL_ONLY = 10,     // v_cndmask_b32 with a mask fixed in SGPRs
    MOV_B32 = 11,
    MIN3_F32 = 12,
    ADD_DPP = 13,      // v_add_f32 with a DPP row shift on its first source
    ADD_MED3 = 14,     // add and med3 alternating in each chain
    ADD_F64 = 15,
    MED3_K0 = 16,      // med3 with the inline constant 0 as one source
    FMA_K = 17,        // fma with the inline constant 0.5 as one source
    FMA_SGPR = 18,     // fma with an SGPR source
    MAX_ABS = 19,      // VOP3 max with an absolute-value modifier
    ADD_MED3_ALT = 20, // add and med3 alternating instruction by instruction
    MOTOR_MIX = 21,    // the motor step's mix: of every 9, 3 med3, 2 sub, 1 add, 2 fma, 1 fmac
};

template <int KIND>
__device__ __forceinline__ void op32(float &a, float b, float c, uint64_t m, int u) {
    if constexpr (KIND == FMA_F32) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
    if constexpr (KIND == ADD_F32) asm volatile("v_add_f32 %0, %0, %1" : "+v"(a) : "v"(b));
    if constexpr (KIND == MAX_F32) asm volatile("v_max_f32 %0, %0, %1" : "+v"(a) : "v"(b));
    if constexpr (KIND == MED3_F32) asm volatile("v_med3_f32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
    if constexpr (KIND == MOV_DPP)
        asm volatile("v_mov_b32_dpp %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf" : "+v"(a));
    if constexpr (KIND == CNDMASK)
        asm volatile("v_cmp_gt_f32 vcc, %1, %2\n\tv_cndmask_b32 %0, %0, %1, vcc" : "+v"(a) : "v"(b), "v"(c) : "vcc");
    if constexpr (KIND == FMAC_F32) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
    if constexpr (KIND == MUL_F32) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(a) : "v"(b));
    if constexpr (KIND == SUB_F32) asm volatile("v_sub_f32 %0, %1, %0" : "+v"(a) : "v"(b));
    if constexpr (KIND == SEL_ONLY) asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(a) : "v"(b), "s"(m));
    if constexpr (KIND == MOV_B32) asm volatile("v_mov_b32 %0, %0" : "+v"(a));
    if constexpr (KIND == MIN3_F32) asm volatile("v_min3_f32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
    if constexpr (KIND == ADD_DPP)
        asm volatile("v_add_f32_dpp %0, %0, %1 row_shr:1 row_mask:0xf bank_mask:0xf" : "+v"(a) : "v"(b));
    if constexpr (KIND == ADD_MED3) {
        if (u & 1) asm volatile("v_med3_f32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
        else asm volatile("v_add_f32 %0, %0, %1" : "+v"(a) : "v"(b));
    }
    if constexpr (KIND == MED3_K0) asm volatile("v_med3_f32 %0, %0, %1, 0" : "+v"(a) : "v"(b));
    if constexpr (KIND == FMA_K) asm volatile("v_fma_f32 %0, %1, 0.5, %0" : "+v"(a) : "v"(b));
    if constexpr (KIND == FMA_SGPR) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a) : "s"(b), "v"(c));
    if constexpr (KIND == MAX_ABS) asm volatile("v_max_f32_e64 %0, |%0|, %1" : "+v"(a) : "v"(b));
    if constexpr (KIND == ADD_MED3_ALT) {
        if (u & 1) asm volatile("v_med3_f32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
        else asm volatile("v_add_f32 %0, %0, %1" : "+v"(a) : "v"(b));
    }
    if constexpr (KIND == MOTOR_MIX) {
        switch (u % 9) {
            case 0: case 1: case 2: asm volatile("v_med3_f32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c)); break;
            case 3: case 4: asm volatile("v_sub_f32 %0, %1, %0" : "+v"(a) : "v"(b)); break;
            case 5: asm volatile("v_add_f32 %0, %0, %1" : "+v"(a) : "v"(b)); break;
            case 6: case 7: asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c)); break;
            default: asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(a) : "v"(b), "v"(c)); break;
        }
    }
}

template <int KIND>
__global__ __launch_bounds__(256) void k_valu32(float *out, int iters, float b, float c) {
    float a[8];
    const uint64_t m = 0x5555555555555555ull;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (float)(threadIdx.x + j);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int j = 0; j < 8; ++j) op32<KIND>(a[j], b, c, m, KIND == ADD_MED3 ? u : 8 * u + j);
    }
    float s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int KIND>
__global__ __launch_bounds__(256) void k_valu64(float *out, int iters, double b, double c) {
    double a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (double)(threadIdx.x + j);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if constexpr (KIND == FMA_F64)
                    asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c));
                else
                    asm volatile("v_add_f64 %0, %0, %1" : "+v"(a[j]) : "v"(b));
            }
    }
    double s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

}  // namespace

// Runs `blocks` blocks of 256 threads, each thread `iters` x 64 instructions of `kind` (the
// CNDMASK kind issues a compare and a select per count); out: blocks * 256 floats (device).
// *ms: elapsed milliseconds of the launch.  Returns 0, or a hipError_t value.
extern "C" int mmk_calib_valu(int kind, int blocks, int iters, float *out, void *stream, double *ms) {
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return (int)e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) return (int)e;
    const dim3 g((unsigned)blocks), t(256);
    e = hipEventRecord(e0, s);
    switch (kind) {
        case FMA_F32: hipLaunchKernelGGL(k_valu32<FMA_F32>, g, t, 0, s, out, iters, 1.0000001f, 1e-7f); break;
        case ADD_F32: hipLaunchKernelGGL(k_valu32<ADD_F32>, g, t, 0, s, out, iters, 1e-7f, 0.f); break;
        case MAX_F32: hipLaunchKernelGGL(k_valu32<MAX_F32>, g, t, 0, s, out, iters, 0.5f, 0.f); break;
        case MED3_F32: hipLaunchKernelGGL(k_valu32<MED3_F32>, g, t, 0, s, out, iters, 0.5f, 2.f); break;
        case FMA_F64: hipLaunchKernelGGL(k_valu64<FMA_F64>, g, t, 0, s, out, iters, 1.0000001, 1e-7); break;
        case ADD_F64: hipLaunchKernelGGL(k_valu64<ADD_F64>, g, t, 0, s, out, iters, 1e-7, 0.0); break;
        case FMAC_F32: hipLaunchKernelGGL(k_valu32<FMAC_F32>, g, t, 0, s, out, iters, 1e-7f, 1e-7f); break;
        case MUL_F32: hipLaunchKernelGGL(k_valu32<MUL_F32>, g, t, 0, s, out, iters, 1.0000001f, 0.f); break;
        case SUB_F32: hipLaunchKernelGGL(k_valu32<SUB_F32>, g, t, 0, s, out, iters, 1e-7f, 0.f); break;
        case SEL_ONLY: hipLaunchKernelGGL(k_valu32<SEL_ONLY>, g, t, 0, s, out, iters, 0.5f, 0.f); break;
        case MOV_B32: hipLaunchKernelGGL(k_valu32<MOV_B32>, g, t, 0, s, out, iters, 0.f, 0.f); break;
        case MIN3_F32: hipLaunchKernelGGL(k_valu32<MIN3_F32>, g, t, 0, s, out, iters, 0.5f, 2.f); break;
        case ADD_DPP: hipLaunchKernelGGL(k_valu32<ADD_DPP>, g, t, 0, s, out, iters, 1e-7f, 0.f); break;
        case ADD_MED3: hipLaunchKernelGGL(k_valu32<ADD_MED3>, g, t, 0, s, out, iters, 1e-7f, 2.f); break;
        case MED3_K0: hipLaunchKernelGGL(k_valu32<MED3_K0>, g, t, 0, s, out, iters, 0.5f, 0.f); break;
        case FMA_K: hipLaunchKernelGGL(k_valu32<FMA_K>, g, t, 0, s, out, iters, 1e-7f, 0.f); break;
        case FMA_SGPR: hipLaunchKernelGGL(k_valu32<FMA_SGPR>, g, t, 0, s, out, iters, 1.0000001f, 1e-7f); break;
        case MAX_ABS: hipLaunchKernelGGL(k_valu32<MAX_ABS>, g, t, 0, s, out, iters, 0.5f, 0.f); break;
        case ADD_MED3_ALT: hipLaunchKernelGGL(k_valu32<ADD_MED3_ALT>, g, t, 0, s, out, iters, 1e-7f, 2.f); break;
        case MOTOR_MIX: hipLaunchKernelGGL(k_valu32<MOTOR_MIX>, g, t, 0, s, out, iters, 1e-7f, 1.0000001f); break;
        case MOV_DPP: hipLaunchKernelGGL(k_valu32<MOV_DPP>, g, t, 0, s, out, iters, 0.f, 0.f); break;
        case CNDMASK: hipLaunchKernelGGL(k_valu32<CNDMASK>, g, t, 0, s, out, iters, 0.5f, 0.25f); break;
        default: return (int)hipErrorInvalidValue;
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float f = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
    *ms = f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (int)e;
}
