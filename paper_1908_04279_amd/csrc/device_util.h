// Device helpers for gfx950 (CDNA4, wave64): DPP lane moves inside 16-lane rows and
// error-free transformations for compensated sums.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mmk {

// DPP control codes (GFX9 encoding).
enum : int {
    DPP_QUAD_XOR1 = 0xB1,        // quad_perm [1,0,3,2]
    DPP_QUAD_XOR2 = 0x4E,        // quad_perm [2,3,0,1]
    DPP_ROW_SHL1 = 0x101,        // lane i <- lane i+1 within the 16-lane row
    DPP_ROW_SHR1 = 0x111,        // lane i <- lane i-1 within the 16-lane row
    DPP_ROW_MIRROR = 0x140,      // lane i <- lane 15-i
    DPP_ROW_HALF_MIRROR = 0x141, // lane i <- lane 7-i within each half row
    DPP_WAVE_SHL1 = 0x130,       // lane i <- lane i+1 across the whole wave
    DPP_WAVE_ROL1 = 0x134,       // lane i <- lane i+1, lane 63 <- lane 0
    DPP_WAVE_SHR1 = 0x138,       // lane i <- lane i-1 across the whole wave
    DPP_WAVE_ROR1 = 0x13C        // lane i <- lane i-1, lane 0 <- lane 63
};

// v from the lane selected by CTRL; lanes whose source is outside the row keep `old`.
template <int CTRL>
__device__ __forceinline__ float dpp(float v, float old) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, old), __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v, double old) {
    const uint64_t vb = __builtin_bit_cast(uint64_t, v), ob = __builtin_bit_cast(uint64_t, old);
    const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)ob, (int)(uint32_t)vb, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(ob >> 32), (int)(uint32_t)(vb >> 32),
                                               CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// v from the lane selected by CTRL where the caller ignores lanes whose source is outside the
// row (no tied old value, so no extra register copy); those lanes read 0.
template <int CTRL>
__device__ __forceinline__ float dpp_any(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_any(double v) {
    const uint64_t vb = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)vb, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(vb >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Lane moves inside groups of G consecutive lanes (G a power of two, 1 .. 64; a group of up to
// 16 lanes sits inside one DPP row, larger groups use the wave-wide shifts).  from_prev: value
// of lane g-1 of the group, `edge` on lane 0.  from_next: value of lane g+1, `edge` on lane G-1.
// A group that fills its row (16) or the wave (64) gets the edge from the DPP old value;
// smaller groups select it (the shift would read the neighbouring group there).
template <int G, typename T>
__device__ __forceinline__ T from_prev(T v, T edge, int g) {
    if constexpr (G == 1) {
        return edge;
    } else if constexpr (G == 16 || G == 64) {
        return dpp<(G == 16 ? DPP_ROW_SHR1 : DPP_WAVE_SHR1)>(v, edge);
    } else {
        const T r = dpp_any<(G < 16 ? DPP_ROW_SHR1 : DPP_WAVE_SHR1)>(v);
        return (g == 0) ? edge : r;
    }
}
template <int G, typename T>
__device__ __forceinline__ T from_next(T v, T edge, int g) {
    if constexpr (G == 1) {
        return edge;
    } else if constexpr (G == 16 || G == 64) {
        return dpp<(G == 16 ? DPP_ROW_SHL1 : DPP_WAVE_SHL1)>(v, edge);
    } else {
        const T r = dpp_any<(G < 16 ? DPP_ROW_SHL1 : DPP_WAVE_SHL1)>(v);
        return (g == G - 1) ? edge : r;
    }
}
// The same with a zero edge: a full row or wave takes the zero that a shift with bound_ctrl
// writes where its source lane is outside the row, with no register holding the old value.
template <int G, typename T>
__device__ __forceinline__ T from_prev0(T v, int g) {
    if constexpr (G == 1) {
        return T(0);
    } else if constexpr (G == 16 || G == 64) {
        return dpp_any<(G == 16 ? DPP_ROW_SHR1 : DPP_WAVE_SHR1)>(v);
    } else {
        const T r = dpp_any<(G < 16 ? DPP_ROW_SHR1 : DPP_WAVE_SHR1)>(v);
        return (g == 0) ? T(0) : r;
    }
}
template <int G, typename T>
__device__ __forceinline__ T from_next0(T v, int g) {
    if constexpr (G == 1) {
        return T(0);
    } else if constexpr (G == 16 || G == 64) {
        return dpp_any<(G == 16 ? DPP_ROW_SHL1 : DPP_WAVE_SHL1)>(v);
    } else {
        const T r = dpp_any<(G < 16 ? DPP_ROW_SHL1 : DPP_WAVE_SHL1)>(v);
        return (g == G - 1) ? T(0) : r;
    }
}

// Sum over the G lanes of a group (butterfly); every lane of the group gets the total.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
    if constexpr (G >= 2) v += dpp_any<DPP_QUAD_XOR1>(v);
    if constexpr (G >= 4) v += dpp_any<DPP_QUAD_XOR2>(v);
    if constexpr (G >= 8) v += dpp_any<DPP_ROW_HALF_MIRROR>(v);
    if constexpr (G >= 16) v += dpp_any<DPP_ROW_MIRROR>(v);
    if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
    if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

// Knuth's TwoSum: s + e == a + b exactly (round-to-nearest, no contraction).
#pragma clang fp contract(off)
template <typename T>
__device__ __forceinline__ void two_sum(T a, T b, T &s, T &e) {
    s = a + b;
    T bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Compensated running sum: hi + lo carries the value; adding x keeps the rounding error.
template <typename T>
struct CSum {
    T hi, lo;
    __device__ __forceinline__ CSum() : hi(0), lo(0) {}
    __device__ __forceinline__ void add(T x) {
        T s, e;
        two_sum(hi, x, s, e);
        hi = s;
        lo += e;
    }
    __device__ __forceinline__ T value() const { return hi + lo; }
};

// Kahan's running sum (4 operations per term).
template <typename T>
struct KahanT {
    T sum = 0, comp = 0;
    __device__ __forceinline__ void add(T x) {
        const T y = x - comp;
        const T t = sum + y;
        comp = (t - sum) - y;
        sum = t;
    }
};
using Kahan = KahanT<float>;

// One Kahan step on a (sum, comp) pair held in registers.
template <typename T>
__device__ __forceinline__ void kahan_add(T &sum, T &comp, T x) {
    const T y = x - comp;
    const T t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

// Compensated butterfly over the G lanes of a group, starting from a Kahan pair
// (value = s - e).  Every lane of the group gets the total.
template <int G, typename T>
__device__ __forceinline__ T group_sum_comp(T s, T kahan_comp) {
    T e = -kahan_comp;
    auto level = [&](auto tag) {
        constexpr int CTRL = decltype(tag)::value;
        T s2 = dpp_any<CTRL>(s), e2 = dpp_any<CTRL>(e);
        T t, err;
        two_sum(s, s2, t, err);
        s = t;
        e = e + e2 + err;
    };
    if constexpr (G >= 2) level(std::integral_constant<int, DPP_QUAD_XOR1>{});
    if constexpr (G >= 4) level(std::integral_constant<int, DPP_QUAD_XOR2>{});
    if constexpr (G >= 8) level(std::integral_constant<int, DPP_ROW_HALF_MIRROR>{});
    if constexpr (G >= 16) level(std::integral_constant<int, DPP_ROW_MIRROR>{});
    auto cross = [&](int m) {
        const T s2 = __shfl_xor(s, m, 64), e2 = __shfl_xor(e, m, 64);
        T t, err;
        two_sum(s, s2, t, err);
        s = t;
        e = e + e2 + err;
    };
    if constexpr (G >= 32) cross(16);
    if constexpr (G >= 64) cross(32);
    return s + e;
}

// Value of the partner lane across the top bit of a group of G lanes (G = 2 .. 64).
template <int G, typename T>
__device__ __forceinline__ T top_xchg(T v) {
    if constexpr (G == 2) return dpp_any<DPP_QUAD_XOR1>(v);
    else if constexpr (G == 4) return dpp_any<DPP_QUAD_XOR2>(v);
    else if constexpr (G == 8) return dpp_any<DPP_ROW_HALF_MIRROR>(v);
    else if constexpr (G == 16) return dpp_any<DPP_ROW_MIRROR>(v);
    else return __shfl_xor(v, G / 2, 64);
}

// Totals of two per-lane quantities q0, q1 over a group of G lanes (G a power of two, 2 .. 64).
// The top level hands q0 to the lower half of the group and q1 to the upper half, each lane
// adding its partner's copy; the remaining levels are a butterfly inside each half.  Lane g of
// the group returns the total of q0 (g < G/2) or q1 (g >= G/2).  COMP (FP32): the inputs are
// Kahan pairs (value = sum - comp) and every level is a TwoSum with the errors carried along;
// otherwise plain sums.  PAIR = false reduces q0 alone in the same order (every lane ends with
// the q0 total, the same bits as lane 0 of the paired form).
template <int G, bool COMP, bool PAIR, typename T>
__device__ __forceinline__ T group_sum_pair(T s0, T c0, T s1, T c1, int g) {
    const bool up = PAIR && (g & (G / 2)) != 0;
    const T ks = up ? s1 : s0, ss = PAIR ? (up ? s0 : s1) : s0;
    const T rs = top_xchg<G>(ss);
    if constexpr (COMP) {
        const T ke = up ? -c1 : -c0, se = PAIR ? (up ? -c0 : -c1) : -c0;
        const T re = top_xchg<G>(se);
        T t, err;
        two_sum(ks, rs, t, err);
        return group_sum_comp<G / 2>(t, -((ke + re) + err));
    } else {
        return group_sum<G / 2>(ks + rs);
    }
}
#pragma clang fp contract(on)

// 16-byte vector loads/stores of CPL consecutive cells (NT: nontemporal, streamed past the
// caches); other sizes fall back to 8-byte or scalar accesses.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T, int CPL, bool NT>
__device__ __forceinline__ void load_cells(const T *p, T (&x)[CPL]) {
    constexpr int B = CPL * (int)sizeof(T);
    if constexpr (B % 16 == 0) {
        const u32x4 *q = reinterpret_cast<const u32x4 *>(p);
#pragma unroll
        for (int i = 0; i < B / 16; ++i) {
            u32x4 w;
            if constexpr (NT)
                w = __builtin_nontemporal_load(q + i);
            else
                w = q[i];
            __builtin_memcpy(&x[i * (16 / sizeof(T))], &w, 16);
        }
    } else if constexpr (B == 8) {
        const uint2 w = *reinterpret_cast<const uint2 *>(p);
        __builtin_memcpy(&x[0], &w, 8);
    } else {
#pragma unroll
        for (int j = 0; j < CPL; ++j) x[j] = p[j];
    }
}

template <typename T, int CPL, bool NT>
__device__ __forceinline__ void store_cells(T *p, const T (&x)[CPL]) {
    constexpr int B = CPL * (int)sizeof(T);
    if constexpr (B % 16 == 0) {
        u32x4 *q = reinterpret_cast<u32x4 *>(p);
#pragma unroll
        for (int i = 0; i < B / 16; ++i) {
            u32x4 w;
            __builtin_memcpy(&w, &x[i * (16 / sizeof(T))], 16);
            if constexpr (NT)
                __builtin_nontemporal_store(w, q + i);
            else
                q[i] = w;
        }
    } else if constexpr (B == 8) {
        uint2 w;
        __builtin_memcpy(&w, &x[0], 8);
        *reinterpret_cast<uint2 *>(p) = w;
    } else {
#pragma unroll
        for (int j = 0; j < CPL; ++j) p[j] = x[j];
    }
}

// Superbee slope of the one-sided differences a (left) and b (right): zero unless a and b
// have the same strict sign, else sgn(b) max(min(2|a|,|b|), min(|a|,2|b|)).
template <typename T>
__device__ __forceinline__ T superbee(T a, T b) {
    const T aa = fabs(a), ab = fabs(b);
    const T m = fmax(fmin(aa + aa, ab), fmin(aa, ab + ab));
    return (a * b > T(0)) ? copysign(m, b) : T(0);
}
// FP32: minmod(x, y) = med3(x, y, 0), and superbee = maxmod(minmod(2a, b), minmod(a, 2b)).
// Both minmods lie between 0 and 2b (|p| <= |b|, |q| <= 2|b|, each with the sign of b or 0), so
// their maxmod is med3(p, q, 2b): the larger for b > 0, the smaller for b < 0, 0 for b = 0.
// Every operation is exact (doubling, median): the value equals the definition, and 2b is the
// doubling the neighbouring cell makes of the same difference.
template <>
__device__ __forceinline__ float superbee<float>(float a, float b) {
    const float b2 = b + b;
    const float p = __builtin_amdgcn_fmed3f(a + a, b, 0.0f);
    const float q = __builtin_amdgcn_fmed3f(a, b2, 0.0f);
    return __builtin_amdgcn_fmed3f(p, q, b2);
}

}  // namespace mmk
