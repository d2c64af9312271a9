// bp_common.hpp -- device helpers shared by the BP forward kernel and the
// weighted-BP adjoint kernel: compile-time loops, the min-sum rule, the window
// index maps and the LDS re-layout of one row across a window boundary.
#pragma once

#include <type_traits>

#include "bp_geom.hpp"
#include "internal.hpp"

namespace polarhip {
namespace bp {

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for_rev(F&& f) {  // E-1 down to B
    if constexpr (B < E) {
        f(std::integral_constant<int, E - 1>{});
        static_for_rev<B, E - 1>(f);
    }
}

__device__ __forceinline__ float g_ms(float a, float b) {
    float m = fminf(fabsf(a), fabsf(b));
    uint32_t s = (__float_as_uint(a) ^ __float_as_uint(b)) & 0x80000000u;
    return __uint_as_float(__float_as_uint(m) | s);
}

// Min-sum g in sign-transfer form: g(a, b) = sgn(a) * clamp(b, -|a|, |a|)
// equals sgn(a) sgn(b) min(|a|, |b|) for every pair (a zero result may carry
// the other sign, which no later value or decision depends on).  A PE's two g
// terms share one operand, so its sign is moved once into the factor that
// multiplies both: sign_to(w, a) = w with its sign flipped where a is negative
// (one bit operation), clamp_mag(b, a) = the clamp (one med3).
__device__ __forceinline__ float sign_to(float w, float a) {
    return __uint_as_float(__float_as_uint(w) ^ (__float_as_uint(a) & 0x80000000u));
}
__device__ __forceinline__ float clamp_mag(float b, float a) { return __builtin_amdgcn_fmed3f(b, -fabsf(a), fabsf(a)); }

// maximum over the wavefront, in every lane
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int q = 1; q < 64; q <<= 1) v = fmaxf(v, __shfl_xor(v, q, 64));
    return v;
}

// clip to [-m, m] (m > 0) in one instruction: the median of v, -m and m is
// min(max(v, -m), m) for every non-NaN v, signed zeros included
__device__ __forceinline__ float clipf(float v, float m) { return __builtin_amdgcn_fmed3f(v, -m, m); }

// The exact check-node rule of Sec. II-B, ln((1 + e^(a+b)) / (e^a + e^b)),
// through the identity sgn(a) sgn(b) min(|a|,|b|) + ln(1 + e^-|a+b|) -
// ln(1 + e^-|a-b|), which never overflows.  The two correction terms use the
// hardware base-2 exponential and logarithm (a few ulp; the terms are below
// ln 2, so the absolute error stays near 1e-7).
__device__ __forceinline__ float g_exact(float a, float b) {
    const float m = g_ms(a, b);
    return (m + __logf(1.0f + __expf(-fabsf(a + b)))) - __logf(1.0f + __expf(-fabsf(a - b)));
}

template <int RULE>
__device__ __forceinline__ float g_rule(float a, float b) {
    if constexpr (RULE == 0) return g_ms(a, b);
    else return g_exact(a, b);
}

// index bits of thread t in window k, register bits zero
template <class G, int K>
__device__ __forceinline__ int idx_base(int t) {
    constexpr int b = G::wbase(K);
    return (t & ((1 << b) - 1)) | ((t >> b) << (b + G::r));
}

// thread part of the LDS word address for boundary J in the layout of window K
template <class G, int J, int K>
__device__ __forceinline__ int lds_base(int t, int slot) {
    int a = 0;
#pragma unroll
    for (int q = 0; q < G::P; ++q)
        if ((t >> q) & 1) a += G::TAB.b[J].c[G::tpb(K, q)];
#pragma unroll
    for (int j = 0; j < G::SLOTB; ++j)
        if ((slot >> j) & 1) a += G::TAB.b[J].c[G::n + j];
    return a;
}

template <class G>
__device__ __forceinline__ void frame_sync() {
    if constexpr (G::NWAVES > 1) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// re-layout one row from window KF to window KT across boundary J
template <class G, int J, int KF, int KT, bool ISR>
__device__ __forceinline__ void transpose_row(float (&row)[G::V], float* tb, int base_from, int base_to) {
    constexpr int buf = ISR ? G::TAB.b[J].buf_r : G::TAB.b[J].buf_l;
    float* p = tb + buf;
#pragma unroll
    for (int v = 0; v < G::V; ++v) p[base_from + G::reg_off(J, KF, v)] = row[v];
    if constexpr (G::TAB.b[J].cross) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int v = 0; v < G::V; ++v) row[v] = p[base_to + G::reg_off(J, KT, v)];
}

}  // namespace bp
}  // namespace polarhip
