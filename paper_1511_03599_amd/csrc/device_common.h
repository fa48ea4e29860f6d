// Device helpers shared by the filter-bank kernels (gfx950, wave64).
//
// Complex samples are (re, im) pairs held in float2 registers. Input streams
// may be stored as complex float32, int16, int8 or float16 (Sec. 3.1); each
// sample is converted to float32 exactly once, when it is loaded.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <utility>

// Marks a lambda's call operator always-inline: the compile-time loops below
// must expand completely so that register arrays indexed by their counters
// stay in registers, however large the enclosing kernel is.
#define PFB_INLINE __attribute__((always_inline))

namespace pfb {

template <int N, class F, int... Is>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
// Compile-time loop: calls f(std::integral_constant<int, i>) for i = 0..N-1,
// so register-array indices derived from i are constants (fully unrolled
// regardless of the unroller's size limits).
template <int N, class F> __device__ __forceinline__ void sfor(F &&f)
{
    sfor_impl<N>(f, std::make_integer_sequence<int, N>{});
}

enum Dtype { DT_C64 = 0, DT_CI16 = 1, DT_CI8 = 2, DT_CF16 = 3 };

template <int DT> struct SampleBytes;
template <> struct SampleBytes<DT_C64> { static constexpr int value = 8; };
template <> struct SampleBytes<DT_CI16> { static constexpr int value = 4; };
template <> struct SampleBytes<DT_CI8> { static constexpr int value = 2; };
template <> struct SampleBytes<DT_CF16> { static constexpr int value = 4; };

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// a * b for complex a, b
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
// a * (-i)
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }
// a * (+i)
__device__ __forceinline__ float2 mul_pi(float2 a) { return make_float2(-a.y, a.x); }
__device__ __forceinline__ float2 conj2(float2 a) { return make_float2(a.x, -a.y); }

// ----------------------------------------------------------------------------
// Loading V consecutive complex samples (V in {1, 2, 4}) starting at sample
// index `i` of a stream stored as DT, converting to float32. The address of
// sample i must be aligned to V * SampleBytes<DT>.
// ----------------------------------------------------------------------------

__device__ __forceinline__ float s16lo(uint32_t w) { return (float)(int32_t)(int16_t)(w & 0xffffu); }
__device__ __forceinline__ float s16hi(uint32_t w) { return (float)((int32_t)w >> 16); }
__device__ __forceinline__ float s8b(uint32_t w, int k) { return (float)(int32_t)(int8_t)((w >> (8 * k)) & 0xffu); }
__device__ __forceinline__ float2 h2f(uint32_t w)
{
    __half2 h = *reinterpret_cast<__half2 *>(&w);
    return __half22float2(h);
}

template <int DT, int V> struct Loader;

template <int V> struct Loader<DT_C64, V> {
    static __device__ __forceinline__ void load(const void *base, int64_t i, float2 (&o)[V])
    {
        const float2 *p = reinterpret_cast<const float2 *>(base) + i;
        if constexpr (V == 1) {
            o[0] = *p;
        } else if constexpr (V == 2) {
            float4 q = *reinterpret_cast<const float4 *>(p);
            o[0] = make_float2(q.x, q.y);
            o[1] = make_float2(q.z, q.w);
        } else {
            float4 q0 = reinterpret_cast<const float4 *>(p)[0];
            float4 q1 = reinterpret_cast<const float4 *>(p)[1];
            o[0] = make_float2(q0.x, q0.y);
            o[1] = make_float2(q0.z, q0.w);
            o[2] = make_float2(q1.x, q1.y);
            o[3] = make_float2(q1.z, q1.w);
        }
    }
};

template <int V> struct Loader<DT_CI16, V> {
    static __device__ __forceinline__ void load(const void *base, int64_t i, float2 (&o)[V])
    {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(base) + i;
        uint32_t w[V];
        if constexpr (V == 1) {
            w[0] = *p;
        } else if constexpr (V == 2) {
            uint2 q = *reinterpret_cast<const uint2 *>(p);
            w[0] = q.x;
            w[1] = q.y;
        } else {
            uint4 q = *reinterpret_cast<const uint4 *>(p);
            w[0] = q.x;
            w[1] = q.y;
            w[2] = q.z;
            w[3] = q.w;
        }
#pragma unroll
        for (int k = 0; k < V; ++k)
            o[k] = make_float2(s16lo(w[k]), s16hi(w[k]));
    }
};

template <int V> struct Loader<DT_CI8, V> {
    static __device__ __forceinline__ void load(const void *base, int64_t i, float2 (&o)[V])
    {
        if constexpr (V == 1) {
            const uint16_t *p = reinterpret_cast<const uint16_t *>(base) + i;
            uint32_t w = *p;
            o[0] = make_float2(s8b(w, 0), s8b(w, 1));
        } else if constexpr (V == 2) {
            const uint32_t *p = reinterpret_cast<const uint32_t *>(reinterpret_cast<const uint16_t *>(base) + i);
            uint32_t w = *p;
            o[0] = make_float2(s8b(w, 0), s8b(w, 1));
            o[1] = make_float2(s8b(w, 2), s8b(w, 3));
        } else {
            const uint2 *p = reinterpret_cast<const uint2 *>(reinterpret_cast<const uint16_t *>(base) + i);
            uint2 q = *p;
            o[0] = make_float2(s8b(q.x, 0), s8b(q.x, 1));
            o[1] = make_float2(s8b(q.x, 2), s8b(q.x, 3));
            o[2] = make_float2(s8b(q.y, 0), s8b(q.y, 1));
            o[3] = make_float2(s8b(q.y, 2), s8b(q.y, 3));
        }
    }
};

template <int V> struct Loader<DT_CF16, V> {
    static __device__ __forceinline__ void load(const void *base, int64_t i, float2 (&o)[V])
    {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(base) + i;
        if constexpr (V == 1) {
            o[0] = h2f(*p);
        } else if constexpr (V == 2) {
            uint2 q = *reinterpret_cast<const uint2 *>(p);
            o[0] = h2f(q.x);
            o[1] = h2f(q.y);
        } else {
            uint4 q = *reinterpret_cast<const uint4 *>(p);
            o[0] = h2f(q.x);
            o[1] = h2f(q.y);
            o[2] = h2f(q.z);
            o[3] = h2f(q.w);
        }
    }
};

typedef float v2f_t __attribute__((ext_vector_type(2)));
typedef float v4f_t __attribute__((ext_vector_type(4)));

// Streaming store of one complex float32 value: output that is written once
// and not read back by this pass is marked non-temporal.
__device__ __forceinline__ void store_nt(float2 *p, float2 v)
{
    v2f_t w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<v2f_t *>(p));
}

// Streaming store of V consecutive complex float32 values (V in {1, 2, 4}).
template <int V>
__device__ __forceinline__ void store_c64_nt(float2 *p, const float2 (&v)[V])
{
    if constexpr (V == 1) {
        store_nt(p, v[0]);
    } else {
#pragma unroll
        for (int k = 0; k < V; k += 2) {
            v4f_t w = {v[k].x, v[k].y, v[k + 1].x, v[k + 1].y};
            __builtin_nontemporal_store(w, reinterpret_cast<v4f_t *>(p + k));
        }
    }
}

// Store V consecutive complex float32 values.
template <int V>
__device__ __forceinline__ void store_c64(float2 *p, const float2 (&v)[V])
{
    if constexpr (V == 1) {
        *p = v[0];
    } else if constexpr (V == 2) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
    } else {
        reinterpret_cast<float4 *>(p)[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
        reinterpret_cast<float4 *>(p)[1] = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
    }
}

// Lane and wave indices for 1-D blocks.
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x >> 6); }

} // namespace pfb
