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

// Workgroup barrier that orders LDS accesses only. __syncthreads() also
// waits for every outstanding global load and store of the wave (its release
// fence covers global memory), which would drain prefetched rows at each
// barrier; where the waves exchange data through LDS alone, this barrier
// lets global loads stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A pointer known to address global memory. Device functions that are not
// inlined receive plain (generic) pointers, whose accesses the compiler must
// issue as flat instructions; rebuilding the pointer in the global address
// space lets it use global loads and stores again. (A flat load also counts
// against the LDS counter, so a wait for it drains the LDS traffic as well.)
template <typename T> __device__ __forceinline__ T *as_global(T *p)
{
    return (T *)(__attribute__((address_space(1))) T *)(uintptr_t)p;
}

// A wave-uniform global pointer, moved into scalar registers. Row bases of
// an unrolled block computed through this stay one scalar value per block:
// otherwise loop strength reduction keeps one 64-bit vector induction
// variable per unrolled row, which exhausts the registers.
template <typename T> __device__ __forceinline__ T *wave_uniform(T *p)
{
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return as_global((T *)(uintptr_t)(((uint64_t)hi << 32) | lo));
}

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

// A row fragment of V consecutive samples as loaded, still in the storage
// type: prefetched rows are held packed (one 32-bit word per int16/fp16
// sample, one per two int8 samples) and converted when they enter the
// filter window, so each sample is still converted exactly once.
template <int DT, int V> struct Packed {
    static constexpr int WORDS = (V * SampleBytes<DT>::value + 3) / 4;
    uint32_t w[WORDS];
};

template <int DT, int V>
__device__ __forceinline__ void load_packed(const void *base, int64_t i, Packed<DT, V> &p)
{
    constexpr int B = V * SampleBytes<DT>::value; // bytes
    const char *a = reinterpret_cast<const char *>(base) + i * SampleBytes<DT>::value;
    if constexpr (B == 2) {
        p.w[0] = *reinterpret_cast<const uint16_t *>(a);
    } else if constexpr (B == 4) {
        p.w[0] = *reinterpret_cast<const uint32_t *>(a);
    } else if constexpr (B == 8) {
        const uint2 q = *reinterpret_cast<const uint2 *>(a);
        p.w[0] = q.x;
        p.w[1] = q.y;
    } else {
        static_assert(B % 16 == 0, "fragment size");
#pragma unroll
        for (int k = 0; k < B / 16; ++k) {
            const uint4 q = reinterpret_cast<const uint4 *>(a)[k];
            p.w[4 * k] = q.x;
            p.w[4 * k + 1] = q.y;
            p.w[4 * k + 2] = q.z;
            p.w[4 * k + 3] = q.w;
        }
    }
}

// Load a packed fragment of V samples at byte offset `off` (32-bit, the
// lane's own) from a wave-uniform base: the address is a scalar base plus a
// zero-extended vector offset, which the memory instruction takes as is (no
// per-lane 64-bit address arithmetic).
template <int DT, int V>
__device__ __forceinline__ void load_packed_off(const char *ubase, uint32_t off, Packed<DT, V> &p)
{
    constexpr int B = V * SampleBytes<DT>::value; // bytes
    const char *a = ubase + off;
    if constexpr (B == 2) {
        p.w[0] = *reinterpret_cast<const uint16_t *>(a);
    } else if constexpr (B == 4) {
        p.w[0] = *reinterpret_cast<const uint32_t *>(a);
    } else if constexpr (B == 8) {
        const uint2 q = *reinterpret_cast<const uint2 *>(a);
        p.w[0] = q.x;
        p.w[1] = q.y;
    } else {
        static_assert(B % 16 == 0, "fragment size");
#pragma unroll
        for (int k = 0; k < B / 16; ++k) {
            const uint4 q = reinterpret_cast<const uint4 *>(a)[k];
            p.w[4 * k] = q.x;
            p.w[4 * k + 1] = q.y;
            p.w[4 * k + 2] = q.z;
            p.w[4 * k + 3] = q.w;
        }
    }
}

template <int DT, int V> __device__ __forceinline__ void zero_packed(Packed<DT, V> &p)
{
#pragma unroll
    for (int k = 0; k < Packed<DT, V>::WORDS; ++k)
        p.w[k] = 0u;
}

// Load the fragment at sample index i when `valid`, zeros otherwise, without
// a branch: the load is always issued (at index `safe`, known to be in
// bounds, when not valid) and the result is masked. A load under a branch
// would leave the number of memory operations in flight unknown to the
// compiler, which then waits for all of them before the next use of any
// prefetched value; issued unconditionally, the waits count exactly.
template <int DT, int V>
__device__ __forceinline__ void load_packed_masked(const void *base, int64_t i, int64_t safe, bool valid,
                                                   Packed<DT, V> &p)
{
    load_packed<DT, V>(base, valid ? i : safe, p);
#pragma unroll
    for (int k = 0; k < Packed<DT, V>::WORDS; ++k)
        p.w[k] = valid ? p.w[k] : 0u;
}

// Convert a packed fragment to float32 (exact for every storage type).
template <int DT, int V>
__device__ __forceinline__ void unpack(const Packed<DT, V> &p, float2 (&o)[V])
{
#pragma unroll
    for (int k = 0; k < V; ++k) {
        if constexpr (DT == DT_C64) {
            o[k] = make_float2(__uint_as_float(p.w[2 * k]), __uint_as_float(p.w[2 * k + 1]));
        } else if constexpr (DT == DT_CI16) {
            o[k] = make_float2(s16lo(p.w[k]), s16hi(p.w[k]));
        } else if constexpr (DT == DT_CF16) {
            o[k] = h2f(p.w[k]);
        } else {
            const uint32_t w = p.w[k / 2];
            o[k] = make_float2(s8b(w, 2 * (k % 2)), s8b(w, 2 * (k % 2) + 1));
        }
    }
}

// Convert sample k of a packed fragment to float32, at every call: the
// stored word passes through an opaque register copy first, so the compiler
// cannot reuse an earlier conversion of the same word (used by the
// convert-per-use comparator, which converts each sample at every tap).
template <int DT, int V> __device__ __forceinline__ float2 unpack_one_fresh(const Packed<DT, V> &p, int k)
{
    if constexpr (DT == DT_C64) {
        return make_float2(__uint_as_float(p.w[2 * k]), __uint_as_float(p.w[2 * k + 1]));
    } else if constexpr (DT == DT_CI16 || DT == DT_CF16) {
        uint32_t w = p.w[k];
        asm volatile("" : "+v"(w));
        if constexpr (DT == DT_CI16)
            return make_float2(s16lo(w), s16hi(w));
        else
            return h2f(w);
    } else {
        uint32_t w = p.w[k / 2];
        asm volatile("" : "+v"(w));
        return make_float2(s8b(w, 2 * (k % 2)), s8b(w, 2 * (k % 2) + 1));
    }
}

// Load V consecutive samples starting at sample index i and convert them.
template <int DT, int V> struct Loader {
    static __device__ __forceinline__ void load(const void *base, int64_t i, float2 (&o)[V])
    {
        Packed<DT, V> p;
        load_packed<DT, V>(base, i, p);
        unpack<DT, V>(p, o);
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

// ----------------------------------------------------------------------------
// Bounded views: a byte range [base, base + bytes) of global memory (a raw
// buffer resource, bytes < 2^31) addressed by 32-bit byte offsets. An access
// whose offset lies outside the range is dropped by the memory unit: a load
// returns zeros without touching memory, a store writes nothing. A negative
// offset, taken as unsigned, is outside too. Kernels use views to issue every
// load and store of a row unconditionally, with rows beyond a tile or a
// stream simply falling outside the range: no memory operation then sits
// under a branch, so the compiler knows how many are in flight and waits for
// exactly the one a value comes from. The whole offset goes in the vector
// offset operand (the scalar one is 0), so the range check covers all of it.
// base and bytes must be wave-uniform.
// ----------------------------------------------------------------------------

struct BufView {
    __amdgpu_buffer_rsrc_t r;
};

// Word 3 of a gfx9 raw buffer resource (32-bit data format, no swizzle).
constexpr int BUF_WORD3 = 0x00020000;

__device__ __forceinline__ BufView buf_view(const void *base, int64_t bytes)
{
    const int n = bytes <= 0 ? 0 : (bytes > 0x7fffffff ? 0x7fffffff : (int)bytes);
    return {__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, n, BUF_WORD3)};
}

typedef unsigned int v2u_t __attribute__((ext_vector_type(2)));
typedef unsigned int v4u_t __attribute__((ext_vector_type(4)));

// Cache-policy bits of a buffer access: non-temporal.
constexpr int BUF_NT = 2;

// Load a packed fragment of V samples at byte offset `off` of view `v`.
template <int DT, int V> __device__ __forceinline__ void buf_load_packed(const BufView &v, int off, Packed<DT, V> &p)
{
    constexpr int B = V * SampleBytes<DT>::value;
    if constexpr (B == 2) {
        p.w[0] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(v.r, off, 0, 0);
    } else if constexpr (B == 4) {
        p.w[0] = __builtin_amdgcn_raw_buffer_load_b32(v.r, off, 0, 0);
    } else if constexpr (B == 8) {
        const v2u_t q = __builtin_amdgcn_raw_buffer_load_b64(v.r, off, 0, 0);
        p.w[0] = q.x;
        p.w[1] = q.y;
    } else {
        static_assert(B % 16 == 0, "fragment size");
#pragma unroll
        for (int k = 0; k < B / 16; ++k) {
            const v4u_t q = __builtin_amdgcn_raw_buffer_load_b128(v.r, off + 16 * k, 0, 0);
            p.w[4 * k] = q.x;
            p.w[4 * k + 1] = q.y;
            p.w[4 * k + 2] = q.z;
            p.w[4 * k + 3] = q.w;
        }
    }
}

// Load V complex float32 values at byte offset `off` of view `v`.
template <int V> __device__ __forceinline__ void buf_load_c64(const BufView &v, int off, float2 (&o)[V])
{
    Packed<DT_C64, V> p;
    buf_load_packed<DT_C64, V>(v, off, p);
    unpack<DT_C64, V>(p, o);
}

// Streaming (non-temporal) store of V complex float32 values at byte offset
// `off` of view `v`.
template <int V> __device__ __forceinline__ void buf_store_c64_nt(const BufView &v, int off, const float2 (&x)[V])
{
    if constexpr (V == 1) {
        const v2u_t q = {__float_as_uint(x[0].x), __float_as_uint(x[0].y)};
        __builtin_amdgcn_raw_buffer_store_b64(q, v.r, off, 0, BUF_NT);
    } else {
#pragma unroll
        for (int k = 0; k < V; k += 2) {
            const v4u_t q = {__float_as_uint(x[k].x), __float_as_uint(x[k].y), __float_as_uint(x[k + 1].x),
                             __float_as_uint(x[k + 1].y)};
            __builtin_amdgcn_raw_buffer_store_b128(q, v.r, off + 8 * k, 0, BUF_NT);
        }
    }
}

// Lane and wave indices for 1-D blocks.
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x >> 6); }
// The same index as a wave-uniform (scalar) value: the compiler cannot see
// that threadIdx.x >> 6 is uniform, and otherwise keeps everything derived
// from it (tile, row and address bases) in vector registers.
__device__ __forceinline__ int wave_id_uniform() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

} // namespace pfb
