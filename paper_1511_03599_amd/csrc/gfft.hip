// Mixed-radix C-point FFT for channel counts that are not powers of two
// (C = 2^a 3^b 5^c 7^d): the DFT of Sec. 2, Eq. (2), unnormalised, natural
// bin order; the inverse (exp(+...)) as conjugate in, conjugate out.
//
// Stockham autosort, one pass per radix of C's factorisation (powers of two
// as radix 16, 8, 4, 2 first, then 7, 5, 3). A pass of radix R and stride L
// (the product of the earlier radices) lets butterfly j (0 <= j < C/R) read
// elements j + i*C/R, multiply element i by W_{RL}^{ik} (k = j mod L), run an
// R-point DFT and write element i to (j - k) R + k + i L. The row lives in
// LDS in two buffers used alternately (the passes are out of place), the
// lanes of a group stride over the butterflies, and the row is loaded and
// stored coalesced. Twiddles come from one table exp(-2 pi i m / C),
// m < C, computed in FP64 on the host: W_{RL}^{ik} = table[i k C/(RL)].
//
// A group of G lanes owns one row: G = 64 (one wave, several rows per block,
// no block barriers) up to C = 1024, G = 256 (one row per block) up to 4096,
// G = 512 above. The two LDS buffers of a row limit how many rows a CU
// holds, so the larger rows take more lanes to keep enough waves in flight
// (T=16, 2^27 samples: 1536 channels 1.32 -> 1.03 ms with 256 lanes instead
// of 64; 6144 channels 1.65 -> 1.36 ms and 7168 1.58 -> 1.32 ms with 512
// instead of 256; 768 channels stay faster with 64).
#include <algorithm>

#include "fft_device.h"
#include "launch.h"

namespace pfb {

// cos(2 pi m / R) and sin(2 pi m / R) for the odd radices.
template <int R> struct OddTw;
template <> struct OddTw<3> {
    static constexpr float c[3] = {1.0f, -0.5f, -0.5f};
    static constexpr float s[3] = {0.0f, 0.86602540378443865f, -0.86602540378443865f};
};
template <> struct OddTw<5> {
    static constexpr float c[5] = {1.0f, 0.30901699437494742f, -0.80901699437494742f, -0.80901699437494742f,
                                   0.30901699437494742f};
    static constexpr float s[5] = {0.0f, 0.95105651629515357f, 0.58778525229247314f, -0.58778525229247314f,
                                   -0.95105651629515357f};
};
template <> struct OddTw<7> {
    static constexpr float c[7] = {1.0f, 0.62348980185873353f, -0.22252093395631440f, -0.90096886790241913f,
                                   -0.90096886790241913f, -0.22252093395631440f, 0.62348980185873353f};
    static constexpr float s[7] = {0.0f, 0.78183148246802981f, 0.97492791218182361f, 0.43388373911755812f,
                                   -0.43388373911755812f, -0.97492791218182361f, -0.78183148246802981f};
};

// R-point DFT (R odd) in place, exp(-2 pi i nk / R), by symmetric pairs:
// with a_n = v_n + v_{R-n}, b_n = v_n - v_{R-n} (n = 1..(R-1)/2),
//   P_k = v_0 + sum_n cos(2 pi nk/R) a_n,  Q_k = sum_n sin(2 pi nk/R) b_n,
//   X_k = P_k - i Q_k,  X_{R-k} = P_k + i Q_k.
template <int R> __device__ __forceinline__ void dft_odd(float2 *v)
{
    constexpr int H = (R - 1) / 2;
    float2 a[H + 1], b[H + 1];
    float2 x0 = v[0];
    sfor<H>([&](auto nc) PFB_INLINE {
        constexpr int n = decltype(nc)::value + 1;
        a[n] = cadd(v[n], v[R - n]);
        b[n] = csub(v[n], v[R - n]);
    });
    float2 s0 = x0;
    sfor<H>([&](auto nc) PFB_INLINE { s0 = cadd(s0, a[decltype(nc)::value + 1]); });
    float2 out[R];
    out[0] = s0;
    sfor<H>([&](auto kc) PFB_INLINE {
        constexpr int k = decltype(kc)::value + 1;
        float px = x0.x, py = x0.y, qx = 0.0f, qy = 0.0f;
        sfor<H>([&](auto nc) PFB_INLINE {
            constexpr int n = decltype(nc)::value + 1;
            constexpr float c = OddTw<R>::c[(n * k) % R];
            constexpr float s = OddTw<R>::s[(n * k) % R];
            px = __builtin_fmaf(c, a[n].x, px);
            py = __builtin_fmaf(c, a[n].y, py);
            qx = __builtin_fmaf(s, b[n].x, qx);
            qy = __builtin_fmaf(s, b[n].y, qy);
        });
        out[k] = make_float2(px + qy, py - qx);     // P - iQ
        out[R - k] = make_float2(px - qy, py + qx); // P + iQ
    });
    sfor<R>([&](auto i) PFB_INLINE { v[i] = out[i]; });
}

template <int R> __device__ __forceinline__ void dft_any(float2 *v)
{
    if constexpr (R == 3 || R == 5 || R == 7)
        dft_odd<R>(v);
    else
        Dft<R>::run(v);
}

template <int G> __device__ __forceinline__ void gf_sync()
{
    if constexpr (G > 64) {
        lds_barrier();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// One pass: `src(idx)` returns input element idx, `dst(idx, v)` takes output
// element idx (LDS rows between passes; the row in global memory for the
// first pass's inputs and the last pass's outputs, both coalesced).
template <int R, int G, class Src, class Dst>
__device__ __forceinline__ void gf_pass(Src &&src, Dst &&dst, int C, int L, const float2 *tw, int lane)
{
    const int CR = C / R;
    const int tstep = C / (R * L);
    for (int j = lane; j < CR; j += G) {
        const int k = j % L;
        float2 v[R];
        sfor<R>([&](auto i) PFB_INLINE { v[i] = src(j + decltype(i)::value * CR); });
        if (L > 1) {
            sfor<R - 1>([&](auto ic) PFB_INLINE {
                constexpr int i = decltype(ic)::value + 1;
                v[i] = cmul(v[i], tw[i * k * tstep]);
            });
        }
        dft_any<R>(v);
        const int o = (j - k) * R + k;
        sfor<R>([&](auto i) PFB_INLINE { dst(o + decltype(i)::value * L, v[i]); });
    }
}

// Pass p of the schedule with radix R (runtime), from src to dst.
template <int G, class Src, class Dst>
__device__ __forceinline__ void gf_pass_any(int R, Src &&src, Dst &&dst, int C, int L, const float2 *tw, int lane)
{
    switch (R) {
    case 16: gf_pass<16, G>(src, dst, C, L, tw, lane); break;
    case 8: gf_pass<8, G>(src, dst, C, L, tw, lane); break;
    case 4: gf_pass<4, G>(src, dst, C, L, tw, lane); break;
    case 2: gf_pass<2, G>(src, dst, C, L, tw, lane); break;
    case 7: gf_pass<7, G>(src, dst, C, L, tw, lane); break;
    case 5: gf_pass<5, G>(src, dst, C, L, tw, lane); break;
    default: gf_pass<3, G>(src, dst, C, L, tw, lane); break;
    }
}

template <int G, bool INV>
__global__ __launch_bounds__((G > 256 ? G : 256)) void gfft_kernel(FftArgs a, GfftSched s)
{
    extern __shared__ float2 gf_lds[];
    const int C = s.C;
    const int grp = (int)threadIdx.x / G;
    const int lane = (int)threadIdx.x % G;
    const int64_t row = (int64_t)blockIdx.x * s.rows_per_block + grp;
    // With G = 64 the groups are waves and use no block barrier, so a group
    // past the last row may leave; with G = 256 there is one row per block.
    if (row >= a.nrows)
        return;
    const int64_t g = row / a.rows_per_group, r = row % a.rows_per_group;
    const float2 *in = a.in + g * a.in_gstride + r * C;
    float2 *out = a.out + g * a.out_gstride + r * C;
    float2 *A = gf_lds + (size_t)grp * 2 * C;
    float2 *B = A + C;
    auto lds_src = [&](const float2 *buf) { return [buf](int idx) { return buf[idx]; }; };
    auto lds_dst = [&](float2 *buf) { return [buf](int idx, float2 v) { buf[idx] = v; }; };
    // the first pass reads the row from global memory and the last writes it
    // there (the schedule always has at least two passes: C >= 32, radix <= 16)
    gf_pass_any<G>(
        s.radix[0], [&](int idx) { const float2 v = in[idx]; return INV ? conj2(v) : v; }, lds_dst(A), C, 1, a.tw,
        lane);
    gf_sync<G>();
    int L = s.radix[0];
    for (int p = 1; p + 1 < s.npass; ++p) {
        gf_pass_any<G>(s.radix[p], lds_src(A), lds_dst(B), C, L, a.tw, lane);
        float2 *t = A;
        A = B;
        B = t;
        L *= s.radix[p];
        gf_sync<G>();
    }
    gf_pass_any<G>(
        s.radix[s.npass - 1], lds_src(A), [&](int idx, float2 v) { store_nt(out + idx, INV ? conj2(v) : v); }, C, L,
        a.tw, lane);
}

// Radix schedule of a 7-smooth C (false if C has another prime factor or
// needs more passes than GfftSched holds).
bool gfft_schedule(int C, GfftSched *s)
{
    GfftSched t{};
    t.C = C;
    int rem = C, np = 0;
    for (int r : {16, 8, 4, 2, 7, 5, 3}) {
        while (rem % r == 0) {
            if (np >= GF_MAX_PASS)
                return false;
            t.radix[np++] = r;
            rem /= r;
        }
    }
    if (rem != 1 || np < 2) // the kernel's first and last passes are distinct
        return false;
    t.npass = np;
    t.group = C <= 1024 ? 64 : C <= 4096 ? 256 : 512;
    const int64_t row_lds = (int64_t)2 * C * 8;
    int f = 1;
    if (t.group == 64)
        f = (int)std::max<int64_t>(1, std::min<int64_t>(4, 65536 / row_lds));
    t.rows_per_block = f;
    *s = t;
    return true;
}

hipError_t launch_gfft(const FftArgs &a, const GfftSched &s, bool inv, hipStream_t st)
{
    const int64_t blocks = (a.nrows + s.rows_per_block - 1) / s.rows_per_block;
    if (blocks <= 0)
        return hipSuccess;
    const size_t lds = (size_t)s.rows_per_block * 2 * s.C * sizeof(float2);
    const dim3 grid((unsigned)blocks), block((unsigned)(s.group * s.rows_per_block));
    if (s.group == 64) {
        auto k = inv ? gfft_kernel<64, true> : gfft_kernel<64, false>;
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        hipLaunchKernelGGL(k, grid, block, lds, st, a, s);
    } else if (s.group == 256) {
        auto k = inv ? gfft_kernel<256, true> : gfft_kernel<256, false>;
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        hipLaunchKernelGGL(k, grid, block, lds, st, a, s);
    } else {
        auto k = inv ? gfft_kernel<512, true> : gfft_kernel<512, false>;
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        hipLaunchKernelGGL(k, grid, block, lds, st, a, s);
    }
    return hipGetLastError();
}

} // namespace pfb
