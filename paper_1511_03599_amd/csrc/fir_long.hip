// Polyphase FIR for tap counts beyond the register window (T > 64): the FIR
// of Algorithm 1, y[s][c] = sum_{t<T} h[t][c] x[s+t][c].
//
// One wave owns 64 adjacent channels (one per lane) of a tile of R = 32
// filtered spectra and keeps the tile's R complex sums in registers. It walks
// the taps in segments of SEG = 32: for each segment it loads the segment's
// taps, fills a register window of SEG raw rows and runs down the tile,
// adding the segment's products to every sum. Each sum still takes its taps
// in ascending order from one accumulator, so the result is the sequential
// sum a single window of T taps would give (the last segment's zero taps add
// exact zeros). Raw rows are re-read once per segment they overlap; those
// re-reads come from the caches, HBM sees about one read of the tile's
// R + T - 1 raw rows.
#include "device_common.h"
#include "launch.h"

namespace pfb {

// Waves per SIMD the registers must allow: two, except for float16 input,
// whose conversions need the whole register file of one wave.
constexpr int fir_long_waves(int dt) { return dt == DT_CF16 ? 1 : 2; }

template <int DT>
__global__ __launch_bounds__(256, fir_long_waves(DT)) void fir_long_kernel(FirArgs a)
{
    constexpr int SEG = 32; // taps per segment = window rows
    constexpr int R = 32;   // filtered spectra per tile
    constexpr int D = 4;    // prefetch depth (rows): the 2T FMA per output hide the rest
    // scalar task index: tile, row and address bases stay in scalar registers
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_id_uniform();
    const int64_t total = (int64_t)a.B * a.n_tiles * a.n_cchunks;
    if (gw >= total)
        return;
    const int cch = (int)(gw % a.n_cchunks);
    const int64_t rest = gw / a.n_cchunks;
    const int tile = (int)(rest % a.n_tiles);
    const int b = (int)(rest / a.n_tiles);
    const int c0 = cch * 64 + lane_id();
    const bool active = c0 < a.C;
    const int64_t s_begin = a.out_first + (int64_t)tile * R;
    const int64_t s_end = a.out_first + a.out_count;
    const int nout = (int)((s_end - s_begin) < R ? (s_end - s_begin) : R);
    const char *xb = reinterpret_cast<const char *>(a.x) + (int64_t)b * a.in_bstride * SampleBytes<DT>::value;
    auto ld = [&](int64_t row, Packed<DT, 1> &o) {
        if (active && row >= 0 && row < a.in_rows)
            load_packed<DT, 1>(xb, row * a.C + c0, o);
        else
            zero_packed<DT, 1>(o);
    };

    float2 acc[R];
    sfor<R>([&](auto o) PFB_INLINE { acc[o] = make_float2(0.0f, 0.0f); });
    const int nseg = (a.T + SEG - 1) / SEG;
    // Wave-uniform: a whole tile, every lane on a channel and every row that
    // any segment's window reads inside the stream. Such tiles issue every
    // load unconditionally, so the compiler waits only for the row that
    // enters the window (a load under a branch makes it wait for all).
    const bool clean = (cch + 1) * 64 <= a.C && nout == R && s_begin >= 0 &&
                       s_begin + (int64_t)nseg * SEG + R - 2 < a.in_rows;
    auto ld_clean = [&](int64_t row, Packed<DT, 1> &o) { load_packed<DT, 1>(xb, row * a.C + c0, o); };
#pragma unroll 1
    for (int g = 0; g < nseg; ++g) {
        float hp[SEG];
        sfor<SEG>([&](auto jc) PFB_INLINE {
            constexpr int j = decltype(jc)::value;
            const int t = g * SEG + j;
            hp[j] = (t < a.T && active) ? a.h[(int64_t)t * a.C + c0] : 0.0f;
        });
        // output o of this segment reads rows r0 + o + j, j < SEG
        const int64_t r0 = s_begin + (int64_t)g * SEG;
        float2 w[SEG][1];
        Packed<DT, 1> pf[D];
        if (clean) {
            sfor<SEG - 1>([&](auto j) PFB_INLINE {
                Packed<DT, 1> t;
                ld_clean(r0 + j, t);
                unpack<DT, 1>(t, w[j]);
            });
            sfor<D>([&](auto k) PFB_INLINE { ld_clean(r0 + SEG - 1 + k, pf[k]); });
            sfor<R>([&](auto oc) PFB_INLINE {
                constexpr int o = decltype(oc)::value;
                unpack<DT, 1>(pf[o % D], w[(o + SEG - 1) % SEG]);
                if constexpr (o + D < R)
                    ld_clean(r0 + o + SEG - 1 + D, pf[o % D]);
                float ar = acc[o].x, ai = acc[o].y;
                sfor<SEG>([&](auto jc) PFB_INLINE {
                    constexpr int j = decltype(jc)::value;
                    ar = __builtin_fmaf(hp[j], w[(o + j) % SEG][0].x, ar);
                    ai = __builtin_fmaf(hp[j], w[(o + j) % SEG][0].y, ai);
                });
                acc[o] = make_float2(ar, ai);
            });
            continue;
        }
        sfor<SEG - 1>([&](auto j) PFB_INLINE {
            Packed<DT, 1> t;
            ld(r0 + j, t);
            unpack<DT, 1>(t, w[j]);
        });
        sfor<D>([&](auto k) PFB_INLINE {
            if (k < nout)
                ld(r0 + SEG - 1 + k, pf[k]);
        });
        sfor<R>([&](auto oc) PFB_INLINE {
            constexpr int o = decltype(oc)::value;
            if (o < nout) {
                unpack<DT, 1>(pf[o % D], w[(o + SEG - 1) % SEG]);
                if (o + D < nout)
                    ld(r0 + o + SEG - 1 + D, pf[o % D]);
                float ar = acc[o].x, ai = acc[o].y;
                sfor<SEG>([&](auto jc) PFB_INLINE {
                    constexpr int j = decltype(jc)::value;
                    ar = __builtin_fmaf(hp[j], w[(o + j) % SEG][0].x, ar);
                    ai = __builtin_fmaf(hp[j], w[(o + j) % SEG][0].y, ai);
                });
                acc[o] = make_float2(ar, ai);
            }
        });
    }
    float2 *yb = a.y + (int64_t)b * a.y_bstride + (s_begin - a.out_first) * a.C + c0;
    sfor<R>([&](auto oc) PFB_INLINE {
        constexpr int o = decltype(oc)::value;
        if (o < nout && active)
            store_nt(yb + (int64_t)o * a.C, acc[o]);
    });
}

hipError_t launch_fir_long(const FirArgs &a, int dtype, hipStream_t st)
{
    const int64_t waves = (int64_t)a.B * a.n_tiles * a.n_cchunks;
    const int64_t blocks = (waves + 3) / 4;
    if (blocks <= 0)
        return hipSuccess;
    const dim3 grid((unsigned)blocks), block(256);
    switch (dtype) {
    case DT_C64: hipLaunchKernelGGL(fir_long_kernel<DT_C64>, grid, block, 0, st, a); break;
    case DT_CI16: hipLaunchKernelGGL(fir_long_kernel<DT_CI16>, grid, block, 0, st, a); break;
    case DT_CI8: hipLaunchKernelGGL(fir_long_kernel<DT_CI8>, grid, block, 0, st, a); break;
    case DT_CF16: hipLaunchKernelGGL(fir_long_kernel<DT_CF16>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace pfb
