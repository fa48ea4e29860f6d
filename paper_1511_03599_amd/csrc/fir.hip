// Polyphase FIR kernels for gfx950.
//
// FIR of Sec. 3.2 (Algorithm 1): y[s][c] = sum_t h[t*C + c] x[s+t][c].
//
// Layout and reuse. Samples are contiguous in channels (Sec. 3.1), so one
// wave owns 64*CPT consecutive channels of a tile of S_B filtered spectra
// (the blocking of Sec. 3.2, Fig. 5, with C_B = 64*CPT) and every row load is
// one coalesced 512*CPT-byte access. Each lane walks down its channels and
// keeps the last TP raw samples of each channel in registers, so every raw
// sample is loaded from HBM once per tile and used for all T taps (the reuse
// principle of Sec. 3.2); only the (T-1)-row halo at the tile start is read
// twice. The taps of the lane's channels also stay in registers. Rows are
// prefetched D outputs ahead. Low-precision samples are converted to float32
// once, at load.
//
// Taps are padded up to the template size TP >= T by leading zeros, so one
// kernel serves every T <= TP: with off = TP - T, window slot j of output s
// holds input row s + j - shift and carries tap j - off (zero for j < off).
// Rows outside [0, in_rows) read as zero. The same kernel computes the
// adjoint in the samples (REV: taps reversed, shift = off + T - 1), which is
// the "full" correlation of the filtered-spectra gradient with the taps.
#include <algorithm>

#include "fir_launch.h"

namespace pfb {

// Tap gradient, first stage: per tile of filtered spectra and per channel,
//   part[tile][t][c] = sum_{s in tile} Re(conj(gy[s][c]) x[s+t][c])
// with the x window of the lane's channel kept in registers (TP rows).
// FORM: GH_BOTH decides per tile between the branch-free form (a tile
// wholly inside the stream) and the tested one; GH_CLEAN and GH_TESTED
// compile one form only, for launches over tiles the host has already
// split (longer windows, where both forms in one kernel would spill).
enum { GH_BOTH = 0, GH_CLEAN = 1, GH_TESTED = 2 };

template <int TP, int D, int FORM>
__global__ __launch_bounds__(256) void gh_partial_kernel(GhArgs a)
{
    constexpr int U = TP > D ? TP : D;
    const int run = a.ntiles_run > 0 ? a.ntiles_run : a.n_tiles;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_id();
    const int64_t total = (int64_t)a.B * run * a.n_cchunks;
    if (gw >= total)
        return;
    const int cch = (int)(gw % a.n_cchunks);
    const int64_t rest = gw / a.n_cchunks;
    const int tile = a.tile0 + (int)(rest % run);
    const int b = (int)(rest / run);
    const int c = cch * 64 + lane_id();
    const bool active = c < a.C;
    const int64_t s_begin = (int64_t)tile * a.SB;
    const int nout = (int)((a.S - s_begin) < a.SB ? (a.S - s_begin) : a.SB);
    const int64_t in_rows = a.S + a.T - 1;
    const float2 *xb = a.x + (int64_t)b * in_rows * a.C + c;
    const float2 *gb = a.gy + (int64_t)b * a.S * a.C + c;

    auto ldx = [&](int64_t row) -> float2 {
        return (active && row < in_rows) ? xb[row * a.C] : make_float2(0.0f, 0.0f);
    };
    auto ldg = [&](int64_t s) -> float2 { return active ? gb[s * a.C] : make_float2(0.0f, 0.0f); };

    float acc[TP];
    sfor<TP>([&](auto j) { acc[j] = 0.0f; });
    float2 w[TP];
    float2 pf[D];
    float2 pg[D];
    auto fma_row = [&](auto jjc, float2 g) PFB_INLINE {
        constexpr int jj = decltype(jjc)::value;
        sfor<TP>([&](auto jc) PFB_INLINE {
            constexpr int j = decltype(jc)::value;
            const float2 xv = w[(jj + j) % TP];
            acc[j] = __builtin_fmaf(g.x, xv.x, __builtin_fmaf(g.y, xv.y, acc[j]));
        });
    };
    // A whole tile inside the stream (every lane's channel, every x row it
    // reads and a whole number of U-row blocks): every load is issued
    // unconditionally, so the compiler waits for exactly the row a step
    // uses. With the tested loads of the general loop below it waited for
    // every load in flight at each row (4096 channels: 648 us, about one
    // memory latency per row).
    const bool clean = FORM == GH_CLEAN || (FORM == GH_BOTH && (cch + 1) * 64 <= a.C && nout == a.SB &&
                                            nout % U == 0 && s_begin + nout + TP - 2 < in_rows);
    if (clean) {
        if constexpr (FORM != GH_TESTED) {
            sfor<TP - 1>([&](auto j) PFB_INLINE { w[j] = xb[(s_begin + j) * a.C]; });
            sfor<D>([&](auto k) PFB_INLINE {
                pf[k] = xb[(s_begin + TP - 1 + k) * a.C];
                pg[k] = gb[(s_begin + k) * a.C];
            });
            // FULL blocks prefetch D rows ahead for every row (the next block
            // exists and D <= U); the LAST block only where that stays inside
            auto block = [&](int base, auto lastc) PFB_INLINE {
                constexpr bool LASTB = decltype(lastc)::value;
                sfor<U>([&](auto jjc) PFB_INLINE {
                    constexpr int jj = decltype(jjc)::value;
                    const int64_t o = base + jj;
                    w[(jj + TP - 1) % TP] = pf[jj % D];
                    const float2 g = pg[jj % D];
                    if constexpr (!LASTB || jj + D < U) {
                        pf[jj % D] = xb[(s_begin + o + D + TP - 1) * a.C];
                        pg[jj % D] = gb[(s_begin + o + D) * a.C];
                    }
                    fma_row(jjc, g);
                });
            };
            int base = 0;
            for (; base + U < nout; base += U)
                block(base, std::false_type{});
            block(base, std::true_type{});
        }
    } else if constexpr (FORM != GH_CLEAN) {
        sfor<TP - 1>([&](auto j) { w[j] = ldx(s_begin + j); });
        sfor<D>([&](auto k) {
            if (k < nout) {
                pf[k] = ldx(s_begin + TP - 1 + k);
                pg[k] = ldg(s_begin + k);
            }
        });
        for (int base = 0; base < nout; base += U) {
            sfor<U>([&](auto jjc) {
                constexpr int jj = decltype(jjc)::value;
                const int o = base + jj;
                if (o < nout) {
                    w[(jj + TP - 1) % TP] = pf[jj % D];
                    const float2 g = pg[jj % D];
                    if (o + D < nout) {
                        pf[jj % D] = ldx(s_begin + o + D + TP - 1);
                        pg[jj % D] = ldg(s_begin + o + D);
                    }
                    fma_row(jjc, g);
                }
            });
        }
    }
    if (active) {
        float *pb = a.part + ((int64_t)b * a.n_tiles + tile) * (int64_t)a.T * a.C + c;
        sfor<TP>([&](auto j) {
            if (j < a.T)
                pb[(int64_t)j * a.C] = acc[j];
        });
    }
}

// Sample gradient and tap-gradient partials in one pass (the split adjoint
// when both are wanted, up to 32 taps): per tile of raw spectra p and per
// channel, with the window of the last TP rows of gy in registers,
//   gx[p][c] = sum_{t < T} h[t][c] gy[p - t][c]           (gy = 0 outside [0, S))
//   part[tile][t][c] = sum_{p in tile} Re(conj(gy[p - t][c]) x[p][c])
// so gy is read once for both, and x once: 24 bytes per sample instead of
// the 32 of the reversed-tap FIR and gh_partial_kernel run one after the
// other. Window slot j of output p holds gy[p - (TP-1) + j], which carries
// tap t = TP-1-j. Tiles wholly inside the stream run with unconditional
// loads and stores, the others with tested ones.
template <int TP, int D>
__global__ __launch_bounds__(256) void gxgh_kernel(GxGhArgs a)
{
    constexpr int U = TP > D ? TP : D;
    static_assert(U % TP == 0 && U % D == 0, "static window and prefetch slots");
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_id();
    const int64_t total = (int64_t)a.B * a.n_tiles * a.n_cchunks;
    if (gw >= total)
        return;
    const int cch = (int)(gw % a.n_cchunks);
    const int64_t rest = gw / a.n_cchunks;
    const int tile = (int)(rest % a.n_tiles);
    const int b = (int)(rest / a.n_tiles);
    const int c = cch * 64 + lane_id();
    const bool active = c < a.C;
    const int64_t rows = a.S + a.T - 1;
    const int64_t p0 = (int64_t)tile * a.SB;
    const int np = (int)((rows - p0) < a.SB ? (rows - p0) : a.SB);
    const float2 *xb = a.x + (int64_t)b * rows * a.C + c;
    const float2 *gb = a.gy + (int64_t)b * a.S * a.C + c;
    float2 *gxb = a.gx + (int64_t)b * rows * a.C + c;
    const int off = TP - a.T;

    float hp[TP];
    sfor<TP>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        hp[j] = (active && j >= off) ? a.h[(int64_t)(TP - 1 - j) * a.C + c] : 0.0f;
    });
    float acc[TP];
    sfor<TP>([&](auto j) { acc[j] = 0.0f; });
    float2 w[TP];
    float2 pg[D], px[D];

    // output row o = base + jj of the tile: gy row p0 + o enters the window,
    // x row p0 + o is consumed, gx row p0 + o is computed
    auto step = [&](auto jjc, float2 g_new, float2 xv, float2 &g_out) PFB_INLINE {
        constexpr int jj = decltype(jjc)::value;
        w[(jj + TP - 1) % TP] = g_new;
        float gr = 0.0f, gi = 0.0f;
        sfor<TP>([&](auto jc) PFB_INLINE {
            constexpr int j = decltype(jc)::value;
            const float2 v = w[(jj + j) % TP];
            gr = __builtin_fmaf(hp[j], v.x, gr);
            gi = __builtin_fmaf(hp[j], v.y, gi);
            acc[j] = __builtin_fmaf(v.x, xv.x, __builtin_fmaf(v.y, xv.y, acc[j]));
        });
        g_out = make_float2(gr, gi);
    };

    const bool clean = (cch + 1) * 64 <= a.C && np == a.SB && np % U == 0 && p0 - (TP - 1) >= 0 &&
                       p0 + np <= a.S;
    if (clean) {
        sfor<TP - 1>([&](auto k) PFB_INLINE { w[k] = gb[(p0 - (TP - 1) + k) * a.C]; });
        sfor<D>([&](auto k) PFB_INLINE {
            pg[k] = gb[(p0 + k) * a.C];
            px[k] = xb[(p0 + k) * a.C];
        });
        // FULL blocks prefetch D rows ahead for every row (the next block
        // exists and D <= U); the LAST block only where that stays inside
        auto block = [&](int base, auto lastc) PFB_INLINE {
            constexpr bool LASTB = decltype(lastc)::value;
            sfor<U>([&](auto jjc) PFB_INLINE {
                constexpr int jj = decltype(jjc)::value;
                const int64_t p = p0 + base + jj;
                const float2 g_new = pg[jj % D], xv = px[jj % D];
                if constexpr (!LASTB || jj + D < U) {
                    pg[jj % D] = gb[(p + D) * a.C];
                    px[jj % D] = xb[(p + D) * a.C];
                }
                float2 g;
                step(jjc, g_new, xv, g);
                store_nt(gxb + p * a.C, g);
            });
        };
        int base = 0;
        for (; base + U < np; base += U)
            block(base, std::false_type{});
        block(base, std::true_type{});
    } else {
        auto ldg = [&](int64_t q) -> float2 {
            return (active && q >= 0 && q < a.S) ? gb[q * a.C] : make_float2(0.0f, 0.0f);
        };
        auto ldx = [&](int64_t p) -> float2 { return (active && p < rows) ? xb[p * a.C] : make_float2(0.0f, 0.0f); };
        sfor<TP - 1>([&](auto k) { w[k] = ldg(p0 - (TP - 1) + k); });
        sfor<D>([&](auto k) {
            if (k < np) {
                pg[k] = ldg(p0 + k);
                px[k] = ldx(p0 + k);
            }
        });
        for (int base = 0; base < np; base += U) {
            sfor<U>([&](auto jjc) {
                constexpr int jj = decltype(jjc)::value;
                const int o = base + jj;
                if (o < np) {
                    const float2 g_new = pg[jj % D], xv = px[jj % D];
                    if (o + D < np) {
                        pg[jj % D] = ldg(p0 + o + D);
                        px[jj % D] = ldx(p0 + o + D);
                    }
                    float2 g;
                    step(jjc, g_new, xv, g);
                    if (active)
                        store_nt(gxb + (p0 + o) * a.C, g);
                }
            });
        }
    }
    if (active) {
        float *pb = a.part + ((int64_t)b * a.n_tiles + tile) * (int64_t)a.T * a.C + c;
        sfor<TP>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            constexpr int t = TP - 1 - j;
            if (t < a.T)
                pb[(int64_t)t * a.C] = acc[j];
        });
    }
}

// Tap gradient, second stage: gh[t][c] = sum over all tiles of the partials.
// Tile p goes to running sum p mod 4 (each sum takes its tiles in ascending
// order), and the four sums are combined as (s0 + s1) + (s2 + s3): a fixed
// order, so the result is bit-reproducible. A block of four waves covers 64
// consecutive elements; wave w keeps running sum w of each of them, so the
// partials are read by four times as many waves as there are element groups.
__global__ __launch_bounds__(256) void gh_reduce_kernel(const float *__restrict__ part, float *__restrict__ gh,
                                                        int64_t n_parts, int64_t tc)
{
    __shared__ float sums[4][64];
    const int w = wave_id(), l = lane_id();
    const int64_t i = (int64_t)blockIdx.x * 64 + l;
    float acc = 0.0f;
    if (i < tc) {
        // eight partials loaded ahead of their additions, which stay in
        // ascending tile order
        int64_t p = w;
        for (; p + 28 < n_parts; p += 32) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                v[k] = part[(p + 4 * k) * tc + i];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                acc += v[k];
        }
        for (; p < n_parts; p += 4)
            acc += part[p * tc + i];
    }
    sums[w][l] = acc;
    __syncthreads();
    if (w == 0 && i < tc)
        gh[i] = (sums[0][l] + sums[1][l]) + (sums[2][l] + sums[3][l]);
}

// ----------------------------------------------------------------------------
// Host launchers
// ----------------------------------------------------------------------------

hipError_t launch_fir(const FirArgs &a, int dtype, int tp, int cpt, bool rev, hipStream_t st, bool per_use)
{
    if (rev)
        return dtype == DT_C64 && !per_use ? launch_fir_adjoint(a, tp, cpt, st) : hipErrorInvalidValue;
    if (per_use && (dtype == DT_C64 || tp > 16))
        return hipErrorInvalidValue;
    switch (dtype) {
    case DT_C64:
        return launch_fir_dt<DT_C64, false>(a, tp, cpt, st);
    case DT_CI16:
        return launch_fir_ci16(a, tp, cpt, per_use, st);
    case DT_CI8:
        return launch_fir_ci8(a, tp, cpt, per_use, st);
    case DT_CF16:
        return launch_fir_cf16(a, tp, cpt, per_use, st);
    default:
        return hipErrorInvalidValue;
    }
}

template <int TP, int FORM> static hipError_t launch_gh_run(const GhArgs &a, hipStream_t st)
{
    constexpr int D = fir_prefetch(TP);
    const int run = a.ntiles_run > 0 ? a.ntiles_run : a.n_tiles;
    const int64_t total = (int64_t)a.B * run * a.n_cchunks;
    const int64_t blocks = (total + 3) / 4;
    if (blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((gh_partial_kernel<TP, D, FORM>), dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int TP> static hipError_t launch_gh_t(const GhArgs &a, hipStream_t st)
{
    if constexpr (TP <= 16) {
        return launch_gh_run<TP, GH_BOTH>(a, st);
    } else if constexpr (TP > 32) {
        return launch_gh_run<TP, GH_TESTED>(a, st); // the branch-free form would halve occupancy
    } else {
        // Tiles wholly inside the stream come first: tile t is one iff its
        // S_B rows are filtered spectra and the x rows it reads, up to
        // (t+1) S_B + TP - 2, exist (S + T - 1 raw spectra). They take the
        // branch-free kernel when every channel chunk is whole and a tile is
        // a whole number of U-row blocks; the rest take the tested one.
        constexpr int D = fir_prefetch(TP);
        constexpr int U = TP > D ? TP : D;
        int64_t n_clean = 0;
        if (a.C % 64 == 0 && a.SB % U == 0 && a.S + a.T - TP >= 0)
            n_clean = std::min<int64_t>(a.n_tiles, (a.S + a.T - TP) / a.SB);
        hipError_t e = hipSuccess;
        if (n_clean > 0) {
            GhArgs c = a;
            c.tile0 = 0;
            c.ntiles_run = (int)n_clean;
            e = launch_gh_run<TP, GH_CLEAN>(c, st);
        }
        if (e == hipSuccess && n_clean < a.n_tiles) {
            GhArgs g = a;
            g.tile0 = (int)n_clean;
            g.ntiles_run = a.n_tiles - (int)n_clean;
            e = launch_gh_run<TP, GH_TESTED>(g, st);
        }
        return e;
    }
}

hipError_t launch_gh(const GhArgs &a, int tp, float *gh, hipStream_t st)
{
    hipError_t e;
    switch (tp) {
    case 4: e = launch_gh_t<4>(a, st); break;
    case 8: e = launch_gh_t<8>(a, st); break;
    case 16: e = launch_gh_t<16>(a, st); break;
    case 32: e = launch_gh_t<32>(a, st); break;
    case 64: e = launch_gh_t<64>(a, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess)
        return e;
    return launch_gh_reduce(a.part, gh, (int64_t)a.B * a.n_tiles, (int64_t)a.T * a.C, st);
}

template <int TP> static hipError_t launch_gxgh_t(const GxGhArgs &a, hipStream_t st)
{
    const int64_t total = (int64_t)a.B * a.n_tiles * a.n_cchunks;
    const int64_t blocks = (total + 3) / 4;
    if (blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((gxgh_kernel<TP, TP <= 16 ? 16 : 8>), dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gxgh(const GxGhArgs &a, int tp, float *gh, hipStream_t st)
{
    hipError_t e;
    switch (tp) {
    case 4: e = launch_gxgh_t<4>(a, st); break;
    case 8: e = launch_gxgh_t<8>(a, st); break;
    case 16: e = launch_gxgh_t<16>(a, st); break;
    case 32: e = launch_gxgh_t<32>(a, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess)
        return e;
    return launch_gh_reduce(a.part, gh, (int64_t)a.B * a.n_tiles, (int64_t)a.T * a.C, st);
}

hipError_t launch_gh_reduce(const float *part, float *gh, int64_t n_parts, int64_t tc, hipStream_t st)
{
    hipLaunchKernelGGL(gh_reduce_kernel, dim3((unsigned)((tc + 63) / 64)), dim3(256), 0, st, part, gh, n_parts, tc);
    return hipGetLastError();
}

} // namespace pfb
