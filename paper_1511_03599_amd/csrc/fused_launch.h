// Fused polyphase FIR + FFT (both steps of the Sec. 2 scheme in one pass).
// The kernel and its launcher are instantiated per input type in separate
// translation units (fused.hip, fused_ci16.hip, fused_ci8.hip,
// fused_cf16.hip) so that they compile in parallel.
//
// One workgroup of C/CPT threads owns every channel of a tile of S_B filtered
// spectra of one stream (C in {256, 512, 1024}). Each thread keeps the last TP
// raw samples of its CPT adjacent channels and their taps in registers (CPT
// channels are loaded as one vector), so each raw sample
// is read from HBM once per tile (Sec. 3.2 reuse principle) and converted to
// float32 once. The tile is processed in chunks of RB filtered spectra:
//   1. FIR: each thread produces RB filtered samples of its channel and
//      writes them into an LDS row buffer [RB][C] (padded);
//   2. FFT: the workgroup transforms the RB rows in LDS (one group of G lanes
//      per row, Stockham passes through that row) and the last pass writes
//      the frequency spectra straight to HBM, coalesced.
// The filtered spectra never leave the chip, so the pass moves only the
// input samples, the taps and the output spectra. Raw rows for the next chunk
// are prefetched into registers before the transforms of the current chunk.
#pragma once

#include "fft_device.h"
#include "launch.h"

namespace pfb {

template <int LOG2C, int TP, int CPT> struct FusedShape {
    static constexpr int C = 1 << LOG2C;
    static constexpr int NT = C / CPT;               // threads per workgroup
    using FL = FftLanes<LOG2C>;
    static constexpr int G = FL::G;
    static constexpr int NG = NT / G;                // rows transformed per round
    static constexpr int RB = 16 > TP ? 16 : TP;     // filtered spectra per chunk
    static constexpr int ROUNDS = RB / NG;
    static constexpr int D = 8;                      // prefetch depth (rows)
    using S = FftShape<LOG2C, G>;
    static constexpr int LDS_BYTES = RB * S::PADDED * 8;
    static_assert(NG >= 1 && RB % TP == 0 && RB % D == 0 && RB % NG == 0, "chunk shape");
};

// CPT used for each transform size: keeps the workgroup at <= 512 threads so
// that a wave may hold up to 256 VGPRs (window, taps, prefetch and the
// transform's 16 elements per lane) without spilling.
constexpr int fused_cpt(int log2c) { return log2c >= 10 ? 2 : 1; }

template <int DT, int TP, int LOG2C, int CPT>
__global__ __launch_bounds__((1 << LOG2C) / CPT) void fused_fwd_kernel(FusedArgs a)
{
    using F = FusedShape<LOG2C, TP, CPT>;
    using S = typename F::S;
    constexpr int C = F::C;
    constexpr int RB = F::RB;
    constexpr int D = F::D;
    constexpr int G = F::G;
    __shared__ float2 lds[RB * S::PADDED];
    // twiddles read from LDS: a wait for a global twiddle load would also
    // wait for the raw rows prefetched before it
    __shared__ float2 tws[fft_tw_entries<LOG2C>()];

    const int64_t lb = blockIdx.x;
    const int tile = (int)(lb % a.n_tiles);
    const int b = (int)(lb / a.n_tiles);
    const int t = (int)threadIdx.x;
    const int c0 = t * CPT;
    const int64_t s_begin = (int64_t)tile * a.SB;
    const int nout = (int)((a.S - s_begin) < a.SB ? (a.S - s_begin) : a.SB);
    const int off = TP - a.T;
    const int64_t row0 = s_begin - off;
    const int64_t in_rows = a.S + a.T - 1;

    stage_twiddles_lds<LOG2C>(tws, a.tw, t, F::NT); // read after the first chunk's barrier

    float hp[TP][CPT];
#pragma unroll
    for (int j = 0; j < TP; ++j)
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            hp[j][k] = (j >= off) ? a.h[(int64_t)(j - off) * C + c0 + k] : 0.0f;

    const char *xb = reinterpret_cast<const char *>(a.x) + (int64_t)b * in_rows * C * SampleBytes<DT>::value;
    auto ldp = [&](int64_t row, Packed<DT, CPT> &o) {
        if (row >= 0 && row < in_rows)
            load_packed<DT, CPT>(xb, row * C + c0, o);
        else
            zero_packed<DT, CPT>(o);
    };

    float2 w[TP][CPT];
    Packed<DT, CPT> pf[D]; // prefetched rows, still packed
    sfor<TP - 1>([&](auto j) PFB_INLINE {
        Packed<DT, CPT> t;
        ldp(row0 + j, t);
        unpack<DT, CPT>(t, w[j]);
    });
    sfor<D>([&](auto k) PFB_INLINE {
        if (k < nout)
            ldp(row0 + TP - 1 + k, pf[k]);
    });

    const int gid = t / G;
    const int lane = t % G;
    float2 *Yb = a.Y + ((int64_t)b * a.S + s_begin) * C;

    // FIR rows of one chunk into the LDS row buffer. FULL chunks (every row
    // and every prefetch inside the tile) and the LAST chunk of a tile (its
    // rows inside the tile; only its first RB-D rows prefetch) issue their
    // loads unconditionally, so the compiler counts the loads in flight and
    // waits only for the row that enters the window; other chunks test each
    // row. (Raw rows of a tile always lie inside the stream.)
    enum { TAIL = 0, FULL = 1, LAST = 2 };
    auto fir_chunk = [&](int base, auto kindc) PFB_INLINE {
        constexpr int KIND = decltype(kindc)::value;
        // raw row prefetched by row jj = 0 of this chunk
        const char *xrow = nullptr;
        if constexpr (KIND != TAIL)
            xrow = wave_uniform(xb + (row0 + base + D + TP - 1) * C * SampleBytes<DT>::value);
        sfor<RB>([&](auto jjc) PFB_INLINE {
            constexpr int jj = decltype(jjc)::value;
            const int o = base + jj;
            if (KIND != TAIL || o < nout) {
                unpack<DT, CPT>(pf[jj % D], w[(jj + TP - 1) % TP]);
                if constexpr (KIND == FULL || (KIND == LAST && jj < RB - D))
                    load_packed<DT, CPT>(xrow, jj * C + c0, pf[jj % D]);
                else if (KIND == TAIL && o + D < nout)
                    ldp(row0 + o + D + TP - 1, pf[jj % D]);
                sfor<CPT>([&](auto kc) PFB_INLINE {
                    constexpr int k = decltype(kc)::value;
                    float ar = 0.0f, ai = 0.0f;
                    sfor<TP>([&](auto jc) PFB_INLINE {
                        constexpr int j = decltype(jc)::value;
                        ar = __builtin_fmaf(hp[j][k], w[(jj + j) % TP][k].x, ar);
                        ai = __builtin_fmaf(hp[j][k], w[(jj + j) % TP][k].y, ai);
                    });
                    lds[jj * S::PADDED + S::pad(c0 + k)] = make_float2(ar, ai);
                });
            }
        });
    };
    // the chunk's transforms, straight to HBM (ALL: every row in the tile)
    auto fft_chunk = [&](int base, auto allc) PFB_INLINE {
        constexpr bool ALL = decltype(allc)::value;
#pragma unroll 1
        for (int round = 0; round < F::ROUNDS; ++round) {
            const int r = round * F::NG + gid;
            const bool valid = ALL || base + r < nout;
            float2 *row = lds + r * S::PADDED;
            float2 *out = Yb + (int64_t)(base + r) * C;
            // opaque lane index: the transform's LDS addresses are formed in
            // each round instead of being hoisted out of the chunk loop and
            // held in registers throughout
            int ln = lane;
            asm volatile("" : "+v"(ln));
            fft_run<LOG2C, G, false, true, true>(
                ln, row, tws, [&](int idx) { return row[S::pad(idx)]; },
                [&](int idx, float2 v) {
                    if (valid)
                        store_nt(out + idx, v);
                });
        }
    };

    for (int base = 0; base < nout; base += RB) {
        if (base + RB + D <= nout)
            fir_chunk(base, std::integral_constant<int, FULL>{});
        else if (base + RB == nout)
            fir_chunk(base, std::integral_constant<int, LAST>{});
        else
            fir_chunk(base, std::integral_constant<int, TAIL>{});
        lds_barrier();
        if (base + RB <= nout)
            fft_chunk(base, std::true_type{});
        else
            fft_chunk(base, std::false_type{});
        lds_barrier();
    }
}

template <int DT, int TP, int LOG2C> hipError_t launch_fused_t(const FusedArgs &a, hipStream_t st)
{
    const int64_t blocks = (int64_t)a.B * a.n_tiles;
    if (blocks <= 0)
        return hipSuccess;
    constexpr int CPT = fused_cpt(LOG2C);
    hipLaunchKernelGGL((fused_fwd_kernel<DT, TP, LOG2C, CPT>), dim3((unsigned)blocks), dim3((1 << LOG2C) / CPT), 0,
                       st, a);
    return hipGetLastError();
}

template <int DT> hipError_t launch_fused_dt(const FusedArgs &a, int tp, int log2c, hipStream_t st)
{
#define PFB_FUSED_C(L2)                                                                                      \
    case L2:                                                                                                 \
        switch (tp) {                                                                                        \
        case 4: return launch_fused_t<DT, 4, L2>(a, st);                                                     \
        case 8: return launch_fused_t<DT, 8, L2>(a, st);                                                     \
        case 16: return launch_fused_t<DT, 16, L2>(a, st);                                                   \
        default: return hipErrorInvalidValue;                                                                \
        }
    switch (log2c) {
        PFB_FUSED_C(8)
        PFB_FUSED_C(9)
        PFB_FUSED_C(10)
    default:
        return hipErrorInvalidValue;
    }
#undef PFB_FUSED_C
}

} // namespace pfb
