// Fused polyphase FIR + FFT (both steps of the Sec. 2 scheme in one pass).
// The kernel and its launcher are instantiated per input type in separate
// translation units (fused.hip, fused_ci16.hip, fused_ci8.hip,
// fused_cf16.hip) so that they compile in parallel.
//
// One workgroup of C/CPT threads owns every channel of a tile of S_B filtered
// spectra of one stream (C in {256, 512, 1024}). Each thread keeps the last TP
// raw samples of its CPT adjacent channels and their taps in registers (CPT
// channels are loaded as one vector), so each raw sample is read from HBM
// once per tile (Sec. 3.2 reuse principle) and converted to float32 once.
// Each thread's FIR writes its channels of a chunk of filtered spectra into an
// LDS row buffer, and groups of G lanes transform the rows (Stockham passes
// through their row), the last pass writing the frequency spectra straight to
// HBM, coalesced. The filtered spectra never leave the chip, so the pass moves
// only the input samples, the taps and the output spectra.
#pragma once

#include "fft_device.h"
#include "launch.h"

namespace pfb {

// CPT used for each transform size: keeps the workgroup at <= 512 threads so
// that a wave may hold up to 256 VGPRs (window, taps, prefetch and the
// transform's 16 elements per lane) without spilling.
constexpr int fused_cpt(int log2c) { return log2c >= 10 ? 2 : 1; }

// ----------------------------------------------------------------------------
// Software pipelining. The chunk is one round of transforms (CH rows: one row
// per group of G lanes) and the LDS holds two chunk buffers. In step k every
// wave transforms its row of chunk k (buffer k mod 2) AND computes the FIR
// rows of chunk k+1 into the other buffer, the FIR rows placed between the
// passes of the transform: each pass's LDS loads are issued before a group of
// FIR rows and used after it, so the FIR arithmetic hides the LDS latency of
// the transform, and raw rows keep streaming in while the transforms run (a
// form that alternates an FIR phase and a transform phase requests no raw row
// during its transform phase, and measured 12% slower at C=1024). One
// barrier per step hands the buffers over.
// Operations and their order per output are fixed by the source (explicit
// FMAs, ascending taps, the same transform code as the split path), so the
// fused, split and batched paths give the same bits.
// ----------------------------------------------------------------------------

template <int LOG2C, int TP, int CPT> struct PipeShape {
    static constexpr int C = 1 << LOG2C;
    static constexpr int NT = C / CPT;               // threads per workgroup
    using FL = FftLanes<LOG2C>;
    static constexpr int G = FL::G;
    static constexpr int CH = NT / G;                // rows per chunk: one transform round
    static constexpr int PAIR = 2 * CH;              // rows per unrolled loop trip
    static constexpr int D = 8;                      // prefetch depth (rows)
    using S = FftShape<LOG2C, G>;
    static constexpr int NPASS = S::NPASS;
    static_assert(G <= 64, "one transform per wave or less");
    static_assert(PAIR % TP == 0 && PAIR % D == 0 && CH >= NPASS, "static window and ring slots");
};

// Rows per loop trip of the pipelined kernel (two chunks of C/CPT/G rows,
// G = C/E lanes per transform): 2 E / CPT.
constexpr int fused_pipe_rows(int log2c) { return 2 * fft_elems_per_lane(log2c) / fused_cpt(log2c); }

template <int DT, int TP, int LOG2C, int CPT>
__global__ __launch_bounds__((1 << LOG2C) / CPT) void fused_fwd_pipe_kernel(FusedArgs a)
{
    using F = PipeShape<LOG2C, TP, CPT>;
    using S = typename F::S;
    constexpr int C = F::C;
    constexpr int CH = F::CH;
    constexpr int D = F::D;
    constexpr int G = F::G;
    constexpr int NPASS = F::NPASS;
    constexpr int E = S::E;
    __shared__ float2 lds[2 * CH * S::PADDED];
    __shared__ float2 tws[fft_tw_entries<LOG2C>()];

    const int64_t lb = blockIdx.x;
    const int tile = (int)(lb % a.n_tiles);
    const int b = (int)(lb / a.n_tiles);
    const int t = (int)threadIdx.x;
    const int c0 = t * CPT;
    const int64_t s_begin = (int64_t)tile * a.SB;
    const int nout = (int)((a.S - s_begin) < a.SB ? (a.S - s_begin) : a.SB);
    const int nchunks = (nout + CH - 1) / CH;
    const int off = TP - a.T;
    const int64_t row0 = s_begin - off;
    const int64_t in_rows = a.S + a.T - 1;

    stage_twiddles_lds<LOG2C>(tws, a.tw, t, F::NT); // read after the first barrier

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
        Packed<DT, CPT> q;
        ldp(row0 + j, q);
        unpack<DT, CPT>(q, w[j]);
    });
    sfor<D>([&](auto k) PFB_INLINE {
        if (k < nout)
            ldp(row0 + TP - 1 + k, pf[k]);
    });

    const uint32_t lane_boff = (uint32_t)c0 * SampleBytes<DT>::value; // the lane's byte offset in a row
    const int gid = t / G;   // this group's row of every chunk
    const int lane = t % G;
    float2 *Yb = a.Y + ((int64_t)b * a.S + s_begin) * C;

    // FIR row jj of the chunk at tile row `base` (HALF: the chunk's position
    // in the loop trip, which fixes its window and ring slots and its LDS
    // buffer). FULL: every row of the chunk and every row it prefetches lies
    // inside the tile, so the loads are issued unconditionally (the compiler
    // then waits only for the row entering the window); TAIL tests each row.
    enum { TAIL = 0, FULL = 1 };
    auto fir_row = [&](int base, const char *xrow, auto halfc, auto kindc, auto jjc) PFB_INLINE {
        constexpr int HALF = decltype(halfc)::value;
        constexpr int KIND = decltype(kindc)::value;
        constexpr int jj = decltype(jjc)::value;
        constexpr int r = HALF * CH + jj; // row within the loop trip
        const int o = base + jj;
        if (KIND == FULL || o < nout) {
            unpack<DT, CPT>(pf[r % D], w[(r + TP - 1) % TP]);
            if constexpr (KIND == FULL)
                load_packed_off<DT, CPT>(wave_uniform(xrow + jj * C * SampleBytes<DT>::value), lane_boff,
                                         pf[r % D]);
            else if (o + D < nout)
                ldp(row0 + o + D + TP - 1, pf[r % D]);
            float2 *dst = lds + (HALF * CH + jj) * S::PADDED;
            sfor<CPT>([&](auto kc) PFB_INLINE {
                constexpr int k = decltype(kc)::value;
                float ar = 0.0f, ai = 0.0f;
                sfor<TP>([&](auto jc) PFB_INLINE {
                    constexpr int j = decltype(jc)::value;
                    ar = __builtin_fmaf(hp[j][k], w[(r + j) % TP][k].x, ar);
                    ai = __builtin_fmaf(hp[j][k], w[(r + j) % TP][k].y, ai);
                });
                dst[S::pad(c0 + k)] = make_float2(ar, ai);
            });
        }
    };
    // FIR rows [LO, HI) of a chunk
    auto fir_rows = [&](int base, const char *xrow, auto halfc, auto kindc, auto loc, auto hic) PFB_INLINE {
        constexpr int LO = decltype(loc)::value, HI = decltype(hic)::value;
        sfor<HI - LO>([&](auto jc) PFB_INLINE {
            fir_row(base, xrow, halfc, kindc, std::integral_constant<int, LO + decltype(jc)::value>{});
        });
    };
    // raw row prefetched by row 0 of the chunk at `base` (FULL chunks)
    auto xrow_of = [&](int base) PFB_INLINE {
        return wave_uniform(xb + (row0 + base + D + TP - 1) * C * SampleBytes<DT>::value);
    };

    // One step: transform this group's row of the chunk at `fbase` (buffer
    // FH) and FIR the chunk at `base` (buffer 1 - FH, which the caller passes
    // as HALF) between the passes; `fir` false: transform only.
    auto step = [&](int fbase, int base, auto halfc, auto kindc, bool fir) PFB_INLINE {
        constexpr int HALF = decltype(halfc)::value;
        constexpr int KIND = decltype(kindc)::value;
        constexpr int FH = 1 - HALF;
        float2 *row = lds + (FH * CH + gid) * S::PADDED;
        const bool valid = fbase + gid < nout;
        float2 *out = Yb + (int64_t)(fbase + gid) * C;
        const char *xrow = nullptr;
        if constexpr (KIND == FULL)
            xrow = xrow_of(base);
        // opaque lane index: LDS addresses formed in each step, not hoisted
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const float2 *twp = fft_twiddle_base<true>(tws);
        float2 v[E];
        fft_gather_first_lds<LOG2C, G>(ln, row, v);
        sfor<NPASS>([&](auto pp) PFB_INLINE {
            constexpr int P = decltype(pp)::value;
            if constexpr (P > 0)
                fft_pass_gather<LOG2C, G, P>(ln, row, v);
            if (fir)
                fir_rows(base, xrow, halfc, kindc, std::integral_constant<int, P * CH / NPASS>{},
                         std::integral_constant<int, (P + 1) * CH / NPASS>{});
            fft_pass_compute<LOG2C, G, false, true, P>(ln, row, twp, v, [&](int idx, float2 val) {
                if (KIND == FULL || valid)
                    store_nt(out + idx, val);
            });
        });
    };

    // prologue: the first chunk's FIR alone (buffer 0)
    if (CH + D <= nout)
        fir_rows(0, xrow_of(0), std::integral_constant<int, 0>{}, std::integral_constant<int, FULL>{},
                 std::integral_constant<int, 0>{}, std::integral_constant<int, CH>{});
    else
        fir_rows(0, nullptr, std::integral_constant<int, 0>{}, std::integral_constant<int, TAIL>{},
                 std::integral_constant<int, 0>{}, std::integral_constant<int, CH>{});
    lds_barrier();
    for (int k = 0; k < nchunks; k += 2) {
        // chunk k (buffer 0) transformed, chunk k+1 filtered into buffer 1
        {
            const int base = (k + 1) * CH;
            if (base + CH + D <= nout)
                step(k * CH, base, std::integral_constant<int, 1>{}, std::integral_constant<int, FULL>{}, true);
            else
                step(k * CH, base, std::integral_constant<int, 1>{}, std::integral_constant<int, TAIL>{},
                     k + 1 < nchunks);
            lds_barrier();
        }
        if (k + 1 < nchunks) {
            // chunk k+1 (buffer 1) transformed, chunk k+2 filtered into buffer 0
            const int base = (k + 2) * CH;
            if (base + CH + D <= nout)
                step((k + 1) * CH, base, std::integral_constant<int, 0>{}, std::integral_constant<int, FULL>{}, true);
            else
                step((k + 1) * CH, base, std::integral_constant<int, 0>{}, std::integral_constant<int, TAIL>{},
                     k + 2 < nchunks);
            lds_barrier();
        }
    }
}

template <int DT, int TP, int LOG2C> hipError_t launch_fused_t(const FusedArgs &a, hipStream_t st)
{
    const int64_t blocks = (int64_t)a.B * a.n_tiles;
    if (blocks <= 0)
        return hipSuccess;
    constexpr int CPT = fused_cpt(LOG2C);
    hipLaunchKernelGGL((fused_fwd_pipe_kernel<DT, TP, LOG2C, CPT>), dim3((unsigned)blocks), dim3((1 << LOG2C) / CPT),
                       0, st, a);
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
