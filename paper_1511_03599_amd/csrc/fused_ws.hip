// Fused polyphase FIR + FFT with specialised waves.
//
// Same arithmetic as fused_fwd_pipe_kernel (fused_launch.h), in the same order, so the
// two kernels give identical bits: the FIR of Algorithm 1 followed by the
// DFT of Sec. 2, Eq. (2), with the filtered spectra kept on chip.
//
// One workgroup owns every channel of a tile of filtered spectra of one
// stream, walked in chunks of RB rows, and its waves take one of two roles:
//   FIR waves  hold, per channel, the window of the last TP raw samples, the
//              taps and a prefetch ring of raw rows in registers, and write
//              the chunk's filtered spectra into an LDS buffer;
//   FFT waves  transform the rows of the other LDS buffer (one transform per
//              group of G lanes) and write the frequency spectra to HBM.
// The buffers are double: the FIR waves fill chunk k+1 while the FFT waves
// transform chunk k, so the FIR waves' raw-sample loads never wait for the
// transforms (in the single-role kernel every wave alternates between the
// two). One workgroup barrier per chunk hands the buffers over; each role
// runs its own loop, with the same number of barriers.
#include "fft_device.h"
#include "launch.h"

namespace pfb {

template <int LOG2C, int TP, int DT> struct FwsShape {
    static constexpr int C = 1 << LOG2C;
    static constexpr int CPT = LOG2C >= 10 ? 2 : 1;    // channels per FIR lane
    static constexpr int NF = C / (64 * CPT);           // FIR waves
    using FL = FftLanes<LOG2C>;
    static constexpr int G = FL::G;                     // lanes per transform
    static constexpr int RB = 4;                        // filtered spectra per chunk
    static constexpr int TPW = 64 / G;                  // transforms per FFT wave
    static constexpr int NX = RB / TPW;                 // FFT waves
    static constexpr int NT = (NF + NX) * 64;
    static constexpr int D = 8;                         // FIR prefetch depth (rows)
    // chunks per unrolled FIR step: whole window periods, even chunk count,
    // and a whole number of prefetch-ring turns, so every register slot and
    // the buffer parity are compile-time constants
    static constexpr int ROWS = (TP > D ? TP : D) > 2 * RB ? (TP > D ? TP : D) : 2 * RB;
    static constexpr int UNR = ROWS / RB;
    using S = FftShape<LOG2C, G>;
    static_assert(G <= 64 && 64 % G == 0 && NX * TPW == RB, "one round of transforms per chunk");
    static_assert(ROWS % TP == 0 && ROWS % D == 0 && UNR % 2 == 0, "static slots and parity");
};

template <int DT, int TP, int LOG2C>
__global__ __launch_bounds__((FwsShape<LOG2C, TP, DT>::NT)) void fused_fwd_ws_kernel(FusedArgs a)
{
    using F = FwsShape<LOG2C, TP, DT>;
    using S = typename F::S;
    constexpr int C = F::C;
    constexpr int CPT = F::CPT;
    constexpr int RB = F::RB;
    constexpr int D = F::D;
    constexpr int G = F::G;
    constexpr int PADDED = S::PADDED;
    __shared__ float2 ybuf[2 * RB * PADDED];

    const int64_t lb = blockIdx.x;
    const int tile = (int)(lb % a.n_tiles);
    const int b = (int)(lb / a.n_tiles);
    const int64_t s_begin = (int64_t)tile * a.SB;
    const int nout = (int)((a.S - s_begin) < a.SB ? (a.S - s_begin) : a.SB);
    const int nchunks = (nout + RB - 1) / RB;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64);

    if (wave >= F::NF) {
        // ---------------- FFT waves ----------------
        const int xl = (int)threadIdx.x - F::NF * 64;
        const int r = (xl / 64) * F::TPW + (xl % 64) / G; // chunk row of this lane's group
        const int lane = xl % G;
        float2 *Yb = a.Y + ((int64_t)b * a.S + s_begin) * C;
        lds_barrier(); // chunk 0 filtered
        for (int k = 0; k < nchunks; ++k) {
            const int o = k * RB + r;
            const bool valid = o < nout;
            float2 *row = ybuf + ((k & 1) * RB + r) * PADDED;
            float2 *out = Yb + (int64_t)o * C;
            fft_run<LOG2C, G, false, true>(
                lane, row, a.tw, [&](int idx) { return row[S::pad(idx)]; },
                [&](int idx, float2 v) {
                    if (valid)
                        store_nt(out + idx, v);
                });
            lds_barrier();
        }
        return;
    }

    // ---------------- FIR waves ----------------
    const int t = (int)threadIdx.x;
    const int c0 = t * CPT;
    const int off = TP - a.T;
    const int64_t row0 = s_begin - off;
    const int64_t in_rows = a.S + a.T - 1;

    float hp[TP][CPT];
    sfor<TP>([&](auto jc) PFB_INLINE {
        constexpr int j = decltype(jc)::value;
        sfor<CPT>([&](auto k) PFB_INLINE { hp[j][k] = (j >= off) ? a.h[(int64_t)(j - off) * C + c0 + k] : 0.0f; });
    });

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
        Packed<DT, CPT> tq;
        ldp(row0 + j, tq);
        unpack<DT, CPT>(tq, w[j]);
    });
    sfor<D>([&](auto k) PFB_INLINE {
        if (k < nout)
            ldp(row0 + TP - 1 + k, pf[k]);
    });

    for (int kb = 0; kb < nchunks; kb += F::UNR) {
        sfor<F::UNR>([&](auto jc) PFB_INLINE {
            constexpr int J = decltype(jc)::value;
            const int k = kb + J;
            if (k < nchunks) {
                float2 *yb = ybuf + (J % 2) * RB * PADDED;
                sfor<RB>([&](auto rc) PFB_INLINE {
                    constexpr int rr = decltype(rc)::value;
                    constexpr int jj = J * RB + rr; // row within the unrolled step
                    const int o = k * RB + rr;      // filtered spectrum s_begin + o
                    if (o < nout) {
                        unpack<DT, CPT>(pf[jj % D], w[(jj + TP - 1) % TP]);
                        if (o + D < nout)
                            ldp(row0 + o + D + TP - 1, pf[jj % D]);
                        sfor<CPT>([&](auto kc) PFB_INLINE {
                            constexpr int kk = decltype(kc)::value;
                            float ar = 0.0f, ai = 0.0f;
                            sfor<TP>([&](auto jc2) PFB_INLINE {
                                constexpr int j = decltype(jc2)::value;
                                ar = __builtin_fmaf(hp[j][kk], w[(jj + j) % TP][kk].x, ar);
                                ai = __builtin_fmaf(hp[j][kk], w[(jj + j) % TP][kk].y, ai);
                            });
                            yb[rr * PADDED + S::pad(c0 + kk)] = make_float2(ar, ai);
                        });
                    }
                });
                lds_barrier();
            }
        });
    }
    lds_barrier(); // the FFT waves' last chunk
}

template <int DT, int TP, int LOG2C> static hipError_t launch_fws_t(const FusedArgs &a, hipStream_t st)
{
    const int64_t blocks = (int64_t)a.B * a.n_tiles;
    if (blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((fused_fwd_ws_kernel<DT, TP, LOG2C>), dim3((unsigned)blocks),
                       dim3(FwsShape<LOG2C, TP, DT>::NT), 0, st, a);
    return hipGetLastError();
}

template <int DT> static hipError_t launch_fws_dt(const FusedArgs &a, int tp, int log2c, hipStream_t st)
{
#define PFB_FWS_C(L2)                                                                                        \
    case L2:                                                                                                 \
        switch (tp) {                                                                                        \
        case 4: return launch_fws_t<DT, 4, L2>(a, st);                                                       \
        case 8: return launch_fws_t<DT, 8, L2>(a, st);                                                       \
        case 16: return launch_fws_t<DT, 16, L2>(a, st);                                                     \
        default: return hipErrorInvalidValue;                                                                \
        }
    switch (log2c) {
        PFB_FWS_C(8)
        PFB_FWS_C(9)
        PFB_FWS_C(10)
    default:
        return hipErrorInvalidValue;
    }
#undef PFB_FWS_C
}

hipError_t launch_fused_ws(const FusedArgs &a, int dtype, int tp, int log2c, hipStream_t st)
{
    switch (dtype) {
    case DT_C64: return launch_fws_dt<DT_C64>(a, tp, log2c, st);
    case DT_CI16: return launch_fws_dt<DT_CI16>(a, tp, log2c, st);
    case DT_CI8: return launch_fws_dt<DT_CI8>(a, tp, log2c, st);
    case DT_CF16: return launch_fws_dt<DT_CF16>(a, tp, log2c, st);
    default: return hipErrorInvalidValue;
    }
}

} // namespace pfb
