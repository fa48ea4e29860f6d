// Register-window FIR wave task, shared by the FIR kernel and the batched
// persistent kernel. See fir.hip for the design.
#pragma once

#include "device_common.h"
#include "launch.h"

namespace pfb {

// Prefetch depth (rows in flight per lane) for each padded tap count: deep
// where the window is small, shallower where registers are scarce.
constexpr int fir_prefetch(int tp) { return tp <= 16 ? 16 : 8; }

// One wave's task: wave task gw of a FIR launch (channel chunk fastest, then
// tile, then stream). NT selects non-temporal stores (results that are not
// read again soon) over plain ones (results read back by the same workgroup).
template <int DT, int TP, int CPT, int D, bool REV, bool NT = true>
__device__ __forceinline__ void fir_wave_task(const FirArgs &a, int64_t gw)
{
    constexpr int U = TP > D ? TP : D; // outputs per unrolled step
    static_assert(U % TP == 0 && U % D == 0, "unroll");
    const int cch = (int)(gw % a.n_cchunks);
    const int64_t rest = gw / a.n_cchunks;
    const int tile = (int)(rest % a.n_tiles);
    const int b = (int)(rest / a.n_tiles);

    const int c0 = (cch * 64 + lane_id()) * CPT;
    const bool active = c0 < a.C;
    const int64_t s_begin = a.out_first + (int64_t)tile * a.SB;
    const int64_t s_end = a.out_first + a.out_count;
    const int nout = (int)((s_end - s_begin) < a.SB ? (s_end - s_begin) : a.SB);
    const int64_t row0 = s_begin - a.shift; // input row of window slot 0
    const int off = TP - a.T;

    float hp[CPT][TP];
    sfor<TP>([&](auto jc) PFB_INLINE {
        constexpr int j = decltype(jc)::value;
        const int t = j - off;
        sfor<CPT>([&](auto k) PFB_INLINE {
            hp[k][j] = (t >= 0 && active) ? a.h[(int64_t)(REV ? a.T - 1 - t : t) * a.C + c0 + k] : 0.0f;
        });
    });

    const char *xb = reinterpret_cast<const char *>(a.x) + (int64_t)b * a.in_bstride * SampleBytes<DT>::value;
    auto ldp = [&](int64_t row, Packed<DT, CPT> &o) {
        if (active && row >= 0 && row < a.in_rows)
            load_packed<DT, CPT>(xb, row * a.C + c0, o);
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

    float2 *yb = a.y + (int64_t)b * a.y_bstride + (s_begin - a.out_first) * a.C + c0;
    for (int base = 0; base < nout; base += U) {
        sfor<U>([&](auto jjc) PFB_INLINE {
            constexpr int jj = decltype(jjc)::value;
            const int o = base + jj;
            if (o < nout) {
                unpack<DT, CPT>(pf[jj % D], w[(jj + TP - 1) % TP]);
                if (o + D < nout)
                    ldp(row0 + o + D + TP - 1, pf[jj % D]);
                float2 acc[CPT];
                sfor<CPT>([&](auto k) PFB_INLINE {
                    float ar = 0.0f, ai = 0.0f;
                    sfor<TP>([&](auto jc) PFB_INLINE {
                        constexpr int j = decltype(jc)::value;
                        ar = __builtin_fmaf(hp[k][j], w[(jj + j) % TP][k].x, ar);
                        ai = __builtin_fmaf(hp[k][j], w[(jj + j) % TP][k].y, ai);
                    });
                    acc[k] = make_float2(ar, ai);
                });
                if (active) {
                    if constexpr (NT)
                        store_c64_nt<CPT>(yb + (int64_t)o * a.C, acc);
                    else
                        store_c64<CPT>(yb + (int64_t)o * a.C, acc);
                }
            }
        });
    }
}

} // namespace pfb
