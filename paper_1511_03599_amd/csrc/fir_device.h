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
// PER_USE selects the convert-per-use comparator (TP <= 16, low-precision
// input): the window holds the samples as stored and each sample is
// converted to float32 at every tap that uses it, 2T conversions per output,
// as in a design that reads the window from a cache or shared memory at
// every tap; otherwise each sample is converted once, when it enters the
// window. Both give the same bits (the conversions are exact).
template <int DT, int TP, int CPT, int D, bool REV, bool NT = true, bool PER_USE = false>
__device__ __forceinline__ void fir_wave_task(const FirArgs &a, int64_t gw)
{
    static_assert(!PER_USE || (TP <= 16 && DT != DT_C64 && !REV), "convert-per-use comparator: TP <= 16");
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
    const int cs = active ? c0 : 0; // an in-bounds channel for every lane
    // Loads are always issued, at a clamped (in-bounds) row, and never under
    // a branch: the compiler then knows how many memory operations are in
    // flight and waits only for the one a value comes from. Rows outside the
    // stream read as zeros; that mask is applied when a row enters the
    // window, not at its load, so no load is waited for early.
    auto ldc = [&](int64_t row, Packed<DT, CPT> &o) {
        const int64_t rs = row < 0 ? 0 : (row < a.in_rows ? row : a.in_rows - 1);
        load_packed<DT, CPT>(xb, rs * a.C + cs, o);
    };
    float2 w[TP][CPT];
    Packed<DT, CPT> wp[PER_USE ? TP : 1]; // the window as stored (PER_USE)
    // a row entering the window: converted (or kept as stored, PER_USE),
    // zeroed when outside the stream or the lane has no channel. The zeroing
    // selects the stored words (all-zero words convert to +0.0 for every
    // type) before the conversion, so the loaded words are always used and
    // the compiler keeps every load unconditional (converting first and then
    // selecting let it move each load and conversion under a branch, with a
    // full wait after each load).
    auto enter = [&](const Packed<DT, CPT> &p, auto slotc, int64_t row, bool test) PFB_INLINE {
        constexpr int slot = decltype(slotc)::value;
        const bool ok = !test || (active && row >= 0 && row < a.in_rows);
        Packed<DT, CPT> m;
        sfor<Packed<DT, CPT>::WORDS>([&](auto q) PFB_INLINE { m.w[q] = ok ? p.w[q] : 0u; });
        if constexpr (PER_USE)
            wp[slot] = m;
        else
            unpack<DT, CPT>(m, w[slot]);
    };
    // window sample of slot `slot`, channel k, for one tap
    auto tap_in = [&](auto slotc, auto kc) PFB_INLINE -> float2 {
        constexpr int slot = decltype(slotc)::value;
        constexpr int k = decltype(kc)::value;
        if constexpr (PER_USE)
            return unpack_one_fresh<DT, CPT>(wp[slot], k);
        else
            return w[slot][k];
    };
    Packed<DT, CPT> pf[D]; // prefetched rows, still packed
    // TP > 16: a tile of one U-row block (MULTI: of whole U-row blocks),
    // every row it reads inside the stream and every lane on a channel
    // (wave-uniform). MULTI only where the loop over blocks still fits the
    // registers without spilling (32 taps, 8-byte complex64 or 4-byte fp16
    // samples, the stand-alone FIR kernel).
    constexpr bool MULTI = TP == 32 && NT && (DT == DT_C64 || DT == DT_CF16);
    const bool tp_clean = TP > 16 && (cch + 1) * 64 * CPT <= a.C && (nout == U || (MULTI && nout > 0 && nout % U == 0)) &&
                          row0 >= 0 && row0 + nout + TP - 2 < a.in_rows;
    sfor<TP - 1>([&](auto j) PFB_INLINE {
        Packed<DT, CPT> t;
        if constexpr (TP <= 16) {
            ldc(row0 + j, t);
            enter(t, j, row0 + j, true);
        } else {
            if (tp_clean) {
                load_packed<DT, CPT>(xb, (row0 + j) * a.C + c0, t);
            } else {
                const int64_t r = row0 + j;
                if (active && r >= 0 && r < a.in_rows)
                    load_packed<DT, CPT>(xb, r * a.C + c0, t);
                else
                    zero_packed<DT, CPT>(t);
            }
            unpack<DT, CPT>(t, w[j]);
        }
    });
    sfor<D>([&](auto k) PFB_INLINE {
        if constexpr (TP <= 16) {
            ldc(row0 + TP - 1 + k, pf[k]); // masked when the row enters the window
        } else {
            const int64_t r = row0 + TP - 1 + k;
            if (tp_clean)
                load_packed<DT, CPT>(xb, r * a.C + c0, pf[k]);
            else if (k < nout && active && r >= 0 && r < a.in_rows)
                load_packed<DT, CPT>(xb, r * a.C + c0, pf[k]);
            else
                zero_packed<DT, CPT>(pf[k]);
        }
    });

    float2 *yb = a.y + (int64_t)b * a.y_bstride + (s_begin - a.out_first) * a.C + c0;
    // One unrolled block of U outputs, of one of three kinds:
    //   FULL  every output in the tile, every entering and prefetched row in
    //         the stream, every lane on a channel: nothing is tested;
    //   LAST  as FULL, but the block ends the tile, so only its first U-D
    //         rows prefetch (a compile-time set): still nothing is tested;
    //   TAIL  anything else (the last tile of a stream, the last partial
    //         channel chunk, a ragged tile end): each row is tested and each
    //         entering row masked.
    enum { TAIL = 0, FULL = 1, LAST = 2 };
    auto block = [&](int base, auto kindc) PFB_INLINE {
        constexpr int KIND = decltype(kindc)::value;
        sfor<U>([&](auto jjc) PFB_INLINE {
            constexpr int jj = decltype(jjc)::value;
            const int o = base + jj;
            const int64_t row_in = row0 + o + TP - 1; // row entering the window
            if (KIND != TAIL || o < nout) {
                if constexpr (KIND == TAIL) {
                    enter(pf[jj % D], std::integral_constant<int, (jj + TP - 1) % TP>{}, row_in, true);
                    ldc(row_in + D, pf[jj % D]);
                } else {
                    enter(pf[jj % D], std::integral_constant<int, (jj + TP - 1) % TP>{}, row_in, false);
                    if constexpr (KIND == FULL || jj < U - D)
                        load_packed<DT, CPT>(xb, (row_in + D) * a.C + c0, pf[jj % D]);
                }
                float2 acc[CPT];
                sfor<CPT>([&](auto k) PFB_INLINE {
                    float ar = 0.0f, ai = 0.0f;
                    sfor<TP>([&](auto jc) PFB_INLINE {
                        constexpr int j = decltype(jc)::value;
                        const float2 xv = tap_in(std::integral_constant<int, (jj + j) % TP>{}, k);
                        ar = __builtin_fmaf(hp[k][j], xv.x, ar);
                        ai = __builtin_fmaf(hp[k][j], xv.y, ai);
                    });
                    acc[k] = make_float2(ar, ai);
                });
                if (KIND != TAIL || active) {
                    if constexpr (NT)
                        store_c64_nt<CPT>(yb + (int64_t)o * a.C, acc);
                    else
                        store_c64<CPT>(yb + (int64_t)o * a.C, acc);
                }
            }
        });
    };
    if constexpr (TP <= 16) {
        int base = 0;
        // wave-uniform: every lane on a channel, every entering row in the stream
        const bool clean =
            (cch + 1) * 64 * CPT <= a.C && row0 + TP - 1 >= 0 && row0 + nout + TP - 2 < a.in_rows;
        if (clean) {
            for (; base + U + D <= nout; base += U)
                block(base, std::integral_constant<int, FULL>{});
            if (base + U == nout) {
                block(base, std::integral_constant<int, LAST>{});
                base += U;
            }
        }
        for (; base < nout; base += U)
            block(base, std::integral_constant<int, TAIL>{});
    } else if (tp_clean) {
        // Windows of 32 taps and more, a tile of whole U-row blocks inside
        // the stream with every lane on a channel (the common case): every
        // load is issued unconditionally, so the compiler waits only for the
        // row that enters the window and D rows stay in flight. Blocks before
        // the last prefetch the next block's first rows; the last block
        // prefetches only inside itself.
        auto clean_block = [&](int base, auto lastc) PFB_INLINE {
            constexpr bool LASTB = decltype(lastc)::value;
            sfor<U>([&](auto jjc) PFB_INLINE {
            constexpr int jj = decltype(jjc)::value;
            const int64_t row_in = row0 + base + jj + TP - 1;
            unpack<DT, CPT>(pf[jj % D], w[(jj + TP - 1) % TP]);
            if constexpr (!LASTB || jj + D < U)
                load_packed<DT, CPT>(xb, (row_in + D) * a.C + c0, pf[jj % D]);
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
            if constexpr (NT)
                store_c64_nt<CPT>(yb + (int64_t)(base + jj) * a.C, acc);
            else
                store_c64<CPT>(yb + (int64_t)(base + jj) * a.C, acc);
            });
        };
        int base = 0;
        if constexpr (MULTI) {
            for (; base + U < nout; base += U)
                clean_block(base, std::false_type{});
        }
        clean_block(base, std::true_type{});
    } else {
        // Windows of 32 taps and more, anything else (ragged tiles, stream
        // edges, the last partial channel chunk): one compact loop; rows
        // outside the stream are not loaded but zeroed, and the prefetch
        // stays inside the tile.
        for (int base = 0; base < nout; base += U) {
            sfor<U>([&](auto jjc) PFB_INLINE {
                constexpr int jj = decltype(jjc)::value;
                const int o = base + jj;
                if (o < nout) {
                    const int64_t row_in = row0 + o + TP - 1;
                    unpack<DT, CPT>(pf[jj % D], w[(jj + TP - 1) % TP]);
                    if (o + D < nout) {
                        const int64_t r = row_in + D;
                        if (active && r >= 0 && r < a.in_rows)
                            load_packed<DT, CPT>(xb, r * a.C + c0, pf[jj % D]);
                        else
                            zero_packed<DT, CPT>(pf[jj % D]);
                    }
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
}

} // namespace pfb
