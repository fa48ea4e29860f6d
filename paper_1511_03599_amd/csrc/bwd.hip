// Fused adjoint of the filter bank: inverse FFT, sample gradient and tap
// gradient in one pass.
//
// For a real loss with frequency-spectra gradient gY (torch convention), the
// adjoint of the DFT of Sec. 2, Eq. (2) gives gy = unnormalised inverse DFT
// of gY, and the adjoint of the FIR of Algorithm 1 gives
//   gx[p][c] = sum_{t < T} h[t][c] gy[p - t][c]      (gy = 0 outside [0, S))
//   gh[t][c] = sum_p Re(conj(gy[p - t][c]) x[p][c])  (p = s + t)
// Both read, for output row p, the same last T rows of gy, so one register
// window of gy per channel serves both.
//
// One workgroup owns all C channels of a tile of gx rows [p0, p0 + S_B) of
// one stream. It walks gy rows q from p0 - (TP-1) upwards in chunks of RB:
//   1. inverse FFT of RB rows of gY (HBM -> registers -> LDS row buffer);
//   2. per channel: push each gy row into the window; for rows q >= p0 also
//      load x[q], write gx[q] and accumulate the tap-gradient partials.
// The first TP-1 rows of a tile only fill the window (they are recomputed
// from gY by the previous tile). At the end each workgroup writes its
// partial tap gradient, which a second small kernel sums in a fixed order.
#include "fft_device.h"
#include "launch.h"

namespace pfb {

template <int LOG2C, int TP, int CPT> struct BwdShape {
    static constexpr int C = 1 << LOG2C;
    static constexpr int NT = C / CPT;
    using FL = FftLanes<LOG2C>;
    static constexpr int G = FL::G;
    static constexpr int NG = NT / G;
    static constexpr int RB = 16 > TP ? 16 : TP;
    static constexpr int ROUNDS = RB / NG;
    // x rows prefetched; shallower for the largest register footprint
    static constexpr int D = (TP >= 16 && CPT == 2) ? 4 : 8;
    using S = FftShape<LOG2C, G>;
    static_assert(G <= 64, "one transform per wave or less");
    static_assert(NG >= 1 && RB % TP == 0 && RB % D == 0 && RB % NG == 0, "chunk shape");
};

constexpr int bwd_cpt(int log2c) { return log2c >= 10 ? 2 : 1; }

template <int TP, int LOG2C, int CPT>
__global__ __launch_bounds__((1 << LOG2C) / CPT) void fused_bwd_kernel(BwdArgs a)
{
    using F = BwdShape<LOG2C, TP, CPT>;
    using S = typename F::S;
    constexpr int C = F::C;
    constexpr int RB = F::RB;
    constexpr int D = F::D;
    constexpr int G = F::G;
    __shared__ float2 lds[RB * S::PADDED];
    // the interleaved form (below) reads its twiddles from LDS
    // twiddles read from LDS: a wait for a global twiddle load would also
    // wait for the x loads and gx stores issued before it
    __shared__ float2 tws[fft_tw_entries<LOG2C>()];

    const int tile = (int)(blockIdx.x % a.n_tiles);
    const int b = (int)(blockIdx.x / a.n_tiles);
    const int t = (int)threadIdx.x;
    const int c0 = t * CPT;
    const int64_t rows = a.S + a.T - 1; // gx rows
    const int64_t p0 = (int64_t)tile * a.SB;
    const int np = (int)((rows - p0) < a.SB ? (rows - p0) : a.SB);
    const int64_t q0 = p0 - (TP - 1);  // first gy row walked
    const int nq = np + TP - 1;        // gy rows walked
    const int off = TP - a.T;
    const bool want_gx = a.gx != nullptr;
    const bool want_gh = a.part != nullptr;
    const bool both = want_gx && want_gh;
    enum { TAIL = 0, FULL = 1, LAST = 2 };
    // BUF: one wave per transform and two transform rounds per chunk
    // (C=512, C=1024): every row runs unconditionally through bounded
    // views, and the rounds interleave with the gradient rows (below);
    // otherwise the chunk forms FULL and TAIL
    constexpr bool BUF = F::G == 64 && F::ROUNDS == 2;

    // window slot j of output p holds gy[p - (TP-1) + j], tap t = TP-1-j
    float hp[TP][CPT];
    sfor<TP>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        sfor<CPT>([&](auto k) { hp[j][k] = (j >= off) ? a.h[(int64_t)(TP - 1 - j) * C + c0 + k] : 0.0f; });
    });
    float acc[TP][CPT];
    sfor<TP>([&](auto j) { sfor<CPT>([&](auto k) { acc[j][k] = 0.0f; }); });

    const float2 *xb = a.x + (int64_t)b * rows * C;
    const float2 *gYb = a.gY + (int64_t)b * a.S * C;
    float2 *gxb = want_gx ? a.gx + (int64_t)b * rows * C : nullptr;
    auto ldx = [&](int64_t row, float2 (&o)[CPT]) {
        if (want_gh && row < rows)
            Loader<DT_C64, CPT>::load(xb, row * C + c0, o);
        else
            sfor<CPT>([&](auto k) { o[k] = make_float2(0.0f, 0.0f); });
    };

    // BUF: every x load and gx store goes through a view of its one row
    // (empty for rows outside the tile, o < 0 or o >= np), so the walk needs
    // no test; the lane's offset in a row is the same for every row.
    const uint32_t lane_off = (uint32_t)c0 * 8u;

    float2 w[TP][CPT];
    float2 pf[D][CPT]; // prefetched x rows: p0 + k (BUF: p0 - (TP-1) + k)
    if constexpr (BUF) {
        // the window's unfilled slots must hold finite values: rows o < 0
        // add their products with zero x rows to the tap-gradient sums
        // the ring starts at x rows o = -(TP-1) .. D-TP (zeros before the tile)
        sfor<TP>([&](auto j) { sfor<CPT>([&](auto k) { w[j][k] = make_float2(0.0f, 0.0f); }); });
        sfor<D>([&](auto j) {
            const int o = (int)j - (TP - 1);
            const bool ok = want_gh && o >= 0 && o < np;
            buf_load_c64<CPT>(buf_view(ok ? xb + (p0 + o) * C : xb, ok ? C * 8 : 0), (int)lane_off, pf[j]);
        });
    } else {
        sfor<D>([&](auto k) {
            if (k < np)
                ldx(p0 + k, pf[k]);
        });
    }

    const int gid = t / G;
    const int lane = t % G;
    // First-pass inputs of the next transform round, loaded one round ahead
    // (the loads of a chunk's first round are in flight during the previous
    // chunk's gradient phase) where registers allow: with two channels per
    // thread the window, taps and tap-gradient sums leave no room, and the
    // loads are issued at the start of each round instead. Rows outside
    // [0, S) transform zeros.
    constexpr int E = S::E;
    constexpr bool AHEAD = CPT == 1;
    float2 gv[E];
    auto gather = [&](int base_, int round_) {
        const int r = round_ * F::NG + gid;
        const int64_t q = q0 + base_ + r;
        if (base_ < nq && q >= 0 && q < a.S && base_ + r < nq) {
            const float2 *src = gYb + q * C;
            fft_gather_first<LOG2C, G>(lane, [&](int idx) { return src[idx]; }, gv);
        } else {
            sfor<E>([&](auto e) PFB_INLINE { gv[e] = make_float2(0.0f, 0.0f); });
        }
    };
    if constexpr (BUF) {
        // Every row through bounded views, and the two transform rounds of
        // a chunk interleaved with its gradient rows:
        //   round 0 (walk rows base..base+7) -> barrier -> gradient rows 0-7,
        //   round 1 (rows base+8..base+15)   -> barrier -> gradient rows 8-15.
        // Each round's gY loads are issued GAT gradient rows before the round
        // starts (into gv, which the gradient rows leave room for), so their
        // latency hides behind those rows. A round writes LDS rows that no
        // wave reads until the barrier after it; the rows it overwrites were
        // last read (by the gradient rows and by the read-back of the other
        // half, both of which every wave finishes before it reaches the
        // previous barrier) before the previous barrier, so one barrier per
        // round suffices.
        static_assert(F::ROUNDS == 2 && F::NG * 2 == RB, "two transform rounds per chunk");
        constexpr int HALF = RB / 2;
        constexpr int GAT0 = HALF / 2, GAT1 = 0;
        const int gw = __builtin_amdgcn_readfirstlane(gid); // this wave's transform
        // first-pass inputs of walk row i (gy row q0 + i), through a view of
        // that one row: rows outside [0, S) or past the walk read as zeros.
        // (One view per row keeps every load's offset the lane's own
        // constant, so no per-row offsets occupy vector registers.)
        auto gather_buf = [&](int i) PFB_INLINE {
            const int64_t q = q0 + i;
            const bool ok = q >= 0 && q < a.S && i < nq;
            const BufView vrow = buf_view(ok ? gYb + q * C : gYb, ok ? C * 8 : 0);
            // the lane's byte offset, opaque so that the per-element offsets
            // (lane offset plus a constant) are formed here and not kept in
            // registers across the loop
            int l8 = lane * 8;
            asm volatile("" : "+v"(l8));
            fft_gather_first<LOG2C, G>(
                lane,
                [&](int idx) {
                    float2 o[1];
                    buf_load_c64<1>(vrow, l8 + (idx - lane) * 8, o);
                    return o[0];
                },
                gv);
        };
        // gradient row jj of the chunk at walk row base: gy row q0 + base + jj
        // serves output row o = base + jj - (TP-1); x row o comes from
        // prefetch slot jj mod D and row o + D is loaded into it
        auto grad_row = [&](int base, auto jjc) PFB_INLINE {
            constexpr int jj = decltype(jjc)::value;
            const int o = base + jj - (TP - 1);
            sfor<CPT>([&](auto k) PFB_INLINE { w[jj % TP][k] = lds[jj * S::PADDED + S::pad(c0 + k)]; });
            float2 xv[CPT];
            sfor<CPT>([&](auto k) PFB_INLINE { xv[k] = pf[jj % D][k]; });
            {
                const int ox = o + D;
                const bool ok = want_gh && ox >= 0 && ox < np;
                buf_load_c64<CPT>(buf_view(ok ? xb + (p0 + ox) * C : xb, ok ? C * 8 : 0), (int)lane_off, pf[jj % D]);
            }
            float2 g[CPT];
            sfor<CPT>([&](auto k) PFB_INLINE {
                float gr = 0.0f, gi = 0.0f;
                sfor<TP>([&](auto jc) PFB_INLINE {
                    constexpr int j = decltype(jc)::value;
                    const float2 v = w[(jj + 1 + j) % TP][k];
                    gr = __builtin_fmaf(hp[j][k], v.x, gr);
                    gi = __builtin_fmaf(hp[j][k], v.y, gi);
                    acc[j][k] = __builtin_fmaf(v.x, xv[k].x, __builtin_fmaf(v.y, xv[k].y, acc[j][k]));
                });
                g[k] = make_float2(gr, gi);
            });
            {
                const bool ok = want_gx && o >= 0 && o < np;
                buf_store_c64_nt<CPT>(buf_view(ok ? gxb + (p0 + o) * C : xb, ok ? C * 8 : 0), (int)lane_off, g);
            }
        };
        // Across a round only the window rows that its transforms overwrite
        // stay in registers: the other half of the window is still in LDS
        // (the previous round's rows) and is read back once the round's
        // transforms are done, before its barrier, so those registers are
        // free during the transforms. Before the first
        // chunk the second-half LDS rows hold zeros (the window's
        // not-yet-walked rows).
        sfor<HALF>([&](auto r) PFB_INLINE {
            sfor<CPT>([&](auto k) PFB_INLINE {
                lds[(HALF + decltype(r)::value) * S::PADDED + S::pad(c0 + k)] = make_float2(0.0f, 0.0f);
            });
        });
        stage_twiddles_lds<LOG2C>(tws, a.tw, t, F::NT);
        lds_barrier();
        gather_buf(gw);
        for (int base = 0; base < nq; base += RB) {
            sfor<2>([&](auto hc) PFB_INLINE {
                constexpr int H = decltype(hc)::value;
                float2 cur[E];
                sfor<E>([&](auto e) PFB_INLINE { cur[e] = gv[e]; });
                float2 *row = lds + (H * F::NG + gw) * S::PADDED;
                // opaque lane index: the transform's LDS addresses are then
                // formed in each round instead of being hoisted out of the
                // loop and held in registers for both rounds
                int ln = lane;
                asm volatile("" : "+v"(ln));
                fft_passes<LOG2C, G, true, false, true>(ln, row, tws, cur, LdsRowDst{row});
                // window slots holding rows of the half this round did not
                // overwrite (the last min(TP, HALF) rows of that half). They
                // are read back before this round's barrier: those rows were
                // written before the previous barrier, and the next round,
                // which overwrites them, starts only after this barrier, so
                // no wave can overwrite a row that another wave is still
                // reading back.
                constexpr int NRR = TP < HALF ? TP : HALF;
                sfor<NRR>([&](auto rc) PFB_INLINE {
                    constexpr int r = (1 - H) * HALF + HALF - NRR + decltype(rc)::value;
                    sfor<CPT>([&](auto k) PFB_INLINE { w[r % TP][k] = lds[r * S::PADDED + S::pad(c0 + k)]; });
                });
                lds_barrier();
                sfor<HALF>([&](auto jc) PFB_INLINE {
                    grad_row(base, std::integral_constant<int, H * HALF + decltype(jc)::value>{});
                    if constexpr (decltype(jc)::value == (H == 0 ? GAT0 : GAT1))
                        gather_buf(H == 0 ? base + F::NG + gw : base + RB + gw);
                });
            });
        }
    } else {
    stage_twiddles_lds<LOG2C>(tws, a.tw, t, F::NT);
    lds_barrier();
    if constexpr (AHEAD)
        gather(0, 0);
    for (int base = 0; base < nq; base += RB) {
        // 1. inverse FFT of gY rows q0+base .. q0+base+RB-1 into LDS
#pragma unroll 1
        for (int round = 0; round < F::ROUNDS; ++round) {
            float2 cur[E];
            if constexpr (AHEAD) {
                sfor<E>([&](auto e) PFB_INLINE { cur[e] = gv[e]; });
                if (round + 1 < F::ROUNDS)
                    gather(base, round + 1);
                else
                    gather(base + RB, 0);
            } else {
                gather(base, round);
                sfor<E>([&](auto e) PFB_INLINE { cur[e] = gv[e]; });
            }
            float2 *row = lds + (round * F::NG + gid) * S::PADDED;
            fft_passes<LOG2C, G, true, false, true>(lane, row, tws, cur, LdsRowDst{row});
        }
        lds_barrier();
        // 2. sample gradient and tap-gradient partials. In FULL chunks (every
        // row an output of the tile, every x prefetch inside it, both
        // gradients wanted) and in the LAST chunk of a tile (the same, with
        // only its first RB-D rows prefetching) nothing is tested, so loads
        // and stores are issued unconditionally and the compiler waits only
        // for the x row a step uses; other chunks test each row.
        auto grad_chunk = [&](auto kindc) PFB_INLINE {
            constexpr int KIND = decltype(kindc)::value;
            // row bases of this chunk (gx row and prefetched x row of jj = 0)
            const float2 *xrow = nullptr;
            float2 *gxrow = nullptr;
            if constexpr (KIND != TAIL) {
                xrow = wave_uniform(xb + (p0 + base - (TP - 1) + D) * C);
                gxrow = wave_uniform(gxb + (p0 + base - (TP - 1)) * C);
            }
            sfor<RB>([&](auto jjc) PFB_INLINE {
                constexpr int jj = decltype(jjc)::value;
                const int i = base + jj; // gy row q0 + i
                if (KIND != TAIL || i < nq) {
                    sfor<CPT>([&](auto k) PFB_INLINE { w[jj % TP][k] = lds[jj * S::PADDED + S::pad(c0 + k)]; });
                    const int o = i - (TP - 1); // output row p0 + o
                    if (KIND != TAIL || o >= 0) {
                        // x[p0 + o] arrives from the prefetch ring; its slot,
                        // o mod D, is a constant because base is a multiple of
                        // RB (itself a multiple of D)
                        constexpr int slot = ((jj - (TP - 1)) % D + D) % D;
                        float2 xv[CPT];
                        sfor<CPT>([&](auto k) PFB_INLINE { xv[k] = pf[slot][k]; });
                        if constexpr (KIND == FULL || (KIND == LAST && jj < RB - D))
                            Loader<DT_C64, CPT>::load(xrow, jj * C + c0, pf[slot]);
                        else if (KIND == TAIL && o + D < np)
                            ldx(p0 + o + D, pf[slot]);
                        float2 g[CPT];
                        sfor<CPT>([&](auto k) PFB_INLINE {
                            float gr = 0.0f, gi = 0.0f;
                            sfor<TP>([&](auto jc) PFB_INLINE {
                                constexpr int j = decltype(jc)::value;
                                // slot of gy[p - (TP-1) + j]: (jj - (TP-1) + j) mod TP
                                const float2 v = w[(jj + 1 + j) % TP][k];
                                gr = __builtin_fmaf(hp[j][k], v.x, gr);
                                gi = __builtin_fmaf(hp[j][k], v.y, gi);
                                acc[j][k] = __builtin_fmaf(v.x, xv[k].x, __builtin_fmaf(v.y, xv[k].y, acc[j][k]));
                            });
                            g[k] = make_float2(gr, gi);
                        });
                        if constexpr (KIND != TAIL)
                            store_c64_nt<CPT>(gxrow + jj * C + c0, g);
                        else if (want_gx && o < np)
                            store_c64_nt<CPT>(gxb + (p0 + o) * C + c0, g);
                    }
                }
            });
        };
        if (both && base >= TP - 1 && base + RB <= nq && base + RB - TP + D < np)
            grad_chunk(std::integral_constant<int, FULL>{});
        else
            grad_chunk(std::integral_constant<int, TAIL>{});
        lds_barrier();
    }
    }
    if (want_gh) {
        float *pb = a.part + ((int64_t)b * a.n_tiles + tile) * (int64_t)a.T * C + c0;
        sfor<TP>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const int tt = TP - 1 - j;
            if (tt < a.T)
                sfor<CPT>([&](auto k) { pb[(int64_t)tt * C + k] = acc[j][k]; });
        });
    }
}

bool fused_bwd_supported(int tp, int log2c)
{
    return log2c >= 8 && log2c <= 10 && (tp == 4 || tp == 8 || tp == 16);
}

template <int TP, int LOG2C> static hipError_t launch_bwd_t(const BwdArgs &a, hipStream_t st)
{
    const int64_t blocks = (int64_t)a.B * a.n_tiles;
    if (blocks <= 0)
        return hipSuccess;
    constexpr int CPT = bwd_cpt(LOG2C);
    hipLaunchKernelGGL((fused_bwd_kernel<TP, LOG2C, CPT>), dim3((unsigned)blocks), dim3((1 << LOG2C) / CPT), 0, st,
                       a);
    return hipGetLastError();
}

hipError_t launch_fused_bwd(const BwdArgs &a, int tp, int log2c, hipStream_t st)
{
#define PFB_BWD_C(L2)                                                                                        \
    case L2:                                                                                                 \
        switch (tp) {                                                                                        \
        case 4: return launch_bwd_t<4, L2>(a, st);                                                           \
        case 8: return launch_bwd_t<8, L2>(a, st);                                                           \
        case 16: return launch_bwd_t<16, L2>(a, st);                                                         \
        default: return hipErrorInvalidValue;                                                                \
        }
    switch (log2c) {
        PFB_BWD_C(8)
        PFB_BWD_C(9)
        PFB_BWD_C(10)
    default:
        return hipErrorInvalidValue;
    }
#undef PFB_BWD_C
}

} // namespace pfb
