// Fused adjoint of the filter bank with specialised waves.
//
// Same arithmetic as fused_bwd_kernel (bwd.hip): for a real loss with
// frequency-spectra gradient gY, gy = unnormalised inverse DFT of gY (adjoint
// of Sec. 2, Eq. (2)), and the adjoint of the FIR of Algorithm 1 gives
//   gx[p][c] = sum_{t < T} h[t][c] gy[p - t][c]      (gy = 0 outside [0, S))
//   gh[t][c] = sum_p Re(conj(gy[p - t][c]) x[p][c])
// with the same operations in the same order, so the two kernels give
// identical bits.
//
// One workgroup owns all C channels of a tile of gx rows, walked in chunks of
// RB gy rows, and its waves take one of two roles:
//   producers  inverse-transform the chunk's gY rows into an LDS buffer and
//              stage the matching x rows into a second one;
//   consumers  hold, per channel, the window of the last TP gy rows, the taps
//              and the tap-gradient sums in registers; they read gy and x
//              rows from LDS, write gx and accumulate the tap gradient.
// The buffers are double: while the consumers work on chunk k, the producers
// fill chunk k+1 from registers loaded one step earlier and issue the loads
// of chunk k+2, so HBM loads are in flight while both roles compute (in a
// single-role kernel every wave alternates between the two and the loads
// wait for the arithmetic). One workgroup barrier per chunk hands
// the buffers over. Each role runs its own loop, so the consumers' window
// and sums are not held by the producer waves; both loops pass the same
// number of barriers.
#include "fft_device.h"
#include "launch.h"

namespace pfb {

template <int LOG2C, int TP> struct WsShape {
    static constexpr int C = 1 << LOG2C;
    static constexpr int CPT = LOG2C >= 10 ? 2 : 1;    // channels per consumer lane
    static constexpr int NC = C / (64 * CPT);           // consumer waves
    using FL = FftLanes<LOG2C>;
    static constexpr int G = FL::G;                     // lanes per transform
    static constexpr int E = FL::E;
    static constexpr int RB = 4;                        // gy rows per chunk
    static constexpr int TPW = 64 / G;                  // transforms per producer wave
    static constexpr int NP = RB / TPW;                 // producer waves
    static constexpr int NT = (NC + NP) * 64;
    static constexpr int XQ = RB * C / 2 / (NP * 64);   // x float4 per producer lane
    // producers prefetch the next chunk where registers allow (C <= 512)
    static constexpr bool PREFETCH = LOG2C <= 9;
    // chunks per unrolled consumer step: a whole number of window periods and
    // an even number of chunks, so window slots and buffer parity are static
    static constexpr int UNR = (TP / RB) > 2 ? (TP / RB) : 2;
    using S = FftShape<LOG2C, G>;
    static_assert(G <= 64 && 64 % G == 0 && NP * TPW == RB, "one round of transforms per chunk");
    static_assert((UNR * RB) % TP == 0 && UNR % 2 == 0, "static window slots and parity");
    static_assert(XQ >= 1 && RB * C / 2 == XQ * NP * 64, "x staging");
};

template <int TP, int LOG2C>
__global__ __launch_bounds__((WsShape<LOG2C, TP>::NT)) void fused_bwd_ws_kernel(BwdArgs a)
{
    using W = WsShape<LOG2C, TP>;
    using S = typename W::S;
    constexpr int C = W::C;
    constexpr int CPT = W::CPT;
    constexpr int RB = W::RB;
    constexpr int G = W::G;
    constexpr int E = W::E;
    constexpr int PADDED = S::PADDED;
    __shared__ float2 gy_buf[2 * RB * PADDED];
    __shared__ float4 x_buf[2 * RB * C / 2];

    const int tile = (int)(blockIdx.x % a.n_tiles);
    const int b = (int)(blockIdx.x / a.n_tiles);
    const int64_t rows = a.S + a.T - 1; // gx rows
    const int64_t p0 = (int64_t)tile * a.SB;
    const int np = (int)((rows - p0) < a.SB ? (rows - p0) : a.SB);
    const int64_t q0 = p0 - (TP - 1);   // first gy row walked
    const int nq = np + TP - 1;         // gy rows walked
    const int nchunks = (nq + RB - 1) / RB;
    const bool want_gx = a.gx != nullptr;
    const bool want_gh = a.part != nullptr;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64);

    if (wave >= W::NC) {
        // ---------------- producers ----------------
        const int pl = (int)threadIdx.x - W::NC * 64;
        const int pw = pl / 64, lw = pl % 64;
        const int r = pw * W::TPW + lw / G; // chunk row transformed by this lane's group
        const int lane = lw % G;
        const float2 *xb = a.x + (int64_t)b * rows * C;
        const float2 *gYb = a.gY + (int64_t)b * a.S * C;
        // x row f of chunk k (gy row k*RB + rr pairs with gx row p0 + o,
        // o = k*RB + rr - (TP-1))
        auto ldx = [&](int k, int e) {
            const int f = pl + W::NP * 64 * e;
            const int rr = f / (C / 2);
            const int cf = f % (C / 2);
            const int o = k * RB + rr - (TP - 1);
            const int64_t xr = p0 + o;
            if (o >= 0 && o < np && xr < rows)
                return *reinterpret_cast<const float4 *>(xb + xr * C + 2 * cf);
            return make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        };
        auto gather = [&](int k, float2 (&v)[E]) {
            const int64_t q = q0 + (int64_t)k * RB + r;
            if (q >= 0 && q < a.S) {
                const float2 *src = gYb + q * C;
                fft_gather_first<LOG2C, G>(lane, [&](int idx) { return src[idx]; }, v);
            } else {
                sfor<E>([&](auto e) PFB_INLINE { v[e] = make_float2(0.0f, 0.0f); });
            }
        };
        if constexpr (W::PREFETCH) {
            // Loads for chunk k+1 are issued before chunk k is transformed
            // and staged, so they are in flight through the transform and
            // the wait at the barrier.
            float2 vn[E];     // first-pass inputs (gY) of the next chunk
            float4 xn[W::XQ]; // x rows of the next chunk
            auto issue = [&](int k) {
                gather(k, vn);
                if (want_gh)
                    sfor<W::XQ>([&](auto ec) PFB_INLINE { xn[decltype(ec)::value] = ldx(k, decltype(ec)::value); });
            };
            auto finish = [&](int k, int buf) {
                float2 v[E];
                sfor<E>([&](auto e) PFB_INLINE { v[e] = vn[e]; });
                if (want_gh) {
                    float4 *xd = x_buf + buf * (RB * C / 2);
                    sfor<W::XQ>([&](auto ec) PFB_INLINE {
                        constexpr int e = decltype(ec)::value;
                        xd[pl + W::NP * 64 * e] = xn[e];
                    });
                }
                if (k + 1 < nchunks)
                    issue(k + 1);
                float2 *row = gy_buf + (buf * RB + r) * PADDED;
                fft_passes<LOG2C, G, true, false, false, false>(lane, row, a.tw, v, LdsRowDst{row});
            };
            issue(0);
            finish(0, 0);
            lds_barrier();
            for (int k = 0; k < nchunks; ++k) {
                if (k + 1 < nchunks)
                    finish(k + 1, (k + 1) & 1);
                lds_barrier();
            }
        } else {
            // Register budget too small to hold the next chunk's loads: each
            // chunk's loads are issued at the start of its own step, x in two
            // halves (the second one in flight during the transform).
            constexpr int XH = (W::XQ + 1) / 2;
            auto produce = [&](int k, int buf) {
                float2 v[E];
                gather(k, v);
                float4 *xd = x_buf + buf * (RB * C / 2);
                float4 xh[XH];
                if (want_gh) {
                    sfor<XH>([&](auto ec) PFB_INLINE { xh[decltype(ec)::value] = ldx(k, decltype(ec)::value); });
                    sfor<XH>([&](auto ec) PFB_INLINE {
                        constexpr int e = decltype(ec)::value;
                        xd[pl + W::NP * 64 * e] = xh[e];
                    });
                    sfor<W::XQ - XH>([&](auto ec) PFB_INLINE {
                        xh[decltype(ec)::value] = ldx(k, XH + decltype(ec)::value);
                    });
                }
                float2 *row = gy_buf + (buf * RB + r) * PADDED;
                fft_passes<LOG2C, G, true, false, false, false>(lane, row, a.tw, v, LdsRowDst{row});
                if (want_gh) {
                    sfor<W::XQ - XH>([&](auto ec) PFB_INLINE {
                        constexpr int e = decltype(ec)::value;
                        xd[pl + W::NP * 64 * (XH + e)] = xh[e];
                    });
                }
            };
            produce(0, 0);
            lds_barrier();
            for (int k = 0; k < nchunks; ++k) {
                if (k + 1 < nchunks)
                    produce(k + 1, (k + 1) & 1);
                lds_barrier();
            }
        }
        return;
    }

    // ---------------- consumers ----------------
    const int t = (int)threadIdx.x;
    const int c0 = t * CPT;
    // window slot j of output p holds gy[p - (TP-1) + j], tap t = TP-1-j
    const int off = TP - a.T;
    float hp[TP][CPT];
    sfor<TP>([&](auto jc) PFB_INLINE {
        constexpr int j = decltype(jc)::value;
        sfor<CPT>([&](auto k) PFB_INLINE {
            hp[j][k] = (j >= off) ? a.h[(int64_t)(TP - 1 - j) * C + c0 + k] : 0.0f;
        });
    });
    float acc[TP][CPT];
    sfor<TP>([&](auto j) PFB_INLINE { sfor<CPT>([&](auto k) PFB_INLINE { acc[j][k] = 0.0f; }); });
    float2 w[TP][CPT];
    float2 *gxb = want_gx ? a.gx + (int64_t)b * rows * C : nullptr;

    lds_barrier(); // chunk 0 staged
    for (int kb = 0; kb < nchunks; kb += W::UNR) {
        sfor<W::UNR>([&](auto jc) PFB_INLINE {
            constexpr int J = decltype(jc)::value;
            constexpr int buf = J % 2;
            const int k = kb + J;
            if (k < nchunks) {
                const float2 *gyr = gy_buf + buf * RB * PADDED;
                const float2 *xr = reinterpret_cast<const float2 *>(x_buf + buf * (RB * C / 2));
                sfor<RB>([&](auto rc) PFB_INLINE {
                    constexpr int rr = decltype(rc)::value;
                    constexpr int jr = J * RB + rr; // row within the unrolled step
                    const int i = k * RB + rr;      // gy row q0 + i
                    if (i < nq) {
                        sfor<CPT>([&](auto kk) PFB_INLINE {
                            w[jr % TP][kk] = gyr[rr * PADDED + S::pad(c0 + kk)];
                        });
                        const int o = i - (TP - 1); // gx row p0 + o
                        if (o >= 0) {
                            float2 xv[CPT];
                            sfor<CPT>([&](auto kk) PFB_INLINE { xv[kk] = xr[rr * C + c0 + kk]; });
                            float2 g[CPT];
                            sfor<CPT>([&](auto kk) PFB_INLINE {
                                float gr = 0.0f, gi = 0.0f;
                                sfor<TP>([&](auto jc2) PFB_INLINE {
                                    constexpr int j = decltype(jc2)::value;
                                    const float2 v = w[(jr + 1 + j) % TP][kk];
                                    gr = __builtin_fmaf(hp[j][kk], v.x, gr);
                                    gi = __builtin_fmaf(hp[j][kk], v.y, gi);
                                    acc[j][kk] =
                                        __builtin_fmaf(v.x, xv[kk].x, __builtin_fmaf(v.y, xv[kk].y, acc[j][kk]));
                                });
                                g[kk] = make_float2(gr, gi);
                            });
                            if (want_gx)
                                store_c64_nt<CPT>(gxb + (p0 + o) * C + c0, g);
                        }
                    }
                });
                lds_barrier();
            }
        });
    }
    if (want_gh) {
        float *pb = a.part + ((int64_t)b * a.n_tiles + tile) * (int64_t)a.T * C + c0;
        sfor<TP>([&](auto jc) PFB_INLINE {
            constexpr int j = decltype(jc)::value;
            const int tt = TP - 1 - j;
            if (tt < a.T)
                sfor<CPT>([&](auto k) PFB_INLINE { pb[(int64_t)tt * C + k] = acc[j][k]; });
        });
    }
}

template <int TP, int LOG2C> static hipError_t launch_bwd_ws_t(const BwdArgs &a, hipStream_t st)
{
    const int64_t blocks = (int64_t)a.B * a.n_tiles;
    if (blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((fused_bwd_ws_kernel<TP, LOG2C>), dim3((unsigned)blocks), dim3(WsShape<LOG2C, TP>::NT), 0,
                       st, a);
    return hipGetLastError();
}

hipError_t launch_fused_bwd_ws(const BwdArgs &a, int tp, int log2c, hipStream_t st)
{
#define PFB_BWD_WS_C(L2)                                                                                     \
    case L2:                                                                                                 \
        switch (tp) {                                                                                        \
        case 4: return launch_bwd_ws_t<4, L2>(a, st);                                                        \
        case 8: return launch_bwd_ws_t<8, L2>(a, st);                                                        \
        case 16: return launch_bwd_ws_t<16, L2>(a, st);                                                      \
        default: return hipErrorInvalidValue;                                                                \
        }
    switch (log2c) {
        PFB_BWD_WS_C(8)
        PFB_BWD_WS_C(9)
        PFB_BWD_WS_C(10)
    default:
        return hipErrorInvalidValue;
    }
#undef PFB_BWD_WS_C
}

} // namespace pfb
