// Stockham autosort FFT for one C-point transform held by a group of G lanes
// (C a power of two, E = C/G elements per lane, E in {8, 16, 32}).
//
// The transform is the DFT of Sec. 2, Eq. (2): unnormalised, bins in natural
// order, exp(-2 pi i n m / C). The inverse (exp(+...), unnormalised) is the
// same network with every constant and twiddle conjugated. Negation is
// exact and every operation here rounds symmetrically, so this gives the
// values of the conjugate-in, conjugate-out form of the forward network
// (up to the sign of an exact zero) without flipping the signs of the input
// and output elements.
//
// Each pass of radix R with stride L (the product of the radices of earlier
// passes) lets every butterfly j (0 <= j < C/R) read elements j + i*C/R,
// multiply element i by W_{R L}^{i k} (k = j mod L), run an R-point DFT in
// registers and write element i to (j - k) R + k + i L. After the last pass
// the output is in natural order. The first pass reads its inputs straight
// from the source (global memory or an LDS row) and the last pass writes its
// outputs straight to the destination with consecutive lanes on consecutive
// elements, so both are coalesced. Between passes the data goes through this
// group's LDS row, padded by one element in sixteen against bank conflicts.
//
// Twiddles come from a per-transform-size table computed in FP64 on the host
// and rounded once to float32: for every pass P > 0 (radix R, stride L) it
// holds W_{RL}^{ik} = exp(-2 pi i (ik mod RL) / (RL)) at
// [pass_offset(P) + k*R + i], so the R twiddles of one butterfly are
// contiguous and load as R/2 aligned 16-byte vectors.
#pragma once

#include <type_traits>

#include "device_common.h"
#include "fft_schedule.h"

namespace pfb {

// cos(2 pi e / 32) and sin(2 pi e / 32).
constexpr float cos32(int e)
{
    constexpr float c[32] = {1.0f, 0.98078528040323045f, 0.92387953251128674f, 0.83146961230254524f,
                             0.70710678118654757f, 0.55557023301960222f, 0.38268343236508978f, 0.19509032201612827f,
                             0.0f, -0.19509032201612827f, -0.38268343236508978f, -0.55557023301960222f,
                             -0.70710678118654757f, -0.83146961230254524f, -0.92387953251128674f, -0.98078528040323045f,
                             -1.0f, -0.98078528040323045f, -0.92387953251128674f, -0.83146961230254524f,
                             -0.70710678118654757f, -0.55557023301960222f, -0.38268343236508978f, -0.19509032201612827f,
                             0.0f, 0.19509032201612827f, 0.38268343236508978f, 0.55557023301960222f,
                             0.70710678118654757f, 0.83146961230254524f, 0.92387953251128674f, 0.98078528040323045f};
    return c[e & 31];
}
constexpr float sin32(int e) { return cos32(e - 8); }

// v * W_N^E with W_N = exp(-2 pi i / N), N dividing 32.
template <int N, int E> __device__ __forceinline__ float2 twc(float2 v)
{
    constexpr int e = (E * (32 / N)) & 31;
    if constexpr (e == 0) {
        return v;
    } else if constexpr (e == 8) {
        return mul_mi(v);
    } else if constexpr (e == 16) {
        return make_float2(-v.x, -v.y);
    } else if constexpr (e == 24) {
        return mul_pi(v);
    } else {
        constexpr float c = cos32(e), s = sin32(e);
        return make_float2(__builtin_fmaf(v.x, c, v.y * s), __builtin_fmaf(v.y, c, -(v.x * s)));
    }
}

// R-point DFT in registers; INV: exp(+...) (conjugated constants).
template <int R, bool INV = false> struct Dft;
template <bool INV> struct Dft<1, INV> {
    static __device__ __forceinline__ void run(float2 *) {}
};
template <bool INV> struct Dft<2, INV> {
    static __device__ __forceinline__ void run(float2 *v)
    {
        float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};
template <bool INV> struct Dft<4, INV> {
    static __device__ __forceinline__ void run(float2 *v)
    {
        const float2 d = csub(v[1], v[3]);
        float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        float2 t2 = cadd(v[1], v[3]), t3 = INV ? mul_pi(d) : mul_mi(d);
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

// R = N1 * N2 by one Cooley-Tukey step: n = N2 n1 + n2, k = k1 + N1 k2.
// INV multiplies by W_N^{-e} = W_N^{N-e}.
template <int N1, int N2, bool INV = false> __device__ __forceinline__ void dft_ct(float2 *v)
{
    constexpr int N = N1 * N2;
    float2 a[N2][N1];
    sfor<N2>([&](auto n2) PFB_INLINE {
        sfor<N1>([&](auto n1) PFB_INLINE { a[n2][n1] = v[N2 * n1 + n2]; });
        Dft<N1, INV>::run(a[n2]);
        sfor<N1>([&](auto k1) PFB_INLINE {
            constexpr int e = (decltype(n2)::value * decltype(k1)::value) % N;
            a[n2][k1] = twc<N, INV ? (N - e) % N : e>(a[n2][k1]);
        });
    });
    sfor<N1>([&](auto k1) PFB_INLINE {
        float2 b[N2];
        sfor<N2>([&](auto n2) PFB_INLINE { b[n2] = a[n2][k1]; });
        Dft<N2, INV>::run(b);
        sfor<N2>([&](auto k2) PFB_INLINE { v[k1 + N1 * k2] = b[k2]; });
    });
}
template <bool INV> struct Dft<8, INV> {
    static __device__ __forceinline__ void run(float2 *v) { dft_ct<4, 2, INV>(v); }
};
template <bool INV> struct Dft<16, INV> {
    static __device__ __forceinline__ void run(float2 *v) { dft_ct<4, 4, INV>(v); }
};
template <bool INV> struct Dft<32, INV> {
    static __device__ __forceinline__ void run(float2 *v) { dft_ct<4, 8, INV>(v); }
};

// v * w, or v * conj(w) for the inverse transform
template <bool INV> __device__ __forceinline__ float2 cmul_tw(float2 v, float2 w)
{
    return cmul(v, INV ? conj2(w) : w);
}

// A destination that is a padded LDS row: output element idx goes to
// row[pad(idx)]. The last pass forms each butterfly's padded address once
// and adds constants (a generic `dst(idx, v)` recomputes pad(idx) per
// element).
struct LdsRowDst {
    float2 *row;
};

// Synchronise the lanes of one FFT group between LDS passes.
template <int G> __device__ __forceinline__ void group_sync()
{
    if constexpr (G > 64) {
        lds_barrier();
    } else {
        // One wave: LDS operations of a wave complete in order; only the
        // compiler has to be kept from moving accesses across this point.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <int LOG2C, int G> struct FftShape {
    static constexpr int C = 1 << LOG2C;
    static constexpr int E = C / G;
    static constexpr FftSchedule SCHED{LOG2C};
    static constexpr int NPASS = SCHED.npass;
    static constexpr int PADDED = C + C / 16; // LDS float2 per transform
    static_assert(E == SCHED.e, "elements per lane");
    static_assert(G * E == C, "shape");

    static __device__ __forceinline__ int pad(int idx) { return idx + (idx >> 4); }
    // pad(a + i*STR) given pa = pad(a): for STR a multiple of 16 the padding
    // grows by exactly i*STR/16, so the address is pa plus a constant and
    // one base register serves every i
    template <int STR> static __device__ __forceinline__ int pad_at(int a, int pa, int i)
    {
        if constexpr (STR % 16 == 0)
            return pa + i * (STR + STR / 16);
        else
            return pad(a + i * STR);
    }
    static constexpr int radix(int p) { return SCHED.radix(p); }
    static constexpr int stride(int p) { return SCHED.stride(p); }
    static constexpr int pass_offset(int p) { return SCHED.pass_offset(p); }
};

// First-pass inputs of one transform, gathered into the lane's registers in
// the order the first pass consumes them: element j + i*C/R of butterfly
// j = lane + G*q goes to v[q*R + i]. Split from the passes so that a caller
// can issue these loads early and overlap their latency with other work.
template <int LOG2C, int G, class Src>
__device__ __forceinline__ void fft_gather_first(int lane, Src &&src, float2 (&v)[FftShape<LOG2C, G>::E])
{
    using S = FftShape<LOG2C, G>;
    constexpr int R = S::radix(0);
    constexpr int NB = S::E / R;
    constexpr int CR = S::C / R;
    sfor<NB>([&](auto q) PFB_INLINE {
        const int j = lane + G * decltype(q)::value;
        sfor<R>([&](auto i) PFB_INLINE { v[decltype(q)::value * R + decltype(i)::value] = src(j + decltype(i)::value * CR); });
    });
}

// The twiddle-table pointer a transform's passes read through (see
// fft_passes): opaque, so that the compiler does not hoist the twiddle loads
// of every pass out of a caller's loop over rows and hold them all in
// registers at once. For an LDS table only an offset is opaque, so the pointer
// keeps its LDS origin; a global one is rebuilt as a global pointer (the
// opaque value has lost its address space, and flat loads would also count
// against the LDS counter).
template <bool TW_LDS> __device__ __forceinline__ const float2 *fft_twiddle_base(const float2 *tw)
{
    if constexpr (TW_LDS) {
        int z = 0;
        asm volatile("" : "+v"(z));
        return tw + z;
    } else {
        const float2 *twp_opaque = tw;
        asm volatile("" : "+v"(twp_opaque));
        return as_global(twp_opaque);
    }
}

// First-pass inputs of one transform read from this group's padded LDS row
// (the same elements, in the same register order, as fft_gather_first with
// src(idx) = row[pad(idx)]). Element j + i*C/R of butterfly j = lane + G*q
// sits at pad(j) + i*(C/R + C/R/16) because C/R is a multiple of 16, so each
// butterfly needs one address and constant offsets (no per-element index
// arithmetic).
template <int LOG2C, int G>
__device__ __forceinline__ void fft_gather_first_lds(int lane, const float2 *row, float2 (&v)[FftShape<LOG2C, G>::E])
{
    using S = FftShape<LOG2C, G>;
    constexpr int R = S::radix(0);
    constexpr int NB = S::E / R;
    constexpr int CR = S::C / R;
    static_assert(CR % 16 == 0 && G % 16 == 0, "constant padded offsets");
    const int pl = S::pad(lane);
    sfor<NB>([&](auto q) PFB_INLINE {
        const int pj = pl + decltype(q)::value * (G + G / 16);
        sfor<R>([&](auto i) PFB_INLINE {
            v[decltype(q)::value * R + decltype(i)::value] = row[pj + decltype(i)::value * (CR + CR / 16)];
        });
    });
}

// Pass P of one transform whose first-pass inputs are already in v (see
// fft_gather_first), in two halves so that callers may run other work
// between them and between the passes of a transform (fft_passes runs them
// back to back):
//   fft_pass_gather   for P > 0, load this pass's inputs from the group's LDS
//                     row into v;
//   fft_pass_compute  apply the twiddles and the radix-R butterflies in
//                     registers, then scatter to the LDS row (and synchronise
//                     the group) or, for the last pass, hand every output
//                     element to `dst(idx, v)`.
// `twp` comes from fft_twiddle_base. A group of more than one wave must
// synchronise between the two halves (fft_pass does).
template <int LOG2C, int G, int P>
__device__ __forceinline__ void fft_pass_gather(int lane, const float2 *lds, float2 (&v)[FftShape<LOG2C, G>::E])
{
    using S = FftShape<LOG2C, G>;
    constexpr int C = S::C;
    constexpr int E = S::E;
    constexpr int R = S::radix(P);
    constexpr int NB = E / R;
    constexpr int CR = C / R;
    static_assert(P > 0, "the first pass's inputs come from fft_gather_first");
    const int plane = S::pad(lane);
    sfor<NB>([&](auto q) PFB_INLINE {
        const int j = lane + G * decltype(q)::value;
        const int pj = S::template pad_at<G>(lane, plane, decltype(q)::value);
        sfor<R>([&](auto i) PFB_INLINE {
            v[decltype(q)::value * R + decltype(i)::value] = lds[S::template pad_at<CR>(j, pj, decltype(i)::value)];
        });
    });
}

// The twiddles of pass P > 0 from the global table for this lane's
// butterflies: R/2 aligned 16-byte vectors per butterfly, E/2 in all for
// every pass (E/R butterflies of R entries). Issued one pass ahead by
// fft_passes, so that their latency hides behind the previous pass instead
// of following a barrier.
template <int LOG2C, int G, int P>
__device__ __forceinline__ void fft_load_twiddles(int lane, const float2 *twp,
                                                  float4 (&w)[FftShape<LOG2C, G>::E / 2])
{
    using S = FftShape<LOG2C, G>;
    constexpr int R = S::radix(P);
    constexpr int L = S::stride(P);
    constexpr int NB = S::E / R;
    constexpr int PO = S::pass_offset(P);
    static_assert(P > 0 && L > 1, "the first pass has no twiddles");
    sfor<NB>([&](auto q) PFB_INLINE {
        constexpr int Q = decltype(q)::value;
        const int k = (lane + G * Q) & (L - 1);
        const float4 *wp = reinterpret_cast<const float4 *>(twp + PO + k * R);
        sfor<R / 2>([&](auto hh) PFB_INLINE { w[Q * (R / 2) + decltype(hh)::value] = wp[decltype(hh)::value]; });
    });
}

// TWR: the pass's twiddles are already in `wpre` (fft_load_twiddles);
// otherwise they are read here, from the LDS copy (TW_LDS) or the global
// table.
template <int LOG2C, int G, bool INV, bool TW_LDS, int P, class Dst, bool TWR = false>
__device__ __forceinline__ void fft_pass_compute(int lane, float2 *lds, const float2 *twp,
                                                 float2 (&v)[FftShape<LOG2C, G>::E], Dst &&dst,
                                                 const float4 *wpre = nullptr)
{
    using S = FftShape<LOG2C, G>;
    constexpr int C = S::C;
    constexpr int E = S::E;
    constexpr int R = S::radix(P);
    constexpr int L = S::stride(P);
    constexpr int NB = E / R;
    constexpr int CR = C / R;

    // twiddle and butterfly
    sfor<NB>([&](auto q) PFB_INLINE {
        constexpr int Q = decltype(q)::value;
        const int j = lane + G * Q;
        if constexpr (L > 1 && TWR) {
            sfor<R / 2>([&](auto hh) PFB_INLINE {
                constexpr int H = decltype(hh)::value;
                const float4 w2 = wpre[Q * (R / 2) + H];
                if constexpr (H > 0)
                    v[Q * R + 2 * H] = cmul_tw<INV>(v[Q * R + 2 * H], make_float2(w2.x, w2.y));
                v[Q * R + 2 * H + 1] = cmul_tw<INV>(v[Q * R + 2 * H + 1], make_float2(w2.z, w2.w));
            });
        } else if constexpr (L > 1 && TW_LDS) {
            const int k = j & (L - 1);
            constexpr int PO = S::pass_offset(P);
            sfor<R - 1>([&](auto ic) PFB_INLINE {
                constexpr int i = decltype(ic)::value + 1;
                v[Q * R + i] = cmul_tw<INV>(v[Q * R + i], twp[PO + i * L + k]);
            });
        } else if constexpr (L > 1) {
            const int k = j & (L - 1);
            constexpr int PO = S::pass_offset(P);
            const float4 *wp = reinterpret_cast<const float4 *>(twp + PO + k * R);
            sfor<R / 2>([&](auto hh) PFB_INLINE {
                constexpr int H = decltype(hh)::value;
                const float4 w2 = wp[H];
                if constexpr (H > 0)
                    v[Q * R + 2 * H] = cmul_tw<INV>(v[Q * R + 2 * H], make_float2(w2.x, w2.y));
                v[Q * R + 2 * H + 1] = cmul_tw<INV>(v[Q * R + 2 * H + 1], make_float2(w2.z, w2.w));
            });
        }
        Dft<R, INV>::run(&v[Q * R]);
    });

    // scatter
    if constexpr (P == S::NPASS - 1) {
        sfor<NB>([&](auto q) PFB_INLINE {
            const int j = lane + G * decltype(q)::value;
            if constexpr (std::is_same_v<std::decay_t<Dst>, LdsRowDst>) {
                const int pj = S::pad(j);
                sfor<R>([&](auto i) PFB_INLINE {
                    dst.row[S::template pad_at<CR>(j, pj, decltype(i)::value)] = v[decltype(q)::value * R + decltype(i)::value];
                });
            } else {
                sfor<R>([&](auto i) PFB_INLINE {
                    dst(j + decltype(i)::value * CR, v[decltype(q)::value * R + decltype(i)::value]);
                });
            }
        });
    } else {
        sfor<NB>([&](auto q) PFB_INLINE {
            const int j = lane + G * decltype(q)::value;
            const int k = j & (L - 1);
            const int o = (j - k) * R + k;
            const int po = S::pad(o);
            sfor<R>([&](auto i) PFB_INLINE {
                lds[S::template pad_at<L>(o, po, decltype(i)::value)] = v[decltype(q)::value * R + decltype(i)::value];
            });
        });
        group_sync<G>();
    }
}

template <int LOG2C, int G, bool INV, bool SRC_IN_LDS, bool TW_LDS, int P, class Dst>
__device__ __forceinline__ void fft_pass(int lane, float2 *lds, const float2 *twp,
                                         float2 (&v)[FftShape<LOG2C, G>::E], Dst &&dst)
{
    using S = FftShape<LOG2C, G>;
    if constexpr (P > 0)
        fft_pass_gather<LOG2C, G, P>(lane, lds, v);
    if constexpr (G > 64 && P < S::NPASS - 1 && (P > 0 || SRC_IN_LDS))
        group_sync<G>(); // every lane has read before any lane overwrites
    fft_pass_compute<LOG2C, G, INV, TW_LDS, P>(lane, lds, twp, v, dst);
}

// The passes of one transform whose first-pass inputs are already in v (see
// fft_gather_first); `dst(idx, v)` receives output element idx from the last
// pass (an LdsRowDst: stored at row[pad(idx)]). When SRC_IN_LDS the inputs
// were read from this group's own LDS row, so a multi-wave group
// synchronises before overwriting it.
//
// TW_LDS: `tw` points to an LDS copy of the table laid out [pass][i][k]
// (stage_twiddles_lds), so that the lanes of a butterfly column read
// consecutive entries; LDS reads are counted apart from the caller's global
// loads and stores, whereas a wait for a global twiddle load also waits for
// every load and store issued before it.
// TW_AHEAD (global table, transforms over several waves): request each
// pass's twiddles one pass early (2E more registers live), so that their
// latency is not exposed after every workgroup barrier; a caller short of
// registers turns it off. A one-wave transform has no barrier to expose it
// and keeps its registers.
template <int LOG2C, int G, bool INV, bool SRC_IN_LDS, bool TW_LDS = false, bool TW_AHEAD = true, class Dst>
__device__ __forceinline__ void fft_passes(int lane, float2 *lds, const float2 *__restrict__ tw,
                                           float2 (&v)[FftShape<LOG2C, G>::E], Dst &&dst)
{
    using S = FftShape<LOG2C, G>;
    const float2 *twp = fft_twiddle_base<TW_LDS>(tw);
    if constexpr (TW_LDS || !TW_AHEAD || G <= 64 || S::NPASS < 2) {
        sfor<S::NPASS>([&](auto pp) PFB_INLINE {
            fft_pass<LOG2C, G, INV, SRC_IN_LDS, TW_LDS, decltype(pp)::value>(lane, lds, twp, v, dst);
        });
    } else {
        // Global table: the twiddles of pass P+1 are requested as pass P
        // starts (those of pass 1 before the first pass), in two register
        // sets used alternately.
        float4 tw_odd[S::E / 2], tw_even[S::E / 2];
        fft_load_twiddles<LOG2C, G, 1>(lane, twp, tw_odd);
        sfor<S::NPASS>([&](auto pp) PFB_INLINE {
            constexpr int P = decltype(pp)::value;
            if constexpr (P > 0)
                fft_pass_gather<LOG2C, G, P>(lane, lds, v);
            if constexpr (P > 0 && P + 1 < S::NPASS)
                fft_load_twiddles<LOG2C, G, P + 1>(lane, twp, (P + 1) % 2 ? tw_odd : tw_even);
            if constexpr (G > 64 && P < S::NPASS - 1 && (P > 0 || SRC_IN_LDS))
                group_sync<G>(); // every lane has read before any lane overwrites
            fft_pass_compute<LOG2C, G, INV, false, P, Dst &, true>(lane, lds, twp, v, dst,
                                                                   P % 2 ? tw_odd : tw_even);
        });
    }
}

// The twiddles of every pass P > 0 that this lane applies (those
// fft_load_twiddles reads), for callers that keep them in registers across
// many transforms: they depend on the lane index only (k = j mod L for the
// lane's butterflies j), never on the row.
template <int LOG2C, int G> struct FftResidentTwiddles {
    using S = FftShape<LOG2C, G>;
    static_assert(S::NPASS >= 2, "a one-pass transform has no twiddles");
    float4 w[S::NPASS - 1][S::E / 2];
    __device__ __forceinline__ void load(int lane, const float2 *tw)
    {
        const float2 *twp = as_global(tw);
        sfor<S::NPASS - 1>([&](auto pp) PFB_INLINE {
            fft_load_twiddles<LOG2C, G, decltype(pp)::value + 1>(lane, twp, w[decltype(pp)::value]);
        });
    }
};

// fft_passes with the twiddles already in registers (same arithmetic, in
// the same order: same bits). SYNC_FIRST: lanes of the group may still be
// reading the LDS row (the previous transform's last pass), so synchronise
// before the first pass overwrites it.
template <int LOG2C, int G, bool INV, bool SYNC_FIRST, class Dst>
__device__ __forceinline__ void fft_passes_resident(int lane, float2 *lds, const FftResidentTwiddles<LOG2C, G> &tw,
                                                    float2 (&v)[FftShape<LOG2C, G>::E], Dst &&dst)
{
    constexpr int NP = FftShape<LOG2C, G>::NPASS;
    sfor<NP>([&](auto pp) PFB_INLINE {
        constexpr int P = decltype(pp)::value;
        if constexpr (P > 0)
            fft_pass_gather<LOG2C, G, P>(lane, lds, v);
        // every lane has read before any lane overwrites
        if constexpr (G > 64 && P < NP - 1 && (P > 0 || SYNC_FIRST))
            group_sync<G>();
        fft_pass_compute<LOG2C, G, INV, false, P, Dst &, true>(lane, lds, nullptr, v, dst, tw.w[P > 0 ? P - 1 : 0]);
    });
}

// Run one transform. `src(idx)` returns input element idx (first pass);
// `dst(idx, v)` receives output element idx (last pass). When SRC_IN_LDS the
// first pass reads this group's own LDS row. INV selects exp(+...).
template <int LOG2C, int G, bool INV, bool SRC_IN_LDS, bool TW_LDS = false, class Src, class Dst>
__device__ __forceinline__ void fft_run(int lane, float2 *lds, const float2 *__restrict__ tw, Src &&src,
                                        Dst &&dst)
{
    float2 v[FftShape<LOG2C, G>::E];
    fft_gather_first<LOG2C, G>(lane, src, v);
    fft_passes<LOG2C, G, INV, SRC_IN_LDS, TW_LDS>(lane, lds, tw, v, dst);
}

// Entries of a C = 2^LOG2C point transform's twiddle table (at least 1, for
// array sizes).
template <int LOG2C> constexpr int fft_tw_entries()
{
    return FftSchedule(LOG2C).table_size() > 0 ? FftSchedule(LOG2C).table_size() : 1;
}

// Copy the twiddle table (global layout [pass][k][i]) into LDS as
// [pass][i][k], thread t of nt; a workgroup barrier must follow before the
// first transform reads it.
template <int LOG2C> __device__ __forceinline__ void stage_twiddles_lds(float2 *dst, const float2 *tw, int t, int nt)
{
    constexpr FftSchedule SC{LOG2C};
    sfor<SC.npass>([&](auto pp) PFB_INLINE {
        constexpr int P = decltype(pp)::value;
        if constexpr (P > 0) {
            constexpr int R = SC.radix(P), L = SC.stride(P), PO = SC.pass_offset(P);
            for (int e = t; e < R * L; e += nt)
                dst[PO + (e % R) * L + e / R] = tw[PO + e];
        }
    });
}

// Lanes per transform: C <= 1024 lives in one wave (or part of one); larger C
// spans several waves: 128 lanes of 16 elements at C = 2048, C/32 lanes of 32
// elements (radix-32 passes) from C = 4096.
template <int LOG2C> struct FftLanes {
    static constexpr int C = 1 << LOG2C;
    static constexpr int E = fft_elems_per_lane(LOG2C);
    static constexpr int G = C / E;
};

} // namespace pfb
