// Stand-alone batched C-point FFT (the DFT step of Sec. 2, Eq. (2)) for the
// split path: reads complex float32 rows, writes their transforms. One group
// of G lanes per row (several rows per block when G < 256); the Stockham
// passes exchange data through the group's padded LDS row.
#include <atomic>

#include "fft_device.h"
#include "launch.h"

namespace pfb {

template <int LOG2C> struct FftKernelShape {
    using FL = FftLanes<LOG2C>;
    static constexpr int G = FL::G;
    static constexpr int NT = G > 64 ? G : 256; // threads per block (one row when G > 64)
    static constexpr int F = NT / G;             // rows per block
    // waves per SIMD the register allocation must allow (launch-bounds
    // minimum): 4 lets two 512-thread blocks (C = 8192) share a CU, which
    // at the unconstrained 169 VGPRs would run alone
    static constexpr int MIN_WAVES = NT >= 512 ? 4 : 1;
};

template <int LOG2C, bool INV>
__global__ __launch_bounds__(FftKernelShape<LOG2C>::NT, FftKernelShape<LOG2C>::MIN_WAVES) void fft_kernel(FftArgs a)
{
    using K = FftKernelShape<LOG2C>;
    constexpr int G = K::G;
    constexpr int C = 1 << LOG2C;
    using S = FftShape<LOG2C, G>;
    __shared__ float2 lds[K::F * S::PADDED];

    const int gid = (int)threadIdx.x / G;
    const int lane = (int)threadIdx.x % G;
    const int64_t row = (int64_t)blockIdx.x * K::F + gid;
    // With G > 64 there is one row per block, so this exit is block-uniform;
    // with G <= 64 the passes use no block-wide barrier.
    if (row >= a.nrows)
        return;
    const int64_t g = row / a.rows_per_group, r = row % a.rows_per_group;
    const float2 *in = a.in + g * a.in_gstride + r * C;
    float2 *out = a.out + g * a.out_gstride + r * C;
    fft_run<LOG2C, G, INV, false>(
        lane, lds + gid * S::PADDED, a.tw, [&](int idx) { return in[idx]; },
        [&](int idx, float2 v) { store_nt(out + idx, v); });
}

// Transforms of C >= 4096 points: persistent workgroups of one transform
// group each (rows blockIdx.x, blockIdx.x + gridDim.x, ...). The twiddles a
// lane applies depend on its lane index only, so each lane loads those of
// every pass once and keeps them in registers for all its rows; one
// workgroup per row re-read them from L2 for every row (twice the row's own
// bytes). Same arithmetic, in the same order, as fft_kernel: the bits agree.
// Measured (split path, T=16, 2^27 samples): 4096 channels 0.874 -> 0.825 ms,
// 8192 channels 0.904 -> 0.795 ms. Not used at 2048 channels (no gain: that
// transform already keeps eight rows per CU in flight) nor for the sub-band
// pairs (1.22 against 0.92 ms for fft_pol2_kernel); also requesting part of
// the next row's inputs before each transform gained nothing at 4096
// channels and lost at 8192 (registers).
template <int LOG2C> struct FftPersistShape {
    using FL = FftLanes<LOG2C>;
    static constexpr int G = FL::G;
    static constexpr int NT = G;
    // LDS holds at most four 4096-point (two 8192-point) rows per CU, i.e.
    // two waves per SIMD with 256 registers each
    static constexpr int MIN_WAVES = 2;
};

template <int LOG2C, bool INV>
__global__ __launch_bounds__(FftPersistShape<LOG2C>::NT, FftPersistShape<LOG2C>::MIN_WAVES) void fft_persist_kernel(
    FftArgs a)
{
    constexpr int G = FftPersistShape<LOG2C>::G;
    constexpr int C = 1 << LOG2C;
    using S = FftShape<LOG2C, G>;
    static_assert(G > 64, "multi-wave transforms");
    __shared__ float2 lds[S::PADDED];
    const int lane = (int)threadIdx.x;
    FftResidentTwiddles<LOG2C, G> tw;
    tw.load(lane, a.tw);
    // rows are block-uniform, so every lane reaches the same barriers
    for (int64_t row = blockIdx.x; row < a.nrows; row += gridDim.x) {
        const int64_t g = row / a.rows_per_group, r = row % a.rows_per_group;
        const float2 *in = a.in + g * a.in_gstride + r * C;
        float2 *out = a.out + g * a.out_gstride + r * C;
        float2 v[S::E];
        fft_gather_first<LOG2C, G>(lane, [&](int idx) { return in[idx]; }, v);
        fft_passes_resident<LOG2C, G, INV, true>(lane, lds, tw, v,
                                                 [&](int idx, float2 t) { store_nt(out + idx, t); });
    }
}

// Workgroups of fft_persist_kernel resident per CU (LDS- and
// register-limited), asked once; 0 if the runtime cannot tell.
template <int LOG2C, bool INV> static int persist_blocks_per_cu()
{
    static std::atomic<int> per_cu{-1};
    int n = per_cu.load(std::memory_order_relaxed);
    if (n < 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fft_persist_kernel<LOG2C, INV>,
                                                         FftPersistShape<LOG2C>::NT, 0) != hipSuccess ||
            n < 0)
            n = 0;
        per_cu.store(n, std::memory_order_relaxed);
    }
    return n;
}

// Transforms of polarisation-interleaved sub-bands (the VEGAS-style layout:
// per spectrum, nsub sub-bands of C channels, each channel holding 2
// interleaved polarisations). Row r = (s * nsub + sub) * 2 + pol transforms
// the C elements at base + 2*idx, base = (s * nsub + sub) * 2C + pol, and
// writes its bins to the same positions of out. A workgroup takes both
// polarisations of a sub-band spectrum, so the two transforms that share
// every 16-byte pair of the row read and write it from one CU (one
// polarisation per workgroup left each line to two CUs, often on two XCDs:
// 4096 channels, 8 sub-bands, int8, 16 taps 1.23 -> 0.92 ms).
template <int LOG2C> struct FftPol2Shape {
    using FL = FftLanes<LOG2C>;
    static constexpr int G = FL::G;
    static constexpr int NT = G > 64 ? 2 * G : 256; // threads per block
    static constexpr int F = NT / G;                // rows per block: both polarisations together
    static constexpr int MIN_WAVES = NT >= 512 ? 2 : 1;
};

template <int LOG2C, bool INV>
__global__ __launch_bounds__(FftPol2Shape<LOG2C>::NT, FftPol2Shape<LOG2C>::MIN_WAVES) void fft_pol2_kernel(
    FftArgs a)
{
    using K = FftPol2Shape<LOG2C>;
    constexpr int G = K::G;
    constexpr int C = 1 << LOG2C;
    using S = FftShape<LOG2C, G>;
    __shared__ float2 lds[K::F * S::PADDED];
    const int gid = (int)threadIdx.x / G;
    const int lane = (int)threadIdx.x % G;
    const int64_t row = (int64_t)blockIdx.x * K::F + gid;
    // rows come in polarisation pairs and a block holds whole pairs, so with
    // G > 64 (block barriers) both groups of a block are in range
    if (row >= a.nrows)
        return;
    const int64_t base = (row >> 1) * 2 * C + (row & 1);
    const float2 *in = a.in + base;
    float2 *out = a.out + base;
    fft_run<LOG2C, G, INV, false>(
        lane, lds + gid * S::PADDED, a.tw, [&](int idx) { return in[2 * idx]; },
        [&](int idx, float2 v) { store_nt(out + 2 * idx, v); });
}

hipError_t launch_fft_pol2(const FftArgs &a, int log2c, hipStream_t st)
{
    switch (log2c) {
#define PFB_POL2_C(L2)                                                                                       \
    case L2: {                                                                                               \
        using K = FftPol2Shape<L2>;                                                                          \
        const int64_t blocks = (a.nrows + K::F - 1) / K::F;                                                  \
        if (blocks <= 0)                                                                                     \
            return hipSuccess;                                                                               \
        hipLaunchKernelGGL((fft_pol2_kernel<L2, false>), dim3((unsigned)blocks), dim3(K::NT), 0, st, a);     \
        return hipGetLastError();                                                                            \
    }
        PFB_POL2_C(5)
        PFB_POL2_C(6)
        PFB_POL2_C(7)
        PFB_POL2_C(8)
        PFB_POL2_C(9)
        PFB_POL2_C(10)
        PFB_POL2_C(11)
        PFB_POL2_C(12)
        PFB_POL2_C(13)
#undef PFB_POL2_C
    default:
        return hipErrorInvalidValue;
    }
}

template <int LOG2C, bool INV> static hipError_t launch_fft_dir(const FftArgs &a, hipStream_t st)
{
    if constexpr (LOG2C >= 12) {
        // persistent workgroups where each gets at least two rows (it loads
        // its twiddles once)
        const int64_t grid = (int64_t)persist_blocks_per_cu<LOG2C, INV>() * a.num_cus;
        if (grid > 0 && a.nrows >= 2 * grid) {
            hipLaunchKernelGGL((fft_persist_kernel<LOG2C, INV>), dim3((unsigned)grid),
                               dim3(FftPersistShape<LOG2C>::NT), 0, st, a);
            return hipGetLastError();
        }
    }
    using K = FftKernelShape<LOG2C>;
    const int64_t blocks = (a.nrows + K::F - 1) / K::F;
    if (blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((fft_kernel<LOG2C, INV>), dim3((unsigned)blocks), dim3(K::NT), 0, st, a);
    return hipGetLastError();
}

template <int LOG2C> static hipError_t launch_fft_t(const FftArgs &a, bool inv, hipStream_t st)
{
    return inv ? launch_fft_dir<LOG2C, true>(a, st) : launch_fft_dir<LOG2C, false>(a, st);
}

hipError_t launch_fft(const FftArgs &a, int log2c, bool inv, hipStream_t st)
{
    switch (log2c) {
    case 5: return launch_fft_t<5>(a, inv, st);
    case 6: return launch_fft_t<6>(a, inv, st);
    case 7: return launch_fft_t<7>(a, inv, st);
    case 8: return launch_fft_t<8>(a, inv, st);
    case 9: return launch_fft_t<9>(a, inv, st);
    case 10: return launch_fft_t<10>(a, inv, st);
    case 11: return launch_fft_t<11>(a, inv, st);
    case 12: return launch_fft_t<12>(a, inv, st);
    case 13: return launch_fft_t<13>(a, inv, st);
    default: return hipErrorInvalidValue;
    }
}

} // namespace pfb
