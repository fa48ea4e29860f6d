// Stand-alone batched C-point FFT (the DFT step of Sec. 2, Eq. (2)) for the
// split path: reads complex float32 rows, writes their transforms. One group
// of G lanes per row (several rows per block when G < 256); the Stockham
// passes exchange data through the group's padded LDS row.
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

template <int LOG2C> static hipError_t launch_fft_t(const FftArgs &a, bool inv, hipStream_t st)
{
    using K = FftKernelShape<LOG2C>;
    const int64_t blocks = (a.nrows + K::F - 1) / K::F;
    if (blocks <= 0)
        return hipSuccess;
    if (inv)
        hipLaunchKernelGGL((fft_kernel<LOG2C, true>), dim3((unsigned)blocks), dim3(K::NT), 0, st, a);
    else
        hipLaunchKernelGGL((fft_kernel<LOG2C, false>), dim3((unsigned)blocks), dim3(K::NT), 0, st, a);
    return hipGetLastError();
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
