// Radix schedule of the C-point Stockham transforms (shared by the kernels
// and the host code that builds their twiddle tables).
#pragma once

namespace pfb {

// Elements per lane for a C = 2^log2c point transform: 16 where the pass
// radices come out even, 8 otherwise, and 32 from C = 4096, where radix-32
// passes need one LDS exchange fewer (C = 8192: 32 x 32 x 8 instead of
// 16 x 16 x 16 x 2) and half as many waves meet at each barrier.
constexpr int fft_elems_per_lane(int log2c)
{
    return (log2c == 5 || log2c == 6 || log2c == 7 || log2c == 9) ? 8 : log2c >= 12 ? 32 : 16;
}

constexpr int fft_ilog2(int v) { return v <= 1 ? 0 : 1 + fft_ilog2(v / 2); }

// Passes: radix E while it divides what is left, then one smaller radix.
struct FftSchedule {
    int log2c, e, log2e, nfull, log2rem, npass;
    constexpr explicit FftSchedule(int l2c)
        : log2c(l2c), e(fft_elems_per_lane(l2c)), log2e(fft_ilog2(fft_elems_per_lane(l2c))),
          nfull(l2c / fft_ilog2(fft_elems_per_lane(l2c))), log2rem(l2c % fft_ilog2(fft_elems_per_lane(l2c))),
          npass(l2c / fft_ilog2(fft_elems_per_lane(l2c)) + (l2c % fft_ilog2(fft_elems_per_lane(l2c)) ? 1 : 0))
    {
    }
    constexpr int radix(int p) const { return p < nfull ? e : (1 << log2rem); }
    constexpr int stride(int p) const { return p == 0 ? 1 : stride(p - 1) * radix(p - 1); }
    // offset of pass p's twiddles in the table (pass 0 has none)
    constexpr int pass_offset(int p) const { return p <= 1 ? 0 : pass_offset(p - 1) + stride(p - 1) * radix(p - 1); }
    constexpr int table_size() const { return pass_offset(npass); }
};

} // namespace pfb
