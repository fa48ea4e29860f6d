// Internal launch interface between the C ABI (api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfb {

// FIR launch over output rows [out_first, out_first + out_count) of each of B
// streams. Output row s of stream b goes to y + b*y_bstride + (s - out_first)*C.
struct FirArgs {
    const void *x;       // stream 0, row 0
    const float *h;      // taps [T][C]
    float2 *y;
    int C, T, B;
    int SB;              // output rows per tile
    int n_tiles;         // tiles per stream
    int n_cchunks;       // channel chunks of 64*CPT
    int64_t in_rows;     // rows readable per stream; others read as zero
    int64_t in_bstride;  // samples between streams in x
    int64_t shift;       // window slot 0 of output s reads input row s - shift
    int64_t out_first;
    int64_t out_count;
    int64_t y_bstride;   // complex values between streams in y
};

// Tap-gradient partials over tiles of S_B filtered spectra.
struct GhArgs {
    const float2 *x;     // [B][S+T-1][C]
    const float2 *gy;    // [B][S][C]
    float *part;         // [B*n_tiles][T][C]
    int C, T, B;
    int SB, n_tiles, n_cchunks;
    int64_t S;
    int tile0 = 0;       // first tile of this launch
    int ntiles_run = 0;  // tiles of this launch (0: all n_tiles)
};

// Sample gradient and tap-gradient partials of the split adjoint in one pass
// over tiles of S_B raw spectra (rows of gx).
struct GxGhArgs {
    const float2 *x;     // [B][S+T-1][C]
    const float2 *gy;    // [B][S][C]
    const float *h;      // [T][C]
    float2 *gx;          // [B][S+T-1][C]
    float *part;         // [B*n_tiles][T][C]
    int C, T, B;
    int SB, n_tiles, n_cchunks;
    int64_t S;
};

// Batched C-point transforms of `nrows` rows. Row r lives at
// in + (r / rows_per_group)*in_gstride + (r % rows_per_group)*C, and likewise
// for out.
struct FftArgs {
    const float2 *in;
    float2 *out;
    const float2 *tw;    // twiddle table of the C-point schedule (fft_device.h)
    int64_t nrows;
    int64_t rows_per_group;
    int64_t in_gstride;
    int64_t out_gstride;
    int num_cus = 0;     // compute units of the device (sizes persistent grids; 0: one block per row)
};

// Fused FIR + FFT: one workgroup holds all C channels of a tile of S_B
// filtered spectra of one stream.
struct FusedArgs {
    const void *x;       // [B][S+T-1][C]
    const float *h;      // [T][C]
    float2 *Y;           // [B][S][C]
    const float2 *tw;
    int T, B;
    int SB, n_tiles;
    int64_t S;
};

// Fused adjoint: one workgroup per tile of S_B gx rows of one stream.
struct BwdArgs {
    const float2 *x;     // [B][S+T-1][C]
    const float *h;      // [T][C]
    const float2 *gY;    // [B][S][C]
    float2 *gx;          // [B][S+T-1][C] or NULL
    float *part;         // [B*n_tiles][T][C] tap-gradient partials, or NULL
    const float2 *tw;
    int T, B;
    int SB, n_tiles;     // gx rows per tile, tiles per stream
    int64_t S;
};

// per_use: the convert-per-use comparator (low-precision input, tp <= 16)
hipError_t launch_fir(const FirArgs &a, int dtype, int tp, int cpt, bool rev, hipStream_t st, bool per_use = false);
// per input type (each in its own translation unit)
hipError_t launch_fir_ci16(const FirArgs &a, int tp, int cpt, bool per_use, hipStream_t st);
hipError_t launch_fir_ci8(const FirArgs &a, int tp, int cpt, bool per_use, hipStream_t st);
hipError_t launch_fir_cf16(const FirArgs &a, int tp, int cpt, bool per_use, hipStream_t st);
hipError_t launch_fir_adjoint(const FirArgs &a, int tp, int cpt, hipStream_t st); // reversed taps, c64
// FIR for T beyond the register window: tiles of 32 rows (SB = 32), one
// channel per lane (64 per wave task), no tap padding (shift = 0).
hipError_t launch_fir_long(const FirArgs &a, int dtype, hipStream_t st);
hipError_t launch_gh(const GhArgs &a, int tp, float *gh, hipStream_t st);
// padded taps tp <= 32; also runs the reduction into gh
hipError_t launch_gxgh(const GxGhArgs &a, int tp, float *gh, hipStream_t st);
hipError_t launch_fft(const FftArgs &a, int log2c, bool inv, hipStream_t st);
// Forward transforms of polarisation-interleaved sub-bands: a.nrows =
// spectra * nsub * 2 rows, row r at a.in + (r/2)*2C + (r%2), element stride 2
// (a.rows_per_group and the group strides are not used).
hipError_t launch_fft_pol2(const FftArgs &a, int log2c, hipStream_t st);
// Replicate C_V-channel taps over polarisation-interleaved sub-bands:
// out[t][(sub*cv + c)*2 + pol] = in[t][c].
hipError_t launch_vegas_taps(const float *in, float *out, int T, int cv, int nsub, hipStream_t st);

// Mixed-radix transform for C = 2^a 3^b 5^c 7^d (not a power of two).
constexpr int GF_MAX_PASS = 16;
struct GfftSched {
    int C;
    int npass;
    int group;           // lanes per row: 64, 256 or 512
    int rows_per_block;
    int radix[GF_MAX_PASS];
};
bool gfft_schedule(int C, GfftSched *s);
hipError_t launch_gfft(const FftArgs &a, const GfftSched &s, bool inv, hipStream_t st);
hipError_t launch_fused(const FusedArgs &a, int dtype, int tp, int log2c, hipStream_t st);
// per input type (each in its own translation unit)
hipError_t launch_fused_ci16(const FusedArgs &a, int tp, int log2c, hipStream_t st);
hipError_t launch_fused_ci8(const FusedArgs &a, int tp, int log2c, hipStream_t st);
hipError_t launch_fused_cf16(const FusedArgs &a, int tp, int log2c, hipStream_t st);
hipError_t launch_fused_ws(const FusedArgs &a, int dtype, int tp, int log2c, hipStream_t st);
// nblk blocks of `bytes` bytes from src + b*src_stride to dst + b*dst_stride
// (src NULL: zeros).
hipError_t launch_copy_blocks(const void *src, int64_t src_stride, void *dst, int64_t dst_stride, int64_t bytes,
                              int64_t nblk, hipStream_t st);
bool fused_supported(int dtype, int tp, int log2c);
hipError_t launch_fused_bwd(const BwdArgs &a, int tp, int log2c, hipStream_t st);
hipError_t launch_fused_bwd_ws(const BwdArgs &a, int tp, int log2c, hipStream_t st);
bool fused_bwd_supported(int tp, int log2c);
hipError_t launch_gh_reduce(const float *part, float *gh, int64_t n_parts, int64_t tc, hipStream_t st);
int fused_rows_per_chunk(int tp, int log2c);

} // namespace pfb
