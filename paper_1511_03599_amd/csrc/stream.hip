// Small layout kernels.
// Block copies for streaming plans: the carried raw spectra (T-1 rows per
// stream) go into the headroom of the caller's buffer before a call and the
// last T-1 rows of the buffer come back into the plan after it. A few KiB to
// MiB per call; explicit kernels (no memset or copy nodes) so that a caller
// may capture the calls in a graph.
// Tap replication for the polarisation-interleaved sub-band layout.
#include "device_common.h"
#include "launch.h"

namespace pfb {

// nblk blocks of `bytes` bytes: block b goes from src + b*src_stride to
// dst + b*dst_stride (src == nullptr writes zeros). VEC: 16-byte units
// (bytes, strides and bases all multiples of 16).
template <bool VEC>
__global__ __launch_bounds__(256) void copy_blocks_kernel(const char *src, int64_t src_stride, char *dst,
                                                          int64_t dst_stride, int64_t bytes, int64_t nblk)
{
    const int64_t units = VEC ? bytes / 16 : bytes;
    const int64_t total = units * nblk;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = g / units, i = g % units;
        char *d = dst + b * dst_stride;
        if constexpr (VEC) {
            const uint4 v = src ? reinterpret_cast<const uint4 *>(src + b * src_stride)[i] : make_uint4(0, 0, 0, 0);
            reinterpret_cast<uint4 *>(d)[i] = v;
        } else {
            d[i] = src ? src[b * src_stride + i] : (char)0;
        }
    }
}

hipError_t launch_copy_blocks(const void *src, int64_t src_stride, void *dst, int64_t dst_stride, int64_t bytes,
                              int64_t nblk, hipStream_t st)
{
    if (bytes <= 0 || nblk <= 0)
        return hipSuccess;
    const bool vec = bytes % 16 == 0 && src_stride % 16 == 0 && dst_stride % 16 == 0 &&
                     ((uintptr_t)src | (uintptr_t)dst) % 16 == 0;
    const int64_t total = (vec ? bytes / 16 : bytes) * nblk;
    const int64_t blocks = (total + 255) / 256 < 2048 ? (total + 255) / 256 : 2048;
    if (vec)
        hipLaunchKernelGGL(copy_blocks_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, st,
                           static_cast<const char *>(src), src_stride, static_cast<char *>(dst), dst_stride, bytes,
                           nblk);
    else
        hipLaunchKernelGGL(copy_blocks_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st,
                           static_cast<const char *>(src), src_stride, static_cast<char *>(dst), dst_stride, bytes,
                           nblk);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void vegas_taps_kernel(const float *in, float *out, int T, int cv, int nsub)
{
    const int64_t cols = (int64_t)2 * cv * nsub;
    const int64_t total = (int64_t)T * cols;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / cols, col = i % cols;
        out[i] = in[t * cv + (col >> 1) % cv];
    }
}

hipError_t launch_vegas_taps(const float *in, float *out, int T, int cv, int nsub, hipStream_t st)
{
    const int64_t total = (int64_t)T * 2 * cv * nsub;
    const int64_t blocks = (total + 255) / 256 < 1024 ? (total + 255) / 256 : 1024;
    if (blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(vegas_taps_kernel, dim3((unsigned)blocks), dim3(256), 0, st, in, out, T, cv, nsub);
    return hipGetLastError();
}

} // namespace pfb
