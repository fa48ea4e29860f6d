// Adjoint of the filter bank without a plan and without any allocation
// (pfb_backward_noalloc in include/pfb.h), for callers that cannot allocate
// device memory.
//
// It runs the same fused adjoint kernel and the same fixed-order tap-gradient
// reduction as pfb_backward. The two buffers a plan would own live in one
// file-scope device array instead: the transform's twiddle table (written by
// a small kernel on every call) and the per-tile tap-gradient partials (every
// tile overwrites its own partial, so nothing needs clearing). Each GPU holds
// its own copy of the array, at its own address, until the process ends; the
// host looks that address up once per device and never uses the array's name
// in host code. All calls on one GPU share its array, so calls that overlap
// on one GPU (two streams, two threads) race; calls ordered on one stream do
// not.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/pfb.h"
#include "fft_schedule.h"
#include "launch.h"
#include "tune.h"

// The scratch array (one copy per GPU). Host code never names it except to
// look its address up.
static __device__ __align__(256) unsigned char scratch[PFB_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int64_t SCRATCH_BYTES = (int64_t)PFB_NOALLOC_SCRATCH_BYTES;
constexpr int64_t TW_BYTES = 16384;   // twiddle region: the 1024-point table is 10 KiB
constexpr int MAX_DEVICES = 64;
constexpr int MAX_PASSES = 8;

std::mutex g_mutex;
void *g_scratch[MAX_DEVICES];          // the array's address on each device

struct TwPasses {
    int n;                             // passes with twiddles (pass 1 ..)
    int radix[MAX_PASSES], stride[MAX_PASSES], offset[MAX_PASSES];
    int entries;
};

// The twiddle table of the Stockham schedule: for every pass after the
// first (radix R, stride L, offset PO), entry PO + k*R + i holds
// exp(-2 pi i (i k mod R L) / (R L)), computed in FP64 and rounded once.
__global__ void noalloc_twiddles(float2 *tw, TwPasses ps)
{
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= ps.entries)
        return;
    int p = 0;
    while (p + 1 < ps.n && e >= ps.offset[p + 1])
        ++p;
    const int R = ps.radix[p], L = ps.stride[p];
    const int local = e - ps.offset[p];
    const int k = local / R, i = local % R;
    const int64_t RL = (int64_t)R * L;
    const int64_t red = ((int64_t)i * k) % RL; // exact integer reduction
    const double a = -2.0 * M_PI * (double)red / (double)RL;
    tw[e] = make_float2((float)cos(a), (float)sin(a));
}

pfb_status scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "hipGetDevice failed");
    if (dev < 0 || dev >= MAX_DEVICES)
        return pfb_internal_fail(PFB_E_UNSUPPORTED, "device index beyond the allocation-free table");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return pfb_internal_fail(PFB_E_HIP, (std::string("hipGetSymbolAddress(scratch): ") +
                                                 hipGetErrorString(e)).c_str());
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return PFB_OK;
}

int ilog2_pow2(int v)
{
    if (v <= 0 || (v & (v - 1)))
        return -1;
    int l = 0;
    while ((1 << l) < v)
        ++l;
    return l;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

} // namespace

extern "C" pfb_status pfb_backward_noalloc(const pfb_desc *d, const void *x, const float *taps, const void *gY,
                                           void *gx, float *gh, void *stream)
{
    using namespace pfb;
    pfb_status st = pfb_internal_validate(d, false);
    if (st != PFB_OK)
        return st;
    if (d->dtype != PFB_C64)
        return pfb_internal_fail(PFB_E_UNSUPPORTED, "pfb_backward_noalloc needs complex float32 input");
    if (d->flags != 0)
        return pfb_internal_fail(PFB_E_INVALID, "pfb_backward_noalloc takes no flags");
    const int log2c = ilog2_pow2(d->channels);
    int tp = 4;
    while (tp < d->taps)
        tp *= 2;
    if (log2c < 0 || !fused_bwd_supported(tp, log2c))
        return pfb_internal_fail(PFB_E_UNSUPPORTED,
                                 "pfb_backward_noalloc supports C in {256, 512, 1024} and T <= 16");
    if (!gY || !taps || (gh && !x))
        return pfb_internal_fail(PFB_E_INVALID, "gY and taps (and x for gh) must be non-NULL");
    if (!aligned16(gY) || !aligned16(taps) || (x && !aligned16(x)) || (gx && !aligned16(gx)) ||
        (gh && !aligned16(gh)))
        return pfb_internal_fail(PFB_E_INVALID, "device pointers must be 16-byte aligned");
    if (!gx && !gh)
        return PFB_OK;

    // tile rows as a plan would choose them, lengthened until the partials fit
    const int64_t B = d->batch, S = d->spectra, T = d->taps, C = d->channels;
    const int64_t rows = S + T - 1;
    const int64_t part_bytes = T * C * 4;
    int cus = 256;
    {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
    }
    int64_t sb = pfb_internal_bwd_tile_rows(B, S, (int)T, (int)C, cus);
    const int64_t rows16 = (rows + 15) / 16 * 16;
    auto parts_for = [&](int64_t r) { return B * ((rows + r - 1) / r); };
    while (parts_for(sb) * part_bytes > SCRATCH_BYTES - TW_BYTES && sb < rows16)
        sb = std::min<int64_t>(sb * 2, rows16);
    if (parts_for(sb) * part_bytes > SCRATCH_BYTES - TW_BYTES)
        return pfb_internal_fail(PFB_E_UNSUPPORTED,
                                 (std::string("pfb_backward_noalloc: the tap-gradient partials of ") +
                                  std::to_string(B) + " streams exceed its " +
                                  std::to_string(SCRATCH_BYTES >> 20) +
                                  " MiB scratch (batch * taps * channels * 4 bytes must fit)")
                                     .c_str());
    if (sb > (int64_t)0x7fffffff / (C * 8))
        return pfb_internal_fail(PFB_E_UNSUPPORTED, "pfb_backward_noalloc: tile beyond a 2 GiB row view");

    void *base = nullptr;
    st = scratch_address(&base);
    if (st != PFB_OK)
        return st;
    float2 *tw = reinterpret_cast<float2 *>(base);
    float *part = reinterpret_cast<float *>(static_cast<unsigned char *>(base) + TW_BYTES);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    const FftSchedule sch(log2c);
    if (sch.npass - 1 > MAX_PASSES || (int64_t)sch.table_size() * 8 > TW_BYTES)
        return pfb_internal_fail(PFB_E_UNSUPPORTED, "pfb_backward_noalloc: twiddle table too large");
    TwPasses ps{};
    ps.n = sch.npass - 1;
    for (int p = 1; p < sch.npass; ++p) {
        ps.radix[p - 1] = sch.radix(p);
        ps.stride[p - 1] = sch.stride(p);
        ps.offset[p - 1] = sch.pass_offset(p);
    }
    ps.entries = sch.table_size();
    if (ps.entries > 0) {
        hipLaunchKernelGGL(noalloc_twiddles, dim3((unsigned)((ps.entries + 255) / 256)), dim3(256), 0, s, tw, ps);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return pfb_internal_fail(PFB_E_HIP, (std::string("twiddle launch: ") + hipGetErrorString(e)).c_str());
    }

    BwdArgs a{};
    a.x = reinterpret_cast<const float2 *>(x);
    a.h = taps;
    a.gY = reinterpret_cast<const float2 *>(gY);
    a.gx = reinterpret_cast<float2 *>(gx);
    a.part = gh ? part : nullptr;
    a.tw = tw;
    a.T = (int)T;
    a.B = (int)B;
    a.SB = (int)sb;
    a.n_tiles = (int)((rows + sb - 1) / sb);
    a.S = S;
    hipError_t e = launch_fused_bwd(a, tp, log2c, s);
    if (e == hipSuccess && gh)
        e = launch_gh_reduce(part, gh, B * a.n_tiles, T * C, s);
    if (e != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, (std::string("allocation-free adjoint launch: ") +
                                             hipGetErrorString(e)).c_str());
    return PFB_OK;
}
