// C ABI of the polyphase filter bank library (declared in include/pfb.h).
//
// Host side only: descriptor validation, plan construction (FP64-derived
// twiddle tables, tile shapes, workspaces), and the launch sequence of each
// call. Every step of the computation runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pfb.h"
#include "fft_schedule.h"
#include "launch.h"
#include "tune.h"

using namespace pfb;

namespace {

thread_local std::string g_last_error;

pfb_status fail(pfb_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

pfb_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return PFB_E_HIP;
}

int bytes_per_sample(int dt)
{
    switch (dt) {
    case PFB_C64: return 8;
    case PFB_CI16: return 4;
    case PFB_CI8: return 2;
    case PFB_CF16: return 4;
    default: return 0;
    }
}

int ilog2_exact(int64_t v)
{
    if (v <= 0 || (v & (v - 1)))
        return -1;
    int l = 0;
    while ((int64_t(1) << l) < v)
        ++l;
    return l;
}

int padded_taps(int T)
{
    int tp = 4;
    while (tp < T)
        tp *= 2;
    return tp;
}

bool mul_ok(int64_t a, int64_t b, int64_t *out)
{
    if (a < 0 || b < 0)
        return false;
    if (a != 0 && b > INT64_MAX / a)
        return false;
    *out = a * b;
    return true;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

} // namespace

enum PlanKind { KIND_SINGLE = 1, KIND_BATCHED = 2 };
enum Path { PATH_FUSED = 0, PATH_SPLIT = 1, PATH_FIR_ONLY = 2 };

struct pfb_plan {
    int kind = KIND_SINGLE;
    pfb_desc d{};
    int device = 0;
    int log2c = -1;
    int tp = 4;
    Path path = PATH_SPLIT;
    // FIR tiling (split path and backward)
    int fir_sb = 256;
    int fir_cpt = 1;
    // fused tiling
    int fused_sb = 0;
    bool fused_ws = false;       // wave-specialised fused kernel
    // split path chunking
    int64_t chunk_rows = 0;
    float2 *twiddle = nullptr;   // FFT twiddle table for C
    bool mixed = false;          // C not a power of two: mixed-radix transform
    bool long_fir = false;       // T beyond the register window
    GfftSched gf{};
    float2 *ws_y = nullptr;      // filtered spectra workspace (split path)
    int64_t ws_y_bytes = 0;
    float2 *ws_gy = nullptr;     // backward: inverse-transformed gradient
    int64_t ws_gy_bytes = 0;
    float *ws_gh = nullptr;      // backward: tap-gradient partials
    int64_t ws_gh_bytes = 0;
    int gh_sb = 256;
    bool bwd_fused = false;      // fused adjoint kernel
    bool bwd_ws = false;         // ... its wave-specialised form
    int bwd_sb = 256;            // gx rows per fused adjoint tile
    int num_cus = 256;           // compute units of the plan's device
    // polarisation-interleaved sub-band layout: per spectrum vegas_nsub
    // sub-bands of vegas_cv channels x 2 polarisations; d describes the FIR
    // over all 2*cv*nsub columns (FIR_ONLY), h_rep holds the replicated taps
    int vegas_cv = 0, vegas_nsub = 0, vegas_log2cv = -1;
    float *h_rep = nullptr;
    // streaming: the last T-1 raw spectra of each stream, [B][T-1][C]
    char *hist = nullptr;
    int64_t hist_bytes = 0;
    // batched
    struct Batched *batched = nullptr;
};

// ----------------------------------------------------------------------------
// Twiddles
// ----------------------------------------------------------------------------

// exp(-2 pi i m / C) for m < C (mixed-radix transforms), FP64 rounded once.
static pfb_status make_twiddles_mixed(int C, float2 **out)
{
    std::vector<float2> host((size_t)C);
    for (int m = 0; m < C; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)C;
        host[(size_t)m] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(float2) * (size_t)C);
    if (e != hipSuccess)
        return fail(PFB_E_NOMEM, std::string("hipMalloc(twiddles): ") + hipGetErrorString(e));
    e = hipMemcpy(p, host.data(), sizeof(float2) * (size_t)C, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p);
        return hip_fail(e, "hipMemcpy(twiddles)");
    }
    *out = reinterpret_cast<float2 *>(p);
    return PFB_OK;
}

static pfb_status make_twiddles(int log2c, float2 **out)
{
    const FftSchedule sch(log2c);
    const int n = sch.table_size() > 0 ? sch.table_size() : 1;
    std::vector<float2> host((size_t)n, make_float2(1.0f, 0.0f));
    for (int p = 1; p < sch.npass; ++p) {
        const int R = sch.radix(p), L = sch.stride(p), RL = R * L;
        for (int k = 0; k < L; ++k)
            for (int i = 0; i < R; ++i) {
                const int64_t e = ((int64_t)i * k) % RL; // exact integer reduction
                const double a = -2.0 * M_PI * (double)e / (double)RL;
                host[(size_t)sch.pass_offset(p) + (size_t)k * R + i] = make_float2((float)std::cos(a), (float)std::sin(a));
            }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(float2) * (size_t)n);
    if (e != hipSuccess)
        return fail(PFB_E_NOMEM, std::string("hipMalloc(twiddles): ") + hipGetErrorString(e));
    e = hipMemcpy(p, host.data(), sizeof(float2) * (size_t)n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p);
        return hip_fail(e, "hipMemcpy(twiddles)");
    }
    *out = reinterpret_cast<float2 *>(p);
    return PFB_OK;
}

// ----------------------------------------------------------------------------
// Validation
// ----------------------------------------------------------------------------

static pfb_status validate_desc(const pfb_desc *d, bool batched_beam)
{
    if (!d)
        return fail(PFB_E_INVALID, "descriptor is NULL");
    if (d->channels < 1)
        return fail(PFB_E_INVALID, "channels must be >= 1");
    if (d->taps < 1)
        return fail(PFB_E_INVALID, "taps must be >= 1");
    if (d->taps > PFB_MAX_TAPS)
        return fail(PFB_E_UNSUPPORTED, "taps above PFB_MAX_TAPS");
    if (d->spectra < 1)
        return fail(PFB_E_INVALID, "spectra must be >= 1");
    if (d->batch < 1)
        return fail(PFB_E_INVALID, "batch must be >= 1");
    if (bytes_per_sample(d->dtype) == 0)
        return fail(PFB_E_INVALID, "unknown dtype");
    const uint32_t known = PFB_FIR_ONLY | PFB_NO_FUSE | PFB_PLAIN | PFB_STREAMING | PFB_CONVERT_PER_USE;
    if (!batched_beam && (d->flags & ~known))
        return fail(PFB_E_INVALID, "unknown flag bits");
    if (!batched_beam && (d->flags & PFB_CONVERT_PER_USE) && (d->dtype == PFB_C64 || d->taps > 16))
        return fail(PFB_E_UNSUPPORTED, "PFB_CONVERT_PER_USE needs int16, int8 or float16 input and T <= 16");
    const bool fir_only = !batched_beam && (d->flags & PFB_FIR_ONLY);
    if (!fir_only) {
        const int l2 = ilog2_exact(d->channels);
        GfftSched gs;
        if (d->channels < PFB_MIN_FFT_CHANNELS || d->channels > PFB_MAX_FFT_CHANNELS)
            return fail(PFB_E_UNSUPPORTED, "the FFT needs channels in [32, 8192]");
        if (batched_beam && l2 < 0)
            return fail(PFB_E_UNSUPPORTED, "batched beams need channels a power of two");
        if (l2 < 0 && !gfft_schedule(d->channels, &gs))
            return fail(PFB_E_UNSUPPORTED, "the FFT needs channels of the form 2^a 3^b 5^c 7^d");
    }
    // every element count must fit comfortably in int64
    int64_t rows = d->spectra + d->taps - 1, t = 0, u = 0;
    if (!mul_ok(rows, d->channels, &t) || !mul_ok(t, d->batch, &u) || !mul_ok(u, 16, &t))
        return fail(PFB_E_INVALID, "problem size overflows 64-bit byte counts");
    return PFB_OK;
}

// ----------------------------------------------------------------------------
// Plans
// ----------------------------------------------------------------------------

static void free_plan_memory(pfb_plan *p)
{
    if (p->twiddle)
        (void)hipFree(p->twiddle);
    if (p->ws_y)
        (void)hipFree(p->ws_y);
    if (p->ws_gy)
        (void)hipFree(p->ws_gy);
    if (p->ws_gh)
        (void)hipFree(p->ws_gh);
    if (p->hist)
        (void)hipFree(p->hist);
    if (p->h_rep)
        (void)hipFree(p->h_rep);
    p->twiddle = nullptr;
    p->ws_y = p->ws_gy = nullptr;
    p->ws_gh = nullptr;
    p->hist = nullptr;
    p->h_rep = nullptr;
}

static pfb_status dev_alloc(void **p, int64_t bytes, const char *what)
{
    *p = nullptr;
    if (bytes <= 0)
        return PFB_OK;
    hipError_t e = hipMalloc(p, (size_t)bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(PFB_E_NOMEM, std::string("hipMalloc(") + what + "): " + hipGetErrorString(e));
    }
    return PFB_OK;
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Rows per tile for a kernel that runs one workgroup per CU at a time: the
// smallest multiple of `rb` that is at least `min_rows` and splits the
// B*rows work into a whole number of rounds over the CUs (so that no CU
// runs one tile more than the others at the end).
static int balanced_tile_rows(int64_t B, int64_t rows, int rb, int64_t min_rows, int cus)
{
    const int64_t max_tiles = B * ceil_div(rows, ceil_div(min_rows, rb) * rb);
    int64_t best_sb = ceil_div(min_rows, rb) * rb;
    double best_eff = 0.0;
    for (int64_t rounds = 1; rounds * cus <= max_tiles * 2 + cus; ++rounds) {
        // tiles per stream needed for `rounds` full rounds
        const int64_t tiles_total = rounds * cus;
        const int64_t tiles_per_stream = ceil_div(tiles_total, B);
        int64_t sb = ceil_div(ceil_div(rows, tiles_per_stream), rb) * rb;
        if (sb < rb)
            sb = rb;
        const int64_t n = B * ceil_div(rows, sb);
        const double eff = (double)n / (double)(ceil_div(n, cus) * cus);
        if (sb >= min_rows && (eff > best_eff + 1e-9 || (eff >= best_eff - 1e-9 && sb > best_sb && eff > 0.97))) {
            best_eff = eff;
            best_sb = sb;
        }
    }
    return (int)best_sb;
}

// Largest tile height (a multiple of rb) whose rows plus `extra` halo rows
// fit one bounded view (under 2 GiB) at row_bytes per row: the fused adjoint
// addresses a tile's rows through such views.
static int view_rows_cap(int64_t row_bytes, int rb, int extra)
{
    const int64_t cap = ((int64_t)0x7fffffff / row_bytes - extra) / rb * rb;
    return (int)(cap < rb ? rb : (cap > INT32_MAX ? INT32_MAX / rb * rb : cap));
}

// Rows per fused tile: whole rounds over the workgroups that fit at once
// (`slots`), at least 256 rows so that the T-1 halo rows a tile re-reads stay
// a small fraction of its input (measured: 64-row tiles fetched 1.24x the
// input bytes; their halo rows are not served by the cache, because
// neighbouring tiles run at the same time and the halo is the start of one
// tile's walk but the end of the other's).
static int choose_fused_sb(const pfb_desc &d, int rb, int slots)
{
    return balanced_tile_rows(d.batch, d.spectra, rb, 256, slots);
}

static pfb_status plan_single(const pfb_desc *d, pfb_plan *p)
{
    p->kind = KIND_SINGLE;
    p->d = *d;
    (void)hipGetDevice(&p->device);
    p->tp = padded_taps(d->taps);
    p->long_fir = d->taps > PFB_MAX_TAPS_WINDOW;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, p->device) == hipSuccess && prop.multiProcessorCount > 0)
            p->num_cus = prop.multiProcessorCount;
    }
    const bool fir_only = d->flags & PFB_FIR_ONLY;
    p->log2c = fir_only ? -1 : ilog2_exact(d->channels);

    TuneEntry te;
    const bool tuned = tune_lookup(*d, &te);
    // Two channels per lane (16-byte complex64 loads) where the doubled
    // register window fits (padded taps <= 16) and C is even; short tiles of
    // 32 filtered spectra keep many waves resident (the halo rows they re-read
    // are served by the caches). For int8 input at 16 taps, tiles of 64 rows
    // measured faster (4096 channels: 0.31 -> 0.27 ms with inputs beyond the
    // last-level cache; at 8 taps 64 rows were slower, 0.25 -> 0.28 ms, and
    // the other input types were slower with 64 too).
    // Longer windows re-read T-1 halo rows per tile, so their tiles are
    // longer: 128 rows at 32 taps (1024 channels: 0.25 -> 0.22 ms), 64 rows
    // at 64 taps (faster than 32 or 128).
    // From 2048 channels complex64 input, and from 4096 int8 input, run
    // faster with one channel per lane and 32-row tiles (twice the waves;
    // T=16, 2^27 samples: complex64 FIR 0.393 -> 0.381 ms at 2048 channels,
    // 0.391 -> 0.377 at 4096, 0.398 -> 0.376 at 8192; int8 0.280 -> 0.26 at
    // 4096, 0.273 -> 0.267 at 8192); int16 and fp16 input do not gain.
    const bool cpt2_ok = p->tp <= 16 && d->channels % 2 == 0;
    const bool wide_one = (d->dtype == PFB_C64 && d->channels >= 2048) || (d->dtype == PFB_CI8 && d->channels >= 4096);
    p->fir_cpt = cpt2_ok && !wide_one ? 2 : 1;
    p->fir_sb = p->tp >= 64                                          ? 64
                : p->tp == 32                                        ? 128
                : (d->dtype == PFB_CI8 && p->tp == 16 && !wide_one) ? 64
                                                                     : 32;
    if (tuned) {
        if (te.fir_cpt == 1 || (te.fir_cpt == 2 && cpt2_ok))
            p->fir_cpt = te.fir_cpt;
        if (te.fir_sb >= 16 && te.fir_sb <= 8192)
            p->fir_sb = te.fir_sb;
    }
    if (d->flags & PFB_PLAIN) {
        // the untuned comparator: one channel per lane, long tiles
        p->fir_cpt = 1;
        p->fir_sb = 256;
    }

    if (fir_only) {
        p->path = PATH_FIR_ONLY;
    } else if (!(d->flags & (PFB_NO_FUSE | PFB_PLAIN | PFB_CONVERT_PER_USE)) &&
               fused_supported(d->dtype, p->tp, p->log2c) &&
               !(tuned && te.path == PATH_SPLIT)) {
        p->path = PATH_FUSED;
        const int rb = fused_rows_per_chunk(p->tp, p->log2c);
        if (tuned && te.fused_ws >= 0)
            p->fused_ws = te.fused_ws != 0;
        // the wave-specialised kernel pays a pipeline fill per tile: longer
        // tiles, balanced over the CUs
        // workgroups per CU at once: LDS-bound (two chunk buffers of C
        // padded complex rows and the twiddles)
        const int slots = p->num_cus * (p->log2c >= 10 ? 1 : 2);
        p->fused_sb = p->fused_ws ? balanced_tile_rows(d->batch, d->spectra, rb, 128, p->num_cus)
                                  : choose_fused_sb(*d, rb, slots);
        if (tuned && te.fused_sb >= rb && te.fused_sb % rb == 0)
            p->fused_sb = te.fused_sb;
    } else {
        p->path = PATH_SPLIT;
    }

    pfb_status st;
    if (!fir_only) {
        if (p->log2c < 0) {
            p->mixed = true;
            if (!gfft_schedule(d->channels, &p->gf))
                return fail(PFB_E_UNSUPPORTED, "no radix schedule for this channel count");
            st = make_twiddles_mixed(d->channels, &p->twiddle);
        } else {
            st = make_twiddles(p->log2c, &p->twiddle);
        }
        if (st != PFB_OK)
            return st;
        // Split path workspace (only the split path without a caller-given
        // y uses it): by default the whole filtered-spectra array, so the
        // FIR and the FFT each run as one launch (measured: chunks sized
        // for the last-level cache lose more to per-launch ramps and tails
        // than they gain); above 4 GiB, or with a tuned chunk size, the
        // rows are processed in chunks.
        const int64_t row_bytes = (int64_t)d->channels * 8;
        if (p->path == PATH_SPLIT) {
            if (d->flags & PFB_PLAIN) {
                p->chunk_rows = d->spectra;
            } else {
                int64_t target = (int64_t)4 << 30;
                if (tuned && te.chunk_mib > 0)
                    target = (int64_t)te.chunk_mib << 20;
                p->chunk_rows = target / (row_bytes * d->batch);
                if (p->chunk_rows < 1)
                    p->chunk_rows = 1;
                if (p->chunk_rows > d->spectra)
                    p->chunk_rows = d->spectra;
            }
            p->ws_y_bytes = p->chunk_rows * row_bytes * d->batch;
            st = dev_alloc(reinterpret_cast<void **>(&p->ws_y), p->ws_y_bytes, "split workspace");
            if (st != PFB_OK)
                return st;
        }
        if (d->dtype == PFB_C64 && d->taps <= PFB_MAX_TAPS_WINDOW) {
            p->bwd_fused = !(d->flags & (PFB_NO_FUSE | PFB_PLAIN)) && fused_bwd_supported(p->tp, p->log2c);
            // at least 128 gx rows per tile (the T-1 halo rows are transformed
            // twice and every tile writes a tap-gradient partial)
            p->bwd_sb = balanced_tile_rows(d->batch, d->spectra + d->taps - 1, 16, 128, p->num_cus);
            if (tuned && te.bwd_sb >= 16 && te.bwd_sb <= 65536)
                p->bwd_sb = te.bwd_sb;
            p->bwd_sb = std::min(p->bwd_sb, view_rows_cap((int64_t)d->channels * 8, 16, 0));
            // measured: the single-role adjoint is the faster default at
            // every supported size (the tuner may still pick the other)
            p->bwd_ws = false;
            if (tuned && te.bwd_ws >= 0)
                p->bwd_ws = te.bwd_ws != 0;
            int64_t parts;
            if (p->bwd_fused) {
                parts = (int64_t)d->batch * ceil_div(d->spectra + d->taps - 1, p->bwd_sb);
            } else {
                p->ws_gy_bytes = (int64_t)d->batch * d->spectra * row_bytes;
                st = dev_alloc(reinterpret_cast<void **>(&p->ws_gy), p->ws_gy_bytes, "backward workspace");
                if (st != PFB_OK)
                    return st;
                // tiles of gh_sb filtered spectra (gh_partial_kernel) or of
                // gh_sb raw spectra (gxgh_kernel), whichever is more
                parts = (int64_t)d->batch * ceil_div(d->spectra + d->taps - 1, p->gh_sb);
            }
            p->ws_gh_bytes = parts * d->taps * d->channels * 4;
            st = dev_alloc(reinterpret_cast<void **>(&p->ws_gh), p->ws_gh_bytes, "tap-gradient partials");
            if (st != PFB_OK)
                return st;
        }
    }
    if ((d->flags & PFB_STREAMING) && d->taps > 1) {
        p->hist_bytes = (int64_t)d->batch * (d->taps - 1) * d->channels * bytes_per_sample(d->dtype);
        pfb_status st2 = dev_alloc(reinterpret_cast<void **>(&p->hist), p->hist_bytes, "streaming history");
        if (st2 != PFB_OK)
            return st2;
        if (hipMemset(p->hist, 0, (size_t)p->hist_bytes) != hipSuccess)
            return fail(PFB_E_HIP, "hipMemset(streaming history)");
    }
    return PFB_OK;
}

extern "C" pfb_status pfb_plan_create(const pfb_desc *desc, pfb_plan **out)
{
    if (!out)
        return fail(PFB_E_INVALID, "out is NULL");
    *out = nullptr;
    pfb_status st = validate_desc(desc, false);
    if (st != PFB_OK)
        return st;
    pfb_plan *p = new (std::nothrow) pfb_plan();
    if (!p)
        return fail(PFB_E_NOMEM, "host allocation of the plan failed");
    st = plan_single(desc, p);
    if (st != PFB_OK) {
        free_plan_memory(p);
        delete p;
        return st;
    }
    *out = p;
    return PFB_OK;
}

extern "C" pfb_status pfb_plan_get_info(const pfb_plan *p, pfb_plan_info *info)
{
    if (!p || !info)
        return fail(PFB_E_INVALID, "NULL argument");
    if (p->kind != KIND_SINGLE)
        return fail(PFB_E_STATE, "not a single-problem plan");
    info->path = (int32_t)p->path;
    info->fir_rows = p->path == PATH_FUSED ? p->fused_sb : p->fir_sb;
    info->fir_cpt = p->fir_cpt;
    info->padded_taps = p->tp;
    info->workspace_bytes = p->ws_y_bytes + p->ws_gy_bytes + p->ws_gh_bytes;
    info->backward_fused = p->bwd_fused ? (p->bwd_ws ? 2 : 1) : 0;
    info->fused_ws = (p->path == PATH_FUSED && p->fused_ws) ? 1 : 0;
    info->chunk_rows = p->chunk_rows;
    info->backward_rows = p->bwd_fused ? p->bwd_sb : p->fir_sb;
    return PFB_OK;
}

// ----------------------------------------------------------------------------
// Forward
// ----------------------------------------------------------------------------

// FIR over output rows [s_a, s_a + n) of every stream into y, where output
// row s of stream b lands at y + b*y_bstride + (s - s_a)*C.
static hipError_t run_fir(const pfb_plan *p, const void *x, const float *h, float2 *y, int64_t s_a, int64_t n,
                          int64_t y_bstride, hipStream_t st)
{
    const pfb_desc &d = p->d;
    FirArgs a{};
    a.x = x;
    a.h = h;
    a.y = y;
    a.C = d.channels;
    a.T = d.taps;
    a.B = d.batch;
    a.SB = p->fir_sb;
    a.n_tiles = (int)ceil_div(n, a.SB);
    a.n_cchunks = (int)ceil_div(d.channels, 64 * p->fir_cpt);
    a.in_rows = d.spectra + d.taps - 1;
    a.in_bstride = a.in_rows * d.channels;
    a.shift = p->tp - d.taps;
    a.out_first = s_a;
    a.out_count = n;
    a.y_bstride = y_bstride;
    if (p->long_fir) {
        a.SB = 32;
        a.n_tiles = (int)ceil_div(n, a.SB);
        a.n_cchunks = (int)ceil_div(d.channels, 64);
        a.shift = 0;
        return launch_fir_long(a, d.dtype, st);
    }
    return launch_fir(a, d.dtype, p->tp, p->fir_cpt, false, st, (d.flags & PFB_CONVERT_PER_USE) != 0);
}

static hipError_t run_fft(const pfb_plan *p, const float2 *in, float2 *out, int64_t nrows, int64_t rows_per_group,
                          int64_t in_gstride, int64_t out_gstride, bool inv, hipStream_t st)
{
    FftArgs a{};
    a.in = in;
    a.out = out;
    a.tw = p->twiddle;
    a.nrows = nrows;
    a.rows_per_group = rows_per_group;
    a.in_gstride = in_gstride;
    a.out_gstride = out_gstride;
    a.num_cus = p->num_cus;
    if (p->mixed)
        return launch_gfft(a, p->gf, inv, st);
    return launch_fft(a, p->log2c, inv, st);
}

// Argument checks of a forward call (before anything is launched).
static pfb_status check_execute_args(const pfb_plan *p, const void *x, const float *taps, const void *y,
                                     const void *Y)
{
    if (!p)
        return fail(PFB_E_INVALID, "plan is NULL");
    if (p->kind != KIND_SINGLE || p->vegas_cv > 0)
        return fail(PFB_E_STATE, "pfb_execute needs a single-problem plan");
    if (!x || !taps)
        return fail(PFB_E_INVALID, "x and taps must be non-NULL");
    const bool fir_only = p->path == PATH_FIR_ONLY;
    if (fir_only && !y)
        return fail(PFB_E_INVALID, "a FIR-only plan needs y");
    if (!fir_only && !Y)
        return fail(PFB_E_INVALID, "Y must be non-NULL");
    if (!aligned16(x) || !aligned16(taps) || (y && !aligned16(y)) || (!fir_only && !aligned16(Y)))
        return fail(PFB_E_INVALID, "device pointers must be 16-byte aligned");
    return PFB_OK;
}

extern "C" pfb_status pfb_execute(pfb_plan *p, const void *x, const float *taps, void *y, void *Y, void *stream)
{
    const pfb_status chk = check_execute_args(p, x, taps, y, Y);
    if (chk != PFB_OK)
        return chk;
    const pfb_desc &d = p->d;
    const bool fir_only = p->path == PATH_FIR_ONLY;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t C = d.channels, S = d.spectra;
    hipError_t e;

    if (fir_only) {
        e = run_fir(p, x, taps, reinterpret_cast<float2 *>(y), 0, S, S * C, st);
        return e == hipSuccess ? PFB_OK : hip_fail(e, "FIR launch");
    }
    float2 *Yo = reinterpret_cast<float2 *>(Y);
    if (p->path == PATH_FUSED && !y) {
        FusedArgs a{};
        a.x = x;
        a.h = taps;
        a.Y = Yo;
        a.tw = p->twiddle;
        a.T = d.taps;
        a.B = d.batch;
        a.SB = p->fused_sb;
        a.n_tiles = (int)ceil_div(S, a.SB);
        a.S = S;
        e = p->fused_ws ? launch_fused_ws(a, d.dtype, p->tp, p->log2c, st)
                        : launch_fused(a, d.dtype, p->tp, p->log2c, st);
        return e == hipSuccess ? PFB_OK : hip_fail(e, "fused FIR+FFT launch");
    }
    if (y) {
        // the caller keeps the filtered spectra: whole FIR, then whole FFT
        float2 *yo = reinterpret_cast<float2 *>(y);
        e = run_fir(p, x, taps, yo, 0, S, S * C, st);
        if (e == hipSuccess)
            e = run_fft(p, yo, Yo, (int64_t)d.batch * S, S, S * C, S * C, false, st);
        return e == hipSuccess ? PFB_OK : hip_fail(e, "split FIR/FFT launch");
    }
    // chunked split path through the plan's workspace
    for (int64_t s_a = 0; s_a < S; s_a += p->chunk_rows) {
        const int64_t n = (S - s_a) < p->chunk_rows ? (S - s_a) : p->chunk_rows;
        e = run_fir(p, x, taps, p->ws_y, s_a, n, n * C, st);
        if (e != hipSuccess)
            return hip_fail(e, "FIR launch");
        e = run_fft(p, p->ws_y, Yo + s_a * C, (int64_t)d.batch * n, n, n * C, S * C, false, st);
        if (e != hipSuccess)
            return hip_fail(e, "FFT launch");
    }
    return PFB_OK;
}

// ----------------------------------------------------------------------------
// Streaming
// ----------------------------------------------------------------------------

extern "C" pfb_status pfb_execute_stream(pfb_plan *p, void *xbuf, const float *taps, void *y, void *Y,
                                         void *stream)
{
    if (!p)
        return fail(PFB_E_INVALID, "plan is NULL");
    if (p->kind != KIND_SINGLE || !(p->d.flags & PFB_STREAMING))
        return fail(PFB_E_STATE, "pfb_execute_stream needs a plan created with PFB_STREAMING");
    const pfb_status chk = check_execute_args(p, xbuf, taps, y, Y);
    if (chk != PFB_OK)
        return chk;
    const pfb_desc &d = p->d;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t bs = bytes_per_sample(d.dtype);
    const int64_t row_bytes = (int64_t)d.channels * bs;
    const int64_t stream_bytes = (d.spectra + d.taps - 1) * row_bytes; // per stream in xbuf
    const int64_t head = (int64_t)(d.taps - 1) * row_bytes;           // carried rows per stream
    char *xb = static_cast<char *>(xbuf);
    if (head > 0) {
        // carried spectra into the headroom rows
        hipError_t e = launch_copy_blocks(p->hist, head, xb, stream_bytes, head, d.batch, st);
        if (e != hipSuccess)
            return hip_fail(e, "streaming history copy-in");
    }
    pfb_status r = pfb_execute(p, xbuf, taps, y, Y, stream);
    if (r != PFB_OK || head == 0)
        return r;
    // the last T-1 rows of every stream become the carried spectra
    hipError_t e = launch_copy_blocks(xb + d.spectra * row_bytes, stream_bytes, p->hist, head, head, d.batch, st);
    return e == hipSuccess ? PFB_OK : hip_fail(e, "streaming history copy-out");
}

extern "C" pfb_status pfb_stream_reset(pfb_plan *p, void *stream)
{
    if (!p)
        return fail(PFB_E_INVALID, "plan is NULL");
    if (p->kind != KIND_SINGLE || !(p->d.flags & PFB_STREAMING))
        return fail(PFB_E_STATE, "pfb_stream_reset needs a plan created with PFB_STREAMING");
    if (!p->hist)
        return PFB_OK;
    hipError_t e = launch_copy_blocks(nullptr, 0, p->hist, p->hist_bytes, p->hist_bytes, 1,
                                      reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? PFB_OK : hip_fail(e, "streaming history reset");
}

// ----------------------------------------------------------------------------
// Polarisation-interleaved sub-band layout
// ----------------------------------------------------------------------------

extern "C" pfb_status pfb_plan_create_vegas(int32_t channels, int32_t subbands, int32_t taps, int64_t spectra,
                                            int32_t dtype, pfb_plan **out)
{
    if (!out)
        return fail(PFB_E_INVALID, "out is NULL");
    *out = nullptr;
    const int l2 = ilog2_exact(channels);
    if (l2 < 0 || channels < PFB_MIN_FFT_CHANNELS || channels > PFB_MAX_FFT_CHANNELS)
        return fail(PFB_E_UNSUPPORTED, "channels per sub-band must be a power of two in [32, 8192]");
    if (subbands < 1)
        return fail(PFB_E_INVALID, "subbands must be >= 1");
    int64_t cols = 0;
    if (!mul_ok((int64_t)2 * channels, subbands, &cols) || cols > INT32_MAX)
        return fail(PFB_E_INVALID, "2 * channels * subbands overflows");
    pfb_desc d{};
    d.channels = (int32_t)cols;
    d.taps = taps;
    d.spectra = spectra;
    d.batch = 1;
    d.dtype = dtype;
    d.flags = PFB_FIR_ONLY;
    pfb_status st = validate_desc(&d, false);
    if (st != PFB_OK)
        return st;
    pfb_plan *p = new (std::nothrow) pfb_plan();
    if (!p)
        return fail(PFB_E_NOMEM, "host allocation of the plan failed");
    st = plan_single(&d, p);
    if (st == PFB_OK) {
        p->vegas_cv = channels;
        p->vegas_nsub = subbands;
        p->vegas_log2cv = l2;
        st = make_twiddles(l2, &p->twiddle);
    }
    if (st == PFB_OK) {
        p->ws_y_bytes = spectra * cols * 8;
        st = dev_alloc(reinterpret_cast<void **>(&p->ws_y), p->ws_y_bytes, "filtered spectra");
    }
    if (st == PFB_OK)
        st = dev_alloc(reinterpret_cast<void **>(&p->h_rep), (int64_t)taps * cols * 4, "replicated taps");
    if (st != PFB_OK) {
        free_plan_memory(p);
        delete p;
        return st;
    }
    *out = p;
    return PFB_OK;
}

extern "C" pfb_status pfb_execute_vegas(pfb_plan *p, const void *x, const float *taps, void *Y, void *stream)
{
    if (!p)
        return fail(PFB_E_INVALID, "plan is NULL");
    if (p->kind != KIND_SINGLE || p->vegas_cv <= 0)
        return fail(PFB_E_STATE, "pfb_execute_vegas needs a plan from pfb_plan_create_vegas");
    if (!x || !taps || !Y)
        return fail(PFB_E_INVALID, "x, taps and Y must be non-NULL");
    if (!aligned16(x) || !aligned16(taps) || !aligned16(Y))
        return fail(PFB_E_INVALID, "device pointers must be 16-byte aligned");
    const pfb_desc &d = p->d;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = launch_vegas_taps(taps, p->h_rep, d.taps, p->vegas_cv, p->vegas_nsub, st);
    if (e == hipSuccess)
        e = run_fir(p, x, p->h_rep, p->ws_y, 0, d.spectra, d.spectra * d.channels, st);
    if (e == hipSuccess) {
        FftArgs a{};
        a.in = p->ws_y;
        a.out = reinterpret_cast<float2 *>(Y);
        a.tw = p->twiddle;
        a.nrows = d.spectra * p->vegas_nsub * 2;
        e = launch_fft_pol2(a, p->vegas_log2cv, st);
    }
    return e == hipSuccess ? PFB_OK : hip_fail(e, "sub-band filter bank launch");
}

// ----------------------------------------------------------------------------
// Backward
// ----------------------------------------------------------------------------

extern "C" pfb_status pfb_backward(pfb_plan *p, const void *x, const float *taps, const void *gY, void *gx,
                                   float *gh, void *stream)
{
    if (!p)
        return fail(PFB_E_INVALID, "plan is NULL");
    if (p->kind != KIND_SINGLE || p->vegas_cv > 0)
        return fail(PFB_E_STATE, "pfb_backward needs a single-problem plan");
    if (p->path == PATH_FIR_ONLY)
        return fail(PFB_E_STATE, "pfb_backward needs a plan with the FFT step");
    const pfb_desc &d = p->d;
    if (d.dtype != PFB_C64)
        return fail(PFB_E_UNSUPPORTED, "pfb_backward needs complex float32 input");
    if (d.taps > PFB_MAX_TAPS_WINDOW)
        return fail(PFB_E_UNSUPPORTED, "pfb_backward supports up to PFB_MAX_TAPS_WINDOW taps");
    if (!gY || !taps || (gh && !x))
        return fail(PFB_E_INVALID, "gY and taps (and x for gh) must be non-NULL");
    if (!aligned16(gY) || !aligned16(taps) || (x && !aligned16(x)) || (gx && !aligned16(gx)) ||
        (gh && !aligned16(gh)))
        return fail(PFB_E_INVALID, "device pointers must be 16-byte aligned");
    if (!gx && !gh)
        return PFB_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t C = d.channels, S = d.spectra, T = d.taps;
    hipError_t e;
    if (p->bwd_fused) {
        BwdArgs a{};
        a.x = reinterpret_cast<const float2 *>(x);
        a.h = taps;
        a.gY = reinterpret_cast<const float2 *>(gY);
        a.gx = reinterpret_cast<float2 *>(gx);
        a.part = gh ? p->ws_gh : nullptr;
        a.tw = p->twiddle;
        a.T = d.taps;
        a.B = d.batch;
        a.SB = p->bwd_sb;
        a.n_tiles = (int)ceil_div(S + T - 1, a.SB);
        a.S = S;
        e = p->bwd_ws ? launch_fused_bwd_ws(a, p->tp, p->log2c, st) : launch_fused_bwd(a, p->tp, p->log2c, st);
        if (e == hipSuccess && gh)
            e = launch_gh_reduce(p->ws_gh, gh, (int64_t)d.batch * a.n_tiles, T * C, st);
        return e == hipSuccess ? PFB_OK : hip_fail(e, "fused adjoint launch");
    }
    // 1. gy = unnormalised inverse DFT of gY (adjoint of Eq. (2))
    e = run_fft(p, reinterpret_cast<const float2 *>(gY), p->ws_gy, (int64_t)d.batch * S, S, S * C, S * C, true, st);
    if (e != hipSuccess)
        return hip_fail(e, "inverse FFT launch");
    // 2 and 3 in one pass when both are wanted (up to 32 taps): gy and x are
    // read once for the sample gradient and the tap-gradient partials
    if (gx && gh && p->tp <= 32) {
        GxGhArgs a{};
        a.x = reinterpret_cast<const float2 *>(x);
        a.gy = p->ws_gy;
        a.h = taps;
        a.gx = reinterpret_cast<float2 *>(gx);
        a.part = p->ws_gh;
        a.C = d.channels;
        a.T = d.taps;
        a.B = d.batch;
        a.SB = p->gh_sb;
        a.n_tiles = (int)ceil_div(S + T - 1, a.SB);
        a.n_cchunks = (int)ceil_div(C, 64);
        a.S = S;
        e = launch_gxgh(a, p->tp, gh, st);
        return e == hipSuccess ? PFB_OK : hip_fail(e, "adjoint launch");
    }
    // 2. gx = adjoint FIR: reversed taps over gy, zero outside [0, S)
    if (gx) {
        FirArgs a{};
        a.x = p->ws_gy;
        a.h = taps;
        a.y = reinterpret_cast<float2 *>(gx);
        a.C = d.channels;
        a.T = d.taps;
        a.B = d.batch;
        a.SB = p->fir_sb;
        const int64_t rows = S + T - 1;
        a.n_tiles = (int)ceil_div(rows, a.SB);
        a.n_cchunks = (int)ceil_div(C, 64 * p->fir_cpt);
        a.in_rows = S;
        a.in_bstride = S * C;
        a.shift = (p->tp - T) + T - 1;
        a.out_first = 0;
        a.out_count = rows;
        a.y_bstride = rows * C;
        e = launch_fir(a, PFB_C64, p->tp, p->fir_cpt, true, st);
        if (e != hipSuccess)
            return hip_fail(e, "adjoint FIR launch");
    }
    // 3. gh = sum over streams and spectra of Re(conj(gy) x), two fixed-order stages
    if (gh) {
        GhArgs a{};
        a.x = reinterpret_cast<const float2 *>(x);
        a.gy = p->ws_gy;
        a.part = p->ws_gh;
        a.C = d.channels;
        a.T = d.taps;
        a.B = d.batch;
        a.SB = p->gh_sb;
        a.n_tiles = (int)ceil_div(S, a.SB);
        a.n_cchunks = (int)ceil_div(C, 64);
        a.S = S;
        e = launch_gh(a, p->tp, gh, st);
        if (e != hipSuccess)
            return hip_fail(e, "tap-gradient launch");
    }
    return PFB_OK;
}

// ----------------------------------------------------------------------------
// Misc
// ----------------------------------------------------------------------------

extern "C" pfb_status pfb_plan_destroy(pfb_plan *p)
{
    if (!p)
        return PFB_OK;
    if (p->batched)
        batched_free(p->batched);
    free_plan_memory(p);
    delete p;
    return PFB_OK;
}

extern "C" const char *pfb_status_str(pfb_status s)
{
    switch (s) {
    case PFB_OK: return "PFB_OK";
    case PFB_E_INVALID: return "PFB_E_INVALID: invalid argument";
    case PFB_E_UNSUPPORTED: return "PFB_E_UNSUPPORTED: unsupported request";
    case PFB_E_NOMEM: return "PFB_E_NOMEM: allocation failed";
    case PFB_E_HIP: return "PFB_E_HIP: HIP runtime error";
    case PFB_E_STATE: return "PFB_E_STATE: wrong plan kind for this call";
    default: return "unknown pfb_status";
    }
}

extern "C" const char *pfb_last_error(void) { return g_last_error.c_str(); }

// Internal hooks for the batched and tuning modules.
pfb_status pfb_internal_fail(pfb_status st, const char *msg) { return fail(st, msg); }
// gx rows per fused adjoint tile, as a plan chooses it (no tuning cache)
int pfb_internal_bwd_tile_rows(int64_t B, int64_t S, int T, int C, int cus)
{
    const int sb = balanced_tile_rows(B, S + T - 1, 16, 128, cus);
    return std::min(sb, view_rows_cap((int64_t)C * 8, 16, 0));
}
pfb_status pfb_internal_validate(const pfb_desc *d, bool batched_beam) { return validate_desc(d, batched_beam); }
pfb_plan *pfb_internal_new_plan() { return new (std::nothrow) pfb_plan(); }
void pfb_internal_set_batched(pfb_plan *p, Batched *b) { p->kind = KIND_BATCHED; p->batched = b; }
Batched *pfb_internal_get_batched(pfb_plan *p) { return p->kind == KIND_BATCHED ? p->batched : nullptr; }
