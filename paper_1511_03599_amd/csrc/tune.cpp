// Tuning cache: a small text file, one entry per line,
//   <arch> <dtype> <C> <T> <B> <S> path=<p> fir_cpt=<n> fir_sb=<n> fused_sb=<n> fused_ws=<n> chunk_mib=<n>
//   bwd_sb=<n> bwd_ws=<n>
// for single plans, and
//   <arch> batched <nbeams> <total samples> tile_kib=<n>
// for batched plans.
// Lines that do not parse are ignored, so a damaged cache degrades to the
// built-in defaults rather than to an error.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <string>
#include <vector>

#include "launch.h"
#include "tune.h"

namespace pfb {

std::string device_arch_name()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return "unknown";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

static bool parse_kv(const char *tok, const char *key, int *val)
{
    const size_t n = std::strlen(key);
    if (std::strncmp(tok, key, n) != 0 || tok[n] != '=')
        return false;
    char *end = nullptr;
    long v = std::strtol(tok + n + 1, &end, 10);
    if (end == tok + n + 1)
        return false;
    *val = (int)v;
    return true;
}

static thread_local const TuneEntry *g_override = nullptr;

void tune_set_override(const TuneEntry *e) { g_override = e; }

// The entry for a descriptor: the last line with the same arch, dtype, C and
// T and the same B and S; failing that, the line with the same arch, dtype,
// C and T whose B*S is nearest in ratio (the last of equals), from which only
// the shape-independent choices carry over (path, FIR channels per lane, the
// wave-specialised forms); tile heights, chunk sizes and the adjoint tile then
// keep the built-in defaults, which are sized for the actual shape.
bool tune_lookup(const pfb_desc &d, TuneEntry *out)
{
    if (g_override) {
        *out = *g_override;
        return true;
    }
    const char *path = std::getenv("PFB_TUNE_CACHE");
    if (!path || !*path)
        return false;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return false;
    const std::string arch = device_arch_name();
    const double want = std::log((double)d.batch * (double)d.spectra);
    char line[512];
    bool exact = false, near = false;
    double near_dist = 0.0;
    TuneEntry best_exact, best_near;
    while (std::fgets(line, sizeof line, f)) {
        char a[64];
        int dt, C, T, B;
        long long S;
        int used = 0;
        if (std::sscanf(line, "%63s %d %d %d %d %lld%n", a, &dt, &C, &T, &B, &S, &used) != 6)
            continue;
        if (arch != a || dt != d.dtype || C != d.channels || T != d.taps || B < 1 || S < 1)
            continue;
        TuneEntry e;
        char *rest = line + used;
        for (char *tok = std::strtok(rest, " \t\r\n"); tok; tok = std::strtok(nullptr, " \t\r\n")) {
            parse_kv(tok, "path", &e.path);
            parse_kv(tok, "fir_cpt", &e.fir_cpt);
            parse_kv(tok, "fir_sb", &e.fir_sb);
            parse_kv(tok, "fused_sb", &e.fused_sb);
            parse_kv(tok, "fused_ws", &e.fused_ws);
            parse_kv(tok, "chunk_mib", &e.chunk_mib);
            parse_kv(tok, "bwd_sb", &e.bwd_sb);
            parse_kv(tok, "bwd_ws", &e.bwd_ws);
        }
        if (B == d.batch && S == d.spectra) {
            best_exact = e; // the last matching line wins
            exact = true;
            continue;
        }
        const double dist = std::fabs(std::log((double)B * (double)S) - want);
        if (!near || dist <= near_dist) {
            best_near = e;
            near_dist = dist;
            near = true;
        }
    }
    std::fclose(f);
    if (exact) {
        *out = best_exact;
        return true;
    }
    if (near) {
        TuneEntry e;
        e.path = best_near.path;
        e.fir_cpt = best_near.fir_cpt;
        e.fused_ws = best_near.fused_ws;
        e.bwd_ws = best_near.bwd_ws;
        *out = e;
        return true;
    }
    return false;
}

static thread_local int g_batched_override = 0;

void batched_tile_set_override(int kib) { g_batched_override = kib; }

static long long batched_total_samples(int32_t nbeams, const pfb_desc *beams)
{
    long long tot = 0;
    for (int i = 0; i < nbeams; ++i)
        tot += (long long)beams[i].spectra * beams[i].channels;
    return tot;
}

int batched_tile_kib(int32_t nbeams, const pfb_desc *beams)
{
    if (g_batched_override > 0)
        return g_batched_override;
    int kib = BATCHED_TILE_KIB_DEFAULT;
    const char *path = std::getenv("PFB_TUNE_CACHE");
    if (!path || !*path)
        return kib;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return kib;
    const std::string arch = device_arch_name();
    const long long tot = batched_total_samples(nbeams, beams);
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char a[64], kw[16];
        int nb = 0;
        long long t = 0;
        int used = 0;
        if (std::sscanf(line, "%63s %15s %d %lld%n", a, kw, &nb, &t, &used) != 4)
            continue;
        if (arch != a || std::strcmp(kw, "batched") != 0 || nb != nbeams || t != tot)
            continue;
        char *rest = line + used;
        for (char *tok = std::strtok(rest, " \t\r\n"); tok; tok = std::strtok(nullptr, " \t\r\n")) {
            int v = 0;
            if (parse_kv(tok, "tile_kib", &v) && v >= 16 && v <= (1 << 20))
                kib = v; // the last matching line wins
        }
    }
    std::fclose(f);
    return kib;
}

} // namespace pfb

// ----------------------------------------------------------------------------
// The tuner
// ----------------------------------------------------------------------------

namespace {

struct Buffers {
    void *x = nullptr, *taps = nullptr, *y = nullptr, *gx = nullptr, *gh = nullptr;
    ~Buffers()
    {
        for (void *p : {x, taps, y, gx, gh})
            if (p)
                (void)hipFree(p);
    }
};

int bytes_per_sample(int dt) { return dt == PFB_C64 ? 8 : dt == PFB_CI8 ? 2 : 4; }

int padded_taps(int T)
{
    int tp = 4;
    while (tp < T)
        tp *= 2;
    return tp;
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

} // namespace

using namespace pfb;

// Time one forward (or, with `backward`, adjoint) call of a plan built with
// configuration `e` (median of `reps` event-timed calls after two warm-up
// calls). Returns < 0 on failure.
static double time_candidate(const pfb_desc &d, const TuneEntry &e, Buffers &buf, hipStream_t st, int reps,
                             bool backward = false)
{
    tune_set_override(&e);
    pfb_plan *p = nullptr;
    pfb_status s = pfb_plan_create(&d, &p);
    tune_set_override(nullptr);
    if (s != PFB_OK)
        return -1.0;
    const bool fir_only = d.flags & PFB_FIR_ONLY;
    void *y = fir_only ? buf.y : nullptr;
    void *Y = fir_only ? nullptr : buf.y;
    auto call = [&]() {
        if (backward)
            return pfb_backward(p, buf.x, (const float *)buf.taps, buf.y, buf.gx, (float *)buf.gh, st);
        return pfb_execute(p, buf.x, (const float *)buf.taps, y, Y, st);
    };
    double best = -1.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        bool ok = true;
        for (int i = 0; i < 2 && ok; ++i)
            ok = call() == PFB_OK;
        std::vector<float> ts;
        for (int i = 0; i < reps && ok; ++i) {
            ok = hipEventRecord(e0, st) == hipSuccess && call() == PFB_OK &&
                 hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.0f;
            if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
                ts.push_back(ms);
        }
        if (ok && !ts.empty()) {
            std::sort(ts.begin(), ts.end());
            best = ts[ts.size() / 2];
        }
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    pfb_plan_destroy(p);
    return best;
}

extern "C" pfb_status pfb_tune(const pfb_desc *desc, const char *cache_path)
{
    pfb_status st = pfb_internal_validate(desc, false);
    if (st != PFB_OK)
        return st;
    if (!cache_path || !*cache_path)
        return pfb_internal_fail(PFB_E_INVALID, "cache_path is empty");
    const pfb_desc d = *desc;
    const int64_t rows = d.spectra + d.taps - 1;
    Buffers buf;
    const size_t xbytes = (size_t)(d.batch * rows * d.channels) * bytes_per_sample(d.dtype);
    const size_t ybytes = (size_t)(d.batch * d.spectra * d.channels) * 8;
    if (hipMalloc(&buf.x, xbytes) != hipSuccess || hipMalloc(&buf.taps, (size_t)d.taps * d.channels * 4) != hipSuccess ||
        hipMalloc(&buf.y, ybytes) != hipSuccess)
        return pfb_internal_fail(PFB_E_NOMEM, "tuner buffers");
    // a small non-zero pattern (timing does not depend on the values)
    if (hipMemset(buf.x, 0x11, xbytes) != hipSuccess || hipMemset(buf.taps, 0x11, (size_t)d.taps * d.channels * 4) != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "tuner buffer fill");
    hipStream_t s = nullptr;
    const bool verbose = std::getenv("PFB_TUNE_VERBOSE") != nullptr;

    std::vector<TuneEntry> cands;
    const int tp = padded_taps(d.taps);
    const bool fir_only = d.flags & PFB_FIR_ONLY;
    const bool cpt2 = tp <= 16 && d.channels % 2 == 0;
    auto add_split = [&](int path) {
        for (int cpt : {1, 2}) {
            if (cpt == 2 && !cpt2)
                continue;
            for (int sb : {16, 32, 64, 128}) {
                if (path == 2) {
                    TuneEntry e;
                    e.fir_cpt = cpt;
                    e.fir_sb = sb;
                    cands.push_back(e);
                } else {
                    for (int mib : {0, 64, 256, 1024}) { // 0: one chunk
                        TuneEntry e;
                        e.path = 1;
                        e.fir_cpt = cpt;
                        e.fir_sb = sb;
                        e.chunk_mib = mib;
                        cands.push_back(e);
                    }
                }
            }
        }
    };
    if (fir_only) {
        add_split(2);
    } else {
        const int l2 = ilog2_exact(d.channels);
        if (!(d.flags & (PFB_NO_FUSE | PFB_PLAIN)) && fused_supported(d.dtype, tp, l2)) {
            const int rb = tp > 16 ? tp : 16;
            for (int ws : {1, 0})
                for (int m : {0, 1, 2, 4, 8, 16, 32}) {
                    TuneEntry e;
                    e.path = 0;
                    e.fused_ws = ws;
                    e.fused_sb = rb * m; // 0: the built-in choice
                    cands.push_back(e);
                }
        }
        add_split(1);
    }
    const int reps = 7;
    double best_t = -1.0;
    TuneEntry best;
    for (const TuneEntry &e : cands) {
        const double t = time_candidate(d, e, buf, s, reps);
        if (verbose)
            std::fprintf(stderr, "pfb_tune: path=%d fir_cpt=%d fir_sb=%d fused_ws=%d fused_sb=%d chunk_mib=%d -> %.4f ms\n",
                         e.path, e.fir_cpt, e.fir_sb, e.fused_ws, e.fused_sb, e.chunk_mib, t);
        if (t > 0 && (best_t < 0 || t < best_t)) {
            best_t = t;
            best = e;
        }
    }
    if (best_t < 0)
        return pfb_internal_fail(PFB_E_HIP, "no tuning candidate ran");
    // the adjoint's tile height, timed with the forward configuration chosen
    if (!fir_only && d.dtype == PFB_C64 && d.taps <= PFB_MAX_TAPS_WINDOW) {
        const size_t gxbytes = (size_t)(d.batch * rows * d.channels) * 8;
        if (hipMalloc(&buf.gx, gxbytes) == hipSuccess &&
            hipMalloc(&buf.gh, (size_t)d.taps * d.channels * 4) == hipSuccess &&
            hipMemset(buf.y, 0x11, ybytes) == hipSuccess) {
            double best_b = -1.0;
            int best_sb = 0, best_ws = -1;
            for (int ws : {1, 0}) {
                for (int sb : {0, 128, 256, 512, 1024}) {
                    TuneEntry e = best;
                    e.bwd_sb = sb;
                    e.bwd_ws = ws;
                    const double t = time_candidate(d, e, buf, s, reps, true);
                    if (verbose)
                        std::fprintf(stderr, "pfb_tune: backward bwd_ws=%d bwd_sb=%d -> %.4f ms\n", ws, sb, t);
                    if (t > 0 && (best_b < 0 || t < best_b)) {
                        best_b = t;
                        best_sb = sb;
                        best_ws = ws;
                    }
                }
            }
            best.bwd_sb = best_sb;
            best.bwd_ws = best_ws;
        }
    }
    FILE *f = std::fopen(cache_path, "a");
    if (!f)
        return pfb_internal_fail(PFB_E_INVALID, "cannot open the tuning cache for writing");
    std::fprintf(f,
                 "%s %d %d %d %d %lld path=%d fir_cpt=%d fir_sb=%d fused_sb=%d fused_ws=%d chunk_mib=%d bwd_sb=%d "
                 "bwd_ws=%d ms=%.5f\n",
                 device_arch_name().c_str(), d.dtype, d.channels, d.taps, d.batch, (long long)d.spectra, best.path,
                 best.fir_cpt, best.fir_sb, best.fused_sb, best.fused_ws, best.chunk_mib, best.bwd_sb, best.bwd_ws,
                 best_t);
    std::fclose(f);
    return PFB_OK;
}

extern "C" pfb_status pfb_tune_batched(int32_t nbeams, const pfb_desc *beams, const char *cache_path)
{
    if (nbeams < 1 || !beams)
        return pfb_internal_fail(PFB_E_INVALID, "nbeams must be >= 1 and beams non-NULL");
    if (!cache_path || !*cache_path)
        return pfb_internal_fail(PFB_E_INVALID, "cache_path is empty");
    for (int i = 0; i < nbeams; ++i) {
        pfb_status st = pfb_internal_validate(&beams[i], true);
        if (st != PFB_OK)
            return st;
    }
    struct BeamBuf {
        void *x = nullptr, *h = nullptr, *Y = nullptr;
    };
    std::vector<BeamBuf> bufs((size_t)nbeams);
    auto release = [&]() {
        for (BeamBuf &b : bufs)
            for (void *p : {b.x, b.h, b.Y})
                if (p)
                    (void)hipFree(p);
    };
    for (int i = 0; i < nbeams; ++i) {
        const pfb_desc &d = beams[i];
        const size_t xb = (size_t)((d.spectra + d.taps - 1) * d.channels) * 8;
        const size_t hb = (size_t)d.taps * d.channels * 4;
        const size_t yb = (size_t)(d.spectra * d.channels) * 8;
        BeamBuf &b = bufs[(size_t)i];
        if (hipMalloc(&b.x, xb) != hipSuccess || hipMalloc(&b.h, hb) != hipSuccess ||
            hipMalloc(&b.Y, yb) != hipSuccess || hipMemset(b.x, 0x11, xb) != hipSuccess ||
            hipMemset(b.h, 0x11, hb) != hipSuccess) {
            release();
            return pfb_internal_fail(PFB_E_NOMEM, "tuner buffers");
        }
    }
    std::vector<const void *> xs((size_t)nbeams);
    std::vector<const float *> hs((size_t)nbeams);
    std::vector<void *> Ys((size_t)nbeams);
    for (int i = 0; i < nbeams; ++i) {
        xs[(size_t)i] = bufs[(size_t)i].x;
        hs[(size_t)i] = (const float *)bufs[(size_t)i].h;
        Ys[(size_t)i] = bufs[(size_t)i].Y;
    }
    const bool verbose = std::getenv("PFB_TUNE_VERBOSE") != nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        release();
        return pfb_internal_fail(PFB_E_HIP, "hipEventCreate");
    }
    double best_t = -1.0;
    int best_kib = 0;
    for (int kib : {64, 128, 256, 512, 1024, 2048, 4096}) {
        batched_tile_set_override(kib);
        pfb_plan *p = nullptr;
        const pfb_status cs = pfb_plan_create_batched(nbeams, beams, &p);
        batched_tile_set_override(0);
        if (cs != PFB_OK)
            continue;
        auto call = [&]() { return pfb_execute_batched(p, xs.data(), hs.data(), Ys.data(), s); };
        bool ok = call() == PFB_OK && call() == PFB_OK;
        std::vector<float> ts;
        for (int r = 0; r < 5 && ok; ++r) {
            ok = hipEventRecord(e0, s) == hipSuccess && call() == PFB_OK && hipEventRecord(e1, s) == hipSuccess &&
                 hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.0f;
            if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
                ts.push_back(ms);
        }
        (void)hipStreamSynchronize(s);
        pfb_plan_destroy(p);
        if (!ok || ts.empty())
            continue;
        std::sort(ts.begin(), ts.end());
        const double t = ts[ts.size() / 2];
        if (verbose)
            std::fprintf(stderr, "pfb_tune_batched: tile_kib=%d -> %.4f ms\n", kib, t);
        if (best_t < 0 || t < best_t) {
            best_t = t;
            best_kib = kib;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    release();
    if (best_t < 0)
        return pfb_internal_fail(PFB_E_HIP, "no batched tuning candidate ran");
    FILE *f = std::fopen(cache_path, "a");
    if (!f)
        return pfb_internal_fail(PFB_E_INVALID, "cannot open the tuning cache for writing");
    std::fprintf(f, "%s batched %d %lld tile_kib=%d ms=%.5f\n", device_arch_name().c_str(), nbeams,
                 pfb::batched_total_samples(nbeams, beams), best_kib, best_t);
    std::fclose(f);
    return PFB_OK;
}
