// Batched multi-beam filter bank: many independent beams, each with its own
// C, T and S, processed by ONE persistent kernel launch per call.
//
// Work is a table of tiles built on the host when the plan is created. A tile
// is a run of consecutive filtered spectra of one beam, over all of its
// channels. A persistent workgroup takes the next tile from an atomic counter
// and does all of the tile's work itself:
//   1. the register-window FIR of every channel of the tile's rows (wave
//      tasks of 64*CPT channels x 32 rows spread over the workgroup's waves),
//      written to the workgroup's own slot of filtered spectra;
//   2. a workgroup barrier;
//   3. the C-point transforms of the slot's rows, written to the beam's
//      frequency spectra.
// No tile depends on another, so no workgroup ever waits for another and no
// device-scope fences are needed: those would write back or invalidate the
// whole L2 of an XCD on every tile. The slot is reused tile after tile; it is
// small enough that the filtered spectra mostly travel through the caches
// rather than HBM. Tiles of one beam are consecutive in the table, so rows
// shared by neighbouring tiles (the T-1 history rows) are read while still
// cached. Beams are ordered by tile work, largest first.
//
// The counter reset and the persistent kernel are recorded once into a HIP
// graph (explicit kernel nodes, no memset nodes) and replayed on each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fft_device.h"
#include "fft_schedule.h"
#include "fir_device.h"
#include "launch.h"
#include "tune.h"

namespace pfb {

// Two persistent workgroups of four waves share a CU (registers allow two
// waves per SIMD, LDS two 8192-point rows), so one can run its FIR while the
// other transforms; a single eight-wave workgroup per CU alternated the two
// phases (64-beam table 13.5 -> 13.1 ms, same bits). Four waves are also the
// fewest that hold an 8192-point transform.
constexpr int BT_THREADS = 256;          // threads per persistent workgroup
constexpr int BT_WAVES = BT_THREADS / 64;
constexpr int BT_TASK_ROWS = 32;         // filtered spectra per FIR wave task
constexpr int BT_LDS = 8704;             // float2: the largest transform round (one 8192-point row)
constexpr int BT_MAX_TAPS = PFB_MAX_TAPS_WINDOW;

struct BeamInfo {
    const float2 *tw;      // twiddles for C
    int C, T, TP, log2c, cpt;
    int n_cchunks;         // channel chunks of 64*cpt
    int tile_rows;         // filtered spectra per tile
    int pad;
    int64_t S;
};

struct BeamPtrs {
    const void *x;
    const float *h;
    float2 *Y;
    const void *pad;       // keeps the entry 32 bytes
};

struct TileDesc {
    int beam;
    int nrows;
    int64_t row0;          // first filtered spectrum of the tile
    int cls;               // tile class (bt_class of the beam's TP and C)
    int pad;
};

struct BatchedArgs {
    const BeamInfo *beams;
    const BeamPtrs *ptrs;
    const TileDesc *tiles;
    int *queue;            // next tile to take
    float2 *slots;         // one slot of filtered spectra per workgroup
    int64_t slot_elems;
    int ntiles;
};

__global__ __launch_bounds__(64) void batched_reset_kernel(BatchedArgs a)
{
    if (threadIdx.x == 0)
        *a.queue = 0;
}

// FIR shape per padded tap count, chosen so that the FIR and the largest
// transform fit the register budget together: two channels per lane
// (16-byte loads) for short windows, one otherwise; a shallower prefetch for
// the longest window.
constexpr int batched_cpt(int tp) { return tp <= 8 ? 2 : 1; }
constexpr int batched_prefetch(int tp) { return tp >= 64 ? 4 : 8; }

// FIR of every channel of rows [row0, row0 + nrows) of one beam into the
// slot (row r of the tile at slot + r*C); this wave takes wave tasks
// wave_id(), wave_id() + BT_WAVES, ...
template <int TP, int CPT>
__device__ __forceinline__ void batched_fir(const BeamInfo bm, const void *x, const float *h, float2 *slot,
                                         int64_t row0, int nrows)
{
    FirArgs f{};
    f.x = x;
    f.h = h;
    f.y = slot;
    f.C = bm.C;
    f.T = bm.T;
    f.B = 1;
    f.SB = BT_TASK_ROWS;
    f.n_tiles = (nrows + BT_TASK_ROWS - 1) / BT_TASK_ROWS;
    f.n_cchunks = bm.n_cchunks;
    f.in_rows = bm.S + bm.T - 1;
    f.in_bstride = 0;
    f.shift = TP - bm.T;
    f.out_first = row0;
    f.out_count = nrows;
    f.y_bstride = 0;
    const int ntasks = f.n_tiles * f.n_cchunks;
    for (int task = wave_id(); task < ntasks; task += BT_WAVES)
        fir_wave_task<DT_C64, TP, CPT, batched_prefetch(TP), false, false>(f, task);
}

// The C-point transforms of the slot's first nrows rows into out (row r at
// out + r*C).
template <int LOG2C>
__device__ __forceinline__ void batched_fft(const float2 *tw, const float2 *slot, float2 *out, int nrows, float2 *lds)
{
    constexpr int C = 1 << LOG2C;
    constexpr int G = FftLanes<LOG2C>::G;
    constexpr int F = BT_THREADS / G; // rows per round
    using S = FftShape<LOG2C, G>;
    static_assert(F * S::PADDED <= BT_LDS, "LDS");
    const int gid = (int)threadIdx.x / G;
    const int lane = (int)threadIdx.x % G;
    if constexpr (G > 64) {
        // Transforms span several waves and synchronise the block, so every
        // group runs the passes (a group past the last row repeats the last
        // row without storing it). The twiddles depend on the lane only:
        // loaded once for all rounds of the tile.
        FftResidentTwiddles<LOG2C, G> twr;
        twr.load(lane, tw);
        for (int base = 0; base < nrows; base += F) {
            const int r = base + gid;
            const bool valid = r < nrows;
            const int rr = valid ? r : nrows - 1;
            const float2 *in = slot + (int64_t)rr * C;
            float2 *o = out + (int64_t)rr * C;
            float2 v[S::E];
            fft_gather_first<LOG2C, G>(lane, [&](int idx) { return in[idx]; }, v);
            fft_passes_resident<LOG2C, G, false, false>(lane, lds + gid * S::PADDED, twr, v, [&](int idx, float2 t) {
                if (valid)
                    store_nt(o + idx, t);
            });
            lds_barrier(); // the LDS rows are reused by the next round
        }
        return;
    }
    for (int base = 0; base < nrows; base += F) {
        const int r = base + gid;
        const bool valid = r < nrows;
        // a group past the last row repeats the last row without storing it
        const int rr = valid ? r : nrows - 1;
        const float2 *in = slot + (int64_t)rr * C;
        float2 *o = out + (int64_t)rr * C;
        if (valid) {
            fft_run<LOG2C, G, false, false>(
                lane, lds + gid * S::PADDED, tw, [&](int idx) { return in[idx]; },
                [&](int idx, float2 v) { store_nt(o + idx, v); });
        }
        lds_barrier(); // the LDS rows are reused by the next round
    }
}

// Tile classes: (padded taps, channels per lane) x transform size. Tiles of
// one class are consecutive in the table.
constexpr int fir_variant(int tp) { return tp == 4 ? 0 : tp == 8 ? 1 : tp == 16 ? 2 : tp == 32 ? 3 : 4; }
constexpr int bt_class(int tp, int log2c) { return fir_variant(tp) * 9 + (log2c - 5); }

// Takes tiles from the queue while they belong to class (TP, LOG2C) and does
// their work; returns the first tile of another class (or ntiles when the
// queue is drained). One call covers a whole run of same-class tiles, so the
// cost of the call itself is paid a few times per workgroup, not per tile.
template <int TP, int LOG2C>
__device__ __noinline__ int batched_run(const BatchedArgs &a, float2 *slot, float2 *lds, int *s_tile, int t)
{
    constexpr int CPT = batched_cpt(TP);
    const TileDesc *tiles = as_global(a.tiles);
    slot = as_global(slot);
    for (;;) {
        const TileDesc td = tiles[t];
        const BeamInfo bm = as_global(a.beams)[td.beam];
        const BeamPtrs bp = as_global(a.ptrs)[td.beam];
        batched_fir<TP, CPT>(bm, as_global(bp.x), as_global(bp.h), slot, td.row0, td.nrows);
        // the slot's rows, written to global memory by every wave, are read
        // back by others: a full barrier (waits for the stores)
        __syncthreads();
        batched_fft<LOG2C>(as_global(bm.tw), slot, as_global(bp.Y) + td.row0 * bm.C, td.nrows, lds);
        // (batched_fft ends with a barrier: the slot and LDS are free again)
        if (threadIdx.x == 0)
            *s_tile = __hip_atomic_fetch_add(as_global(a.queue), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        lds_barrier();
        t = *s_tile;
        lds_barrier();
        if (t >= a.ntiles || tiles[t].cls != bt_class(TP, LOG2C))
            return t;
    }
}

template <int TP>
__device__ __forceinline__ int batched_dispatch_c(const BatchedArgs &a, float2 *slot, float2 *lds, int *s_tile, int t,
                                                  int log2c)
{
    switch (log2c) {
    case 5: return batched_run<TP, 5>(a, slot, lds, s_tile, t);
    case 6: return batched_run<TP, 6>(a, slot, lds, s_tile, t);
    case 7: return batched_run<TP, 7>(a, slot, lds, s_tile, t);
    case 8: return batched_run<TP, 8>(a, slot, lds, s_tile, t);
    case 9: return batched_run<TP, 9>(a, slot, lds, s_tile, t);
    case 10: return batched_run<TP, 10>(a, slot, lds, s_tile, t);
    case 11: return batched_run<TP, 11>(a, slot, lds, s_tile, t);
    case 12: return batched_run<TP, 12>(a, slot, lds, s_tile, t);
    default: return batched_run<TP, 13>(a, slot, lds, s_tile, t);
    }
}

__global__ __launch_bounds__(BT_THREADS, 2) void batched_kernel(BatchedArgs a)
{
    __shared__ float2 lds[BT_LDS];
    __shared__ int s_tile;
    float2 *slot = a.slots + (int64_t)blockIdx.x * a.slot_elems;
    if (threadIdx.x == 0)
        s_tile = __hip_atomic_fetch_add(a.queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    lds_barrier();
    int t = s_tile;
    lds_barrier();
    while (t < a.ntiles) {
        const int cls = a.tiles[t].cls;
        const int log2c = 5 + cls % 9;
        switch (cls / 9) {
        case 0: t = batched_dispatch_c<4>(a, slot, lds, &s_tile, t, log2c); break;
        case 1: t = batched_dispatch_c<8>(a, slot, lds, &s_tile, t, log2c); break;
        case 2: t = batched_dispatch_c<16>(a, slot, lds, &s_tile, t, log2c); break;
        case 3: t = batched_dispatch_c<32>(a, slot, lds, &s_tile, t, log2c); break;
        default: t = batched_dispatch_c<64>(a, slot, lds, &s_tile, t, log2c); break;
        }
    }
}

} // namespace pfb

using namespace pfb;

struct Batched {
    int nbeams = 0;
    std::vector<pfb_desc> descs;
    std::vector<BeamInfo> info;         // host copy (pointers to device memory)
    BeamInfo *d_info = nullptr;
    BeamPtrs *d_ptrs = nullptr;
    BeamPtrs *h_ptrs = nullptr;         // pinned staging for the pointer table
    std::vector<BeamPtrs> last_ptrs;    // what the device table holds
    TileDesc *d_tiles = nullptr;
    int *d_queue = nullptr;
    float2 *d_slots = nullptr;
    std::vector<void *> allocs;         // twiddle tables
    int ntiles = 0;
    int grid = 0;
    int64_t slot_elems = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool launched = false;
    BatchedArgs args{};
};

void batched_free(Batched *b)
{
    if (!b)
        return;
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    if (b->done)
        (void)hipEventDestroy(b->done);
    for (void *p : b->allocs)
        (void)hipFree(p);
    for (void *p : {(void *)b->d_info, (void *)b->d_ptrs, (void *)b->d_tiles, (void *)b->d_queue, (void *)b->d_slots})
        if (p)
            (void)hipFree(p);
    if (b->h_ptrs)
        (void)hipHostFree(b->h_ptrs);
    delete b;
}

static int ilog2_exact(int64_t v)
{
    if (v <= 0 || (v & (v - 1)))
        return -1;
    int l = 0;
    while ((int64_t(1) << l) < v)
        ++l;
    return l;
}

static pfb_status twiddle_table(int log2c, float2 **out)
{
    const FftSchedule sch(log2c);
    const int n = sch.table_size() > 0 ? sch.table_size() : 1;
    std::vector<float2> host((size_t)n, make_float2(1.0f, 0.0f));
    for (int p = 1; p < sch.npass; ++p) {
        const int R = sch.radix(p), L = sch.stride(p), RL = R * L;
        for (int k = 0; k < L; ++k)
            for (int i = 0; i < R; ++i) {
                const int64_t e = ((int64_t)i * k) % RL;
                const double ang = -2.0 * M_PI * (double)e / (double)RL;
                host[(size_t)sch.pass_offset(p) + (size_t)k * R + i] =
                    make_float2((float)std::cos(ang), (float)std::sin(ang));
            }
    }
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(float2) * (size_t)n) != hipSuccess)
        return pfb_internal_fail(PFB_E_NOMEM, "hipMalloc(batched twiddles)");
    if (hipMemcpy(p, host.data(), sizeof(float2) * (size_t)n, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p);
        return pfb_internal_fail(PFB_E_HIP, "hipMemcpy(batched twiddles)");
    }
    *out = reinterpret_cast<float2 *>(p);
    return PFB_OK;
}

// Filtered spectra per tile of a beam with C channels: about tile_kib KiB of
// filtered spectra, a whole number of FIR wave tasks, at least one.
static int batched_tile_rows(int C, int64_t S, int tile_kib)
{
    int64_t r = ((int64_t)tile_kib << 10) / ((int64_t)C * 8);
    r = std::max<int64_t>(BT_TASK_ROWS, r / BT_TASK_ROWS * BT_TASK_ROWS);
    const int64_t s_up = (S + BT_TASK_ROWS - 1) / BT_TASK_ROWS * BT_TASK_ROWS;
    return (int)std::min<int64_t>(r, std::max<int64_t>(BT_TASK_ROWS, s_up));
}

static pfb_status build_batched(int32_t nbeams, const pfb_desc *beams, Batched *B)
{
    B->nbeams = nbeams;
    B->descs.assign(beams, beams + nbeams);
    B->info.resize((size_t)nbeams);
    const int tile_kib = batched_tile_kib(nbeams, beams);
    float2 *tw_by_log2c[14] = {};
    for (int i = 0; i < nbeams; ++i) {
        const pfb_desc &d = beams[i];
        BeamInfo &bi = B->info[(size_t)i];
        bi.C = d.channels;
        bi.T = d.taps;
        bi.TP = 4;
        while (bi.TP < d.taps)
            bi.TP *= 2;
        bi.log2c = ilog2_exact(d.channels);
        bi.cpt = batched_cpt(bi.TP);
        bi.n_cchunks = (d.channels + 64 * bi.cpt - 1) / (64 * bi.cpt);
        bi.S = d.spectra;
        bi.tile_rows = batched_tile_rows(d.channels, d.spectra, tile_kib);
        bi.pad = 0;
        if (!tw_by_log2c[bi.log2c]) {
            pfb_status st = twiddle_table(bi.log2c, &tw_by_log2c[bi.log2c]);
            if (st != PFB_OK)
                return st;
            B->allocs.push_back(tw_by_log2c[bi.log2c]);
        }
        bi.tw = tw_by_log2c[bi.log2c];
        B->slot_elems = std::max<int64_t>(B->slot_elems, (int64_t)bi.tile_rows * bi.C);
    }

    // tile table: beams by tile size, largest first; each beam's tiles in
    // row order
    std::vector<int> order((size_t)nbeams);
    for (int i = 0; i < nbeams; ++i)
        order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const BeamInfo &x = B->info[(size_t)a], &y = B->info[(size_t)b];
        const int64_t wx = (int64_t)x.tile_rows * x.C, wy = (int64_t)y.tile_rows * y.C;
        if (wx != wy)
            return wx > wy;
        return bt_class(x.TP, x.log2c) < bt_class(y.TP, y.log2c);
    });
    std::vector<TileDesc> tiles;
    for (int bidx : order) {
        const BeamInfo &bi = B->info[(size_t)bidx];
        for (int64_t r0 = 0; r0 < bi.S; r0 += bi.tile_rows) {
            TileDesc t{};
            t.beam = bidx;
            t.row0 = r0;
            t.nrows = (int)std::min<int64_t>(bi.tile_rows, bi.S - r0);
            t.cls = bt_class(bi.TP, bi.log2c);
            tiles.push_back(t);
        }
    }
    if (tiles.size() > (size_t)INT32_MAX - ((size_t)1 << 20))
        return pfb_internal_fail(PFB_E_UNSUPPORTED, "batched tile table too large");
    B->ntiles = (int)tiles.size();

    int dev = 0, cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        cus = prop.multiProcessorCount;
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_kernel, BT_THREADS, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    B->grid = std::min(cus * per_cu, B->ntiles);

    if (hipMalloc(&B->d_info, sizeof(BeamInfo) * (size_t)nbeams) != hipSuccess ||
        hipMalloc(&B->d_ptrs, sizeof(BeamPtrs) * (size_t)nbeams) != hipSuccess ||
        hipMalloc(&B->d_tiles, sizeof(TileDesc) * tiles.size()) != hipSuccess ||
        hipMalloc(&B->d_queue, sizeof(int)) != hipSuccess ||
        hipMalloc(&B->d_slots, sizeof(float2) * (size_t)B->slot_elems * (size_t)B->grid) != hipSuccess ||
        hipHostMalloc(&B->h_ptrs, sizeof(BeamPtrs) * (size_t)nbeams, hipHostMallocDefault) != hipSuccess)
        return pfb_internal_fail(PFB_E_NOMEM, "batched plan tables and slots");
    if (hipMemcpy(B->d_info, B->info.data(), sizeof(BeamInfo) * (size_t)nbeams, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(B->d_tiles, tiles.data(), sizeof(TileDesc) * tiles.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(B->d_ptrs, 0, sizeof(BeamPtrs) * (size_t)nbeams) != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "batched plan upload");
    B->last_ptrs.assign((size_t)nbeams, BeamPtrs{nullptr, nullptr, nullptr, nullptr});

    BatchedArgs &a = B->args;
    a.beams = B->d_info;
    a.ptrs = B->d_ptrs;
    a.tiles = B->d_tiles;
    a.queue = B->d_queue;
    a.slots = B->d_slots;
    a.slot_elems = B->slot_elems;
    a.ntiles = B->ntiles;

    // graph: reset the tile counter, then the persistent kernel
    if (hipGraphCreate(&B->graph, 0) != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "hipGraphCreate");
    void *kargs[] = {&B->args};
    hipKernelNodeParams rp{};
    rp.func = reinterpret_cast<void *>(batched_reset_kernel);
    rp.gridDim = dim3(1);
    rp.blockDim = dim3(64);
    rp.sharedMemBytes = 0;
    rp.kernelParams = kargs;
    rp.extra = nullptr;
    hipGraphNode_t n_reset = nullptr, n_main = nullptr;
    if (hipGraphAddKernelNode(&n_reset, B->graph, nullptr, 0, &rp) != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "graph reset node");
    hipKernelNodeParams mp = rp;
    mp.func = reinterpret_cast<void *>(batched_kernel);
    mp.gridDim = dim3((unsigned)B->grid);
    mp.blockDim = dim3(BT_THREADS);
    if (hipGraphAddKernelNode(&n_main, B->graph, &n_reset, 1, &mp) != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "graph kernel node");
    if (hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0) != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "hipGraphInstantiate");
    if (hipEventCreateWithFlags(&B->done, hipEventDisableTiming) != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "hipEventCreate");
    return PFB_OK;
}

extern "C" pfb_status pfb_plan_create_batched(int32_t nbeams, const pfb_desc *beams, pfb_plan **out)
{
    if (!out)
        return pfb_internal_fail(PFB_E_INVALID, "out is NULL");
    *out = nullptr;
    if (nbeams < 1 || !beams)
        return pfb_internal_fail(PFB_E_INVALID, "nbeams must be >= 1 and beams non-NULL");
    for (int i = 0; i < nbeams; ++i) {
        pfb_status st = pfb_internal_validate(&beams[i], true);
        if (st != PFB_OK)
            return st;
        if (beams[i].batch != 1)
            return pfb_internal_fail(PFB_E_INVALID, "batched beams are single streams (batch == 1)");
        if (beams[i].dtype != PFB_C64)
            return pfb_internal_fail(PFB_E_UNSUPPORTED, "batched beams take complex float32 input");
        if (beams[i].taps > BT_MAX_TAPS)
            return pfb_internal_fail(PFB_E_UNSUPPORTED, "batched beams support up to 64 taps");
    }
    Batched *B = new (std::nothrow) Batched();
    pfb_plan *p = pfb_internal_new_plan();
    if (!B || !p) {
        delete B;
        if (p)
            pfb_plan_destroy(p);
        return pfb_internal_fail(PFB_E_NOMEM, "host allocation of the batched plan failed");
    }
    pfb_internal_set_batched(p, B);
    pfb_status st = build_batched(nbeams, beams, B);
    if (st != PFB_OK) {
        pfb_plan_destroy(p);
        return st;
    }
    *out = p;
    return PFB_OK;
}

extern "C" pfb_status pfb_execute_batched(pfb_plan *p, const void *const *x, const float *const *taps,
                                          void *const *Y, void *stream)
{
    if (!p)
        return pfb_internal_fail(PFB_E_INVALID, "plan is NULL");
    Batched *B = pfb_internal_get_batched(p);
    if (!B)
        return pfb_internal_fail(PFB_E_STATE, "pfb_execute_batched needs a batched plan");
    if (!x || !taps || !Y)
        return pfb_internal_fail(PFB_E_INVALID, "pointer arrays must be non-NULL");
    for (int i = 0; i < B->nbeams; ++i) {
        if (!x[i] || !taps[i] || !Y[i])
            return pfb_internal_fail(PFB_E_INVALID, "every beam needs x, taps and Y");
        if (((uintptr_t)x[i] | (uintptr_t)taps[i] | (uintptr_t)Y[i]) & 15u)
            return pfb_internal_fail(PFB_E_INVALID, "device pointers must be 16-byte aligned");
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    bool changed = false;
    for (int i = 0; i < B->nbeams; ++i) {
        const BeamPtrs &op = B->last_ptrs[(size_t)i];
        if (x[i] != op.x || taps[i] != op.h || Y[i] != (void *)op.Y)
            changed = true;
    }
    if (changed) {
        // the staging buffer may still be read by an earlier copy
        if (B->launched && hipEventSynchronize(B->done) != hipSuccess)
            return pfb_internal_fail(PFB_E_HIP, "hipEventSynchronize");
        for (int i = 0; i < B->nbeams; ++i) {
            B->h_ptrs[i] = BeamPtrs{x[i], taps[i], reinterpret_cast<float2 *>(Y[i]), nullptr};
            B->last_ptrs[(size_t)i] = B->h_ptrs[i];
        }
        if (hipMemcpyAsync(B->d_ptrs, B->h_ptrs, sizeof(BeamPtrs) * (size_t)B->nbeams, hipMemcpyHostToDevice, st) !=
            hipSuccess)
            return pfb_internal_fail(PFB_E_HIP, "pointer table upload");
    }
    if (hipGraphLaunch(B->exec, st) != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "hipGraphLaunch");
    if (hipEventRecord(B->done, st) != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "batched completion record");
    B->launched = true;
    return PFB_OK;
}
