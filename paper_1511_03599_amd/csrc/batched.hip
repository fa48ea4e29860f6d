// Batched multi-beam filter bank: many independent beams, each with its own
// C, T and S, processed by ONE persistent kernel launch per call.
//
// Work is a table of tiles built on the host when the plan is created:
//   FIR tile: up to 8 wave tasks of one beam (a wave task is 64*CPT channels
//             x 32 filtered spectra, the register-window FIR of fir.hip),
//             writing the beam's filtered spectra into the plan's workspace;
//   FFT tile: the C-point transforms of one group of rows of one beam,
//             reading the filtered spectra back and writing the frequency
//             spectra.
// Rows of a beam are split into groups (about 2 MiB of filtered spectra each);
// a group's FFT tile may start once all of its FIR tiles have finished. The
// tile table is ordered beam by beam, largest beams first, with each group's
// FFT tile placed after the FIR tiles of the NEXT group, so a transform
// rarely waits and reads its rows back while they are still cached.
//
// The persistent workgroups take tiles in table order from an atomic counter.
// A FIR tile publishes its completion with a release increment of its
// group's counter; an FFT tile waits (bounded spin, acquire) for that counter
// to reach the group's FIR tile count. Every tile a wait can depend on has a
// smaller table index, so it was taken earlier by a workgroup that is already
// running and never waits itself: the waits always end. A wait that exceeds
// its bound (a library bug) raises an error flag instead of hanging.
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

constexpr int BT_THREADS = 512;          // threads per persistent workgroup
constexpr int BT_WAVES = BT_THREADS / 64;
constexpr int BT_TASK_ROWS = 32;         // filtered spectra per FIR wave task
constexpr int BT_LDS = 8704;             // float2: the largest transform round

struct BeamInfo {
    float2 *yws;           // filtered spectra workspace of this beam [S][C]
    const float2 *tw;      // twiddles for C
    int C, T, TP, log2c, cpt;
    int n_cchunks, n_tiles;
    int64_t S;
};

struct BeamPtrs {
    const void *x;
    const float *h;
    float2 *Y;
    const void *pad;       // keeps the entry 32 bytes
};

struct TileDesc {
    int kind;              // 0 FIR, 1 FFT
    int beam;
    int64_t first;         // FIR: first wave task; FFT: first row
    int count;             // FIR: wave tasks (<= 8); FFT: rows
    int group;             // dependency counter
    int need;              // FFT: FIR tiles of the group
    int pad;
};

struct BatchedArgs {
    const BeamInfo *beams;
    const BeamPtrs *ptrs;
    const TileDesc *tiles;
    int *queue;            // next tile to take
    int *deps;             // per-group finished FIR tiles
    int *err;              // set when a wait exceeds its bound
    int ntiles;
    int ngroups;
    long long spin_limit;
};

__global__ __launch_bounds__(256) void batched_reset_kernel(BatchedArgs a)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i == 0) {
        *a.queue = 0;
        *a.err = 0;
    }
    for (int g = i; g < a.ngroups; g += (int)(gridDim.x * blockDim.x))
        a.deps[g] = 0;
}

template <int TP, int CPT>
__device__ __forceinline__ void batched_fir(const BeamInfo &bm, const BeamPtrs &bp, int64_t task)
{
    FirArgs f{};
    f.x = bp.x;
    f.h = bp.h;
    f.y = bm.yws;
    f.C = bm.C;
    f.T = bm.T;
    f.B = 1;
    f.SB = BT_TASK_ROWS;
    f.n_tiles = bm.n_tiles;
    f.n_cchunks = bm.n_cchunks;
    f.in_rows = bm.S + bm.T - 1;
    f.in_bstride = 0;
    f.shift = TP - bm.T;
    f.out_first = 0;
    f.out_count = bm.S;
    f.y_bstride = 0;
    fir_wave_task<DT_C64, TP, CPT, 8, false>(f, task);
}

// The transform of each size is a separate (not inlined) device function:
// merged into one body with the other sizes and the FIR variants, the
// transforms spill heavily. The call costs one save and restore of the
// callee-saved registers per tile.
template <int LOG2C>
__device__ __noinline__ void batched_fft(const BeamInfo &bm, const BeamPtrs &bp, int64_t row0, int nrows,
                                         float2 *lds)
{
    constexpr int C = 1 << LOG2C;
    constexpr int G = FftLanes<LOG2C>::G;
    constexpr int F = BT_THREADS / G; // rows per round
    using S = FftShape<LOG2C, G>;
    static_assert(F * S::PADDED <= BT_LDS, "LDS");
    const int gid = (int)threadIdx.x / G;
    const int lane = (int)threadIdx.x % G;
    for (int base = 0; base < nrows; base += F) {
        const int r = base + gid;
        const bool valid = r < nrows;
        // a group past the last row repeats the last row without storing it
        const int rr = valid ? r : nrows - 1;
        const float2 *in = bm.yws + (row0 + rr) * C;
        float2 *out = bp.Y + (row0 + rr) * C;
        if constexpr (F == 1) {
            fft_run<LOG2C, G, false, false>(
                lane, lds, bm.tw, [&](int idx) { return in[idx]; },
                [&](int idx, float2 v) { store_nt(out + idx, v); });
        } else if constexpr (G > 64) {
            // transforms span several waves and synchronise the block, so
            // every group runs the passes
            fft_run<LOG2C, G, false, false>(
                lane, lds + gid * S::PADDED, bm.tw, [&](int idx) { return in[idx]; },
                [&](int idx, float2 v) {
                    if (valid)
                        store_nt(out + idx, v);
                });
        } else if (valid) {
            fft_run<LOG2C, G, false, false>(
                lane, lds + gid * S::PADDED, bm.tw, [&](int idx) { return in[idx]; },
                [&](int idx, float2 v) { store_nt(out + idx, v); });
        }
        __syncthreads(); // the LDS rows are reused by the next round
    }
}

__global__ __launch_bounds__(BT_THREADS) void batched_kernel(BatchedArgs a)
{
    __shared__ float2 lds[BT_LDS];
    __shared__ int s_tile;
    for (;;) {
        if (threadIdx.x == 0)
            s_tile = __hip_atomic_fetch_add(a.queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();
        if (t >= a.ntiles)
            break;
        const TileDesc td = a.tiles[t];
        const BeamInfo bm = a.beams[td.beam];
        const BeamPtrs bp = a.ptrs[td.beam];
        if (td.kind == 0) {
            const int w = wave_id();
            if (w < td.count) {
                const int64_t task = td.first + w;
                switch (bm.TP) {
                case 4: batched_fir<4, 1>(bm, bp, task); break;
                case 8: batched_fir<8, 1>(bm, bp, task); break;
                case 16: batched_fir<16, 1>(bm, bp, task); break;
                default: batched_fir<32, 1>(bm, bp, task); break;
                }
            }
            // publish: every thread's stores are made visible at device
            // scope before the group counter moves
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_fetch_add(a.deps + td.group, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (threadIdx.x == 0) {
                long long spins = 0;
                while (__hip_atomic_load(a.deps + td.group, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < td.need) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > a.spin_limit) {
                        __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                }
            }
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            switch (bm.log2c) {
            case 5: batched_fft<5>(bm, bp, td.first, td.count, lds); break;
            case 6: batched_fft<6>(bm, bp, td.first, td.count, lds); break;
            case 7: batched_fft<7>(bm, bp, td.first, td.count, lds); break;
            case 8: batched_fft<8>(bm, bp, td.first, td.count, lds); break;
            case 9: batched_fft<9>(bm, bp, td.first, td.count, lds); break;
            case 10: batched_fft<10>(bm, bp, td.first, td.count, lds); break;
            case 11: batched_fft<11>(bm, bp, td.first, td.count, lds); break;
            case 12: batched_fft<12>(bm, bp, td.first, td.count, lds); break;
            default: batched_fft<13>(bm, bp, td.first, td.count, lds); break;
            }
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
    int *d_counters = nullptr;          // [0] queue, [1] err, [2..] deps
    int *h_err = nullptr;               // pinned copy of the error flag
    std::vector<void *> allocs;         // workspaces and twiddle tables
    int ntiles = 0, ngroups = 0;
    int grid = 0;
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
    for (void *p : {(void *)b->d_info, (void *)b->d_ptrs, (void *)b->d_tiles, (void *)b->d_counters})
        if (p)
            (void)hipFree(p);
    if (b->h_ptrs)
        (void)hipHostFree(b->h_ptrs);
    if (b->h_err)
        (void)hipHostFree(b->h_err);
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

static pfb_status build_batched(int32_t nbeams, const pfb_desc *beams, Batched *B)
{
    B->nbeams = nbeams;
    B->descs.assign(beams, beams + nbeams);
    B->info.resize((size_t)nbeams);
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
        // one channel per lane: the persistent kernel's register budget is
        // the maximum over every tap count and transform size it serves
        bi.cpt = 1;
        bi.n_cchunks = (d.channels + 64 * bi.cpt - 1) / (64 * bi.cpt);
        bi.n_tiles = (int)((d.spectra + BT_TASK_ROWS - 1) / BT_TASK_ROWS);
        bi.S = d.spectra;
        if (!tw_by_log2c[bi.log2c]) {
            pfb_status st = twiddle_table(bi.log2c, &tw_by_log2c[bi.log2c]);
            if (st != PFB_OK)
                return st;
            B->allocs.push_back(tw_by_log2c[bi.log2c]);
        }
        bi.tw = tw_by_log2c[bi.log2c];
        void *ws = nullptr;
        if (hipMalloc(&ws, (size_t)d.spectra * d.channels * 8) != hipSuccess)
            return pfb_internal_fail(PFB_E_NOMEM, "hipMalloc(batched filtered-spectra workspace)");
        B->allocs.push_back(ws);
        bi.yws = reinterpret_cast<float2 *>(ws);
    }

    // tile table: beams largest first; per beam, groups of rows
    std::vector<int> order((size_t)nbeams);
    for (int i = 0; i < nbeams; ++i)
        order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return beams[a].spectra * beams[a].channels > beams[b].spectra * beams[b].channels;
    });
    std::vector<TileDesc> tiles;
    int ngroups = 0;
    for (int bidx : order) {
        const BeamInfo &bi = B->info[(size_t)bidx];
        // rows per group: about 2 MiB of filtered spectra, a multiple of the
        // FIR task height
        int64_t rg = ((int64_t)2 << 20) / ((int64_t)bi.C * 8);
        rg = std::max<int64_t>(BT_TASK_ROWS, rg / BT_TASK_ROWS * BT_TASK_ROWS);
        const int64_t ngr = (bi.S + rg - 1) / rg;
        std::vector<TileDesc> pending_fft;
        for (int64_t g = 0; g < ngr; ++g) {
            const int64_t r0 = g * rg;
            const int64_t nr = std::min<int64_t>(rg, bi.S - r0);
            const int64_t t0 = r0 / BT_TASK_ROWS, t1 = (r0 + nr + BT_TASK_ROWS - 1) / BT_TASK_ROWS;
            const int64_t task0 = t0 * bi.n_cchunks, task1 = t1 * bi.n_cchunks;
            const int gid = ngroups++;
            int nfir = 0;
            for (int64_t k = task0; k < task1; k += BT_WAVES) {
                TileDesc t{};
                t.kind = 0;
                t.beam = bidx;
                t.first = k;
                t.count = (int)std::min<int64_t>(BT_WAVES, task1 - k);
                t.group = gid;
                tiles.push_back(t);
                ++nfir;
            }
            // transforms of the previous group follow this group's FIR tiles
            for (const TileDesc &f : pending_fft)
                tiles.push_back(f);
            pending_fft.clear();
            TileDesc f{};
            f.kind = 1;
            f.beam = bidx;
            f.first = r0;
            f.count = (int)nr;
            f.group = gid;
            f.need = nfir;
            pending_fft.push_back(f);
        }
        for (const TileDesc &f : pending_fft)
            tiles.push_back(f);
    }
    B->ntiles = (int)tiles.size();
    B->ngroups = ngroups;

    if (hipMalloc(&B->d_info, sizeof(BeamInfo) * (size_t)nbeams) != hipSuccess ||
        hipMalloc(&B->d_ptrs, sizeof(BeamPtrs) * (size_t)nbeams) != hipSuccess ||
        hipMalloc(&B->d_tiles, sizeof(TileDesc) * tiles.size()) != hipSuccess ||
        hipMalloc(&B->d_counters, sizeof(int) * (size_t)(ngroups + 2)) != hipSuccess ||
        hipHostMalloc(&B->h_ptrs, sizeof(BeamPtrs) * (size_t)nbeams, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&B->h_err, sizeof(int), hipHostMallocDefault) != hipSuccess)
        return pfb_internal_fail(PFB_E_NOMEM, "batched plan tables");
    *B->h_err = 0;
    if (hipMemcpy(B->d_info, B->info.data(), sizeof(BeamInfo) * (size_t)nbeams, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(B->d_tiles, tiles.data(), sizeof(TileDesc) * tiles.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(B->d_ptrs, 0, sizeof(BeamPtrs) * (size_t)nbeams) != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "batched plan upload");
    B->last_ptrs.assign((size_t)nbeams, BeamPtrs{nullptr, nullptr, nullptr, nullptr});

    int dev = 0, cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        cus = prop.multiProcessorCount;
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_kernel, BT_THREADS, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    B->grid = std::min(cus * per_cu, B->ntiles);

    BatchedArgs &a = B->args;
    a.beams = B->d_info;
    a.ptrs = B->d_ptrs;
    a.tiles = B->d_tiles;
    a.queue = B->d_counters;
    a.err = B->d_counters + 1;
    a.deps = B->d_counters + 2;
    a.ntiles = B->ntiles;
    a.ngroups = ngroups;
    a.spin_limit = 1LL << 26;

    // graph: reset the counters, then the persistent kernel
    if (hipGraphCreate(&B->graph, 0) != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "hipGraphCreate");
    void *kargs[] = {&B->args};
    hipKernelNodeParams rp{};
    rp.func = reinterpret_cast<void *>(batched_reset_kernel);
    rp.gridDim = dim3((unsigned)std::max(1, std::min(1024, (ngroups + 255) / 256)));
    rp.blockDim = dim3(256);
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
        if (beams[i].taps > 32)
            return pfb_internal_fail(PFB_E_UNSUPPORTED, "batched beams support up to 32 taps");
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
    // report a wait that overran its bound in an earlier call
    if (B->launched && hipEventQuery(B->done) == hipSuccess && *B->h_err) {
        *B->h_err = 0;
        return pfb_internal_fail(PFB_E_HIP, "a batched dependency wait exceeded its bound in an earlier call");
    }
    bool changed = false;
    for (int i = 0; i < B->nbeams; ++i) {
        const BeamPtrs np{x[i], taps[i], reinterpret_cast<float2 *>(Y[i]), nullptr};
        const BeamPtrs &op = B->last_ptrs[(size_t)i];
        if (np.x != op.x || np.h != op.h || np.Y != op.Y)
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
    if (hipMemcpyAsync(B->h_err, B->d_counters + 1, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipEventRecord(B->done, st) != hipSuccess)
        return pfb_internal_fail(PFB_E_HIP, "batched completion record");
    B->launched = true;
    return PFB_OK;
}
