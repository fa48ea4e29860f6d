// Register-window FIR kernel and its launcher, instantiated per input type
// in separate translation units (fir.hip for complex float32,
// fir_adjoint.hip for the reversed-tap adjoint, fir_ci16.hip, fir_ci8.hip,
// fir_cf16.hip) so that they compile in parallel. See fir.hip for the design.
#pragma once

#include "fir_device.h"
#include "launch.h"

namespace pfb {

template <int DT, int TP, int CPT, int D, bool REV, bool PER_USE = false>
__global__ __launch_bounds__(256, 2) void fir_kernel(FirArgs a)
{
    // Consecutive waves take consecutive channel chunks, then consecutive
    // tiles, so the waves resident at any time sweep one narrow band of rows.
    // Up to 16 taps the task index is made scalar, so that row and address
    // bases stay in scalar registers (above that the longer windows
    // allocate better from the vector form).
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (TP <= 16 ? wave_id_uniform() : wave_id());
    const int64_t total = (int64_t)a.B * a.n_tiles * a.n_cchunks;
    if (gw >= total)
        return;
    fir_wave_task<DT, TP, CPT, D, REV, true, PER_USE>(a, gw);
}

template <int DT, int TP, int CPT, bool REV, bool PER_USE = false>
hipError_t launch_fir_t(const FirArgs &a, hipStream_t st)
{
    constexpr int D = fir_prefetch(TP);
    const int64_t total = (int64_t)a.B * a.n_tiles * a.n_cchunks;
    const int64_t blocks = (total + 3) / 4;
    if (blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((fir_kernel<DT, TP, CPT, D, REV, PER_USE>), dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int DT, bool REV>
hipError_t launch_fir_dt(const FirArgs &a, int tp, int cpt, hipStream_t st)
{
#define PFB_FIR_CASE(TPV)                                                                                    \
    case TPV:                                                                                                \
        return cpt == 2 ? launch_fir_t<DT, TPV, 2, REV>(a, st) : launch_fir_t<DT, TPV, 1, REV>(a, st);
    // two channels per lane only where the doubled window still fits in
    // registers; the larger windows run one channel per lane
    switch (tp) {
        PFB_FIR_CASE(4)
        PFB_FIR_CASE(8)
        PFB_FIR_CASE(16)
    case 32:
        return launch_fir_t<DT, 32, 1, REV>(a, st);
    case 64:
        return launch_fir_t<DT, 64, 1, REV>(a, st);
    default:
        return hipErrorInvalidValue;
    }
#undef PFB_FIR_CASE
}

// The convert-per-use comparator (fir_wave_task, PER_USE) for one
// low-precision input type, padded taps <= 16.
template <int DT> hipError_t launch_fir_per_use_dt(const FirArgs &a, int tp, int cpt, hipStream_t st)
{
#define PFB_FIR_PU_CASE(TPV)                                                                                 \
    case TPV:                                                                                                \
        return cpt == 2 ? launch_fir_t<DT, TPV, 2, false, true>(a, st) : launch_fir_t<DT, TPV, 1, false, true>(a, st);
    switch (tp) {
        PFB_FIR_PU_CASE(4)
        PFB_FIR_PU_CASE(8)
        PFB_FIR_PU_CASE(16)
    default:
        return hipErrorInvalidValue;
    }
#undef PFB_FIR_PU_CASE
}

} // namespace pfb
