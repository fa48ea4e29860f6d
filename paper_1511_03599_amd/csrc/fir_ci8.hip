// Register-window FIR (fir_launch.h) for ci8 input, and its convert-per-use
// comparator.
#include "fir_launch.h"

namespace pfb {

hipError_t launch_fir_ci8(const FirArgs &a, int tp, int cpt, bool per_use, hipStream_t st)
{
    return per_use ? launch_fir_per_use_dt<DT_CI8>(a, tp, cpt, st) : launch_fir_dt<DT_CI8, false>(a, tp, cpt, st);
}

} // namespace pfb
