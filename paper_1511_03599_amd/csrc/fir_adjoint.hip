// Register-window FIR (fir_launch.h) with reversed taps: the adjoint of the
// FIR of Algorithm 1 in the samples, over complex float32 gradients.
#include "fir_launch.h"

namespace pfb {

hipError_t launch_fir_adjoint(const FirArgs &a, int tp, int cpt, hipStream_t st)
{
    return launch_fir_dt<DT_C64, true>(a, tp, cpt, st);
}

} // namespace pfb
