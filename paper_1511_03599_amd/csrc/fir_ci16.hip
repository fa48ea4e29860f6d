// Register-window FIR (fir_launch.h) for ci16 input.
#include "fir_launch.h"

namespace pfb {

hipError_t launch_fir_ci16(const FirArgs &a, int tp, int cpt, hipStream_t st)
{
    return launch_fir_dt<DT_CI16, false>(a, tp, cpt, st);
}

} // namespace pfb
