// Register-window FIR (fir_launch.h) for cf16 input.
#include "fir_launch.h"

namespace pfb {

hipError_t launch_fir_cf16(const FirArgs &a, int tp, int cpt, hipStream_t st)
{
    return launch_fir_dt<DT_CF16, false>(a, tp, cpt, st);
}

} // namespace pfb
