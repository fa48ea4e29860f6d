// Fused FIR + FFT (fused_launch.h) for ci8 input.
#include "fused_launch.h"

namespace pfb {

hipError_t launch_fused_ci8(const FusedArgs &a, int tp, int log2c, hipStream_t st)
{
    return launch_fused_dt<DT_CI8>(a, tp, log2c, st);
}

} // namespace pfb
