// Fused FIR + FFT (fused_launch.h) for ci16 input.
#include "fused_launch.h"

namespace pfb {

hipError_t launch_fused_ci16(const FusedArgs &a, int tp, int log2c, hipStream_t st)
{
    return launch_fused_dt<DT_CI16>(a, tp, log2c, st);
}

} // namespace pfb
