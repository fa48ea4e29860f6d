// Fused polyphase FIR + FFT: which shapes take it, and the launcher for each
// input type (the kernel is in fused_launch.h).
#include "fused_launch.h"

namespace pfb {

bool fused_supported(int dtype, int tp, int log2c)
{
    if (dtype < 0 || dtype > 3)
        return false;
    if (log2c < 8 || log2c > 10)
        return false;
    return tp == 4 || tp == 8 || tp == 16;
}

int fused_rows_per_chunk(int tp, int log2c)
{
    (void)tp;
    return fused_pipe_rows(log2c);
}

hipError_t launch_fused(const FusedArgs &a, int dtype, int tp, int log2c, hipStream_t st)
{
    switch (dtype) {
    case DT_C64: return launch_fused_dt<DT_C64>(a, tp, log2c, st);
    case DT_CI16: return launch_fused_ci16(a, tp, log2c, st);
    case DT_CI8: return launch_fused_ci8(a, tp, log2c, st);
    case DT_CF16: return launch_fused_cf16(a, tp, log2c, st);
    default: return hipErrorInvalidValue;
    }
}

} // namespace pfb
