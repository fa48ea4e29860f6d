// Batched multi-beam plans (placeholder until the persistent kernel lands).
#include <hip/hip_runtime.h>

#include "tune.h"

struct Batched {
    int nbeams = 0;
};

void batched_free(Batched *b) { delete b; }

extern "C" pfb_status pfb_plan_create_batched(int32_t nbeams, const pfb_desc *beams, pfb_plan **out)
{
    (void)nbeams;
    (void)beams;
    if (out)
        *out = nullptr;
    return pfb_internal_fail(PFB_E_UNSUPPORTED, "batched plans are not built yet");
}

extern "C" pfb_status pfb_execute_batched(pfb_plan *p, const void *const *x, const float *const *taps,
                                          void *const *Y, void *stream)
{
    (void)p;
    (void)x;
    (void)taps;
    (void)Y;
    (void)stream;
    return pfb_internal_fail(PFB_E_UNSUPPORTED, "batched plans are not built yet");
}

