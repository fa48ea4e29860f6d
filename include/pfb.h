/*
 * pfb.h -- C ABI of the MI355X (gfx950) polyphase filter bank library.
 *
 * The library computes the two-step polyphase filter bank of Sec. 2:
 *
 *   raw spectra --FIR--> filtered spectra --DFT--> frequency spectra
 *
 * Data model (Sec. 2 and Sec. 3.1). A stream of complex samples is split into
 * spectra of C channels, contiguous in channels. Complex values are stored as
 * interleaved (re, im) pairs of the element type. For one plan:
 *
 *   x     [batch][spectra + taps - 1][channels]  complex, element type `dtype`
 *   taps  [taps][channels]                       float32, h[t*C + c]
 *   y     [batch][spectra][channels]             complex float32 (filtered)
 *   Y     [batch][spectra][channels]             complex float32 (frequency)
 *
 * FIR (Sec. 3.2, Algorithm 1), in "valid" mode (S filtered spectra from
 * S+T-1 raw spectra, no zero padding, no state between calls):
 *   y[b][s][c] = sum_{t=0}^{T-1} h[t*C + c] * x[b][s+t][c]
 * accumulated in float32 in ascending t. Coefficients are real, unique per
 * (tap, channel) and float32 for every input type (Sec. 3.1).
 * DFT (Sec. 2, Eq. (2)), per filtered spectrum, unnormalised, bins in natural
 * order 0..C-1:
 *   Y[b][s][m] = sum_{n=0}^{C-1} y[b][s][n] * exp(-2 pi i n m / C)
 *
 * Input element types (Sec. 3.1: 32-, 16- and 8-bit input): complex float32,
 * complex int16, complex int8 (signed) and complex float16. Each sample is
 * converted to float32 once, in registers; outputs are always complex
 * float32 (Sec. 3.1).
 *
 * Memory. Every array argument is a DEVICE pointer owned by the caller, dense
 * in the layout above and aligned to 16 bytes. The library never frees or
 * keeps caller memory beyond a call. A plan owns its twiddle tables, tile
 * tables, workspace and captured graphs; all of them are allocated when the
 * plan is created, so the execute and backward calls allocate nothing.
 *
 * Streams. `stream` is a hipStream_t passed as void* (NULL = the default
 * stream). All work of a call is enqueued on that stream in order; the calls
 * return once the work is enqueued. A plan must not be used by two streams at
 * the same time, and must be destroyed only after its work has completed.
 *
 * Errors. Every entry point returns a pfb_status. Arguments are validated on
 * the host before anything is enqueued; a failed validation returns
 * PFB_E_INVALID or PFB_E_UNSUPPORTED and enqueues nothing. Launch failures
 * return PFB_E_HIP. Faults that happen on the device surface at the caller's
 * next synchronisation. The library never aborts the process and no C++
 * exception crosses this interface. pfb_last_error() returns a description of
 * the last failure on the calling thread.
 */
#ifndef PFB_H
#define PFB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PFB_OK = 0,
    PFB_E_INVALID = 1,     /* bad argument: null pointer, size, alignment   */
    PFB_E_UNSUPPORTED = 2, /* valid request outside what the library does   */
    PFB_E_NOMEM = 3,       /* device or host allocation failed              */
    PFB_E_HIP = 4,         /* a HIP runtime call or kernel launch failed    */
    PFB_E_STATE = 5        /* plan of the wrong kind for this call          */
} pfb_status;

typedef enum {
    PFB_C64 = 0,  /* complex float32: 8 bytes per sample                */
    PFB_CI16 = 1, /* complex int16:   4 bytes per sample                */
    PFB_CI8 = 2,  /* complex int8:    2 bytes per sample                */
    PFB_CF16 = 3  /* complex float16: 4 bytes per sample                */
} pfb_dtype;

/* Plan flags. */
enum {
    PFB_FIR_ONLY = 1u,      /* stop after the FIR: y is the output, Y unused  */
    PFB_NO_FUSE = 4u,       /* run FIR and FFT as separate passes             */
    PFB_PLAIN = 8u,         /* the untuned single-stream comparator: one FIR
                               launch over the whole stream into a workspace,
                               then one FFT launch; no fusion, no chunking   */
    PFB_STREAMING = 16u,    /* the plan carries the last T-1 raw spectra of
                               each stream from one pfb_execute_stream call
                               to the next (real-time use, Sec. 5)          */
    PFB_CONVERT_PER_USE = 32u /* comparator for the conversion study of
                               Sec. 4.2: the FIR converts each 8- or 16-bit
                               sample at every tap that uses it (2T
                               conversions per output, as a kernel that
                               re-reads its window from a cache or shared
                               memory does) instead of once when it is
                               loaded. Same results. Needs an int16, int8 or
                               float16 plan with T <= 16; forces the split
                               path. PFB_E_UNSUPPORTED otherwise.          */
};

/* Limits. */
#define PFB_MAX_TAPS 1024        /* forward and FIR-only plans            */
#define PFB_MAX_TAPS_WINDOW 64   /* register-window kernels; pfb_backward
                                    and batched plans accept up to this   */
#define PFB_MIN_FFT_CHANNELS 32
#define PFB_MAX_FFT_CHANNELS 8192

/* One filter-bank problem. `spectra` counts filtered (output) spectra; the
 * input has spectra + taps - 1 raw spectra per stream. */
typedef struct {
    int32_t channels;  /* C >= 1; unless FIR_ONLY, C in [32, 8192] and of the
                          form 2^a 3^b 5^c 7^d (powers of two take the fused
                          paths, other sizes the split path with a
                          mixed-radix transform)                            */
    int32_t taps;      /* T in [1, PFB_MAX_TAPS]; above PFB_MAX_TAPS_WINDOW the
                          forward runs the long-tap FIR on the split path  */
    int64_t spectra;   /* S >= 1                                               */
    int32_t batch;     /* B >= 1 independent streams                           */
    int32_t dtype;     /* a pfb_dtype                                          */
    uint32_t flags;    /* PFB_* flags                                          */
} pfb_desc;

typedef struct pfb_plan pfb_plan;

/* Description of what a plan will run, for reports and tests. */
typedef struct {
    int32_t path;          /* 0 fused FIR+FFT, 1 split FIR then FFT, 2 FIR only */
    int32_t fir_rows;      /* filtered spectra per FIR tile (S_B)              */
    int32_t fir_cpt;       /* channels per thread in the FIR kernel            */
    int32_t padded_taps;   /* taps rounded up to the kernel's template size    */
    int64_t workspace_bytes;
    int64_t chunk_rows;    /* spectra per FIR/FFT chunk on the split path      */
    int32_t backward_fused;/* pfb_backward runs: 0 the split adjoint (inverse
                              FFT, reversed-tap FIR, tap-gradient pass),
                              1 the fused adjoint kernel, 2 its
                              wave-specialised form (same results)          */
    int32_t fused_ws;      /* 1 if the fused forward runs its wave-specialised
                              form (same results as the single-role kernel)  */
    int32_t backward_rows; /* sample-gradient rows per adjoint tile (fused
                              adjoint) or per adjoint FIR tile (split)      */
} pfb_plan_info;

/*
 * Create a plan for one problem (all streams share C, T, S and the taps).
 * Validates the descriptor, builds the FP64-derived twiddle table and
 * allocates the workspace on the current HIP device.
 * out: receives the plan (set to NULL on failure).
 */
pfb_status pfb_plan_create(const pfb_desc *desc, pfb_plan **out);

/*
 * Forward filter bank (Sec. 2 scheme).
 *   x     device, [B][S+T-1][C] samples of the plan's dtype
 *   taps  device, [T][C] float32
 *   y     device, [B][S][C] complex float32, or NULL. When non-NULL the
 *         filtered spectra are written there too (this forces the split
 *         path). With PFB_FIR_ONLY, y is required and Y is ignored.
 *   Y     device, [B][S][C] complex float32 (required unless FIR_ONLY)
 * Outputs are overwritten. Inputs are not modified.
 */
pfb_status pfb_execute(pfb_plan *plan, const void *x, const float *taps, void *y, void *Y,
                       void *stream);

/*
 * Streaming forward filter bank (plans created with PFB_STREAMING): the
 * streams continue across calls, as if every call's new raw spectra were
 * appended to one long input. Output s of a call is the filter bank of Alg. 1
 * and Eq. (2) over the T raw spectra ending at its new raw spectrum s, the
 * first T-1 of which may come from earlier calls (zeros before the first
 * call or after pfb_stream_reset).
 *   xbuf  device, [B][S+T-1][C] samples of the plan's dtype: per stream, the
 *         last S rows hold the call's S new raw spectra and the first T-1
 *         rows are headroom that the library overwrites with the carried
 *         spectra (so the new data are never copied). The caller may reuse
 *         the same buffer on every call.
 *   taps, y, Y  as for pfb_execute (S filtered / frequency spectra per call).
 * After the call the plan keeps the last T-1 rows of xbuf per stream.
 * Calls on one plan must be ordered (same stream, or synchronised).
 * Errors: PFB_E_STATE for a plan without PFB_STREAMING; otherwise those of
 * pfb_execute.
 */
pfb_status pfb_execute_stream(pfb_plan *plan, void *xbuf, const float *taps, void *y, void *Y,
                              void *stream);

/* Zero the carried spectra of a streaming plan (on `stream`). */
pfb_status pfb_stream_reset(pfb_plan *plan, void *stream);

/*
 * Polarisation-interleaved sub-band layout (as in the VEGAS spectrometer the
 * paper compares with, Sec. 5): every raw spectrum holds `subbands`
 * sub-bands of `channels` channels, each channel 2 interleaved complex
 * polarisations: x [spectra+taps-1][subbands][channels][2] of `dtype`. The
 * plan runs, for every sub-band and polarisation, the filter bank of Alg. 1
 * and Eq. (2) over that sub-band's channels with the same C_V-channel taps:
 * the FIR treats all 2*channels*subbands columns as independent channels
 * (the mapping C = 2 C_V N_sub of Sec. 5), and the transform reads each
 * polarisation of each sub-band with element stride 2.
 *   channels  C_V, a power of two in [32, 8192]; subbands >= 1; taps as for
 *             pfb_plan_create (T <= PFB_MAX_TAPS); dtype any pfb_dtype.
 *   taps      device, [T][channels] float32 (replicated by the library)
 *   Y         device, [spectra][subbands][channels][2] complex float32:
 *             bin k of polarisation p of sub-band b at Y[s][b][k][p].
 * The plan owns a filtered-spectra workspace (spectra*2*channels*subbands
 * complex values) and the replicated taps. pfb_execute/pfb_backward reject
 * these plans (PFB_E_STATE).
 */
pfb_status pfb_plan_create_vegas(int32_t channels, int32_t subbands, int32_t taps, int64_t spectra,
                                 int32_t dtype, pfb_plan **out);
pfb_status pfb_execute_vegas(pfb_plan *plan, const void *x, const float *taps, void *Y, void *stream);

/*
 * Adjoint (backward) of the forward filter bank for a real loss, given
 * gY = dL/dRe(Y) + i dL/dIm(Y) (the frequency-spectra gradient):
 *   gy[b][s][c] = sum_m gY[b][s][m] exp(+2 pi i m c / C)   (adjoint of Eq. (2))
 *   gx[b][p][c] = sum_{t: 0 <= p-t < S} h[t*C+c] gy[b][p-t][c]  (adjoint of Alg. 1)
 *   gh[t*C+c]   = sum_b sum_s Re(conj(gy[b][s][c]) x[b][s+t][c])
 *   x     device, [B][S+T-1][C] complex float32 (the plan's dtype must be C64)
 *   taps  device, [T][C] float32
 *   gY    device, [B][S][C] complex float32
 *   gx    device, [B][S+T-1][C] complex float32, or NULL to skip
 *   gh    device, [T][C] float32, or NULL to skip; summed over the batch and
 *         OVERWRITTEN (never accumulated into). Its reduction runs in a fixed
 *         order, so repeated calls give identical bits.
 * Requires a plan without FIR_ONLY.
 */
pfb_status pfb_backward(pfb_plan *plan, const void *x, const float *taps, const void *gY,
                        void *gx, float *gh, void *stream);

/* Size of the device scratch of pfb_backward_noalloc (bytes, one per GPU). */
#define PFB_NOALLOC_SCRATCH_BYTES (32u << 20)

/*
 * pfb_backward without a plan and without any allocation, for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. Same results as pfb_backward with a
 * plan of the same descriptor (the same fused adjoint kernel and fixed-order
 * tap-gradient reduction; its twiddle table is computed on the device by
 * every call, in FP64 rounded once, like the plan's host-built table).
 *   desc  C in {256, 512, 1024}, T <= 16, dtype PFB_C64, flags 0; other
 *         descriptors return PFB_E_UNSUPPORTED (or PFB_E_INVALID).
 *   x, taps, gY, gx, gh  as for pfb_backward (gx or gh may be NULL).
 * The library keeps the twiddle table and the per-tile tap-gradient partials
 * in a device array of PFB_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends: batch * taps * channels * 4 bytes of partials must fit in it
 * (at C=1024, T=16: up to 511 streams); larger problems return
 * PFB_E_UNSUPPORTED before anything is enqueued. The call makes no hipMalloc,
 * hipFree or other allocating call. All calls on one GPU share its array:
 * calls that overlap on one GPU (different streams or threads) race; calls
 * ordered on one stream are safe.
 */
pfb_status pfb_backward_noalloc(const pfb_desc *desc, const void *x, const float *taps, const void *gY,
                                void *gx, float *gh, void *stream);

/*
 * Many independent beams with their own C, T, S (one stream each, complex
 * float32, C a power of two in [32, 8192], T <= PFB_MAX_TAPS_WINDOW) in one
 * persistent launch
 * per call, recorded into a HIP graph when the plan is created. Each beam's
 * result is the forward filter bank of its descriptor (Alg. 1 then Eq. (2)),
 * bit-identical to a separate single-beam plan.
 *   nbeams  >= 1; beams: host array of nbeams descriptors (batch must be 1,
 *           dtype C64; flags ignored)
 * The plan owns its tile table and one slot of filtered spectra per
 * persistent workgroup (about 1 MiB each with the default tile size, or the
 * tuned one from the cache named by PFB_TUNE_CACHE). Errors:
 * PFB_E_UNSUPPORTED for other dtypes or T > 64, PFB_E_NOMEM if the device
 * allocations fail.
 */
pfb_status pfb_plan_create_batched(int32_t nbeams, const pfb_desc *beams, pfb_plan **out);

/*
 * Execute a batched plan.
 *   x, taps, Y: HOST arrays of nbeams DEVICE pointers, beam i laid out as a
 *   single stream of its own descriptor. The pointer values are baked into
 *   the plan's graph on the first call; later calls with different pointers
 *   rebuild the device-side pointer table (no allocation).
 */
pfb_status pfb_execute_batched(pfb_plan *plan, const void *const *x, const float *const *taps,
                               void *const *Y, void *stream);

/*
 * Time the candidate tile configurations for one descriptor on the current
 * device (temporary buffers are allocated and freed inside this call) and
 * store the fastest in the tuning cache file `cache_path` (a small text file,
 * created or updated). Plans created afterwards read the cache named by the
 * PFB_TUNE_CACHE environment variable; a missing or unreadable cache means
 * built-in defaults.
 */
pfb_status pfb_tune(const pfb_desc *desc, const char *cache_path);

/*
 * Time the candidate tile sizes of a batched plan for this beam table (the
 * same descriptors pfb_plan_create_batched takes; temporary buffers for every
 * beam are allocated and freed inside this call) and append the fastest to
 * the tuning cache file `cache_path`, keyed by the device, the beam count and
 * the total sample count. Batched plans created afterwards read it from the
 * cache named by PFB_TUNE_CACHE.
 */
pfb_status pfb_tune_batched(int32_t nbeams, const pfb_desc *beams, const char *cache_path);

/* Report what a plan will run. */
pfb_status pfb_plan_get_info(const pfb_plan *plan, pfb_plan_info *info);

/* Release a plan and everything it owns. NULL is accepted. */
pfb_status pfb_plan_destroy(pfb_plan *plan);

/* Static description of a status code. */
const char *pfb_status_str(pfb_status status);

/* Description of the last failure on the calling thread ("" if none). */
const char *pfb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PFB_H */
