// Internal declarations shared by the C-ABI translation units: the tuning
// cache and the batched-plan module.
#pragma once

#include <string>

#include "../../include/pfb.h"

namespace pfb {

// One tuned configuration for a descriptor (arch, dtype, C, T, flags class).
struct TuneEntry {
    int path = -1;       // 0 fused, 1 split, -1 not set
    int fir_cpt = 0;     // FIR channels per thread
    int fir_sb = 0;      // FIR rows per tile
    int fused_sb = 0;    // fused rows per tile
    int fused_ws = -1;   // fused forward: 1 wave-specialised, 0 single-role, -1 not set
    int chunk_mib = 0;   // split-path chunk size
    int bwd_sb = 0;      // fused adjoint rows per tile
    int bwd_ws = -1;     // fused adjoint: 1 wave-specialised, 0 single-role, -1 not set
};

// Look the descriptor up in the cache file named by PFB_TUNE_CACHE. Returns
// false (and leaves *out untouched) when the variable is unset, the file is
// missing or unreadable, or has no entry for this descriptor.
bool tune_lookup(const pfb_desc &d, TuneEntry *out);

// While non-NULL on the calling thread, plans take this configuration instead
// of the cache (used by the tuner to time candidates).
void tune_set_override(const TuneEntry *e);

std::string device_arch_name();

// Batched plans: the tile size (KiB of filtered spectra per tile) for this
// beam table, from the thread's override, else the cache (lines
//   <arch> batched <nbeams> <total samples> tile_kib=<k>
// ), else the built-in default.
int batched_tile_kib(int32_t nbeams, const pfb_desc *beams);
void batched_tile_set_override(int kib); // 0 clears

// Built-in batched tile size: the tuner's choice on a 64-beam table of
// 128 - 8192 channels (256 KiB: 14.0 ms against 14.4 ms with 1 MiB tiles).
constexpr int BATCHED_TILE_KIB_DEFAULT = 256;

} // namespace pfb

struct Batched;
void batched_free(Batched *b);

pfb_status pfb_internal_fail(pfb_status st, const char *msg);
int pfb_internal_bwd_tile_rows(int64_t B, int64_t S, int T, int C, int cus);
pfb_status pfb_internal_validate(const pfb_desc *d, bool batched_beam);
pfb_plan *pfb_internal_new_plan();
void pfb_internal_set_batched(pfb_plan *p, Batched *b);
Batched *pfb_internal_get_batched(pfb_plan *p);
