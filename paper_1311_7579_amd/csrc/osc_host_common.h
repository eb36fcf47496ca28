// Host-side helpers of libosc shared by the plain entry points and the
// batched form (defined in osc_host.hip).
#pragma once

#include "../../include/osc.h"
#include "osc_internal.h"

namespace osc {
namespace host {

// Parameter-only quantities of one set (mixing matrix, flavour-basis
// vacuum mass matrix and its square, cubic constants, channel table).
SetConsts set_consts(const osc_params& p);
// sin / cos of k pi / 32 rounded to FP64 (from long double sinl / cosl).
const SinCosTable& sincos_table();
PathConsts path_consts(const osc_sample* s);
BinConsts bin_consts(const osc_binning* b);
bool sample_ok(const osc_sample* s, bool needs_hist_inputs);
bool binning_ok(const osc_ctx* ctx, const osc_binning* b);
int ctx_device(const osc_ctx* ctx);
// Copy of parameter set `set` of the context; false when out of range.
bool ctx_set(osc_ctx* ctx, int32_t set, SetConsts* out);

// Device scratch one osc_fill_pdf-style histogram of n events needs.
size_t fill_scratch_bytes(int64_t n, int nbins);

// Enqueues the per-event kernel and the merge of one histogram on `stream`
// with caller-provided scratch (fill_scratch_bytes).  With `bins` (the
// sample's cached histogram slots for this binning, enqueue_bin_slots) the
// reco energies are not read.  Arguments are assumed validated.
hipError_t enqueue_fill(const SetConsts& sc, const osc_sample* sample, const uint16_t* bins,
                        const osc_binning* binning, bool mixed, double* scratch,
                        double* hist_out, double* p_out, hipStream_t stream);

// Enqueues the computation of the sample's cached histogram slots (n
// 16-bit entries at `bins`) for `binning` on `stream`.
hipError_t enqueue_bin_slots(const osc_sample* sample, const osc_binning* binning,
                             uint16_t* bins, hipStream_t stream);

}  // namespace host
}  // namespace osc
