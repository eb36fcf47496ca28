// Kernel launchers of libosc (defined in osc_kernels.hip).
#pragma once

#include "osc_internal.h"

namespace osc {

// mode: 0 = probabilities only, 1 = probabilities + histogram partials,
// 2 = histogram partials of given values, 3 = mode 1 with the events'
// histogram slots read from `bins` (launch_bin_slots) instead of computed
// from e_reco.  partial holds ntiles x (nbins + 2) FP64 entries, tile-major.
// mixed selects the FP32-mixed tier (FP64 eigenvalues and phases, FP32
// sine/cosine and amplitude assembly).  ev_begin / ev_end (optional,
// created by the caller) receive the kernel's own begin and end times.
hipError_t launch_tiles(int mode, bool write_p, bool mixed, const SetConsts& sc,
                        const PathConsts& pc, const BinConsts& bc, int64_t n,
                        const double* e_true, const uint8_t* flags, const double* weight,
                        const double* e_reco, const uint16_t* bins, const double* value,
                        double* p_out, double* partial, hipStream_t stream,
                        hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);

// The cached histogram slot of each of n events (reco energies e_reco,
// binning bc) for mode 3: out holds n 16-bit entries.
hipError_t launch_bin_slots(int64_t n, const double* e_reco, const BinConsts& bc, uint16_t* out,
                            hipStream_t stream);

// launch_tiles with P through a layered path (FP64; mode 0 or 1).
hipError_t launch_layered_tiles(int mode, bool write_p, const SetConsts& sc,
                                const LayerPath& lp, const BinConsts& bc, int64_t n,
                                const double* e_true, const uint8_t* flags, const double* weight,
                                const double* e_reco, double* p_out, double* partial,
                                hipStream_t stream, hipEvent_t ev_begin = nullptr,
                                hipEvent_t ev_end = nullptr);

// The levels of the histogram merge for n_samples samples of tiles[s]
// tiles each (per parameter set), and the scratch strides they need.  A
// fixed-capacity value: planning a merge allocates nothing.  A sample has
// at most kMaxEvents / kTileEvents = 2^22 tiles, which two levels of
// kMergeChunkRows = 2^14 rows reduce to one.
constexpr int kMaxMergeLevels = 3;
struct MergePlan {
    int nbt = 0;
    int n_samples = 0;
    int n_levels = 0;
    MergeLevel levels[kMaxMergeLevels];
    int64_t tile_set_stride = 0;   // elements of tile results per set
    int64_t level_set_stride = 0;  // elements of each of the two level buffers per set
};

MergePlan plan_merge(const int64_t* tiles, int n_samples, int nbt);

// Scratch (bytes) for the tile results and the level buffers of n_sets sets.
size_t merge_scratch_bytes(const MergePlan& p, int64_t n_sets);

// Runs the merge levels on `stream`: tile results at the start of scratch,
// histograms hist_out[set][sample][bin].
hipError_t launch_merge(const MergePlan& p, int64_t n_sets, double* scratch, double* hist_out,
                        hipStream_t stream);

// -2 ln L (Eq. 2, Poisson per regular bin, mu = scale * hist) of n_hist
// histograms (nbins + 2 entries each) against data rows (nbins entries;
// histogram k uses row k % n_data).
hipError_t launch_poisson_nll(const double* hist, int64_t n_hist, double scale,
                              const double* data, int64_t n_data, int nbins, double* out,
                              hipStream_t stream);

// Adds to bad[0] the events of the sample whose true energy is not finite
// and positive and to bad[1] those with an invalid flag byte.
hipError_t launch_validate_sample(int64_t n, const double* e_true, const uint8_t* flags,
                                  unsigned long long* bad, hipStream_t stream);

// Resident one-wave blocks per CU of the per-event kernel of `mode` for
// histograms of nbins bins.
hipError_t occupancy(int mode, int nbins, int* blocks_per_cu);

// Raises the dynamic-LDS limit of the histogram kernels.
hipError_t set_kernel_attributes(size_t max_dyn_lds);

}  // namespace osc
