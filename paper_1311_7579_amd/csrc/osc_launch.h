// Kernel launchers of libosc (defined in osc_kernels.hip).
#pragma once

#include "osc_internal.h"

namespace osc {

// mode: 0 = probabilities only, 1 = probabilities + histogram partials,
// 2 = histogram partials of given values.  partial holds ntiles x
// (nbins + 2) FP64 entries, tile-major.
// mixed selects the FP32-mixed tier (FP64 eigenvalues and phases, FP32
// sine/cosine and amplitude assembly).
hipError_t launch_tiles(int mode, bool write_p, bool mixed, const SetConsts& sc,
                        const PathConsts& pc, const BinConsts& bc, int64_t n,
                        const double* e_true, const uint8_t* flags, const double* weight,
                        const double* e_reco, const double* value, double* p_out,
                        double* partial, hipStream_t stream);

// Bytes of scratch one histogram needs: merge counter, tile results,
// chunk results.
size_t merge_scratch_bytes(int64_t n, int nbt);

// Tile results of the scratch buffer (after the merge counter).
inline double* scratch_partials(void* scratch)
{
    return reinterpret_cast<double*>(static_cast<char*>(scratch) + kMergeCounterBytes);
}

// Adds the tile results of every histogram entry into hist_out.
hipError_t launch_merge(void* scratch, int64_t n, int nbt, double* hist_out, hipStream_t stream);

// Resident one-wave blocks per CU of the per-event kernel of `mode` for
// histograms of nbins bins.
hipError_t occupancy(int mode, int nbins, int* blocks_per_cu);

// Raises the dynamic-LDS limit of the histogram kernels.
hipError_t set_kernel_attributes(size_t max_dyn_lds);

}  // namespace osc
