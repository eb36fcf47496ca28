// Kernel launchers of libosc (defined in osc_kernels.hip).
#pragma once

#include "osc_internal.h"

namespace osc {

// mode: 0 = probabilities only, 1 = probabilities + histogram partials,
// 2 = histogram partials of given values.  partial holds (nbins + 2) x
// ntiles FP64 entries, bin-major.
hipError_t launch_tiles(int mode, bool write_p, const SetConsts& sc, const PathConsts& pc,
                        const BinConsts& bc, int64_t n, const double* e_true,
                        const uint8_t* flags, const double* weight, const double* e_reco,
                        const double* value, double* p_out, double* partial,
                        hipStream_t stream);

// Adds the tile partials of every histogram entry into hist_out.
hipError_t launch_merge(const double* partial, int64_t n, int nbt, double* hist_out,
                        hipStream_t stream);

// Raises the dynamic-LDS limit of the histogram kernels.
hipError_t set_kernel_attributes(size_t max_dyn_lds);

}  // namespace osc
