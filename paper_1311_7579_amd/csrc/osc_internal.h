// Internal layout shared by the host side and the kernels of libosc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osc {

// Reduction contract of the binned PDF: a tile is kTileLanes lanes x
// kLaneEvents events per lane (one wave64 per tile).
constexpr int kTileLanes = 64;
constexpr int kLaneEvents = 16;
constexpr int kTileEvents = kTileLanes * kLaneEvents;

// Largest event count accepted.
constexpr int64_t kMaxEvents = int64_t(1) << 32;
// Histogram merge: launches of 256-thread blocks, each reducing an aligned
// chunk of kMergeChunkTiles rows (tile results, then chunk results) per bin,
// level by level until one row per histogram is left.  Rows are stored
// bin-major within each chunk (partial_index).
constexpr int kMergeThreads = 256;
constexpr int kMergeChunkTiles = 128;
constexpr int kMaxBatchSamples = 16;

// One level of the merge for n_samples samples (x any number of parameter
// sets, one set per grid row): sample s has rows[s] input rows stored from
// row 128 * chunk0[s] of the set's input region and produces
// ceil(rows[s] / 128) (at least one) output rows, stored from row
// out_row0[s] of the set's output region.  The final level writes
// hist[set][sample][bin] instead.
struct MergeLevel {
    int32_t n_samples;
    int32_t nbt;
    int64_t total_chunks;                 // blocks per set
    int64_t set_stride_in, set_stride_out;
    int64_t rows[kMaxBatchSamples];
    int64_t chunk0[kMaxBatchSamples];
    int64_t out_row0[kMaxBatchSamples];
};

// Position of the result of (tile, bin) among the tile results.
__host__ __device__ inline int64_t partial_index(int64_t tile, int bin, int nbt)
{
    return (tile / kMergeChunkTiles) * int64_t(nbt) * kMergeChunkTiles +
           int64_t(bin) * kMergeChunkTiles + (tile % kMergeChunkTiles);
}

// One flavour channel (beta <- alpha) of the vacuum mass matrix H0 =
// U diag(0, dm21, dm31) U^+ in the flavour basis, for neutrinos.
// With M = H0 + A e_e e_e^T:
//   M_ba      = m + A [a = b = e]
//   (M^2)_ba  = m2 + A g + A^2 [a = b = e],  g = [b = e] H0_ea + H0_be [a = e]
// Antineutrinos use the complex conjugates and the opposite sign of A.
struct Chan {
    double m_re, m_im;
    double m2_re, m2_im;
    double g_re, g_im;
};

// Parameter-only quantities of one oscillation parameter set.
// Characteristic polynomial of M: x^3 - tr x^2 + c1 x - det with
//   tr = T0 + A,  c1 = C0 + A CA,  det = A DA.
struct SetConsts {
    double T0, C0, CA, DA;
    Chan ch[16];   // index (beta << 2) | alpha; entries with a 3 hold NaN
};

// Path constants of one sample.
struct PathConsts {
    double kA;   // matter term per GeV: A = +-kA * E (eV^2)
    double kL;   // phase per eV^2 per 1/GeV: phase = kL * lambda / E
};

struct BinConsts {
    double lo;
    double wb;      // (hi - lo) / nbins, computed on the host in FP64
    double inv_wb;  // 1 / wb rounded to FP64 (fast path of the bin index)
    double scale;   // 1 + e_scale rounded to FP64; the bin is taken for x * scale
    int32_t nb;     // regular bins; entries nb and nb + 1 are under/overflow
};

}  // namespace osc
