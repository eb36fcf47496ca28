// Internal layout shared by the host side and the kernels of libosc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osc {

// Reduction contract of the binned PDF: a tile is kTileLanes lanes x
// kLaneEvents events per lane (one wave64 per tile).
constexpr int kTileLanes = 64;
#ifndef OSC_LANE_EVENTS
#define OSC_LANE_EVENTS 16
#endif
constexpr int kLaneEvents = OSC_LANE_EVENTS;
constexpr int kTileEvents = kTileLanes * kLaneEvents;
// Histogram accumulators per bin of a tile: lane l adds into accumulator
// l mod kHistLanes, so kLaneShare lanes share one accumulator and add into
// it in ascending lane order.  Small accumulator rows keep the LDS per wave
// low (occupancy is bounded by registers, not by the histograms).  The
// value is part of the reduction contract (the bits of every histogram
// depend on it); the macro exists for build-time tuning sweeps.
#ifndef OSC_HIST_LANES
#define OSC_HIST_LANES 8
#endif
constexpr int kHistLanes = OSC_HIST_LANES;
constexpr int kLaneShare = kTileLanes / kHistLanes;
// Waves per SIMD the per-event kernels are compiled for (register caps
// that the compiler meets without spilling).
#ifndef OSC_TILE_WAVES
#define OSC_TILE_WAVES 6
#endif
constexpr int kTileWavesPerSimd = OSC_TILE_WAVES;
constexpr int kBatchWavesPerSimd = 4;
constexpr int kLayeredWavesPerSimd = 3;

// Largest event count accepted.
constexpr int64_t kMaxEvents = int64_t(1) << 32;
// Histogram merge: launches of 1024-thread blocks, one block per (chunk of
// kMergeChunkRows = 16384 rows, bin, parameter set); thread t of a block
// adds rows 16 t .. 16 t + 15 of its chunk as a binary tree, and the
// block's threads meet in a binary tree (the 64 lanes of a wave, then the
// 16 waves) -- one aligned subtree of the tile tree per block, so the
// thread count changes no bits (1024 threads ran the one-level merge of
// 9766 tiles in 7.1 us per call against 8.1 us with 256).  Levels repeat
// until one row per histogram is left (one level up to kMergeChunkRows
// tiles, i.e. 1.6e7 events, per sample).  Rows are stored bin-major
// within chunks of kLayoutChunk rows (partial_index), so a thread's rows
// of one bin are contiguous.  The macro exists for build-time sweeps.
#ifndef OSC_MERGE_THREADS
#define OSC_MERGE_THREADS 1024
#endif
constexpr int kMergeThreads = OSC_MERGE_THREADS;
constexpr int kMergeWaves = kMergeThreads / 64;
constexpr int kMergeThreadRows = 16384 / kMergeThreads;
constexpr int64_t kMergeChunkRows = int64_t(kMergeThreads) * kMergeThreadRows;
constexpr int kLayoutChunk = 128;
constexpr int kMaxBatchSamples = 16;
// Largest number of parameter sets of one batch (the merge grid's z extent).
constexpr int kMaxBatchSets = 65535;

// One level of the merge for n_samples samples (x any number of parameter
// sets, one set per grid layer z): sample s has rows[s] input rows stored
// from row in_row0[s] (a multiple of kLayoutChunk) of the set's input
// region, takes blocks chunk0[s] .. and produces ceil(rows[s] /
// kMergeChunkRows) (at least one) output rows, stored from row out_row0[s]
// (a multiple of kLayoutChunk) of the set's output region.  The final level
// writes hist[set][sample][bin] instead.
struct MergeLevel {
    int32_t n_samples;
    int32_t nbt;
    int64_t total_chunks;                 // blocks per (bin, set)
    int64_t set_stride_in, set_stride_out;
    int64_t rows[kMaxBatchSamples];
    int64_t in_row0[kMaxBatchSamples];
    int64_t chunk0[kMaxBatchSamples];
    int64_t out_row0[kMaxBatchSamples];
};

// Position of the result of (tile, bin) among the tile results.
__host__ __device__ inline int64_t partial_index(int64_t tile, int bin, int nbt)
{
    return (tile / kLayoutChunk) * int64_t(nbt) * kLayoutChunk + int64_t(bin) * kLayoutChunk +
           (tile % kLayoutChunk);
}

// One flavour channel (beta <- alpha) of the vacuum mass matrix H0 =
// U diag(0, dm21, dm31) U^+ in the flavour basis, for neutrinos.
// With M = H0 + A e_e e_e^T:
//   M_ba      = m + A [a = b = e]
//   (M^2)_ba  = m2 + A g + A^2 [a = b = e],  g = [b = e] H0_ea + H0_be [a = e]
// Antineutrinos use the complex conjugates and the opposite sign of A.
// dee = [a = b = e] is stored as 0.0 / 1.0 so that the kernel applies it
// with FMAs.  The kernels expand these 9 entries into the flag-indexed LDS
// tables of TileTables (conjugated copies for antineutrinos, [a = b]).
struct Chan {
    double m_re, m_im;
    double m2_re, m2_im;
    double g_re, g_im;
    double dee;
};

constexpr int kChannels = 9;   // index 3 beta + alpha

// Parameter-only quantities of one oscillation parameter set.
// Characteristic polynomial of M: x^3 - tr x^2 + c1 x - det with
//   tr = T0 + A,  c1 = C0 + A CA,  det = A DA.
// The trigonometric seed of its roots uses q/2 with q = 2 tr^3 - 9 tr c1 +
// 27 det, expanded in A as q/2 = ((A + QH2) A + QH1) A + QH0.
struct SetConsts {
    double T0, C0, CA, DA;
    double QH0, QH1, QH2;
    Chan ch[kChannels];
};

// sin and cos of k pi / 32, k = 0..63 (the anchors of the FP64 phase
// sine/cosine), computed once on the host in extended precision.
struct SinCos {
    double s, c;
};
struct SinCosTable {
    SinCos e[64];
};
// The LDS form of an anchor adds cm1 = c - 1, so that cos(phase) - 1 is
// formed without cancellation.
struct SinCosL {
    double s, c, cm1;
};

// Path constants of one sample.
struct PathConsts {
    double kA;   // matter term per GeV: A = +-kA * E (eV^2)
    double kL;   // phase per eV^2 per 1/GeV in units of pi/32:
                 // phase = (pi/32) * kL * lambda / E
};

// A path of piecewise-constant density: layers in the order the neutrino
// crosses them, each with its own PathConsts.
constexpr int kMaxLayers = 32;
struct LayerPath {
    int32_t n;
    PathConsts layer[kMaxLayers];
};

// The fast bin index is exact for quotients below this magnitude, so no
// binning may have more regular bins (under/overflow included).
constexpr double kFastBinLimit = 4096.0;
constexpr int32_t kMaxBins = 4094;

struct BinConsts {
    double lo;
    double wb;      // (hi - lo) / nbins, computed on the host in FP64
    double inv_wb;  // 1 / wb rounded to FP64 (fast path of the bin index)
    double scale;   // 1 + e_scale rounded to FP64; the bin is taken for x * scale
    int32_t nb;     // regular bins; entries nb and nb + 1 are under/overflow
};

// Flag bytes f < 32 with alpha = f & 3 < 3 and beta = (f >> 2) & 3 < 3, as
// a bit mask over f.
constexpr uint32_t kValidFlags = 0x07770777u;

// Tables a per-event kernel keeps in LDS, built by each block from a
// SetConsts and the SinCosTable:
//  * ch: the channel table per (alpha, beta, antineutrino): entries
//    3 beta + alpha for neutrinos, 9 + 3 beta + alpha for antineutrinos
//    (complex conjugates: m_im, m2_im and g_im negated), each with
//    dba = [alpha = beta]; entry 18 (invalid flag bytes) is zero with
//    dba = NaN, so P comes out NaN;
//  * flag: for each flag byte f < 32 the byte offset of its ch entry and
//    the sign bit of A (set for antineutrinos); bytes >= 32 use entry 31,
//    which is invalid;
//  * sct: the phase sine/cosine anchors (24 B each: the table grows the
//    per-wave LDS by 512 B, which still leaves room for the six waves per
//    SIMD of a 50-bin histogram).
// The per-event decode of a flag byte is then one min, one LDS read and one
// XOR.
struct ChanL {
    double m_re, m_im;
    double m2_re, m2_im;
    double g_re, g_im;
    double dee, dba;
};
constexpr int kLdsChannels = 2 * kChannels + 1;
constexpr int kInvalidChannel = 2 * kChannels;
constexpr int kFlagEntries = 32;
struct FlagInfo {
    uint32_t ch_off;   // byte offset into the table's ch array
    uint32_t sign;     // 0 or 0x80000000: the sign bit of A
};
struct TileTables {
    ChanL ch[kLdsChannels];
    FlagInfo flag[kFlagEntries];
    SinCosL sct[64];
};

// The FP32-mixed tier assembles the amplitude in FP32 from the same channel
// entries rounded to FP32 (M_ba and (M^2)_ba are then formed from them in
// FP32), and its phases use the hardware sine and cosine, so its tables
// hold FP32 channel entries and no sin/cos anchors.
struct ChanF {
    float m_re, m_im;
    float m2_re, m2_im;
    float g_re, g_im;
    float dee, dba;
};
struct TileTablesMixed {
    ChanF ch[kLdsChannels];
    FlagInfo flag[kFlagEntries];
};
template <bool MIXED>
struct TablesOf {
    using type = TileTables;
};
template <>
struct TablesOf<true> {
    using type = TileTablesMixed;
};
template <bool MIXED>
using Tables = typename TablesOf<MIXED>::type;

}  // namespace osc
