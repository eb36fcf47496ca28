// HIP kernels of libosc for gfx950 (CDNA4, wave64).
//
// One wave64 owns one tile of kTileEvents consecutive events.  Lane l of
// tile t handles events t*T + m*64 + l, m = 0..K-1 (coalesced SoA loads,
// software-pipelined one group of kGroup events ahead), computes the oscillation
// probability of each event in FP64 (flavour basis, one amplitude element
// per event), optionally writes it, and adds w * P into a per-wave
// histogram held in LDS (kHistLanes accumulators per bin, each shared by
// kLaneShare lanes that add in ascending lane order: masked LDS atomic adds,
// one lane group after the other).  The accumulators of the tile meet in a
// fixed binary tree; a merge kernel adds the tile results per bin in a
// fixed binary tree.  Every addition has a fixed place in that order, so
// the bits of the histogram do not depend on the launch shape or timing.
#include <hip/hip_ext.h>

#include <algorithm>

#include "osc_device.h"
#include "osc_host_common.h"
#include "osc_internal.h"
#include "osc_launch.h"

namespace osc {

namespace {

using namespace dev;

// Register budget for kTileWavesPerSimd resident waves per SIMD.
template <int MODE, bool WRITE_P, bool MIXED = false>
__global__ __launch_bounds__(kTileLanes) __attribute__((amdgpu_waves_per_eu(kTileWavesPerSimd)))
void tile_kernel(
    SetConsts sc, SinCosTable sctab, PathConsts pc, BinConsts bc, int64_t n,
    [[maybe_unused]] int64_t ntiles,
    const double* __restrict__ e_true, const uint8_t* __restrict__ flags,
    const double* __restrict__ weight, const double* __restrict__ e_reco,
    const uint16_t* __restrict__ bins, const double* __restrict__ value,
    double* __restrict__ p_out, double* __restrict__ partial)
{
    extern __shared__ double hist[];
    __shared__ Tables<MIXED> tabs;

    const int lane = threadIdx.x;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int nbt = bc.nb + 2;

    if (MODE != kHist) {
        load_tab<MIXED>(sc, tabs, lane);
        if constexpr (!MIXED) load_sincos(sctab, tabs, lane);
    }
    if (MODE != kReweight) hist_zero(hist, lane, nbt);
    __syncthreads();

    const ConstDensityProb<MIXED> prob{&sc, &tabs, pc.kA, pc.kL,
                                       MIXED ? PolyRegs{} : PolyRegs::in_vgprs()};
    const TileArrays t = tile_arrays(tile, n, e_true, flags, weight, e_reco, bins, value, p_out);
    if (t.n == kTileEvents)
        tile_events<MODE, WRITE_P, true, WRITE_P>(prob, bc, hist, lane, t.n, t.e_true, t.flags,
                                                  t.weight, t.e_reco, t.bins, t.value, t.p_out);
    else
        tile_events<MODE, WRITE_P, false, WRITE_P>(prob, bc, hist, lane, t.n, t.e_true, t.flags,
                                                   t.weight, t.e_reco, t.bins, t.value, t.p_out);

    if (MODE != kReweight) {
        __syncthreads();
        tile_write(hist, lane, nbt, tile, partial);
    }
}

// The same tile body with P through a layered path (FP64 only).  The event
// loop stays rolled: the layer loop is large, and 16 unrolled copies of it
// would not fit the instruction cache.
#ifndef OSC_LAYERED_ROLL
#define OSC_LAYERED_ROLL 1
#endif
constexpr bool kLayeredRoll = OSC_LAYERED_ROLL;
template <int MODE, bool WRITE_P>
__global__ __launch_bounds__(kTileLanes) __attribute__((amdgpu_waves_per_eu(kLayeredWavesPerSimd)))
void layered_tile_kernel(SetConsts sc, SinCosTable sctab, LayerPath lp, BinConsts bc, int64_t n,
                         const double* __restrict__ e_true, const uint8_t* __restrict__ flags,
                         const double* __restrict__ weight, const double* __restrict__ e_reco,
                         double* __restrict__ p_out, double* __restrict__ partial)
{
    extern __shared__ double hist[];
    __shared__ TileTables tabs;

    const int lane = threadIdx.x;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int nbt = bc.nb + 2;

    load_tab(sc, tabs, lane);
    load_sincos(sctab, tabs, lane);
    if (MODE != kReweight) hist_zero(hist, lane, nbt);
    __syncthreads();

    const LayeredProb prob{&sc, &tabs, &lp};
    const TileArrays t =
        tile_arrays(tile, n, e_true, flags, weight, e_reco, nullptr, nullptr, p_out);
    if (t.n == kTileEvents)
        tile_events<MODE, WRITE_P, true, kLayeredRoll>(prob, bc, hist, lane, t.n, t.e_true, t.flags,
                                                       t.weight, t.e_reco, nullptr, nullptr, t.p_out);
    else
        tile_events<MODE, WRITE_P, false, kLayeredRoll>(prob, bc, hist, lane, t.n, t.e_true, t.flags,
                                                        t.weight, t.e_reco, nullptr, nullptr, t.p_out);

    if (MODE != kReweight) {
        __syncthreads();
        tile_write(hist, lane, nbt, tile, partial);
    }
}

template <bool FINAL>
__global__ __launch_bounds__(kMergeThreads) void merge_level_kernel(MergeLevel L,
                                                                   const double* __restrict__ in,
                                                                   double* __restrict__ out)
{
    merge_level_block<FINAL>(L, in, out);
}

// Eq. (2) as a product of Poisson probabilities over the regular bins:
// -2 ln L = 2 sum_b (mu_b - d_b ln mu_b + lgamma(d_b + 1)), mu_b = scale *
// hist_b.  One wave per histogram; lane l adds bins l, l + 64, ... in
// ascending order, then the lanes meet in the wave's butterfly tree (a
// fixed order).
__global__ __launch_bounds__(64) void poisson_nll_kernel(const double* __restrict__ hist,
                                                         double scale, int64_t n_data,
                                                         const double* __restrict__ data,
                                                         int nbins, double* __restrict__ out)
{
    const int64_t k = blockIdx.x;
    const int lane = threadIdx.x;
    const double* mu = hist + k * (nbins + 2);
    const double* d = data + (k % n_data) * nbins;
    double acc = 0.0;
    for (int b = lane; b < nbins; b += 64) {
        const double m = scale * mu[b], x = d[b];
        const double term = m == 0.0 ? (x == 0.0 ? 0.0 : __builtin_inf())
                                     : m - x * log(m) + lgamma(x + 1.0);
        acc = acc + term;
    }
    acc = wave_tree(acc);
    if (lane == 0) out[k] = 2.0 * acc;
}

// The cached histogram slot of every event of a sample: the LDS slot
// (hslot) its contribution goes to in the per-event kernels, from the bin
// of e_reco by the exact rule (a correctly rounded division) and the
// accumulator of its lane, event index mod kHistLanes (tiles start at
// multiples of kTileEvents, so an event's lane is its index mod 64).
__global__ __launch_bounds__(256) void bin_slot_kernel(int64_t n, const double* __restrict__ e_reco,
                                                       BinConsts bc, uint16_t* __restrict__ out)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        out[i] = uint16_t(hslot(lds_bin(bin_floor_exact(e_reco[i], bc), bc),
                                int(i & (kHistLanes - 1))));
}

// One-time domain check of a sample: counts of events whose true energy
// is not finite and positive, and of events with an invalid flag byte.
// Grid-stride loop; per-wave sums, one integer atomic per wave and counter
// (integer sums: the totals do not depend on the order).
__global__ __launch_bounds__(256) void validate_sample_kernel(int64_t n,
                                                              const double* __restrict__ e_true,
                                                              const uint8_t* __restrict__ flags,
                                                              unsigned long long* __restrict__ bad)
{
    unsigned long long be = 0, bf = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const double e = e_true[i];
        const uint32_t f = flags[i];
        be += (e > 0.0 && e <= __DBL_MAX__) ? 0ull : 1ull;   // NaN fails both tests
        bf += ((f < 32u) && ((kValidFlags >> (f & 31u)) & 1u)) ? 0ull : 1ull;
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        be += __shfl_xor(be, s, 64);
        bf += __shfl_xor(bf, s, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (be) atomicAdd(&bad[0], be);
        if (bf) atomicAdd(&bad[1], bf);
    }
}

}  // namespace

hipError_t launch_validate_sample(int64_t n, const double* e_true, const uint8_t* flags,
                                  unsigned long long* bad, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(validate_sample_kernel, dim3(unsigned(blocks)), dim3(256), 0, stream, n,
                       e_true, flags, bad);
    return hipGetLastError();
}

hipError_t launch_bin_slots(int64_t n, const double* e_reco, const BinConsts& bc, uint16_t* out,
                            hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(bin_slot_kernel, dim3(unsigned(blocks)), dim3(256), 0, stream, n, e_reco,
                       bc, out);
    return hipGetLastError();
}

hipError_t launch_poisson_nll(const double* hist, int64_t n_hist, double scale,
                              const double* data, int64_t n_data, int nbins, double* out,
                              hipStream_t stream)
{
    if (n_hist == 0) return hipSuccess;
    hipLaunchKernelGGL(poisson_nll_kernel, dim3(unsigned(n_hist)), dim3(64), 0, stream, hist,
                       scale, n_data, data, nbins, out);
    return hipGetLastError();
}

hipError_t launch_tiles(int mode, bool write_p, bool mixed, const SetConsts& sc,
                        const PathConsts& pc, const BinConsts& bc, int64_t n,
                        const double* e_true, const uint8_t* flags, const double* weight,
                        const double* e_reco, const uint16_t* bins, const double* value,
                        double* p_out, double* partial, hipStream_t stream, hipEvent_t ev_begin,
                        hipEvent_t ev_end)
{
    const int64_t ntiles = (n + kTileEvents - 1) / kTileEvents;
    if (ntiles == 0) return hipSuccess;
    const size_t lds = mode == kReweight ? 0 : size_t(bc.nb + 2) * kHistLanes * sizeof(double);
    const dim3 grid{unsigned(ntiles)}, block{unsigned(kTileLanes)};
    const SinCosTable& sctab = host::sincos_table();
#define OSC_LAUNCH(M, W, X)                                                                      \
    hipExtLaunchKernelGGL((tile_kernel<M, W, X>), grid, block, lds, stream, ev_begin, ev_end, 0,  \
                          sc, sctab, pc, bc, n, ntiles, e_true, flags, weight, e_reco, bins,      \
                          value, p_out, partial)
    if (mode == kReweight) {
        if (mixed) OSC_LAUNCH(kReweight, true, true);
        else OSC_LAUNCH(kReweight, true, false);
    } else if (mode == kPdf) {
        if (write_p && mixed) OSC_LAUNCH(kPdf, true, true);
        else if (write_p) OSC_LAUNCH(kPdf, true, false);
        else if (mixed) OSC_LAUNCH(kPdf, false, true);
        else OSC_LAUNCH(kPdf, false, false);
    } else if (mode == kPdfBinned) {
        if (write_p && mixed) OSC_LAUNCH(kPdfBinned, true, true);
        else if (write_p) OSC_LAUNCH(kPdfBinned, true, false);
        else if (mixed) OSC_LAUNCH(kPdfBinned, false, true);
        else OSC_LAUNCH(kPdfBinned, false, false);
    } else {
        OSC_LAUNCH(kHist, false, false);
    }
#undef OSC_LAUNCH
    return hipGetLastError();
}

hipError_t launch_layered_tiles(int mode, bool write_p, const SetConsts& sc,
                                const LayerPath& lp, const BinConsts& bc, int64_t n,
                                const double* e_true, const uint8_t* flags, const double* weight,
                                const double* e_reco, double* p_out, double* partial,
                                hipStream_t stream, hipEvent_t ev_begin, hipEvent_t ev_end)
{
    const int64_t ntiles = (n + kTileEvents - 1) / kTileEvents;
    if (ntiles == 0) return hipSuccess;
    const size_t lds = mode == kReweight ? 0 : size_t(bc.nb + 2) * kHistLanes * sizeof(double);
    const dim3 grid{unsigned(ntiles)}, block{unsigned(kTileLanes)};
    const SinCosTable& sctab = host::sincos_table();
    if (mode == kReweight)
        hipExtLaunchKernelGGL((layered_tile_kernel<kReweight, true>), grid, block, lds, stream,
                              ev_begin, ev_end, 0, sc, sctab, lp, bc, n, e_true, flags, weight,
                              e_reco, p_out, partial);
    else if (write_p)
        hipExtLaunchKernelGGL((layered_tile_kernel<kPdf, true>), grid, block, lds, stream,
                              ev_begin, ev_end, 0, sc, sctab, lp, bc, n, e_true, flags, weight,
                              e_reco, p_out, partial);
    else
        hipExtLaunchKernelGGL((layered_tile_kernel<kPdf, false>), grid, block, lds, stream,
                              ev_begin, ev_end, 0, sc, sctab, lp, bc, n, e_true, flags, weight,
                              e_reco, p_out, partial);
    return hipGetLastError();
}

// A level divides every sample's row count by kMergeChunkRows (rounding
// up), so two levels reduce the largest accepted sample to one row.
static_assert(kMaxEvents / kTileEvents <= kMergeChunkRows * kMergeChunkRows &&
                  kMaxMergeLevels >= 2,
              "the merge plan's level capacity covers every accepted sample");

MergePlan plan_merge(const int64_t* tiles, int n_samples, int nbt)
{
    auto align = [](int64_t r) { return (r + kLayoutChunk - 1) / kLayoutChunk * kLayoutChunk; };
    MergePlan p;
    p.nbt = nbt;
    p.n_samples = n_samples;
    int64_t rows[kMaxBatchSamples], row0[kMaxBatchSamples];
    int64_t in_rows = 0;
    for (int s = 0; s < n_samples; ++s) {
        rows[s] = tiles[s];
        row0[s] = in_rows;
        in_rows += align(rows[s]);
    }
    int64_t level_max = 0;
    for (bool first = true;; first = false) {
        MergeLevel L{};
        L.n_samples = n_samples;
        L.nbt = nbt;
        int64_t chunks = 0, out_rows = 0;
        bool final_level = true;
        for (int s = 0; s < n_samples; ++s) {
            const int64_t r = rows[s];
            const int64_t ch = r > kMergeChunkRows ? (r + kMergeChunkRows - 1) / kMergeChunkRows : 1;
            L.rows[s] = r;
            L.in_row0[s] = row0[s];
            L.chunk0[s] = chunks;
            L.out_row0[s] = out_rows;
            chunks += ch;
            out_rows += align(ch);
            if (ch > 1) final_level = false;
            rows[s] = ch;
            row0[s] = L.out_row0[s];
        }
        L.total_chunks = chunks;
        L.set_stride_in = in_rows * nbt;
        L.set_stride_out = final_level ? 0 : out_rows * nbt;
        if (first) p.tile_set_stride = L.set_stride_in;
        else level_max = std::max(level_max, L.set_stride_in);
        if (!final_level) level_max = std::max(level_max, L.set_stride_out);
        p.levels[p.n_levels++] = L;
        in_rows = out_rows;
        if (final_level) break;
    }
    p.level_set_stride = level_max;
    return p;
}

size_t merge_scratch_bytes(const MergePlan& p, int64_t n_sets)
{
    return size_t(n_sets) * size_t(p.tile_set_stride + 2 * p.level_set_stride) * sizeof(double);
}

hipError_t launch_merge(const MergePlan& p, int64_t n_sets, double* scratch, double* hist_out,
                        hipStream_t stream)
{
    double* bufs[2] = {scratch + n_sets * p.tile_set_stride,
                       scratch + n_sets * (p.tile_set_stride + p.level_set_stride)};
    const double* in = scratch;
    for (int l = 0; l < p.n_levels; ++l) {
        const MergeLevel& L = p.levels[l];
        const dim3 grid{unsigned(L.total_chunks), unsigned(p.nbt), unsigned(n_sets)};
        const bool final_level = l + 1 == p.n_levels;
        double* out = final_level ? hist_out : bufs[l % 2];
        if (final_level)
            hipLaunchKernelGGL(merge_level_kernel<true>, grid, dim3(kMergeThreads), 0, stream, L,
                               in, out);
        else
            hipLaunchKernelGGL(merge_level_kernel<false>, grid, dim3(kMergeThreads), 0, stream, L,
                               in, out);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        in = out;
    }
    return hipSuccess;
}

hipError_t occupancy(int mode, int nbins, int* blocks_per_cu)
{
    const size_t lds = mode == kReweight ? 0 : size_t(nbins + 2) * kHistLanes * sizeof(double);
    const void* f = mode == kReweight ? reinterpret_cast<const void*>(&tile_kernel<kReweight, true>)
                  : mode == kPdf      ? reinterpret_cast<const void*>(&tile_kernel<kPdf, true>)
                                      : reinterpret_cast<const void*>(&tile_kernel<kHist, false>);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, kTileLanes, lds);
}

hipError_t set_kernel_attributes(size_t max_dyn_lds)
{
    const void* fns[] = {
        reinterpret_cast<const void*>(&tile_kernel<kPdf, true, false>),
        reinterpret_cast<const void*>(&tile_kernel<kPdf, false, false>),
        reinterpret_cast<const void*>(&tile_kernel<kPdf, true, true>),
        reinterpret_cast<const void*>(&tile_kernel<kPdf, false, true>),
        reinterpret_cast<const void*>(&tile_kernel<kHist, false, false>),
        reinterpret_cast<const void*>(&tile_kernel<kPdfBinned, true, false>),
        reinterpret_cast<const void*>(&tile_kernel<kPdfBinned, false, false>),
        reinterpret_cast<const void*>(&tile_kernel<kPdfBinned, true, true>),
        reinterpret_cast<const void*>(&tile_kernel<kPdfBinned, false, true>),
        reinterpret_cast<const void*>(&layered_tile_kernel<kPdf, true>),
        reinterpret_cast<const void*>(&layered_tile_kernel<kPdf, false>),
    };
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           int(max_dyn_lds));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace osc
