// Batched form of libosc: every parameter set x every sample of a list in
// one launch of a persistent kernel plus the histogram merge, replayed from
// a captured HIP graph, with launch shapes chosen by an autotuner.
//
// A work item is (group of sets_per_item parameter sets, sample, tile).  The
// wave that takes it runs, for each set of the group, the same tile body as
// osc_fill_pdf (same per-event arithmetic, same lane order, same lane tree)
// and writes the tile row into that set's region of the merge plan; the
// merge then reduces every (set, sample) in the contract's order.  Hence
// each batched histogram equals the plain call bit for bit, whatever the
// launch shape.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/osc.h"
#include "osc_device.h"
#include "osc_host_common.h"
#include "osc_internal.h"
#include "osc_launch.h"

namespace osc {
namespace {

using namespace dev;

struct BatchSampleDev {
    const double* e_true;
    const uint8_t* flags;
    const double* weight;
    const uint16_t* bins;   // cached histogram slots (made at batch creation)
    int64_t n;
    int64_t tile0;   // first work tile of this sample among all samples
    int64_t row0;    // first tile row of this sample in a set's tile-result region
    PathConsts pc;
};

struct BatchArgs {
    int32_t n_samples;
    int32_t n_sets;
    int32_t sets_per_item;
    int32_t nbt;
    int32_t schedule;      // Schedule
    int64_t groups;        // ceil(n_sets / sets_per_item)
    int64_t n_items;       // total tiles x groups
    int64_t set_stride;    // tile-result elements per set
    BinConsts bc;
};

enum Schedule { kDynamic = 0, kStatic = 1, kOnePerBlock = 2 };

// Work items are tile-major (the set groups of one tile are consecutive).
// The persistent schedules give each XCD one contiguous range of them, so
// that the set groups of a tile run on one XCD and read the tile's events
// from one L2: workgroups reach the XCDs round-robin, so workgroup b of a
// grid of G serves part b mod X of X = min(8, G) parts, and the dynamic
// schedule keeps one queue counter per part, kQueueStride counters apart.
// On the 256-set x 4-sample workload this cut the bytes fetched 8-10x and
// the dynamic schedule's time 1 %.  With one workgroup per item, items stay
// in workgroup order (every XCD takes a share of every tile): the
// contiguous ranges there fetched 9x less but ran 1.4 % slower, since the
// samples' costs differ and contiguous ranges load the XCDs unevenly.
constexpr int kQueueStride = 32;
constexpr int kQueueParts = 8;
constexpr size_t kQueueBytes = size_t(kQueueParts) * kQueueStride * sizeof(unsigned);

struct ItemRange {
    int64_t begin, end;
};

__device__ __forceinline__ ItemRange part_items(int64_t x, int64_t parts, int64_t n)
{
    const int64_t q = n / parts, r = n % parts;
    const int64_t begin = x * q + (x < r ? x : r);
    return ItemRange{begin, begin + q + (x < r ? 1 : 0)};
}

__device__ __forceinline__ int64_t take_item(unsigned* queue, int lane)
{
    unsigned v = 0;
    if (lane == 0) v = atomicAdd(queue, 1u);
    return int64_t(__builtin_amdgcn_readfirstlane(v));
}

__global__ void reset_queue(unsigned* queue)
{
    if (threadIdx.x < kQueueParts) queue[threadIdx.x * kQueueStride] = 0u;
}

template <bool MIXED>
__global__ __launch_bounds__(kTileLanes) __attribute__((amdgpu_waves_per_eu(kBatchWavesPerSimd)))
void batch_kernel(BatchArgs a, SinCosTable sctab, const BatchSampleDev* __restrict__ samples,
                  const SetConsts* __restrict__ sets, double* __restrict__ partial,
                  unsigned* __restrict__ queue)
{
    extern __shared__ double hist[];
    __shared__ Tables<MIXED> tabs;
    const int lane = threadIdx.x;
    const int nbt = a.nbt;
    if constexpr (!MIXED) load_sincos(sctab, tabs, lane);   // read after the first barrier below

    const int64_t G = gridDim.x, b = blockIdx.x;
    int64_t item, end, stride = 0, base = 0;
    unsigned* q = nullptr;
    if (a.schedule == kOnePerBlock) {
        item = b;
        end = item + 1;
    } else {
        const int64_t parts = min(int64_t(kQueueParts), G), x = b % parts;
        const ItemRange r = part_items(x, parts, a.n_items);
        end = r.end;
        if (a.schedule == kDynamic) {
            q = queue + x * kQueueStride;
            base = r.begin;
            item = base + take_item(q, lane);
        } else {
            item = r.begin + b / parts;
            stride = G / parts + (x < G % parts ? 1 : 0);   // workgroups serving part x
        }
    }
    while (item < end) {
        // the next item is taken before this one runs (the queue's
        // latency overlaps the work); one workgroup per item stops here
        const int64_t next = q ? base + take_item(q, lane) : (stride ? item + stride : end);
        // items are tile-major, so the groups of one tile run close together
        // and share the tile's events in L2
        const int64_t gtile = item / a.groups;
        const int64_t g = item - gtile * a.groups;
        int s = 0;
        while (s + 1 < a.n_samples && gtile >= samples[s + 1].tile0) ++s;
        const BatchSampleDev& S = samples[s];
        const int64_t tile = gtile - S.tile0;
        const TileArrays t = tile_arrays(tile, S.n, S.e_true, S.flags, S.weight, nullptr, S.bins,
                                         nullptr, nullptr);
        const int set_end = int(min(int64_t(a.n_sets), (g + 1) * a.sets_per_item));
        for (int set = int(g) * a.sets_per_item; set < set_end; ++set) {
            const SetConsts& sc = sets[set];
            __syncthreads();   // the previous set's table and histogram are read
            load_tab<MIXED>(sc, tabs, lane);
            hist_zero(hist, lane, nbt);
            __syncthreads();
            const ConstDensityProb<MIXED> prob{&sc, &tabs, S.pc.kA, S.pc.kL};
            if (t.n == kTileEvents)
                tile_events<kPdfBinned, false, true, true, false>(
                    prob, a.bc, hist, lane, t.n, t.e_true, t.flags, t.weight, nullptr, t.bins,
                    nullptr, nullptr);
            else
                tile_events<kPdfBinned, false, false, true, false>(
                    prob, a.bc, hist, lane, t.n, t.e_true, t.flags, t.weight, nullptr, t.bins,
                    nullptr, nullptr);
            __syncthreads();
            tile_write(hist, lane, nbt, S.row0 + tile, partial + int64_t(set) * a.set_stride);
        }
        item = next;
    }
}

}  // namespace
}  // namespace osc

struct osc_batch {
    osc_ctx* ctx = nullptr;
    int device = 0;
    int n_samples = 0;
    int max_sets = 0;
    osc_binning binning{};
    osc_precision precision = OSC_FP64;
    std::vector<int64_t> tiles;
    osc::MergePlan plan;
    osc::BatchSampleDev* d_samples = nullptr;
    uint16_t* d_bins = nullptr;   // the samples' cached histogram slots, back to back
    osc::SetConsts* d_sets = nullptr;
    osc::SetConsts* h_sets = nullptr;   // pinned staging
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    double* d_scratch = nullptr;
    unsigned* d_queue = nullptr;
    double* d_hist = nullptr;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_sets = -1;
    osc_batch_config graph_cfg{};
    osc_batch_config cfg{};
    int num_cus = 0;
    int occupancy = 1;
    std::mutex mu;
};

namespace {

bool same_cfg(const osc_batch_config& a, const osc_batch_config& b)
{
    return a.sets_per_item == b.sets_per_item && a.schedule == b.schedule &&
           a.waves_per_cu == b.waves_per_cu && a.use_graph == b.use_graph;
}

bool cfg_ok(const osc_batch_config& c)
{
    return c.sets_per_item >= 1 && c.sets_per_item <= 64 && c.schedule >= 0 && c.schedule <= 2 &&
           c.waves_per_cu >= 0 && c.waves_per_cu <= 32 && (c.use_graph == 0 || c.use_graph == 1);
}

osc::BatchArgs batch_args(const osc_batch* b, int n_sets, const osc_batch_config& c)
{
    osc::BatchArgs a{};
    a.n_samples = b->n_samples;
    a.n_sets = n_sets;
    a.sets_per_item = std::min(c.sets_per_item, n_sets);
    a.nbt = b->binning.nbins + 2;
    a.schedule = c.schedule;
    a.groups = (n_sets + a.sets_per_item - 1) / a.sets_per_item;
    int64_t total_tiles = 0;
    for (int64_t t : b->tiles) total_tiles += t;
    a.n_items = total_tiles * a.groups;
    a.set_stride = b->plan.tile_set_stride;
    a.bc = osc::host::bin_consts(&b->binning);
    return a;
}

// Limits of one launch: a one-workgroup-per-item grid must fit the 32-bit
// count of work-items (64 per workgroup), and the persistent waves of the
// dynamic schedule take n_items + grid tickets from a 32-bit counter.
constexpr int64_t kMaxGridItems = ((int64_t(1) << 32) - 1) / osc::kTileLanes;
constexpr int64_t kMaxTickets = (int64_t(1) << 32) - 1;
constexpr int kMaxWavesPerCu = 32;

bool launchable(const osc_batch* b, int n_sets, const osc_batch_config& c)
{
    const osc::BatchArgs a = batch_args(b, n_sets, c);
    if (c.schedule == osc::kOnePerBlock) return a.n_items <= kMaxGridItems;
    return a.n_items + int64_t(b->num_cus) * kMaxWavesPerCu <= kMaxTickets;
}

// Enqueues one batched evaluation of n_sets sets (parameters already in
// d_sets) on `stream`: queue reset, persistent kernel, merge levels.
hipError_t enqueue(osc_batch* b, int n_sets, const osc_batch_config& c, hipStream_t stream)
{
    const osc::BatchArgs a = batch_args(b, n_sets, c);
    const size_t lds = size_t(a.nbt) * osc::kHistLanes * sizeof(double);
    int64_t grid = a.n_items;
    if (c.schedule != osc::kOnePerBlock) {
        const int wpc = c.waves_per_cu > 0 ? c.waves_per_cu : b->occupancy;
        grid = std::min<int64_t>(a.n_items, int64_t(b->num_cus) * wpc);
    }
    if (a.n_items > 0) {
        if (a.schedule == osc::kDynamic) {
            hipLaunchKernelGGL(osc::reset_queue, dim3(1), dim3(64), 0, stream, b->d_queue);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        const osc::SinCosTable& sct = osc::host::sincos_table();
        if (b->precision == OSC_FP32_MIXED)
            hipLaunchKernelGGL(osc::batch_kernel<true>, dim3(unsigned(grid)), dim3(osc::kTileLanes),
                               lds, stream, a, sct, b->d_samples, b->d_sets, b->d_scratch,
                               b->d_queue);
        else
            hipLaunchKernelGGL(osc::batch_kernel<false>, dim3(unsigned(grid)), dim3(osc::kTileLanes),
                               lds, stream, a, sct, b->d_samples, b->d_sets, b->d_scratch,
                               b->d_queue);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return osc::launch_merge(b->plan, n_sets, b->d_scratch, b->d_hist, stream);
}

// Stages n_sets parameter sets (host precompute, pinned copy) and enqueues
// their upload on `stream`.
osc_status stage_sets(osc_batch* b, const osc_params* sets, int n_sets, hipStream_t stream)
{
    if (b->staged_pending && hipEventSynchronize(b->staged) != hipSuccess) return OSC_ERR_DEVICE;
    for (int k = 0; k < n_sets; ++k) b->h_sets[k] = osc::host::set_consts(sets[k]);
    if (hipMemcpyAsync(b->d_sets, b->h_sets, size_t(n_sets) * sizeof(osc::SetConsts),
                       hipMemcpyHostToDevice, stream) != hipSuccess)
        return OSC_ERR_DEVICE;
    if (hipEventRecord(b->staged, stream) != hipSuccess) return OSC_ERR_DEVICE;
    b->staged_pending = true;
    return OSC_OK;
}

osc_status run_locked(osc_batch* b, int n_sets, const osc_batch_config& c, hipStream_t stream)
{
    if (!c.use_graph) return enqueue(b, n_sets, c, stream) == hipSuccess ? OSC_OK : OSC_ERR_DEVICE;
    if (!b->exec || b->graph_sets != n_sets || !same_cfg(b->graph_cfg, c)) {
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return OSC_ERR_DEVICE;
        const hipError_t e1 = enqueue(b, n_sets, c, b->capture_stream);
        const hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
        if (e1 != hipSuccess || e2 != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return OSC_ERR_DEVICE;
        }
        const hipError_t e3 = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) {
            b->exec = nullptr;
            return OSC_ERR_DEVICE;
        }
        b->graph_sets = n_sets;
        b->graph_cfg = c;
    }
    return hipGraphLaunch(b->exec, stream) == hipSuccess ? OSC_OK : OSC_ERR_DEVICE;
}

void free_batch(osc_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->h_sets) (void)hipHostFree(b->h_sets);
    for (void* p : {static_cast<void*>(b->d_samples), static_cast<void*>(b->d_sets),
                    static_cast<void*>(b->d_scratch), static_cast<void*>(b->d_queue),
                    static_cast<void*>(b->d_hist), static_cast<void*>(b->d_bins)})
        if (p) (void)hipFree(p);
    delete b;
}

std::string tune_key(const osc_batch* b, int n_sets)
{
    int64_t events = 0;
    for (int64_t t : b->tiles) events += t;
    const int log2_tiles = events > 0 ? int(std::floor(std::log2(double(events)))) : 0;
    char buf[160];
    std::snprintf(buf, sizeof buf, "batch tier=%d nbins=%d samples=%d sets=%d log2tiles=%d",
                  int(b->precision), b->binning.nbins, b->n_samples, n_sets, log2_tiles);
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, osc_batch_config* out)
{
    if (!path || !*path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        const char* bar = std::strchr(line, '|');
        if (!bar || std::string(line, size_t(bar - line)) != key) continue;
        osc_batch_config c{};
        if (std::sscanf(bar + 1, "%d %d %d %d", &c.sets_per_item, &c.schedule, &c.waves_per_cu,
                        &c.use_graph) == 4 && cfg_ok(c)) {
            *out = c;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, const osc_batch_config& c, double ms)
{
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s|%d %d %d %d  # %.4f ms\n", key.c_str(), c.sets_per_item, c.schedule,
                 c.waves_per_cu, c.use_graph, ms);
    std::fclose(f);
}

}  // namespace

extern "C" {

osc_status osc_batch_create(osc_ctx* ctx, const osc_sample* samples, int32_t n_samples,
                            const osc_binning* binning, osc_precision precision, int32_t max_sets,
                            osc_batch** out)
{
    if (!out) return OSC_ERR_INVALID_ARG;
    *out = nullptr;
    if (!ctx || !samples || n_samples < 1 || n_samples > osc::kMaxBatchSamples || max_sets < 1 ||
        max_sets > osc::kMaxBatchSets)
        return OSC_ERR_INVALID_ARG;
    if (precision != OSC_FP64 && precision != OSC_FP32_MIXED) return OSC_ERR_INVALID_ARG;
    if (!osc::host::binning_ok(ctx, binning)) return OSC_ERR_INVALID_ARG;
    for (int s = 0; s < n_samples; ++s)
        if (!osc::host::sample_ok(&samples[s], true)) return OSC_ERR_INVALID_ARG;
    const int device = osc::host::ctx_device(ctx);
    if (hipSetDevice(device) != hipSuccess) return OSC_ERR_DEVICE;

    osc_batch* b = new (std::nothrow) osc_batch();
    if (!b) return OSC_ERR_OUT_OF_MEMORY;
    b->ctx = ctx;
    b->device = device;
    b->n_samples = n_samples;
    b->max_sets = max_sets;
    b->binning = *binning;
    b->precision = precision;
    const int nbt = binning->nbins + 2;
    std::vector<osc::BatchSampleDev> hs;
    hs.resize(size_t(n_samples));
    int64_t tile0 = 0;
    for (int s = 0; s < n_samples; ++s) {
        const int64_t t = (samples[s].n + osc::kTileEvents - 1) / osc::kTileEvents;
        b->tiles.push_back(t);
        hs[size_t(s)] = osc::BatchSampleDev{samples[s].e_true, samples[s].flags, samples[s].weight,
                                            nullptr, samples[s].n, tile0, 0,
                                            osc::host::path_consts(&samples[s])};
        tile0 += t;
    }
    b->plan = osc::plan_merge(b->tiles.data(), n_samples, nbt);
    for (int s = 0; s < n_samples; ++s)
        hs[size_t(s)].row0 = b->plan.levels[0].in_row0[s];

    hipDeviceProp_t prop;
    int occ = 0;
    const size_t lds = size_t(nbt) * osc::kHistLanes * sizeof(double);
    const bool ok =
        hipGetDeviceProperties(&prop, device) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&osc::batch_kernel<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&osc::batch_kernel<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, reinterpret_cast<const void*>(&osc::batch_kernel<false>), osc::kTileLanes, lds) ==
            hipSuccess;
    if (!ok) {
        free_batch(b);
        return OSC_ERR_DEVICE;
    }
    b->num_cus = prop.multiProcessorCount;
    b->occupancy = std::max(1, occ);
    b->cfg = osc_batch_config{8, osc::kDynamic, 0, 1};
    // the persistent schedules must be able to run every set count up to
    // max_sets with one set per item
    if (!launchable(b, max_sets, osc_batch_config{1, osc::kDynamic, 0, 1})) {
        free_batch(b);
        return OSC_ERR_INVALID_ARG;
    }

    // Only now, with every argument accepted, are the sample arrays read:
    // the reco-energy bins do not change from run to run, so each event's
    // histogram slot is cached once, here.
    int64_t events = 0;
    for (int s = 0; s < n_samples; ++s) events += samples[s].n;
    if (events > 0 && hipMalloc(&b->d_bins, size_t(events) * sizeof(uint16_t)) != hipSuccess) {
        free_batch(b);
        return OSC_ERR_OUT_OF_MEMORY;
    }
    hipError_t be = hipDeviceSynchronize();
    events = 0;
    for (int s = 0; s < n_samples && be == hipSuccess; ++s) {
        uint16_t* bins = samples[s].n > 0 ? b->d_bins + events : nullptr;
        hs[size_t(s)].bins = bins;
        be = osc::host::enqueue_bin_slots(&samples[s], binning, bins, nullptr);
        events += samples[s].n;
    }
    if (be == hipSuccess) be = hipDeviceSynchronize();
    if (be != hipSuccess) {
        free_batch(b);
        return OSC_ERR_DEVICE;
    }

    const size_t scratch = osc::merge_scratch_bytes(b->plan, max_sets);
    const size_t hist_bytes = size_t(max_sets) * n_samples * nbt * sizeof(double);
    if (hipMalloc(&b->d_samples, hs.size() * sizeof(osc::BatchSampleDev)) != hipSuccess ||
        hipMalloc(&b->d_sets, size_t(max_sets) * sizeof(osc::SetConsts)) != hipSuccess ||
        hipMalloc(&b->d_scratch, scratch) != hipSuccess ||
        hipMalloc(&b->d_queue, osc::kQueueBytes) != hipSuccess ||
        hipMalloc(&b->d_hist, hist_bytes) != hipSuccess ||
        hipHostMalloc(&b->h_sets, size_t(max_sets) * sizeof(osc::SetConsts), hipHostMallocDefault) !=
            hipSuccess) {
        free_batch(b);
        return OSC_ERR_OUT_OF_MEMORY;
    }
    if (hipMemcpy(b->d_samples, hs.data(), hs.size() * sizeof(osc::BatchSampleDev),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(b->d_queue, 0, osc::kQueueBytes) != hipSuccess ||
        hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        free_batch(b);
        return OSC_ERR_DEVICE;
    }
    *out = b;
    return OSC_OK;
}

osc_status osc_batch_destroy(osc_batch* b)
{
    if (!b) return OSC_OK;
    osc_status st = hipSetDevice(b->device) == hipSuccess && hipDeviceSynchronize() == hipSuccess
                        ? OSC_OK
                        : OSC_ERR_DEVICE;
    free_batch(b);
    return st;
}

osc_status osc_batch_get_config(const osc_batch* b, osc_batch_config* cfg)
{
    if (!b || !cfg) return OSC_ERR_INVALID_ARG;
    *cfg = b->cfg;
    return OSC_OK;
}

osc_status osc_batch_set_config(osc_batch* b, const osc_batch_config* cfg)
{
    if (!b || !cfg || !cfg_ok(*cfg)) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(b->mu);
    b->cfg = *cfg;
    return OSC_OK;
}

osc_status osc_batch_run(osc_batch* b, const osc_params* sets, int32_t n_sets, double* hist_out,
                         void* stream)
{
    if (!b || !hist_out || n_sets < 1 || n_sets > b->max_sets) return OSC_ERR_INVALID_ARG;
    osc_status st = osc_validate_params(sets, n_sets);
    if (st != OSC_OK) return st;
    std::lock_guard<std::mutex> lock(b->mu);
    if (!launchable(b, n_sets, b->cfg)) return OSC_ERR_INVALID_ARG;
    if (hipSetDevice(b->device) != hipSuccess) return OSC_ERR_DEVICE;
    const hipStream_t hs = static_cast<hipStream_t>(stream);
    st = stage_sets(b, sets, n_sets, hs);
    if (st != OSC_OK) return st;
    st = run_locked(b, n_sets, b->cfg, hs);
    if (st != OSC_OK) return st;
    const size_t bytes = size_t(n_sets) * b->n_samples * (b->binning.nbins + 2) * sizeof(double);
    return hipMemcpyAsync(hist_out, b->d_hist, bytes, hipMemcpyDeviceToDevice, hs) == hipSuccess
               ? OSC_OK
               : OSC_ERR_DEVICE;
}

osc_status osc_batch_tune(osc_batch* b, const osc_params* sets, int32_t n_sets,
                          const char* cache_path, double* best_ms, void* stream)
{
    if (!b || n_sets < 1 || n_sets > b->max_sets) return OSC_ERR_INVALID_ARG;
    osc_status st = osc_validate_params(sets, n_sets);
    if (st != OSC_OK) return st;
    std::lock_guard<std::mutex> lock(b->mu);
    if (hipSetDevice(b->device) != hipSuccess) return OSC_ERR_DEVICE;
    const std::string key = tune_key(b, n_sets);
    osc_batch_config cached{};
    if (cache_lookup(cache_path, key, &cached)) {
        b->cfg = cached;
        if (best_ms) *best_ms = -1.0;
        return OSC_OK;
    }
    const hipStream_t hs = static_cast<hipStream_t>(stream);
    st = stage_sets(b, sets, n_sets, hs);
    if (st != OSC_OK) return st;

    std::vector<osc_batch_config> cands;
    for (int spi : {1, 2, 4, 8, 16})
        if (spi <= n_sets || spi == 1)
            for (int sched : {int(osc::kDynamic), int(osc::kStatic), int(osc::kOnePerBlock)}) {
                const osc_batch_config c{spi, sched, 0, 1};
                if (launchable(b, n_sets, c)) cands.push_back(c);
            }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) return OSC_ERR_DEVICE;
    double best = 1e300;
    osc_batch_config best_cfg = b->cfg;
    for (const osc_batch_config& c : cands) {
        if (run_locked(b, n_sets, c, hs) != OSC_OK) continue;   // warm-up and capture
        float ms = 0.0f;
        double total = 0.0;
        bool good = true;
        for (int rep = 0; rep < 2 && good; ++rep) {
            good = hipEventRecord(t0, hs) == hipSuccess && run_locked(b, n_sets, c, hs) == OSC_OK &&
                   hipEventRecord(t1, hs) == hipSuccess && hipEventSynchronize(t1) == hipSuccess &&
                   hipEventElapsedTime(&ms, t0, t1) == hipSuccess;
            total += ms;
        }
        if (good && total / 2 < best) {
            best = total / 2;
            best_cfg = c;
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (best >= 1e300) return OSC_ERR_DEVICE;
    b->cfg = best_cfg;
    cache_store(cache_path, key, best_cfg, best);
    if (best_ms) *best_ms = best;
    return OSC_OK;
}

}  // extern "C"
