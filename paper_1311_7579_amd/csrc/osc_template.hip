// Bin-centre reweighting (Sec. 1.1.1): the approximation that event-by-event
// reweighting replaces.  A sample is reduced once to a migration template
// T[r][c][t] -- the Monte Carlo weight of channel c (alpha + 3 beta + 9 anti)
// in true-energy bin t and reconstructed-energy bin r -- and a parameter set
// is applied by evaluating P once per channel at every true-bin centre:
//   hist[r] = sum over k = c nt + t of fl(T[r][k] * P[k]).
//
// Template build (once, deterministic): every event gets a cell key, a
// stable radix sort groups the events of a cell in ascending event order,
// and one thread per cell adds the cell's weights in that order.
// Per call: one kernel for the 18 nt probabilities (the same per-event
// arithmetic as the fused kernel), one wave per reconstructed bin for the
// contraction (lane-strided sums, then the wave's binary tree).
#include <hipcub/hipcub.hpp>

#include <cstdint>
#include <new>

#include "../../include/osc.h"
#include "osc_device.h"
#include "osc_host_common.h"
#include "osc_internal.h"

namespace osc {
namespace {

using namespace dev;

constexpr int kTemplateChannels = 18;

struct TrueBins {
    double lo, wb;
    int32_t nt;
};

// Cell key of every event: (r * 18 + c) * nt + t, or n_cells when the flag
// byte is invalid or the true energy is outside the true binning.
__global__ __launch_bounds__(256) void template_keys_kernel(
    int64_t n, const double* __restrict__ e_true, const uint8_t* __restrict__ flags,
    const double* __restrict__ e_reco, TrueBins tb, BinConsts rb, uint32_t n_cells,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ idx)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t f = flags[i];
    const bool valid = (f < 32u) && ((kValidFlags >> (f & 31u)) & 1u);
    double kt, kr;
    {
#pragma clang fp contract(off)
        kt = __builtin_floor((e_true[i] - tb.lo) / tb.wb);
        kr = __builtin_floor((e_reco[i] * rb.scale - rb.lo) / rb.wb);
    }
    const bool inside = kt >= 0.0 && kt < double(tb.nt);
    const int r = (kr < 0.0) ? rb.nb : ((kr < double(rb.nb)) ? int(kr) : rb.nb + 1);
    const uint32_t c = (f & 3u) + 3u * ((f >> 2) & 3u) + 9u * ((f >> 4) & 1u);
    keys[i] = (valid && inside)
                  ? (uint32_t(r) * kTemplateChannels + c) * uint32_t(tb.nt) + uint32_t(kt)
                  : n_cells;
    idx[i] = uint32_t(i);
}

// First and one-past-last position of every cell in the sorted keys.
__global__ __launch_bounds__(256) void template_bounds_kernel(int64_t n,
                                                              const uint32_t* __restrict__ keys,
                                                              uint32_t n_cells,
                                                              uint32_t* __restrict__ first,
                                                              uint32_t* __restrict__ last)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = keys[i];
    if (k >= n_cells) return;
    if (i == 0 || keys[i - 1] != k) first[k] = uint32_t(i);
    if (i == n - 1 || keys[i + 1] != k) last[k] = uint32_t(i + 1);
}

// The weights in sorted order: ws[i] = weight[idx[i]] (independent loads,
// so the per-cell sums below stream contiguous memory instead of waiting
// on one dependent gather per addition).
__global__ __launch_bounds__(256) void template_gather_kernel(int64_t n,
                                                              const uint32_t* __restrict__ idx,
                                                              const double* __restrict__ weight,
                                                              double* __restrict__ ws)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) ws[i] = weight[idx[i]];
}

// Weight sum of every cell, its events in ascending event order from +0.0:
// one thread per cell adds its contiguous run of ws one value after the
// other, with the loads of kSumBatch values issued ahead of their adds.
constexpr uint32_t kSumBatch = 16;
__global__ __launch_bounds__(256) void template_sum_kernel(uint32_t n_cells,
                                                           const uint32_t* __restrict__ first,
                                                           const uint32_t* __restrict__ last,
                                                           const double* __restrict__ ws,
                                                           double* __restrict__ T)
{
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    double s = 0.0;
    uint32_t i = first[c];
    const uint32_t end = last[c];
    for (; end - i >= kSumBatch && i < end; i += kSumBatch) {
        double v[kSumBatch];
#pragma unroll
        for (uint32_t j = 0; j < kSumBatch; ++j) v[j] = ws[i + j];
#pragma unroll
        for (uint32_t j = 0; j < kSumBatch; ++j) s = s + v[j];
    }
    for (; i < end; ++i) s = s + ws[i];
    T[c] = s;
}

// P of the 18 channels at the centre of every true bin, layout P[c][t].
__global__ __launch_bounds__(64) void centre_probs_kernel(SetConsts sc, SinCosTable sctab,
                                                          PathConsts pc, TrueBins tb,
                                                          double* __restrict__ P)
{
    __shared__ TileTables tabs;
    load_tab(sc, tabs, threadIdx.x);
    load_sincos(sctab, tabs, threadIdx.x);
    __syncthreads();
    const int64_t k = int64_t(blockIdx.x) * 64 + threadIdx.x;
    if (k >= int64_t(kTemplateChannels) * tb.nt) return;
    const uint32_t c = uint32_t(k / tb.nt), t = uint32_t(k - int64_t(c) * tb.nt);
    double E;
    {
#pragma clang fp contract(off)
        const double off = (double(t) + 0.5) * tb.wb;
        E = tb.lo + off;
    }
    const uint32_t f = (c % 3u) | (((c / 3u) % 3u) << 2) | ((c / 9u) << 4);
    P[k] = event_prob<false>(sc, tabs, pc.kA, pc.kL, E, f);
}

// hist[r] for one reconstructed bin per wave: lane l adds the terms
// k = l, l + 64, ... in ascending k, then the wave's binary tree.  The
// operands of kContractBatch consecutive terms are loaded before any of
// them is added, so the loads overlap; the additions keep their order.
constexpr int kContractBatch = 8;

__global__ __launch_bounds__(64) void bincentre_contract_kernel(const double* __restrict__ T,
                                                                const double* __restrict__ P,
                                                                int64_t K,
                                                                double* __restrict__ hist)
{
    const int r = blockIdx.x;
    const int lane = threadIdx.x;
    const double* row = T + int64_t(r) * K;
    double acc = 0.0;
    int64_t k = lane;
    for (; k + (kContractBatch - 1) * 64 < K; k += kContractBatch * 64) {
        double t[kContractBatch], p[kContractBatch];
#pragma unroll
        for (int j = 0; j < kContractBatch; ++j) {
            t[j] = row[k + j * 64];
            p[j] = P[k + j * 64];
        }
#pragma unroll
        for (int j = 0; j < kContractBatch; ++j) {
#pragma clang fp contract(off)
            const double term = t[j] * p[j];
            acc = acc + term;
        }
    }
    for (; k < K; k += 64) {
#pragma clang fp contract(off)
        const double term = row[k] * P[k];
        acc = acc + term;
    }
    acc = wave_tree(acc);
    if (lane == 0) hist[r] = acc;
}

}  // namespace
}  // namespace osc

struct osc_template {
    osc_ctx* ctx = nullptr;
    int device = 0;
    osc::TrueBins tb{};
    int32_t nr = 0;
    osc::PathConsts pc{};
    double* d_T = nullptr;   // [nr + 2][18][nt]
    double* d_P = nullptr;   // [18][nt], used when the caller passes no table
};

namespace {

bool true_binning_ok(const osc_binning* b)
{
    if (!b || b->nbins < 1 || b->nbins > 65536) return false;
    if (!(b->lo >= 0.0) || !(b->hi > b->lo) || !(b->hi < 1e300)) return false;
    if (b->e_scale != 0.0) return false;
    const double wb = (b->hi - b->lo) / double(b->nbins);
    return wb > 0.0 && wb < 1e300;
}

unsigned blocks_for(int64_t n, int threads) { return unsigned((n + threads - 1) / threads); }

}  // namespace

extern "C" {

osc_status osc_template_create(osc_ctx* ctx, const osc_sample* sample,
                               const osc_binning* true_binning,
                               const osc_binning* reco_binning, osc_template** out,
                               int64_t* n_used)
{
    if (!out) return OSC_ERR_INVALID_ARG;
    *out = nullptr;
    if (!ctx || !osc::host::sample_ok(sample, true) || !true_binning_ok(true_binning) ||
        !osc::host::binning_ok(ctx, reco_binning))
        return OSC_ERR_INVALID_ARG;
    if (sample->n > int64_t(INT32_MAX)) return OSC_ERR_INVALID_ARG;
    const int64_t nt = true_binning->nbins, nrt = int64_t(reco_binning->nbins) + 2;
    const int64_t cells = nrt * osc::kTemplateChannels * nt;
    if (cells >= int64_t(UINT32_MAX)) return OSC_ERR_INVALID_ARG;
    const uint32_t n_cells = uint32_t(cells);
    const int device = osc::host::ctx_device(ctx);
    if (hipSetDevice(device) != hipSuccess) return OSC_ERR_DEVICE;

    osc_template* tp = new (std::nothrow) osc_template();
    if (!tp) return OSC_ERR_OUT_OF_MEMORY;
    tp->ctx = ctx;
    tp->device = device;
    tp->tb = osc::TrueBins{true_binning->lo,
                           (true_binning->hi - true_binning->lo) / double(true_binning->nbins),
                           true_binning->nbins};
    tp->nr = reco_binning->nbins;
    tp->pc = osc::host::path_consts(sample);
    if (hipMalloc(&tp->d_T, size_t(cells) * sizeof(double)) != hipSuccess ||
        hipMalloc(&tp->d_P, size_t(osc::kTemplateChannels * nt) * sizeof(double)) != hipSuccess) {
        osc_template_destroy(tp);
        return OSC_ERR_OUT_OF_MEMORY;
    }

    const int64_t n = sample->n;
    hipStream_t s = nullptr;
    uint32_t *keys = nullptr, *idx = nullptr, *skeys = nullptr, *sidx = nullptr;
    uint32_t *first = nullptr, *last = nullptr;
    double* ws = nullptr;
    void* tmp = nullptr;
    size_t tmp_bytes = 0;
    osc_status st = OSC_OK;
    int end_bit = 1;
    while (end_bit < 32 && (uint64_t(1) << end_bit) <= uint64_t(n_cells)) ++end_bit;
    // the sample may have been written by work still in flight on any stream
    if (hipDeviceSynchronize() != hipSuccess) st = OSC_ERR_DEVICE;
    if (st == OSC_OK && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        st = OSC_ERR_DEVICE;
    const size_t nb = size_t(n > 0 ? n : 1) * sizeof(uint32_t);
    if (st == OSC_OK &&
        (hipMalloc(&keys, nb) != hipSuccess || hipMalloc(&idx, nb) != hipSuccess ||
         hipMalloc(&skeys, nb) != hipSuccess || hipMalloc(&sidx, nb) != hipSuccess ||
         hipMalloc(&ws, size_t(n > 0 ? n : 1) * sizeof(double)) != hipSuccess ||
         hipMalloc(&first, size_t(n_cells) * sizeof(uint32_t)) != hipSuccess ||
         hipMalloc(&last, size_t(n_cells) * sizeof(uint32_t)) != hipSuccess))
        st = OSC_ERR_OUT_OF_MEMORY;
    if (st == OSC_OK &&
        hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys, skeys, idx, sidx, int(n), 0,
                                           end_bit, s) != hipSuccess)
        st = OSC_ERR_DEVICE;
    if (st == OSC_OK && hipMalloc(&tmp, tmp_bytes > 0 ? tmp_bytes : 1) != hipSuccess)
        st = OSC_ERR_OUT_OF_MEMORY;
    if (st == OSC_OK) {
        hipError_t e = hipMemsetAsync(first, 0, size_t(n_cells) * sizeof(uint32_t), s);
        if (e == hipSuccess) e = hipMemsetAsync(last, 0, size_t(n_cells) * sizeof(uint32_t), s);
        if (e == hipSuccess && n > 0) {
            hipLaunchKernelGGL(osc::template_keys_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                               s, n, sample->e_true, sample->flags, sample->e_reco, tp->tb,
                               osc::host::bin_consts(reco_binning), n_cells, keys, idx);
            e = hipGetLastError();
            if (e == hipSuccess)
                e = hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, skeys, idx, sidx,
                                                       int(n), 0, end_bit, s);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(osc::template_bounds_kernel, dim3(blocks_for(n, 256)),
                                   dim3(256), 0, s, n, skeys, n_cells, first, last);
                e = hipGetLastError();
            }
            if (e == hipSuccess) {
                hipLaunchKernelGGL(osc::template_gather_kernel, dim3(blocks_for(n, 256)),
                                   dim3(256), 0, s, n, sidx, sample->weight, ws);
                e = hipGetLastError();
            }
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(osc::template_sum_kernel, dim3(blocks_for(n_cells, 256)),
                               dim3(256), 0, s, n_cells, first, last, ws, tp->d_T);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = OSC_ERR_DEVICE;
    }
    if (st == OSC_OK && n_used) {
        // events in the template: the sorted keys below n_cells
        uint32_t count = 0;
        if (n > 0) {
            // the sentinel key sorts last; find the first sentinel by bisection
            int64_t lo = 0, hi = n;
            while (lo < hi) {
                const int64_t mid = (lo + hi) / 2;
                uint32_t k = 0;
                if (hipMemcpy(&k, skeys + mid, sizeof(k), hipMemcpyDeviceToHost) != hipSuccess) {
                    st = OSC_ERR_DEVICE;
                    break;
                }
                if (k < n_cells) lo = mid + 1;
                else hi = mid;
            }
            count = uint32_t(lo);
        }
        *n_used = count;
    }
    for (void* p : {static_cast<void*>(keys), static_cast<void*>(idx), static_cast<void*>(skeys),
                    static_cast<void*>(sidx), static_cast<void*>(first), static_cast<void*>(last),
                    static_cast<void*>(ws), tmp})
        if (p) (void)hipFree(p);
    if (s) (void)hipStreamDestroy(s);
    if (st != OSC_OK) {
        osc_template_destroy(tp);
        return st;
    }
    *out = tp;
    return OSC_OK;
}

osc_status osc_template_destroy(osc_template* t)
{
    if (!t) return OSC_OK;
    osc_status st = OSC_OK;
    if (hipSetDevice(t->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        st = OSC_ERR_DEVICE;
    if (t->d_T) (void)hipFree(t->d_T);
    if (t->d_P) (void)hipFree(t->d_P);
    delete t;
    return st;
}

osc_status osc_template_copy(const osc_template* t, double* dst, void* stream)
{
    if (!t || !dst) return OSC_ERR_INVALID_ARG;
    if (hipSetDevice(t->device) != hipSuccess) return OSC_ERR_DEVICE;
    const size_t cells = size_t(t->nr + 2) * osc::kTemplateChannels * size_t(t->tb.nt);
    return hipMemcpyAsync(dst, t->d_T, cells * sizeof(double), hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(stream)) == hipSuccess
               ? OSC_OK
               : OSC_ERR_DEVICE;
}

osc_status osc_fill_pdf_bincentre(osc_ctx* ctx, const osc_template* t, int32_t set,
                                  double* hist_out, double* p_centre_out, void* stream)
{
    if (!ctx || !t || !hist_out || t->ctx != ctx) return OSC_ERR_INVALID_ARG;
    osc::SetConsts sc;
    if (!osc::host::ctx_set(ctx, set, &sc)) return OSC_ERR_INVALID_ARG;
    if (hipSetDevice(t->device) != hipSuccess) return OSC_ERR_DEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* P = p_centre_out ? p_centre_out : t->d_P;
    const int64_t K = int64_t(osc::kTemplateChannels) * t->tb.nt;
    hipLaunchKernelGGL(osc::centre_probs_kernel, dim3(blocks_for(K, 64)), dim3(64), 0, s, sc,
                       osc::host::sincos_table(), t->pc, t->tb, P);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(osc::bincentre_contract_kernel, dim3(unsigned(t->nr + 2)), dim3(64), 0,
                           s, t->d_T, P, K, hist_out);
        e = hipGetLastError();
    }
    return e == hipSuccess ? OSC_OK : OSC_ERR_DEVICE;
}

}  // extern "C"
