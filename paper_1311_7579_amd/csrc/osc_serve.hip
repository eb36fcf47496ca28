// Serving form of libosc: a request loop for fitter proposals.
//
// Requests (one parameter set, one resident sample, one precision tier)
// are queued first-in first-out.  A dispatcher thread admits the request at
// the head of the queue as soon as a slot (a HIP stream with its own
// histogram buffers) is free and the request's merge scratch fits in a
// device arena whose size is the memory budget; admitted requests run
// concurrently on their streams and overlap on the device.  Each request
// reduces its histogram privately in the fixed order of osc_fill_pdf, so its
// result is the same alone and in any mix.  When data rows are set, each
// request also computes -2 ln L (Eq. 2) of its histogram against its
// sample's row on the device.  Completion is signalled by a host function
// enqueued after the device-to-host copy of the histogram (and -2 ln L).
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include <cmath>

#include "../../include/osc.h"
#include "osc_host_common.h"
#include "osc_internal.h"
#include "osc_launch.h"

namespace {

double now_s()
{
    using clock = std::chrono::steady_clock;
    return std::chrono::duration<double>(clock::now().time_since_epoch()).count();
}

constexpr size_t kArenaAlign = 256;

struct Request {
    osc_params params{};
    int32_t sample = 0;
    osc_precision precision = OSC_FP64;
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
    bool done = false;
    bool with_nll = false;
    osc_status status = OSC_OK;
    std::vector<double> hist;
    double nll = NAN;
};

struct Slot {
    hipStream_t stream = nullptr;
    double* d_hist = nullptr;   // nbins + 2 histogram entries, then -2 ln L
    double* h_hist = nullptr;   // pinned, same layout
    bool busy = false;
    uint64_t ticket = 0;
    size_t off = 0, bytes = 0;
    std::atomic<int> finished{0};
    std::atomic<double> t_done{0.0};
};

// First-fit allocator over [0, size) with coalescing frees.
class Arena {
public:
    void reset(size_t size)
    {
        free_.clear();
        free_[0] = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = (bytes + kArenaAlign - 1) & ~(kArenaAlign - 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t next = it->first + bytes;
            free_.erase(it);
            if (rest) free_[next] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + kArenaAlign - 1) & ~(kArenaAlign - 1);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

}  // namespace

struct osc_server {
    osc_ctx* ctx = nullptr;
    int device = 0;
    std::vector<osc_sample> samples;
    std::vector<uint16_t*> bins;   // per sample: cached histogram slots (device)
    std::vector<size_t> need;   // scratch bytes per sample
    osc_binning binning{};
    int nbt = 0;
    double* d_data = nullptr;   // n_samples rows of nbins counts
    double mu_scale = 1.0;
    bool has_data = false;
    osc_server_config cfg{};
    char* arena_mem = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    uint64_t waiting_ticket = 0;   // queue head last seen waiting for budget
    osc_server_stats stats{};
    std::mutex mu;
    std::condition_variable cv_dispatch, cv_done;
    std::thread dispatcher;
    bool stop = false;
};

namespace {

void on_slot_done(void* user)
{
    // runs on a HIP runtime thread once the histogram is on the host:
    // lock-free hand-over to the dispatcher
    Slot* s = static_cast<Slot*>(user);
    s->t_done.store(now_s(), std::memory_order_relaxed);
    s->finished.store(1, std::memory_order_release);
}

// Launch one admitted request on its slot (lock held).
osc_status launch(osc_server* sv, Slot& slot, Request& r)
{
    const osc::SetConsts sc = osc::host::set_consts(r.params);
    double* scratch = reinterpret_cast<double*>(sv->arena_mem + slot.off);
    if (osc::host::enqueue_fill(sc, &sv->samples[size_t(r.sample)], sv->bins[size_t(r.sample)],
                                &sv->binning, r.precision == OSC_FP32_MIXED, scratch,
                                slot.d_hist, nullptr, slot.stream) != hipSuccess)
        return OSC_ERR_DEVICE;
    r.with_nll = sv->has_data;
    const int nb = sv->binning.nbins;
    if (r.with_nll &&
        osc::launch_poisson_nll(slot.d_hist, 1, sv->mu_scale, sv->d_data + size_t(r.sample) * nb,
                                1, nb, slot.d_hist + sv->nbt, slot.stream) != hipSuccess)
        return OSC_ERR_DEVICE;
    if (hipMemcpyAsync(slot.h_hist, slot.d_hist,
                       size_t(sv->nbt + (r.with_nll ? 1 : 0)) * sizeof(double),
                       hipMemcpyDeviceToHost, slot.stream) != hipSuccess)
        return OSC_ERR_DEVICE;
    if (hipLaunchHostFunc(slot.stream, on_slot_done, &slot) != hipSuccess) return OSC_ERR_DEVICE;
    return OSC_OK;
}

void dispatch_loop(osc_server* sv)
{
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lock(sv->mu);
    while (!sv->stop) {
        // retire finished slots
        for (Slot& slot : sv->slots) {
            if (!slot.busy || !slot.finished.load(std::memory_order_acquire)) continue;
            Request& r = sv->reqs[slot.ticket];
            r.hist.assign(slot.h_hist, slot.h_hist + sv->nbt);
            if (r.with_nll) r.nll = slot.h_hist[sv->nbt];
            r.t_done = slot.t_done.load(std::memory_order_relaxed);
            r.done = true;
            sv->arena.release(slot.off, slot.bytes);
            slot.busy = false;
            slot.finished.store(0, std::memory_order_relaxed);
            ++sv->stats.completed;
            --sv->stats.in_flight;
            sv->cv_done.notify_all();
        }
        // admit from the head of the queue while a slot and the budget allow
        while (!sv->pending.empty()) {
            Slot* free_slot = nullptr;
            for (Slot& slot : sv->slots)
                if (!slot.busy) {
                    free_slot = &slot;
                    break;
                }
            if (!free_slot) break;
            const uint64_t ticket = sv->pending.front();
            Request& r = sv->reqs[ticket];
            const size_t bytes = sv->need[size_t(r.sample)];
            size_t off = 0;
            if (!sv->arena.alloc(bytes, &off)) {
                if (sv->waiting_ticket != ticket) {
                    sv->waiting_ticket = ticket;   // count each blocked request once
                    ++sv->stats.budget_waits;
                }
                break;
            }
            sv->pending.pop_front();
            free_slot->busy = true;
            free_slot->ticket = ticket;
            free_slot->off = off;
            free_slot->bytes = bytes;
            r.t_admit = now_s();
            ++sv->stats.admitted;
            ++sv->stats.in_flight;
            sv->stats.max_in_flight = std::max(sv->stats.max_in_flight, sv->stats.in_flight);
            sv->stats.peak_scratch_bytes =
                std::max<int64_t>(sv->stats.peak_scratch_bytes, int64_t(sv->arena.used()));
            const osc_status st = launch(sv, *free_slot, r);
            if (st != OSC_OK) {
                // fail the request and free its resources; kernels that were
                // enqueued before the failure may still use the scratch, so
                // the slot's stream drains first
                (void)hipStreamSynchronize(free_slot->stream);
                r.status = st;
                r.done = true;
                r.t_done = now_s();
                sv->arena.release(off, bytes);
                free_slot->busy = false;
                --sv->stats.in_flight;
                ++sv->stats.failed;
                sv->cv_done.notify_all();
            }
        }
        bool any_busy = false;
        for (const Slot& slot : sv->slots) any_busy |= slot.busy;
        // completions arrive without a notification (lock-free callback), so
        // poll briefly while work is in flight
        sv->cv_dispatch.wait_for(lock, any_busy ? std::chrono::microseconds(20)
                                                : std::chrono::microseconds(2000));
    }
}

void destroy_server(osc_server* sv)
{
    for (Slot& slot : sv->slots) {
        if (slot.stream) {
            (void)hipStreamSynchronize(slot.stream);
            (void)hipStreamDestroy(slot.stream);
        }
        if (slot.d_hist) (void)hipFree(slot.d_hist);
        if (slot.h_hist) (void)hipHostFree(slot.h_hist);
    }
    if (sv->arena_mem) (void)hipFree(sv->arena_mem);
    for (uint16_t* b : sv->bins)
        if (b) (void)hipFree(b);
    if (sv->d_data) (void)hipFree(sv->d_data);
    delete sv;
}

}  // namespace

extern "C" {

osc_status osc_server_create(osc_ctx* ctx, const osc_sample* samples, int32_t n_samples,
                             const osc_binning* binning, const osc_server_config* cfg,
                             osc_server** out)
{
    if (!out) return OSC_ERR_INVALID_ARG;
    *out = nullptr;
    if (!ctx || !samples || n_samples < 1 || !cfg || cfg->slots < 1 || cfg->slots > 64 ||
        cfg->scratch_budget_bytes <= 0 || cfg->queue_capacity < 1)
        return OSC_ERR_INVALID_ARG;
    if (!osc::host::binning_ok(ctx, binning)) return OSC_ERR_INVALID_ARG;
    for (int s = 0; s < n_samples; ++s)
        if (!osc::host::sample_ok(&samples[s], true)) return OSC_ERR_INVALID_ARG;
    const int device = osc::host::ctx_device(ctx);
    if (hipSetDevice(device) != hipSuccess) return OSC_ERR_DEVICE;

    osc_server* sv = new (std::nothrow) osc_server();
    if (!sv) return OSC_ERR_OUT_OF_MEMORY;
    sv->ctx = ctx;
    sv->device = device;
    sv->samples.assign(samples, samples + n_samples);
    sv->binning = *binning;
    sv->nbt = binning->nbins + 2;
    sv->cfg = *cfg;
    for (const osc_sample& s : sv->samples)
        sv->need.push_back(osc::host::fill_scratch_bytes(s.n, binning->nbins));
    sv->slots = std::vector<Slot>(size_t(cfg->slots));
    const size_t budget = size_t(cfg->scratch_budget_bytes) & ~(kArenaAlign - 1);
    bool ok = budget > 0 && hipMalloc(&sv->arena_mem, budget) == hipSuccess;
    // the reco-energy bins of a resident sample do not change from request
    // to request: cache each event's histogram slot once
    sv->bins.assign(sv->samples.size(), nullptr);
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    for (size_t k = 0; ok && k < sv->samples.size(); ++k) {
        const osc_sample& smp = sv->samples[k];
        if (smp.n == 0) continue;
        ok = hipMalloc(&sv->bins[k], size_t(smp.n) * sizeof(uint16_t)) == hipSuccess &&
             osc::host::enqueue_bin_slots(&smp, binning, sv->bins[k], nullptr) == hipSuccess;
    }
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    for (Slot& slot : sv->slots) {
        ok = ok && hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking) == hipSuccess &&
             hipMalloc(&slot.d_hist, size_t(sv->nbt + 1) * sizeof(double)) == hipSuccess &&
             hipHostMalloc(&slot.h_hist, size_t(sv->nbt + 1) * sizeof(double),
                           hipHostMallocDefault) == hipSuccess;
    }
    if (!ok) {
        destroy_server(sv);
        return OSC_ERR_OUT_OF_MEMORY;
    }
    sv->arena.reset(budget);
    try {
        sv->dispatcher = std::thread(dispatch_loop, sv);
    } catch (...) {
        destroy_server(sv);
        return OSC_ERR_DEVICE;
    }
    *out = sv;
    return OSC_OK;
}

osc_status osc_server_destroy(osc_server* sv)
{
    if (!sv) return OSC_OK;
    {
        std::lock_guard<std::mutex> lock(sv->mu);
        sv->stop = true;
    }
    sv->cv_dispatch.notify_all();
    if (sv->dispatcher.joinable()) sv->dispatcher.join();
    destroy_server(sv);
    return OSC_OK;
}

osc_status osc_server_submit(osc_server* sv, const osc_params* set, int32_t sample,
                             osc_precision precision, uint64_t* ticket)
{
    if (!sv || !set || !ticket || sample < 0 || size_t(sample) >= sv->samples.size())
        return OSC_ERR_INVALID_ARG;
    if (precision != OSC_FP64 && precision != OSC_FP32_MIXED) return OSC_ERR_INVALID_ARG;
    if (osc_validate_params(set, 1) != OSC_OK) return OSC_ERR_INVALID_ARG;
    const size_t budget = size_t(sv->cfg.scratch_budget_bytes) & ~(kArenaAlign - 1);
    if (((sv->need[size_t(sample)] + kArenaAlign - 1) & ~(kArenaAlign - 1)) > budget)
        return OSC_ERR_BUDGET;   // could never be admitted
    {
        std::lock_guard<std::mutex> lock(sv->mu);
        if (int32_t(sv->pending.size()) >= sv->cfg.queue_capacity) {
            ++sv->stats.rejected;
            return OSC_ERR_BUDGET;
        }
        const uint64_t t = sv->next_ticket++;
        Request& r = sv->reqs[t];
        r.params = *set;
        r.sample = sample;
        r.precision = precision;
        r.t_submit = now_s();
        sv->pending.push_back(t);
        ++sv->stats.submitted;
        sv->stats.max_queued = std::max<int64_t>(sv->stats.max_queued, int64_t(sv->pending.size()));
        *ticket = t;
    }
    sv->cv_dispatch.notify_one();
    return OSC_OK;
}

osc_status osc_server_set_data(osc_server* sv, const double* data, double mu_scale)
{
    if (!sv) return OSC_ERR_INVALID_ARG;
    if (data && (!std::isfinite(mu_scale) || !(mu_scale > 0.0))) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(sv->mu);
    if (sv->stats.in_flight > 0) return OSC_ERR_NOT_READY;
    if (!data) {
        sv->has_data = false;
        return OSC_OK;
    }
    const size_t bytes = sv->samples.size() * size_t(sv->binning.nbins) * sizeof(double);
    if (hipSetDevice(sv->device) != hipSuccess) return OSC_ERR_DEVICE;
    if (!sv->d_data && hipMalloc(&sv->d_data, bytes) != hipSuccess) return OSC_ERR_OUT_OF_MEMORY;
    if (hipMemcpy(sv->d_data, data, bytes, hipMemcpyHostToDevice) != hipSuccess)
        return OSC_ERR_DEVICE;
    sv->mu_scale = mu_scale;
    sv->has_data = true;
    return OSC_OK;
}

static osc_status take_result(osc_server* sv, uint64_t ticket, double* hist, double* nll,
                              double* latency_s, double* queue_s)
{
    auto it = sv->reqs.find(ticket);
    Request& r = it->second;
    const osc_status st = r.status;
    if (st == OSC_OK && hist) std::copy(r.hist.begin(), r.hist.end(), hist);
    if (nll) *nll = (st == OSC_OK) ? r.nll : NAN;
    if (latency_s) *latency_s = r.t_done - r.t_submit;
    if (queue_s) *queue_s = r.t_admit - r.t_submit;
    sv->reqs.erase(it);
    return st;
}

osc_status osc_server_poll(osc_server* sv, uint64_t ticket, double* hist, double* nll,
                           double* latency_s, double* queue_s)
{
    if (!sv) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return OSC_ERR_INVALID_ARG;
    if (!it->second.done) return OSC_ERR_NOT_READY;
    return take_result(sv, ticket, hist, nll, latency_s, queue_s);
}

osc_status osc_server_wait(osc_server* sv, uint64_t ticket, double* hist, double* nll,
                           double* latency_s, double* queue_s)
{
    if (!sv) return OSC_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lock(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return OSC_ERR_INVALID_ARG;
    sv->cv_done.wait(lock, [&] {
        auto j = sv->reqs.find(ticket);
        return j == sv->reqs.end() || j->second.done;
    });
    if (sv->reqs.find(ticket) == sv->reqs.end()) return OSC_ERR_INVALID_ARG;
    return take_result(sv, ticket, hist, nll, latency_s, queue_s);
}

osc_status osc_server_get_stats(osc_server* sv, osc_server_stats* out)
{
    if (!sv || !out) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(sv->mu);
    *out = sv->stats;
    out->queued = int64_t(sv->pending.size());
    out->scratch_in_use_bytes = int64_t(sv->arena.used());
    return OSC_OK;
}

osc_status osc_server_reset_stats(osc_server* sv)
{
    if (!sv) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(sv->mu);
    const int64_t in_flight = sv->stats.in_flight;
    sv->stats = osc_server_stats{};
    sv->stats.in_flight = in_flight;
    sv->stats.max_in_flight = in_flight;
    sv->stats.max_queued = int64_t(sv->pending.size());
    sv->stats.peak_scratch_bytes = int64_t(sv->arena.used());
    return OSC_OK;
}

osc_status osc_server_request_bytes(const osc_server* sv, int32_t sample, int64_t* bytes)
{
    if (!sv || !bytes || sample < 0 || size_t(sample) >= sv->samples.size())
        return OSC_ERR_INVALID_ARG;
    *bytes = int64_t(sv->need[size_t(sample)]);
    return OSC_OK;
}

}  // extern "C"
