// Host side of libosc: the C ABI of include/osc.h, argument validation,
// the parameter-only precompute (Sec. 2.1 of arXiv:1311.7579 computes these
// on the CPU and ships them to the GPU), device scratch, kernel launches.
#include <algorithm>
#include <cmath>
#include <complex>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/osc.h"
#include "osc_host_common.h"
#include "osc_internal.h"
#include "osc_launch.h"

namespace {

using cplx = std::complex<double>;

// hbar*c = 197.3269804 MeV fm; N_A = 6.02214076e23 / mol (CODATA 2018);
// G_F / (hbar c)^3 = 1.1663787e-5 GeV^-2.
constexpr double kHbarcEvM = 197.3269804e-9;
constexpr double kAvogadro = 6.02214076e23;
constexpr double kFermiGeV = 1.1663787e-5;

// The phase m^2 L / 2E in natural units per (eV^2 / GeV) over L_km
// kilometres, in units of pi/32 (the form the kernels take), rounded once
// from extended precision.
double phase_steps(double L_km)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double k = 1.0e3L / static_cast<long double>(kHbarcEvM) / 2.0e9L;
    return static_cast<double>(k * static_cast<long double>(L_km) * (32.0L / pi));
}

// 2 sqrt(2) G_F N_e E per (g/cm^3 * GeV * Ye), in eV^2
double matter_constant()
{
    const double hbarc_ev_cm = kHbarcEvM * 1.0e2;
    const double ne_ev3 = kAvogadro * hbarc_ev_cm * hbarc_ev_cm * hbarc_ev_cm;  // per g/cm^3
    return 2.0 * std::sqrt(2.0) * (kFermiGeV * 1.0e-18) * ne_ev3 * 1.0e9;
}

bool is_finite(double x) { return std::isfinite(x); }

bool params_ok(const osc_params& p)
{
    const double s[3] = {p.sin2_th12, p.sin2_th23, p.sin2_th13};
    for (double v : s)
        if (!is_finite(v) || v < 0.0 || v > 1.0) return false;
    if (!is_finite(p.dm2_21) || !(p.dm2_21 > 0.0)) return false;
    if (!is_finite(p.dm2_32) || p.dm2_32 == 0.0) return false;
    const double dm31 = p.dm2_32 + p.dm2_21;
    if (!is_finite(dm31) || dm31 == 0.0) return false;
    if (!is_finite(p.delta_cp)) return false;
    return true;
}

// Mixing matrix (PDG form), rows = flavour (e, mu, tau), columns = mass.
void mixing_matrix(const osc_params& p, cplx U[3][3])
{
    const double s12 = std::sqrt(p.sin2_th12), c12 = std::sqrt(1.0 - p.sin2_th12);
    const double s23 = std::sqrt(p.sin2_th23), c23 = std::sqrt(1.0 - p.sin2_th23);
    const double s13 = std::sqrt(p.sin2_th13), c13 = std::sqrt(1.0 - p.sin2_th13);
    const cplx ep = std::polar(1.0, p.delta_cp);     // e^{+i delta}
    const cplx em = std::conj(ep);
    U[0][0] = c12 * c13;
    U[0][1] = s12 * c13;
    U[0][2] = s13 * em;
    U[1][0] = -s12 * c23 - c12 * s23 * s13 * ep;
    U[1][1] = c12 * c23 - s12 * s23 * s13 * ep;
    U[1][2] = s23 * c13;
    U[2][0] = s12 * s23 - c12 * c23 * s13 * ep;
    U[2][1] = -c12 * s23 - s12 * c23 * s13 * ep;
    U[2][2] = c23 * c13;
}

}  // namespace

// Parameter-only quantities of one set for the kernels.
osc::SetConsts osc::host::set_consts(const osc_params& p)
{
    cplx U[3][3];
    mixing_matrix(p, U);
    const double dm21 = p.dm2_21, dm31 = p.dm2_32 + p.dm2_21;
    const double lv[3] = {0.0, dm21, dm31};

    cplx H[3][3], H2[3][3];   // U diag(lv) U^+ and U diag(lv^2) U^+
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
            cplx h = 0.0, h2 = 0.0;
            for (int i = 0; i < 3; ++i) {
                const cplx t = U[b][i] * std::conj(U[a][i]);
                h += lv[i] * t;
                h2 += lv[i] * lv[i] * t;
            }
            H[b][a] = h;
            H2[b][a] = h2;
        }

    osc::SetConsts sc{};
    sc.T0 = dm21 + dm31;                        // trace of H
    sc.C0 = dm21 * dm31;                        // sum of principal 2x2 minors of H
    sc.CA = H[1][1].real() + H[2][2].real();    // d c1 / dA
    sc.DA = dm21 * dm31 * std::norm(U[0][0]);   // d det / dA = cofactor_ee(H)
    // q/2 = tr^3 - 4.5 tr c1 + 13.5 det as a cubic in A
    sc.QH2 = 3.0 * sc.T0 - 4.5 * sc.CA;
    sc.QH1 = 3.0 * sc.T0 * sc.T0 - 4.5 * (sc.C0 + sc.T0 * sc.CA) + 13.5 * sc.DA;
    sc.QH0 = sc.T0 * (sc.T0 * sc.T0 - 4.5 * sc.C0);
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
            cplx g = 0.0;
            if (b == 0) g += H[0][a];
            if (a == 0) g += H[b][0];
            sc.ch[3 * b + a] = osc::Chan{H[b][a].real(), H[b][a].imag(), H2[b][a].real(),
                                         H2[b][a].imag(), g.real(),          g.imag(),
                                         (a == 0 && b == 0) ? 1.0 : 0.0};
        }
    return sc;
}

namespace {

struct Scratch {
    void* ptr = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;      // recorded after the slot's last use
    bool recorded = false;
    hipStream_t last = nullptr;     // stream of the slot's last use
};

constexpr int kScratchSlots = 4;

// hipEvents around the kernels of one call (profiling only)
struct ProfRec {
    hipEvent_t start = nullptr, mid = nullptr, end = nullptr;
};

}  // namespace

struct osc_ctx {
    int device = 0;
    size_t max_dyn_lds = 0;
    int32_t max_nbins = 0;
    std::vector<osc_params> params;
    std::vector<osc::SetConsts> consts;
    Scratch slots[kScratchSlots];
    int next_slot = 0;
    // While every call has used one stream (`sole`), the stream order alone
    // protects the scratch slots and no event is recorded per call.
    bool one_stream = true;
    bool used = false;
    hipStream_t sole = nullptr;
    double* noalloc = nullptr;      // this device's address of the static scratch array
    bool profiling = false;
    std::vector<ProfRec> prof;
    std::mutex mu;
};

namespace {

osc_status device_status(hipError_t e) { return e == hipSuccess ? OSC_OK : OSC_ERR_DEVICE; }

void drop_profile(osc_ctx* ctx)
{
    for (ProfRec& r : ctx->prof) {
        for (hipEvent_t e : {r.start, r.mid, r.end})
            if (e) (void)hipEventDestroy(e);
    }
    ctx->prof.clear();
}

// Starts a profiling record when profiling is on.  `start` and `mid` are
// handed to the launch of the per-event kernel, which records its own
// begin and end time in them (the dispatch's timestamps, so the interval
// is the kernel's execution alone); `end` is recorded on the stream after
// the merge.
ProfRec* prof_begin(osc_ctx* ctx, hipStream_t)
{
    if (!ctx->profiling) return nullptr;
    ProfRec r;
    if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.mid) != hipSuccess ||
        hipEventCreate(&r.end) != hipSuccess) {
        for (hipEvent_t e : {r.start, r.mid, r.end})
            if (e) (void)hipEventDestroy(e);
        return nullptr;
    }
    ctx->prof.push_back(r);
    return &ctx->prof.back();
}

void prof_mark(hipEvent_t ev, hipStream_t stream)
{
    if (ev) (void)hipEventRecord(ev, stream);
}

// Scratch for one call on `stream`: slots are used round-robin.  While the
// context has seen a single stream, that stream's order already puts every
// use of a slot after the previous one.  The first call on a second stream
// waits once for the device to go idle (the first stream may have been
// destroyed since, so no event can be recorded on it now); from then on
// every call records the slot's event after its use, and a slot last used
// on another stream orders the new stream after that use.
osc_status acquire_scratch(osc_ctx* ctx, size_t bytes, hipStream_t stream, Scratch** out)
{
    if (ctx->one_stream) {
        if (!ctx->used) {
            ctx->used = true;
            ctx->sole = stream;
        } else if (stream != ctx->sole) {
            if (hipDeviceSynchronize() != hipSuccess) return OSC_ERR_DEVICE;
            ctx->one_stream = false;
        }
    }
    Scratch& s = ctx->slots[ctx->next_slot];
    ctx->next_slot = (ctx->next_slot + 1) % kScratchSlots;
    if (s.done == nullptr && hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
        return OSC_ERR_DEVICE;
    if (s.cap < bytes) {
        if (s.ptr) {
            // the slot's last use is on `stream` (one stream) or behind its event
            const hipError_t e = ctx->one_stream ? hipStreamSynchronize(stream)
                                 : s.recorded    ? hipEventSynchronize(s.done)
                                                 : hipSuccess;
            if (e != hipSuccess) return OSC_ERR_DEVICE;
            if (hipFree(s.ptr) != hipSuccess) return OSC_ERR_DEVICE;
            s.ptr = nullptr;
            s.cap = 0;
        }
        const size_t want = (bytes + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1);
        if (hipMalloc(&s.ptr, want) != hipSuccess) {
            s.ptr = nullptr;
            return OSC_ERR_OUT_OF_MEMORY;
        }
        s.cap = want;
        s.recorded = false;
    } else if (s.recorded && s.last != stream) {
        if (hipStreamWaitEvent(stream, s.done, 0) != hipSuccess) return OSC_ERR_DEVICE;
    }
    *out = &s;
    return OSC_OK;
}

osc_status release_scratch(osc_ctx* ctx, Scratch* s, hipStream_t stream)
{
    if (ctx->one_stream) return OSC_OK;
    if (hipEventRecord(s->done, stream) != hipSuccess) return OSC_ERR_DEVICE;
    s->recorded = true;
    s->last = stream;
    return OSC_OK;
}

}  // namespace

bool osc::host::sample_ok(const osc_sample* s, bool needs_hist_inputs)
{
    if (!s || s->n < 0 || s->n > osc::kMaxEvents) return false;
    if (!is_finite(s->L_km) || s->L_km < 0.0) return false;
    if (!is_finite(s->rho_gcc) || s->rho_gcc < 0.0) return false;
    if (!is_finite(s->Ye) || s->Ye < 0.0 || s->Ye > 1.0) return false;
    if (s->n > 0) {
        if (!s->e_true || !s->flags) return false;
        if (needs_hist_inputs && (!s->weight || !s->e_reco)) return false;
    }
    return true;
}

bool osc::host::binning_ok(const osc_ctx* ctx, const osc_binning* b)
{
    if (!b || b->nbins < 1 || b->nbins > ctx->max_nbins) return false;
    if (!is_finite(b->lo) || !is_finite(b->hi) || !(b->lo < b->hi)) return false;
    const double wb = (b->hi - b->lo) / double(b->nbins);
    if (!is_finite(b->e_scale) || !(b->e_scale > -1.0)) return false;
    return is_finite(wb) && wb > 0.0;
}

osc::PathConsts osc::host::path_consts(const osc_sample* s)
{
    return osc::PathConsts{matter_constant() * s->Ye * s->rho_gcc, phase_steps(s->L_km)};
}

osc::BinConsts osc::host::bin_consts(const osc_binning* b)
{
    const double wb = (b->hi - b->lo) / double(b->nbins);
    return osc::BinConsts{b->lo, wb, 1.0 / wb, 1.0 + b->e_scale, b->nbins};
}

int osc::host::ctx_device(const osc_ctx* ctx) { return ctx->device; }

const osc::SinCosTable& osc::host::sincos_table()
{
    static const osc::SinCosTable table = [] {
        osc::SinCosTable t{};
        const long double pi = 3.141592653589793238462643383279502884L;
        for (int k = 0; k < 64; ++k) {
            const long double a = pi * static_cast<long double>(k) / 32.0L;
            t.e[k] = osc::SinCos{static_cast<double>(std::sin(a)), static_cast<double>(std::cos(a))};
        }
        return t;
    }();
    return table;
}

bool osc::host::ctx_set(osc_ctx* ctx, int32_t set, osc::SetConsts* out)
{
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (set < 0 || size_t(set) >= ctx->consts.size()) return false;
    *out = ctx->consts[size_t(set)];
    return true;
}

size_t osc::host::fill_scratch_bytes(int64_t n, int nbins)
{
    const int64_t tiles = (n + osc::kTileEvents - 1) / osc::kTileEvents;
    return osc::merge_scratch_bytes(osc::plan_merge(&tiles, 1, nbins + 2), 1);
}

hipError_t osc::host::enqueue_fill(const osc::SetConsts& sc, const osc_sample* sample,
                                   const uint16_t* bins, const osc_binning* binning, bool mixed,
                                   double* partials, double* hist_out, double* p_out,
                                   hipStream_t stream)
{
    const osc::BinConsts bc = bin_consts(binning);
    const int64_t tiles = (sample->n + osc::kTileEvents - 1) / osc::kTileEvents;
    const osc::MergePlan plan = osc::plan_merge(&tiles, 1, bc.nb + 2);
    hipError_t e = osc::launch_tiles(bins ? 3 : 1, p_out != nullptr, mixed, sc,
                                     path_consts(sample), bc, sample->n, sample->e_true,
                                     sample->flags, sample->weight, bins ? nullptr : sample->e_reco,
                                     bins, nullptr, p_out, partials, stream);
    if (e == hipSuccess) e = osc::launch_merge(plan, 1, partials, hist_out, stream);
    return e;
}

hipError_t osc::host::enqueue_bin_slots(const osc_sample* sample, const osc_binning* binning,
                                        uint16_t* bins, hipStream_t stream)
{
    return osc::launch_bin_slots(sample->n, sample->e_reco, bin_consts(binning), bins, stream);
}

namespace {

using osc::host::bin_consts;
using osc::host::binning_ok;
using osc::host::path_consts;
using osc::host::sample_ok;
using osc::host::set_consts;

// The per-event kernel and the merge of one histogram on `stream`, with
// the tile results and level buffers in `partials` (merge_scratch_bytes of
// `plan`).  t0 / t1 (nullable) receive the per-event kernel's own begin and
// end times.
hipError_t enqueue_hist(int mode, bool write_p, bool mixed, const osc::SetConsts& sc,
                        const osc::PathConsts& pc, const osc::BinConsts& bc, int64_t n,
                        const double* e_true, const uint8_t* flags, const double* weight,
                        const double* e_reco, const uint16_t* bins, const double* value,
                        double* p_out, double* hist_out, const osc::MergePlan& plan,
                        double* partials, hipStream_t stream, const osc::LayerPath* lp,
                        hipEvent_t t0, hipEvent_t t1)
{
    hipError_t e = lp ? osc::launch_layered_tiles(mode, write_p, sc, *lp, bc, n, e_true, flags,
                                                  weight, e_reco, p_out, partials, stream, t0,
                                                  t1)
                      : osc::launch_tiles(mode, write_p, mixed, sc, pc, bc, n, e_true, flags,
                                          weight, e_reco, bins, value, p_out, partials, stream,
                                          t0, t1);
    if (e == hipSuccess) e = osc::launch_merge(plan, 1, partials, hist_out, stream);
    return e;
}

// Tile partials + merge for one histogram on `stream`, in a scratch slot of
// the context.
osc_status run_hist(osc_ctx* ctx, int mode, bool write_p, bool mixed, const osc::SetConsts& sc,
                    const osc::PathConsts& pc, const osc::BinConsts& bc, int64_t n,
                    const double* e_true, const uint8_t* flags, const double* weight,
                    const double* e_reco, const uint16_t* bins, const double* value,
                    double* p_out, double* hist_out, hipStream_t stream,
                    const osc::LayerPath* lp = nullptr)
{
    const int64_t tiles = (n + osc::kTileEvents - 1) / osc::kTileEvents;
    const osc::MergePlan plan = osc::plan_merge(&tiles, 1, bc.nb + 2);
    Scratch* s = nullptr;
    osc_status st = acquire_scratch(ctx, osc::merge_scratch_bytes(plan, 1), stream, &s);
    if (st != OSC_OK) return st;
    ProfRec* pr = prof_begin(ctx, stream);
    const hipError_t e = enqueue_hist(mode, write_p, mixed, sc, pc, bc, n, e_true, flags, weight,
                                      e_reco, bins, value, p_out, hist_out, plan,
                                      static_cast<double*>(s->ptr), stream, lp,
                                      pr ? pr->start : nullptr, pr ? pr->mid : nullptr);
    if (pr) prof_mark(pr->end, stream);
    st = release_scratch(ctx, s, stream);
    if (e != hipSuccess) return OSC_ERR_DEVICE;
    return st;
}

// ---- The entry point that allocates nothing --------------------------------
// osc_fill_pdf_noalloc keeps its tile results and merge level buffers in
// this file-scope array instead of a scratch slot of the context.  Each GPU
// the library runs on holds its own copy for the life of the process.  In
// host code the name stands for a host-side shadow, not a device address:
// kernels are only ever given the address that hipGetSymbolAddress returns
// for the current device (noalloc_address).
static __device__ __align__(256) double scratch[OSC_NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device`, which must be current;
// resolved once per device.  nullptr when the runtime cannot resolve it.
double* noalloc_address(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_noalloc_ptr[device] = static_cast<double*>(ptr);
    }
    return g_noalloc_ptr[device];
}

}  // namespace

extern "C" {

osc_status osc_create(osc_ctx** out, int device)
{
    if (!out) return OSC_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return OSC_ERR_DEVICE;
    if (device < 0 || device >= count) return OSC_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return OSC_ERR_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return OSC_ERR_DEVICE;
    osc_ctx* ctx = new (std::nothrow) osc_ctx();
    if (!ctx) return OSC_ERR_OUT_OF_MEMORY;
    ctx->device = device;
    ctx->noalloc = noalloc_address(device);
    // per-wave histograms: (nbins + 2) x kHistLanes accumulators x 8 B of
    // dynamic LDS, next to the static tables (channels, flags, sin/cos)
    const size_t static_lds = sizeof(osc::TileTables);
    size_t lds = prop.sharedMemPerBlock > static_lds ? prop.sharedMemPerBlock - static_lds : 0;
    if (osc::set_kernel_attributes(lds) != hipSuccess) {
        // keep to the default 64 KiB per workgroup when the larger limit is refused
        (void)hipGetLastError();
        lds = std::min<size_t>(lds, 65536 - static_lds);
    }
    const size_t row = size_t(osc::kHistLanes) * sizeof(double);
    ctx->max_nbins = std::min<int32_t>(int32_t(lds / row) - 2, osc::kMaxBins);
    ctx->max_dyn_lds = lds;
    if (ctx->max_nbins < 1) {
        delete ctx;
        return OSC_ERR_DEVICE;
    }
    *out = ctx;
    return OSC_OK;
}

osc_status osc_destroy(osc_ctx* ctx)
{
    if (!ctx) return OSC_OK;
    osc_status st = OSC_OK;
    (void)hipSetDevice(ctx->device);
    drop_profile(ctx);
    // one stream: it may have been destroyed since its last call, so wait
    // for the device
    if (ctx->one_stream && ctx->used && hipDeviceSynchronize() != hipSuccess) st = OSC_ERR_DEVICE;
    for (Scratch& s : ctx->slots) {
        if (s.recorded && hipEventSynchronize(s.done) != hipSuccess) st = OSC_ERR_DEVICE;
        if (s.ptr && hipFree(s.ptr) != hipSuccess) st = OSC_ERR_DEVICE;
        if (s.done && hipEventDestroy(s.done) != hipSuccess) st = OSC_ERR_DEVICE;
    }
    delete ctx;
    return st;
}

osc_status osc_validate_params(const osc_params* sets, int32_t n_sets)
{
    if (!sets || n_sets < 1) return OSC_ERR_INVALID_ARG;
    for (int32_t k = 0; k < n_sets; ++k)
        if (!params_ok(sets[k])) return OSC_ERR_INVALID_ARG;
    return OSC_OK;
}

osc_status osc_set_params(osc_ctx* ctx, const osc_params* sets, int32_t n_sets)
{
    if (!ctx) return OSC_ERR_INVALID_ARG;
    osc_status st = osc_validate_params(sets, n_sets);
    if (st != OSC_OK) return st;
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        ctx->params.assign(sets, sets + n_sets);
        ctx->consts.resize(size_t(n_sets));
    } catch (...) {
        return OSC_ERR_OUT_OF_MEMORY;
    }
    for (int32_t k = 0; k < n_sets; ++k) ctx->consts[size_t(k)] = set_consts(sets[k]);
    return OSC_OK;
}

osc_status osc_reweight(osc_ctx* ctx, const osc_sample* sample, int32_t set, double* p_out,
                        void* stream)
{
    if (!ctx || !sample_ok(sample, false)) return OSC_ERR_INVALID_ARG;
    if (sample->n > 0 && !p_out) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (set < 0 || size_t(set) >= ctx->consts.size()) return OSC_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return OSC_ERR_DEVICE;
    const osc::BinConsts bc{0.0, 1.0, 1.0, 1.0, 1};
    const hipStream_t hs = static_cast<hipStream_t>(stream);
    ProfRec* pr = prof_begin(ctx, hs);
    const hipError_t e = osc::launch_tiles(0, true, false, ctx->consts[size_t(set)],
                                           path_consts(sample), bc,
                                           sample->n, sample->e_true, sample->flags, nullptr,
                                           nullptr, nullptr, nullptr, p_out, nullptr, hs,
                                           pr ? pr->start : nullptr, pr ? pr->mid : nullptr);
    if (pr) {
        (void)hipEventDestroy(pr->end);
        pr->end = nullptr;
    }
    return device_status(e);
}

osc_status osc_fill_pdf(osc_ctx* ctx, const osc_sample* sample, int32_t set,
                        const osc_binning* binning, osc_precision precision, double* hist_out,
                        double* p_out, void* stream)
{
    if (!ctx || !sample_ok(sample, true) || !hist_out) return OSC_ERR_INVALID_ARG;
    if (!binning_ok(ctx, binning)) return OSC_ERR_INVALID_ARG;
    if (precision != OSC_FP64 && precision != OSC_FP32_MIXED) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (set < 0 || size_t(set) >= ctx->consts.size()) return OSC_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return OSC_ERR_DEVICE;
    return run_hist(ctx, 1, p_out != nullptr, precision == OSC_FP32_MIXED, ctx->consts[size_t(set)],
                    path_consts(sample),
                    bin_consts(binning), sample->n, sample->e_true, sample->flags, sample->weight,
                    sample->e_reco, nullptr, nullptr, p_out, hist_out,
                    static_cast<hipStream_t>(stream));
}

osc_status osc_fill_pdf_noalloc(osc_ctx* ctx, const osc_sample* sample, int32_t set,
                                const osc_binning* binning, osc_precision precision,
                                double* hist_out, double* p_out, void* stream)
{
    if (!ctx || !sample_ok(sample, true) || !hist_out) return OSC_ERR_INVALID_ARG;
    if (!binning_ok(ctx, binning)) return OSC_ERR_INVALID_ARG;
    if (precision != OSC_FP64 && precision != OSC_FP32_MIXED) return OSC_ERR_INVALID_ARG;
    const osc::BinConsts bc = bin_consts(binning);
    const int64_t tiles = (sample->n + osc::kTileEvents - 1) / osc::kTileEvents;
    const osc::MergePlan plan = osc::plan_merge(&tiles, 1, bc.nb + 2);
    if (osc::merge_scratch_bytes(plan, 1) > OSC_NOALLOC_SCRATCH_BYTES) return OSC_ERR_BUDGET;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (set < 0 || size_t(set) >= ctx->consts.size()) return OSC_ERR_INVALID_ARG;
    if (!ctx->noalloc) return OSC_ERR_DEVICE;
    if (hipSetDevice(ctx->device) != hipSuccess) return OSC_ERR_DEVICE;
    const hipError_t e = enqueue_hist(
        1, p_out != nullptr, precision == OSC_FP32_MIXED, ctx->consts[size_t(set)],
        path_consts(sample), bc, sample->n, sample->e_true, sample->flags, sample->weight,
        sample->e_reco, nullptr, nullptr, p_out, hist_out, plan, ctx->noalloc,
        static_cast<hipStream_t>(stream), nullptr, nullptr, nullptr);
    return device_status(e);
}

struct osc_binned {
    osc_ctx* ctx = nullptr;
    osc_sample sample{};        // e_reco is not read after creation
    osc_binning binning{};
    uint16_t* slots = nullptr;  // n cached histogram slots (device)
};

osc_status osc_binned_create(osc_ctx* ctx, const osc_sample* sample, const osc_binning* binning,
                             osc_binned** out)
{
    if (!out) return OSC_ERR_INVALID_ARG;
    *out = nullptr;
    if (!ctx || !sample_ok(sample, true) || !binning_ok(ctx, binning)) return OSC_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return OSC_ERR_DEVICE;
    osc_binned* b = new (std::nothrow) osc_binned();
    if (!b) return OSC_ERR_OUT_OF_MEMORY;
    b->ctx = ctx;
    b->sample = *sample;
    b->binning = *binning;
    if (sample->n > 0 &&
        hipMalloc(&b->slots, size_t(sample->n) * sizeof(uint16_t)) != hipSuccess) {
        delete b;
        return OSC_ERR_OUT_OF_MEMORY;
    }
    // synchronous: after earlier work on the device (the caller's uploads),
    // and the slots are ready on return
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = osc::host::enqueue_bin_slots(sample, binning, b->slots, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        if (b->slots) (void)hipFree(b->slots);
        delete b;
        return OSC_ERR_DEVICE;
    }
    *out = b;
    return OSC_OK;
}

osc_status osc_binned_destroy(osc_binned* b)
{
    if (!b) return OSC_OK;
    osc_status st = OSC_OK;
    if (b->slots) {
        if (hipSetDevice(b->ctx->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
            hipFree(b->slots) != hipSuccess)
            st = OSC_ERR_DEVICE;
    }
    delete b;
    return st;
}

osc_status osc_fill_pdf_binned(osc_ctx* ctx, const osc_binned* b, int32_t set,
                               osc_precision precision, double* hist_out, double* p_out,
                               void* stream)
{
    if (!ctx || !b || b->ctx != ctx || !hist_out) return OSC_ERR_INVALID_ARG;
    if (precision != OSC_FP64 && precision != OSC_FP32_MIXED) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (set < 0 || size_t(set) >= ctx->consts.size()) return OSC_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return OSC_ERR_DEVICE;
    const osc_sample& s = b->sample;
    return run_hist(ctx, 3, p_out != nullptr, precision == OSC_FP32_MIXED,
                    ctx->consts[size_t(set)], path_consts(&s), bin_consts(&b->binning), s.n,
                    s.e_true, s.flags, s.weight, nullptr, b->slots, nullptr, p_out, hist_out,
                    static_cast<hipStream_t>(stream));
}

namespace {

// Layers of a piecewise-constant path: 1..kMaxLayers layers, each with
// L >= 0, rho >= 0 (finite) and 0 <= Ye <= 1.
bool layers_ok(const osc_layer* layers, int32_t n_layers)
{
    if (!layers || n_layers < 1 || n_layers > osc::kMaxLayers) return false;
    for (int32_t j = 0; j < n_layers; ++j) {
        const osc_layer& l = layers[j];
        if (!is_finite(l.L_km) || l.L_km < 0.0 || !is_finite(l.rho_gcc) || l.rho_gcc < 0.0 ||
            !is_finite(l.Ye) || l.Ye < 0.0 || l.Ye > 1.0)
            return false;
    }
    return true;
}

osc::LayerPath layer_path(const osc_layer* layers, int32_t n_layers)
{
    osc::LayerPath lp{};
    lp.n = n_layers;
    for (int32_t j = 0; j < n_layers; ++j)
        lp.layer[j] = osc::PathConsts{matter_constant() * layers[j].Ye * layers[j].rho_gcc,
                                      phase_steps(layers[j].L_km)};
    return lp;
}

}  // namespace

osc_status osc_reweight_layered(osc_ctx* ctx, const osc_sample* sample, const osc_layer* layers,
                                int32_t n_layers, int32_t set, double* p_out, void* stream)
{
    if (!ctx || !sample_ok(sample, false) || !layers_ok(layers, n_layers))
        return OSC_ERR_INVALID_ARG;
    if (sample->n > 0 && !p_out) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (set < 0 || size_t(set) >= ctx->consts.size()) return OSC_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return OSC_ERR_DEVICE;
    const osc::BinConsts bc{0.0, 1.0, 1.0, 1.0, 1};
    const hipStream_t hs = static_cast<hipStream_t>(stream);
    ProfRec* pr = prof_begin(ctx, hs);
    const hipError_t e = osc::launch_layered_tiles(
        0, true, ctx->consts[size_t(set)], layer_path(layers, n_layers), bc, sample->n,
        sample->e_true, sample->flags, nullptr, nullptr, p_out, nullptr, hs,
        pr ? pr->start : nullptr, pr ? pr->mid : nullptr);
    if (pr) {
        (void)hipEventDestroy(pr->end);
        pr->end = nullptr;
    }
    return device_status(e);
}

osc_status osc_fill_pdf_layered(osc_ctx* ctx, const osc_sample* sample, const osc_layer* layers,
                                int32_t n_layers, int32_t set, const osc_binning* binning,
                                double* hist_out, double* p_out, void* stream)
{
    if (!ctx || !sample_ok(sample, true) || !hist_out || !layers_ok(layers, n_layers))
        return OSC_ERR_INVALID_ARG;
    if (!binning_ok(ctx, binning)) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (set < 0 || size_t(set) >= ctx->consts.size()) return OSC_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return OSC_ERR_DEVICE;
    const osc::LayerPath lp = layer_path(layers, n_layers);
    return run_hist(ctx, 1, p_out != nullptr, false, ctx->consts[size_t(set)], osc::PathConsts{},
                    bin_consts(binning), sample->n, sample->e_true, sample->flags,
                    sample->weight, sample->e_reco, nullptr, nullptr, p_out, hist_out,
                    static_cast<hipStream_t>(stream), &lp);
}

osc_status osc_fill_hist(osc_ctx* ctx, int64_t n, const double* value, const double* weight,
                         const double* e_reco, const osc_binning* binning, double* hist_out,
                         void* stream)
{
    if (!ctx || n < 0 || n > osc::kMaxEvents || !hist_out) return OSC_ERR_INVALID_ARG;
    if (n > 0 && (!value || !weight || !e_reco)) return OSC_ERR_INVALID_ARG;
    if (!binning_ok(ctx, binning)) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return OSC_ERR_DEVICE;
    const osc::SetConsts sc{};
    const osc::PathConsts pc{0.0, 0.0};
    return run_hist(ctx, 2, false, false, sc, pc, bin_consts(binning), n, nullptr, nullptr, weight,
                    e_reco, nullptr, value, nullptr, hist_out, static_cast<hipStream_t>(stream));
}

osc_status osc_profile_enable(osc_ctx* ctx, int on)
{
    if (!ctx) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(ctx->mu);
    drop_profile(ctx);
    ctx->profiling = on != 0;
    return OSC_OK;
}

osc_status osc_profile_read(osc_ctx* ctx, double* event_kernel_ms, int64_t* event_kernel_launches,
                            double* merge_kernel_ms, int64_t* merge_kernel_launches)
{
    if (!ctx) return OSC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(ctx->mu);
    double tile_ms = 0.0, merge_ms = 0.0;
    int64_t tiles = 0, merges = 0;
    osc_status st = OSC_OK;
    for (const ProfRec& r : ctx->prof) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.mid) != hipSuccess ||
            hipEventElapsedTime(&ms, r.start, r.mid) != hipSuccess) {
            st = OSC_ERR_DEVICE;
            break;
        }
        tile_ms += ms;
        ++tiles;
        if (r.end) {
            if (hipEventSynchronize(r.end) != hipSuccess ||
                hipEventElapsedTime(&ms, r.mid, r.end) != hipSuccess) {
                st = OSC_ERR_DEVICE;
                break;
            }
            merge_ms += ms;
            ++merges;
        }
    }
    drop_profile(ctx);
    if (event_kernel_ms) *event_kernel_ms = tile_ms;
    if (event_kernel_launches) *event_kernel_launches = tiles;
    if (merge_kernel_ms) *merge_kernel_ms = merge_ms;
    if (merge_kernel_launches) *merge_kernel_launches = merges;
    return st;
}

osc_status osc_poisson_nll(osc_ctx* ctx, const double* hist, int64_t n_hist, double mu_scale,
                           const double* data, int64_t n_data, int32_t nbins, double* nll_out,
                           void* stream)
{
    if (!ctx || n_hist < 0 || n_data < 1 || nbins < 1 || nbins > ctx->max_nbins)
        return OSC_ERR_INVALID_ARG;
    if (!is_finite(mu_scale) || !(mu_scale > 0.0)) return OSC_ERR_INVALID_ARG;
    if (n_hist > 0 && (!hist || !data || !nll_out)) return OSC_ERR_INVALID_ARG;
    if (n_hist > int64_t(1) << 31) return OSC_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return OSC_ERR_DEVICE;
    return device_status(osc::launch_poisson_nll(hist, n_hist, mu_scale, data, n_data, nbins,
                                                 nll_out, static_cast<hipStream_t>(stream)));
}

osc_status osc_validate_sample(osc_ctx* ctx, const osc_sample* sample, int64_t* bad_energy,
                               int64_t* bad_flags, void* stream)
{
    if (!ctx || !sample_ok(sample, false)) return OSC_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return OSC_ERR_DEVICE;
    const hipStream_t hs = static_cast<hipStream_t>(stream);
    unsigned long long* d = nullptr;
    unsigned long long h[2] = {0, 0};
    if (hipMalloc(&d, sizeof h) != hipSuccess) return OSC_ERR_OUT_OF_MEMORY;
    hipError_t e = hipMemsetAsync(d, 0, sizeof h, hs);
    if (e == hipSuccess)
        e = osc::launch_validate_sample(sample->n, sample->e_true, sample->flags, d, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    (void)hipFree(d);
    if (e != hipSuccess) return OSC_ERR_DEVICE;
    if (bad_energy) *bad_energy = int64_t(h[0]);
    if (bad_flags) *bad_flags = int64_t(h[1]);
    return OSC_OK;
}

void osc_reduction_layout(int32_t* tile_lanes, int32_t* lane_events, int32_t* accumulators)
{
    if (tile_lanes) *tile_lanes = osc::kTileLanes;
    if (lane_events) *lane_events = osc::kLaneEvents;
    if (accumulators) *accumulators = osc::kHistLanes;
}

int32_t osc_max_nbins(const osc_ctx* ctx) { return ctx ? ctx->max_nbins : 0; }

osc_status osc_occupancy(const osc_ctx* ctx, int32_t nbins, int with_hist, int32_t* waves_per_cu)
{
    if (!ctx || !waves_per_cu) return OSC_ERR_INVALID_ARG;
    if (with_hist && (nbins < 1 || nbins > ctx->max_nbins)) return OSC_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return OSC_ERR_DEVICE;
    int blocks = 0;
    if (osc::occupancy(with_hist ? 1 : 0, nbins, &blocks) != hipSuccess) return OSC_ERR_DEVICE;
    *waves_per_cu = blocks;
    return OSC_OK;
}

const char* osc_status_string(osc_status status)
{
    switch (status) {
        case OSC_OK: return "ok";
        case OSC_ERR_INVALID_ARG: return "invalid argument";
        case OSC_ERR_OUT_OF_MEMORY: return "out of device memory";
        case OSC_ERR_DEVICE: return "no usable device or HIP runtime error";
        case OSC_ERR_BUDGET: return "over memory budget";
        case OSC_ERR_NOT_READY: return "not ready";
    }
    return "unknown status";
}

}  // extern "C"
