/*
 * osc.h -- C ABI of libosc: event-by-event three-flavour neutrino
 * oscillation reweighting through constant-density matter on AMD MI355X
 * (gfx950), after arXiv:1311.7579.
 *
 * The operation (Sec. 1.1, 1.1.1, 2.1 of the paper): for every Monte Carlo
 * event with true energy E, initial flavour alpha, final flavour beta and a
 * neutrino / antineutrino flag, compute the oscillation probability
 * P(alpha -> beta) over a baseline L through matter of constant density
 * (matter effects on nu_e from forward scattering on electrons), in double
 * precision; then weight the event by w * P and fill a binned
 * reconstructed-energy PDF.  Parameter-only quantities are computed on the
 * host (Sec. 2.1) and the per-event work runs in HIP kernels.
 *
 * Units: E in GeV, L in km, mass splittings in eV^2, density in g/cm^3,
 * Ye = electrons per nucleon.  Flavour index 0 = e, 1 = mu, 2 = tau.
 *
 * Execution model: every call that takes a stream enqueues its kernels on
 * that stream (a hipStream_t passed as void*, NULL = the null stream) and
 * returns before they finish; results are valid once the stream has
 * synchronised.  All device pointers are caller-owned device memory (for
 * example torch tensors' data pointers) and must stay alive until then.
 * A context's device scratch is ordered by the stream alone while all its
 * calls use one stream; the first call on a second stream waits once for
 * the device to go idle, and later calls order the scratch through events.
 * Errors are reported as status codes; nothing aborts the process.
 */
#ifndef OSC_H
#define OSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OSC_OK = 0,
    OSC_ERR_INVALID_ARG = 1,   /* a NULL pointer, a value outside its domain */
    OSC_ERR_OUT_OF_MEMORY = 2, /* device scratch could not be allocated      */
    OSC_ERR_DEVICE = 3,        /* no usable GPU, or a HIP runtime failure     */
    OSC_ERR_BUDGET = 4,        /* over a memory budget or a fixed capacity    */
    OSC_ERR_NOT_READY = 5      /* reserved: result not available yet          */
} osc_status;

typedef enum {
    OSC_FP64 = 0,        /* every step in FP64 (the paper's precision, Sec. 2.1) */
    OSC_FP32_MIXED = 1   /* FP64 eigenvalues and phases, FP32 amplitude assembly
                            (eigenvalues refined until within ~1e-11 of their
                            smallest distance, not to the last bit; waves
                            with |A| > 0.01 eV^2 assemble in FP64).
                            Measured |P - P_exact|: <= 1.5e-6 for Table
                            1-like sets at 295 km, <= 6e-6 to 2500 km and
                            for near-measured angles anywhere, <= 1.8e-5
                            for any angles at E <= 20 GeV through rho <= 3
                            g/cm^3, ~5e-5 at worst (any angles, long L/E
                            near the solar resonance)                      */
} osc_precision;

/* Opaque context bound to one device: holds the parameter sets and the
 * device scratch used by the histogram reduction. */
typedef struct osc_ctx osc_ctx;

/* One oscillation parameter set: the six rows of Table 1.
 * sin2_th12, sin2_th23, sin2_th13 in [0, 1]; dm2_21 > 0;
 * dm2_32 != 0 (positive: normal ordering) and dm2_32 + dm2_21 != 0, so the
 * three vacuum levels (0, dm2_21, dm2_32 + dm2_21) are distinct;
 * delta_cp in radians, finite. */
typedef struct {
    double sin2_th12, sin2_th23, sin2_th13;
    double dm2_32, dm2_21;
    double delta_cp;
} osc_params;

/* A Monte Carlo sample in struct-of-arrays layout (Sec. 2.1 keeps the
 * per-event energies in a device array).  All four arrays are device
 * pointers with n entries (they may be NULL when n == 0):
 *   e_true  FP64, true energy in GeV, must be > 0 (not checked per event;
 *           E <= 0 gives an undefined probability);
 *   flags   one byte per event: bits 0-1 alpha, bits 2-3 beta (3 is
 *           invalid), bit 4 antineutrino, bits 5-7 zero.  Invalid flag
 *           bytes give P = NaN;
 *   weight  FP64 Monte Carlo weight, any value (only read by the
 *           histogram calls);
 *   e_reco  FP64 reconstructed energy in GeV (only read by osc_fill_pdf).
 * L_km >= 0, rho_gcc >= 0, 0 <= Ye <= 1 describe the constant-density path. */
typedef struct {
    int64_t n;
    const double* e_true;
    const uint8_t* flags;
    const double* weight;
    const double* e_reco;
    double L_km, rho_gcc, Ye;
} osc_sample;

/* Regular binning of the reconstructed energy: nbins bins of width
 * wb = (hi - lo) / nbins (IEEE FP64).  With x = e_reco * (1 + e_scale)
 * (both operations in FP64, e_scale a relative energy-scale shift, 0 for
 * none; Sec. 1.1.1 names this systematic and the event migration it
 * causes), an event falls into bin floor((x - lo) / wb) (FP64 subtraction
 * and division), into the underflow entry when that quotient is negative,
 * and into the overflow entry when it is >= nbins or NaN.  Histogram
 * layout: nbins bins, underflow, overflow.
 * 1 <= nbins <= osc_max_nbins(); lo < hi, both finite; e_scale > -1. */
typedef struct {
    int32_t nbins;
    double lo, hi;
    double e_scale;
} osc_binning;

/* Create a context on HIP device `device`.  Returns OSC_ERR_DEVICE when no
 * GPU is present or the device index is out of range; *out is then NULL. */
osc_status osc_create(osc_ctx** out, int device);

/* Release a context and its device scratch after waiting for the work it
 * enqueued.  NULL is accepted. */
osc_status osc_destroy(osc_ctx* ctx);

/* Check parameter sets without a device (the domain rules of osc_params).
 * Returns OSC_ERR_INVALID_ARG for the first invalid set. */
osc_status osc_validate_params(const osc_params* sets, int32_t n_sets);

/* Store n_sets >= 1 parameter sets in the context, replacing earlier ones,
 * and compute their parameter-only quantities on the host (Sec. 2.1:
 * mixing matrix, vacuum mass matrix in the flavour basis and its square,
 * the constants of the characteristic cubic).  The host array is copied;
 * the caller may free it on return.  Kernels already enqueued keep the
 * values they were launched with. */
osc_status osc_set_params(osc_ctx* ctx, const osc_params* sets, int32_t n_sets);

/* One-time check of a sample's per-event domain, which the per-event
 * kernels do not make: *bad_energy receives the number of events whose
 * true energy is not finite and > 0 (their P is undefined), *bad_flags the
 * number with an invalid flag byte (their P is NaN).  Either output may be
 * NULL.  Synchronous on `stream` (returns after the counts are on the
 * host). */
osc_status osc_validate_sample(osc_ctx* ctx, const osc_sample* sample, int64_t* bad_energy,
                               int64_t* bad_flags, void* stream);

/* Sec. 2.1 (the paper's kernel): write P(alpha -> beta) of every event of
 * `sample` under parameter set `set` to p_out (device, n FP64 entries,
 * event order).  weight and e_reco are not read.
 * Accuracy domain (all per-event entry points): P is within about 1e-12 of
 * the exact value, plus 2^-53 |A| / gap from the amplitude's own
 * cancellation and 4 * 2^-53 * phi * (1 + spread / gap) from the FP64
 * rounding of the largest phase difference phi (radians), amplified by
 * the eigenvalues' conditioning (gap and spread: the smallest and largest
 * distance between the eigenvalues of the matter Hamiltonian; the phase
 * term reaches 1e-12 where phi * (1 + spread / gap) reaches about 2e3),
 * for matter terms |A| = K_A Ye rho E up to about 1 eV^2 with mixing
 * angles near the measured ones (Table 1: E rho Ye up to ~6500 GeV
 * g/cm^3), and up to about 0.04 eV^2 for arbitrary angles.  Beyond that
 * the FP32 seeds of the eigenvalue solver can no longer resolve the two
 * roots that stay near the vacuum masses and P is not reliable.
 * Exact level crossings: with a zero mixing angle a mass state decouples
 * from nu_e and two eigenvalues cross at one matter term (with a very
 * small angle they nearly do).  Events whose two closest eigenvalues lie
 * within about 7e-4 of the spread (next to the atmospheric crossing with
 * sin2_th13 = 0, a window of about +-7e-4 of its energy; next to the solar
 * one with sin2_th12 = 0, +-2 %) cannot be resolved from the
 * characteristic cubic; their P is NaN, in both precision tiers and on
 * layered paths.  Farther from the crossing the statement above holds
 * (the FP32-mixed tier: within 3e-4). */
osc_status osc_reweight(osc_ctx* ctx, const osc_sample* sample, int32_t set,
                        double* p_out, void* stream);

/* Sec. 1.1.1 event-by-event reweighting: compute P per event, the
 * contribution c = w * P (rounded separately, never fused), the bin of
 * e_reco, and the histogram hist_out (device, nbins + 2 FP64 entries,
 * overwritten).  p_out (device, n entries) may be NULL; when given it
 * receives P.
 *
 * The histogram is bit-reproducible: it is the sum of the c values in a
 * fixed order that depends only on n and the event order, never on the
 * launch shape (see osc_reduction_layout): tiles of W*K consecutive events;
 * lane l of tile t takes events t*W*K + m*W + l (m = 0..K-1) and adds them
 * into accumulator l mod A of their bin; each accumulator starts from +0.0
 * and receives its additions in ascending m and, within one m, in
 * ascending l; per bin, the A accumulators of a tile meet in the complete
 * binary tree over accumulator index; the tile results meet in the
 * complete binary tree over tile index, padded with +0.0 to a power of two.
 * Every addition is an IEEE FP64 round-to-nearest-even addition, for any
 * contribution: negative, +-0, subnormal, infinite and NaN weights (or P)
 * enter the sum as they are, with the same bits as that order of plain
 * FP64 additions (a NaN's payload aside). */
osc_status osc_fill_pdf(osc_ctx* ctx, const osc_sample* sample, int32_t set,
                        const osc_binning* binning, osc_precision precision,
                        double* hist_out, double* p_out, void* stream);

/* ---- Cached reco-energy bins (Sec. 1.1.1) ----
 * Event-by-event reweighting changes only the weights w * P of the events;
 * the bin of each event's reconstructed energy stays the same from one
 * parameter set to the next.  A binned sample computes it once: for every
 * event the histogram slot its contribution goes to (the bin by the rule
 * of osc_binning, and the event's accumulator in the reduction contract),
 * 2 bytes of device memory per event.  osc_fill_pdf_binned then reads
 * those 2 bytes instead of the 8-byte reco energy and skips the bin
 * arithmetic; its results are bit-identical to osc_fill_pdf with the same
 * sample and binning. */
typedef struct osc_binned osc_binned;

/* Bin `sample` (device arrays as in osc_sample; e_reco is read here and
 * never again; e_true, flags and weight must stay valid and unchanged for
 * the life of the binned sample) under `binning` (e_scale included; a
 * different shift needs its own binned sample).  Allocates n 16-bit
 * entries of device memory owned by the binned sample.  Synchronous: waits
 * for all earlier work on the device, returns once the bins are on it. */
osc_status osc_binned_create(osc_ctx* ctx, const osc_sample* sample,
                             const osc_binning* binning, osc_binned** out);

/* Wait for the device and free the binned sample. NULL is accepted. */
osc_status osc_binned_destroy(osc_binned* binned);

/* osc_fill_pdf on a binned sample of the same context (the binning and
 * path are the binned sample's): hist_out (device, nbins + 2 FP64
 * entries) and p_out (device, n entries, nullable) as for osc_fill_pdf,
 * with the same bits. */
osc_status osc_fill_pdf_binned(osc_ctx* ctx, const osc_binned* binned, int32_t set,
                               osc_precision precision, double* hist_out, double* p_out,
                               void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * osc_fill_pdf with the same arguments, kernels and results (bit for bit),
 * that keeps its tile results and merge buffers in a fixed array of
 * OSC_NOALLOC_SCRATCH_BYTES of device memory inside the library instead of
 * the context's scratch.  It calls no hipMalloc, hipFree or other
 * allocating routine.  The array's address on a device is resolved once,
 * by osc_create on that device; each GPU holds its own array until the
 * process ends.  Bytes needed: 8 (nbins + 2) (R + 2 S), with
 * R = 128 ceil(T / 128) rows of tile results for T = ceil(n / 1024) tiles,
 * and S = 0 for T <= 16384, else S = 128 ceil(ceil(T / 16384) / 128)
 * (about 8 MiB for 2e7 events at 50 bins); larger requests return
 * OSC_ERR_BUDGET before anything is enqueued.  Every call on a GPU, from
 * any context, shares that GPU's array: calls whose work overlaps on the
 * device (different streams, or other threads) race and give undefined
 * histograms; calls ordered on one stream are safe.  Nothing in the array
 * needs to start at zero: every call writes what it reads. */
#define OSC_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
osc_status osc_fill_pdf_noalloc(osc_ctx* ctx, const osc_sample* sample, int32_t set,
                                const osc_binning* binning, osc_precision precision,
                                double* hist_out, double* p_out, void* stream);

/* The reduction of osc_fill_pdf on given per-event values: histogram of
 * e_reco with contributions c = weight * value (separately rounded), same
 * binning rule and the same reduction order.  All arrays are device
 * pointers with n entries; hist_out has nbins + 2 entries. */
osc_status osc_fill_hist(osc_ctx* ctx, int64_t n, const double* value,
                         const double* weight, const double* e_reco,
                         const osc_binning* binning, double* hist_out, void* stream);

/* Device-side timing of the kernels this context launches: while enabled,
 * every call records hipEvents on its stream around the per-event kernel
 * and around the histogram merge.  Enabling (on != 0) or disabling drops
 * earlier records. */
osc_status osc_profile_enable(osc_ctx* ctx, int on);

/* Wait for the recorded kernels and return the summed durations in
 * milliseconds and the launch counts of the per-event kernel and of the
 * merge kernel since the last enable or read; then drop the records.
 * Any output pointer may be NULL. */
osc_status osc_profile_read(osc_ctx* ctx, double* event_kernel_ms, int64_t* event_kernel_launches,
                            double* merge_kernel_ms, int64_t* merge_kernel_launches);

/* ---- Piecewise-constant matter ----
 * The paper takes one constant density (Sec. 1.1); a path through layers
 * of different densities (the extension the paper's CPU library, Prob3++,
 * makes for paths through the Earth) evolves the neutrino with the
 * product of the layers' evolution operators, each the constant-density
 * operator of Sec. 1.1 for its own density and length:
 *   S = S_{n-1} ... S_1 S_0,  P(alpha -> beta) = |S_{beta alpha}|^2,
 * layer 0 crossed first.  Computed in FP64 by propagating column alpha
 * through the layers. */
typedef struct {
    double L_km;     /* layer length, >= 0 */
    double rho_gcc;  /* density, >= 0      */
    double Ye;       /* electrons per nucleon, 0..1 */
} osc_layer;

/* osc_reweight through n_layers (1..32) layers, host array, copied; the
 * sample's own L_km, rho_gcc and Ye are not used. */
osc_status osc_reweight_layered(osc_ctx* ctx, const osc_sample* sample, const osc_layer* layers,
                                int32_t n_layers, int32_t set, double* p_out, void* stream);

/* osc_fill_pdf (FP64) through n_layers layers: same binning rule, same
 * reduction contract, so the histogram is bit-identical to osc_fill_hist
 * applied to the P it computes. */
osc_status osc_fill_pdf_layered(osc_ctx* ctx, const osc_sample* sample, const osc_layer* layers,
                                int32_t n_layers, int32_t set, const osc_binning* binning,
                                double* hist_out, double* p_out, void* stream);

/* ---- Bin-centre reweighting (Sec. 1.1.1) ----
 * The approximation that event-by-event reweighting replaces: apply a
 * parameter set at the centre of each true-energy bin and to the whole
 * bin.  The sample is reduced once to a migration template
 *   T[r][c][t] = sum of the weights of the events of channel c in true
 *                bin t and reconstructed bin r,
 * channel c = alpha + 3 beta + 9 anti (18 channels), each cell's weights
 * added in ascending event order from +0.0.  A call then computes
 *   P[c][t] = P_c(E_t),  E_t = lo_t + (t + 1/2) * ((hi_t - lo_t) / nt)
 *   hist[r] = sum over k = c nt + t of fl(T[r][k] * P[k]),
 * the terms of each r in a fixed order: term k goes to lane k mod 64, each
 * lane adds its terms in ascending k from +0.0, and the 64 lane sums meet
 * in the complete binary tree over lane index.  The result is
 * bit-reproducible. */
typedef struct osc_template osc_template;

/* Build the template of `sample` (device arrays as in osc_sample, n up to
 * 2^31 - 1; weight and e_reco are read).  true_binning: the true-energy
 * bins, 1 <= nbins <= 65536, 0 <= lo < hi, e_scale = 0; events whose true
 * energy falls outside [0, nbins) by the binning rule of osc_binning, and
 * events with an invalid flag byte, are left out.  reco_binning: as for
 * osc_fill_pdf (e_scale applies; under/overflow rows kept).  Synchronous:
 * waits for all earlier work on the device, returns once the template is
 * built, after which the sample arrays are no
 * longer read; the path (L, rho, Ye) is taken from `sample`.  *n_used
 * (may be NULL) receives the number of events in the template.  The
 * template holds (nbins_reco + 2) * 18 * nbins_true FP64 values of device
 * memory and belongs to ctx. */
osc_status osc_template_create(osc_ctx* ctx, const osc_sample* sample,
                               const osc_binning* true_binning,
                               const osc_binning* reco_binning, osc_template** out,
                               int64_t* n_used);

/* Wait for the device and free the template. NULL is accepted. */
osc_status osc_template_destroy(osc_template* t);

/* Copy the template, layout [r][c][t], to dst (device, (nbins_reco + 2) *
 * 18 * nbins_true FP64 entries) on `stream`. */
osc_status osc_template_copy(const osc_template* t, double* dst, void* stream);

/* Bin-centre PDF of parameter set `set`: hist_out (device, nbins_reco + 2
 * entries, overwritten).  p_centre_out (device, 18 * nbins_true entries,
 * layout [c][t]) may be NULL; when given it receives the probabilities at
 * the bin centres and serves as the call's table.  Without it the table is
 * the template's own buffer, so calls on one template without
 * p_centre_out must not overlap (one stream at a time). */
osc_status osc_fill_pdf_bincentre(osc_ctx* ctx, const osc_template* t, int32_t set,
                                  double* hist_out, double* p_centre_out, void* stream);

/* Sec. 2.2, Eq. (2): the binned likelihood of the fitter, read as a
 * product over the regular bins of Poisson probabilities of observed counts
 * d_b given the expectation mu_b = mu_scale * hist_b (mu_scale > 0: the
 * exposure that turns the Monte Carlo PDF into expected counts):
 *   -2 ln L = 2 sum_b (mu_b - d_b ln mu_b + ln d_b!)
 * (a bin with mu_b = 0 adds 0 if d_b = 0, else +infinity; under/overflow
 * entries are not used).  hist: device, n_hist histograms of nbins + 2
 * entries (the layout of osc_fill_pdf / osc_batch_run); data: device,
 * n_data rows of nbins counts, histogram k compared with row k % n_data
 * (so batched histograms [set][sample] pair with per-sample data rows);
 * nll_out: device, n_hist values.  The sum over bins has a fixed order. */
osc_status osc_poisson_nll(osc_ctx* ctx, const double* hist, int64_t n_hist, double mu_scale,
                           const double* data, int64_t n_data, int32_t nbins, double* nll_out,
                           void* stream);

/* ---- Batched form ---------------------------------------------------------
 * Every parameter set x every sample of a list in one persistent kernel
 * launch plus the histogram merge (the fitter evaluating many proposals, or
 * one proposal against several samples).  Each (set, sample) histogram is
 * bit-identical to osc_fill_pdf on that set and sample in the same
 * precision, for every launch configuration. */
typedef struct osc_batch osc_batch;

typedef struct {
    int32_t sets_per_item; /* parameter sets one wave evaluates per tile (1..64)   */
    int32_t schedule;      /* 0: persistent waves taking tiles from an atomic queue;
                              1: persistent waves striding over the tiles;
                              2: one workgroup per tile                            */
    int32_t waves_per_cu;  /* persistent grid = CUs x waves_per_cu, 0 = occupancy   */
    int32_t use_graph;     /* 1: replay a captured HIP graph, 0: launch directly    */
} osc_batch_config;

/* Prepare a batched evaluation over n_samples (1..16) resident samples
 * (device arrays as in osc_sample; e_true, flags and weight must stay valid
 * and unchanged for the life of the batch; e_reco is read only here, where
 * every event's histogram slot is cached as for osc_binned_create, 2 bytes
 * per event), one binning and one precision, for up to max_sets
 * (1..65535) parameter sets per run.  Synchronous (waits for earlier work
 * on the device).  Allocates the device scratch (tile results of
 * max_sets sets) and chooses a default configuration.  OSC_ERR_INVALID_ARG
 * also when max_sets x (the samples' tiles of 1024 events) work items
 * would overflow the 32-bit work counter of the persistent schedules. */
osc_status osc_batch_create(osc_ctx* ctx, const osc_sample* samples, int32_t n_samples,
                            const osc_binning* binning, osc_precision precision, int32_t max_sets,
                            osc_batch** out);

/* Wait for the device and free the batch. NULL is accepted. */
osc_status osc_batch_destroy(osc_batch* batch);

osc_status osc_batch_get_config(const osc_batch* batch, osc_batch_config* cfg);
osc_status osc_batch_set_config(osc_batch* batch, const osc_batch_config* cfg);

/* Evaluate n_sets (1..max_sets) parameter sets on every sample (with the
 * one-workgroup-per-tile schedule, OSC_ERR_INVALID_ARG when the work items,
 * (tiles) x ceil(n_sets / sets_per_item), exceed the 2^32 - 1 work-items of
 * one grid at 64 per workgroup; the autotuner skips such candidates): host
 * precompute of the sets (Sec. 2.1), an asynchronous upload, one graph
 * replay (kernel + merge) and a device copy of the histograms to hist_out
 * (device, n_sets x n_samples x (nbins + 2) FP64, set-major).  Runs on
 * `stream`; a batch serves one stream at a time.  The host array may be
 * freed on return. */
osc_status osc_batch_run(osc_batch* batch, const osc_params* sets, int32_t n_sets,
                         double* hist_out, void* stream);

/* Autotuner: time every candidate configuration (sets per item x schedule)
 * on these parameter sets and keep the fastest.  With cache_path, a result
 * recorded there for the same shape (tier, bins, samples, sets, log2 of the
 * tile count) is reused without timing, and new results are appended.
 * best_ms (nullable) receives the winning time, or -1 when cached.
 * Blocks until the timing runs have finished. */
osc_status osc_batch_tune(osc_batch* batch, const osc_params* sets, int32_t n_sets,
                          const char* cache_path, double* best_ms, void* stream);

/* ---- Serving form ----------------------------------------------------------
 * A request loop for fitter proposals: each request is one parameter set on
 * one resident sample in one precision tier.  Requests are queued first in,
 * first out; a dispatcher thread admits the head of the queue when one of
 * `slots` HIP streams is free and the request's device scratch fits in the
 * remaining budget; admitted requests run concurrently.  A request's
 * histogram is the same, bit for bit, as osc_fill_pdf of the same set,
 * sample and tier, alone or in any mix. */
typedef struct osc_server osc_server;

typedef struct {
    int32_t slots;                /* requests in flight at once (1..64)              */
    int32_t queue_capacity;       /* pending requests before submit is refused        */
    int64_t scratch_budget_bytes; /* device scratch shared by the requests in flight   */
} osc_server_config;

typedef struct {
    int64_t submitted, admitted, completed, failed, rejected;
    int64_t in_flight, max_in_flight, queued, max_queued;
    int64_t budget_waits;          /* times the queue head waited for scratch budget */
    int64_t peak_scratch_bytes, scratch_in_use_bytes;
} osc_server_stats;

/* Start a server over n_samples resident samples (device arrays as in
 * osc_sample; e_true, flags and weight valid and unchanged for the
 * server's life; e_reco is read only here, where every event's histogram
 * slot is cached as for osc_binned_create) and one binning.  Synchronous
 * (waits for earlier work on the device).  Allocates the bin caches (2
 * bytes per event, outside the scratch budget), the scratch budget, the
 * slot streams and pinned result buffers, and starts the dispatcher
 * thread. */
osc_status osc_server_create(osc_ctx* ctx, const osc_sample* samples, int32_t n_samples,
                             const osc_binning* binning, const osc_server_config* cfg,
                             osc_server** out);

/* Stop the dispatcher, wait for the requests in flight and free the server.
 * Requests not yet admitted are dropped. NULL is accepted. */
osc_status osc_server_destroy(osc_server* server);

/* Queue one request; *ticket identifies it.  OSC_ERR_BUDGET when the queue
 * is full or the request could never fit in the scratch budget;
 * OSC_ERR_INVALID_ARG for an invalid parameter set or sample index. */
osc_status osc_server_submit(osc_server* server, const osc_params* set, int32_t sample,
                             osc_precision precision, uint64_t* ticket);

/* Data for the fitter's likelihood (Sec. 2.2, Eq. 2): n_samples rows of
 * nbins observed counts (host, copied) and the exposure mu_scale > 0.  Once
 * set, every request admitted afterwards also computes, on the device
 * after its histogram, -2 ln L of mu_scale * histogram against its
 * sample's row (the reduction of osc_poisson_nll).  data = NULL clears
 * them.  OSC_ERR_NOT_READY while requests are in flight. */
osc_status osc_server_set_data(osc_server* server, const double* data, double mu_scale);

/* Non-blocking: OSC_ERR_NOT_READY while the request runs; once done,
 * copies the histogram (nbins + 2 FP64, host memory; nullable), -2 ln L
 * (nullable; NaN when the request ran without data), the latency from
 * submission to the results on the host and the time spent queued
 * (seconds; nullable), forgets the ticket and returns the request's status. */
osc_status osc_server_poll(osc_server* server, uint64_t ticket, double* hist, double* nll,
                           double* latency_s, double* queue_s);

/* Blocking form of osc_server_poll. */
osc_status osc_server_wait(osc_server* server, uint64_t ticket, double* hist, double* nll,
                           double* latency_s, double* queue_s);

osc_status osc_server_get_stats(osc_server* server, osc_server_stats* out);

/* Start a new statistics window: the counters (submitted, admitted,
 * completed, failed, rejected, budget_waits) restart from zero and the
 * maxima (max_in_flight, max_queued, peak_scratch_bytes) from the current
 * in-flight count, queue length and scratch in use, so that a later
 * osc_server_get_stats describes only what happened since.  Requests
 * already queued or in flight are not affected. */
osc_status osc_server_reset_stats(osc_server* server);

/* Device scratch (bytes) one request on `sample` takes from the budget. */
osc_status osc_server_request_bytes(const osc_server* server, int32_t sample, int64_t* bytes);

/* Constants of the reduction contract: W lanes per tile, K events per lane
 * and A accumulators per bin of a tile.  Any pointer may be NULL. */
void osc_reduction_layout(int32_t* tile_lanes, int32_t* lane_events, int32_t* accumulators);

/* Largest nbins osc_fill_pdf accepts on this context's device: the
 * per-wave histograms (nbins + 2 rows of 8 accumulators) live in LDS next
 * to the static tables, and no binning exceeds 4094 bins. */
int32_t osc_max_nbins(const osc_ctx* ctx);

/* Resident waves per compute unit of the per-event kernel (one wave per
 * tile): for osc_fill_pdf with `nbins` bins when with_hist != 0, for
 * osc_reweight otherwise.  *waves_per_cu receives the count. */
osc_status osc_occupancy(const osc_ctx* ctx, int32_t nbins, int with_hist, int32_t* waves_per_cu);

/* Static description of a status code. */
const char* osc_status_string(osc_status status);

#ifdef __cplusplus
}
#endif
#endif
