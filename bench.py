"""Throughput and latency of the plain FP64 reweight + binned PDF on one GPU.

Workload: 1e7 synthetic Monte Carlo events (true E log-uniform on
[0.1, 10] GeV, nu_mu -> nu_mu / nu_mu -> nu_e at 50 % each, 20 %
antineutrinos, weights U(0.5, 1.5), reco E = true E x N(1, 0.1)), Table 1
parameters, 295 km at 2.6 g/cm^3, 50 reco-E bins on [0, 3] GeV, per-event
P written out.  The sample is uploaded once and its reco-energy bins are
cached once (osc_binned_create, 2 bytes per event), outside the timed
region, as a fitter keeps its Monte Carlo resident.  One step = one
osc_fill_pdf_binned call: P of every event, w * P, the histogram.

Prints one JSON line: evals/s over the timed steps, p50/p99 latency of
single calls measured on the host (launch to histogram on the host), the
roofline position of the per-event kernel timed with hipEvents on its own
stream, and the CPU oracle timed on a bounded slice of the same events.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_EVENTS = 10_000_000
SEED = 1
NBINS, LO, HI = 50, 0.0, 3.0

# Algorithmic HBM bytes per event of the fused kernel on a binned sample:
# read E (8), flags (1), weight (8), the cached histogram slot (2); write P
# (8).  Histogram partials add (nbins + 2) * 8 B per 1024-event tile
# (0.4 B/event) and are left out.  With bins computed per call the slot is
# replaced by the 8-byte reco energy (33 B).
BYTES_PER_EVENT = 27
BYTES_PER_EVENT_COMPUTED_BINS = 33
HBM_PEAK_GBS = 8000.0
SETTLE_S = 0.1   # untimed load before the warm-up steps (clock settle)
# Algorithmic FP64 flops per event of the formulation the kernel follows
# (an FMA counts two, a reciprocal estimate one): matter term and amplitude
# inputs 9, cubic coefficients 12 (the trigonometric seeds are FP32), one
# Halley step with its third-order correction on two roots 54, third root 2,
# differences, 1/(E Q) and the phase scale 16, coefficients of the
# projectors X1 and X2 6, two sin and cos - 1 of the phase differences 52
# (the phase products sit inside their reduction FMAs), numerators of X1
# and X2 16, amplitude sum 15, |S|^2 3, weighted add 2 (w * P and the add
# into the histogram).  Computing the bin per call adds 4 (scale, offset,
# quotient, floor).  A wave in which two eigenvalues lie within ~0.85 % of
# their spread adds a Newton step (31); no wave of the benchmark workloads
# does.
FLOPS_PER_EVENT = 187
FLOPS_PER_EVENT_COMPUTED_BINS = 191
# Layered path, per layer: matter term 1, cubic coefficients 9 and its
# solution 59 (as above: p 3, corrected Halley 54, third root 2),
# differences and 1/Q 12, phase scale 1, two sin and cos - 1 52, cos 2,
# c_k 7, eigenvalue sums and products 6, polynomial coefficients a2, a1, a0
# 19, y = M v 74, z = M y 74, v = a2 z + a1 y + a0 v 66: 382.  The first
# layer forms y as column alpha of M (2 instead of 74), the last only
# component beta of z and v (26 + 22 instead of 74 + 66); per event 1/E 7,
# |v_beta|^2 3 and the weighted add 2.
LAYER_FLOPS = 382


def layered_flops_per_event(n_layers):
    return LAYER_FLOPS * n_layers - 72 - 92 + 12


# FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz.
FP64_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# HBM traffic and VALU instruction mix of one launch of the fused kernel on
# this workload (binned sample, FP64, P written), read with rocprofv3 --pmc
# (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, scaled by what the same
# counters read for a plain device copy of known size; SQ_INSTS_VALU and its
# class counters, wave instructions x 64 / events).  Valid only for the
# kernel sources and build flags they were taken on (sha256 over
# KERNEL_SOURCES); reported as null once those change.
KERNEL_SOURCES = ("paper_1311_7579_amd/csrc/osc_device.h",
                  "paper_1311_7579_amd/csrc/osc_internal.h",
                  "paper_1311_7579_amd/csrc/osc_kernels.hip",
                  "paper_1311_7579_amd/build.py")
COUNTER_TRAFFIC = {
    "fetch_kib": 92836.0, "fetch_scale": 2.0,     # copy of 512 MiB: FETCH_SIZE 262157 KiB
    "write_kib": 82562.4, "write_scale": 1.0,     # copy of 512 MiB: WRITE_SIZE 524288 KiB
    "valu_per_event": 170.0,
    "classes_per_event": {"fp64": 119.5, "fp64_trans": 2.0, "fp32": 15.0, "fp32_trans": 4.0,
                          "cvt": 5.0, "int32": 6.69, "int64": 0.375, "other": 17.44},
    "source_sha256": "bda247f22a1b7708bb86df22b451d9748abe6d2a1e6e26a4b6f78e769d704574",
}
# Issue time of one wave instruction on one SIMD, measured on the box with
# probe kernels of independent chains (ns): FP64 FMA/MUL/ADD 2.08, FP32
# 1.06, v_rcp_f64 6.75, v_cos_f32 3.38 and v_sqrt_f32 about 4 (3.7 for the
# FP32 transcendentals, two cos and a sqrt and an rsq per event).
# Conversions and 64-bit integer operations are taken at the FP64 rate and
# the unclassified remainder (moves, selects) at the FP32 rate: assumed,
# not measured.  2.08 ns for a 4-cycle FP64 instruction is an engine clock
# of 1.92 GHz under this load, against the 2.4 GHz of the published peak.
ISSUE_NS = {"fp64": 2.08, "fp64_trans": 6.75, "fp32": 1.06, "fp32_trans": 3.7,
            "cvt": 2.08, "int32": 1.06, "int64": 2.08, "other": 1.06}
VALU_SIMDS = 1024
CLOCK_HZ = 2.4e9


def valu_issue(kernel_ms, flops_per_event):
    """Where the FP64 roofline fraction goes, from the counter mix of the
    current sources (None once they change): the fraction equals
    clock x mix x issue, with clock = the engine clock the measured issue
    rates imply over 2.4 GHz, mix = the time the event's flops would need
    as FP64 FMAs over the time its instruction mix needs, and issue = that
    instruction time over the kernel's duration."""
    if kernel_sources_sha256() != COUNTER_TRAFFIC["source_sha256"]:
        return None
    cls = COUNTER_TRAFFIC["classes_per_event"]
    ns = sum(cls[k] * ISSUE_NS[k] for k in cls)            # per wave-event, one SIMD
    wave_events = N_EVENTS / 64 / VALU_SIMDS
    issue_ms = ns * wave_events * 1e-6
    clock = (4 / (ISSUE_NS["fp64"] * 1e-9)) / CLOCK_HZ
    mix = (flops_per_event / 2 * ISSUE_NS["fp64"]) / ns
    # FP64 VALU instructions per second against the FP64 pipe's instruction
    # peak (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-ops/s)
    fp64_lane_ops = (cls["fp64"] + cls["fp64_trans"]) * N_EVENTS / (kernel_ms * 1e-3)
    return {"valu_insts_per_event": COUNTER_TRAFFIC["valu_per_event"],
            "fp64_pipe_frac": fp64_lane_ops / (FP64_PEAK_TFLOPS * 1e12 / 2),
            "classes_per_event": cls, "issue_ns_per_wave_event": ns,
            "issue_ms_at_measured_rates": issue_ms, "frac": issue_ms / kernel_ms,
            "decomposition": {"clock": clock, "mix": mix, "issue": issue_ms / kernel_ms,
                              "product": clock * mix * issue_ms / kernel_ms}}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-calls", type=int, default=1000)
    ap.add_argument("--cpu-events", type=int, default=10_000_000,
                    help="events of the oracle's timed slice (all host threads)")
    ap.add_argument("--cpu-events-1t", type=int, default=1_000_000,
                    help="events of the oracle's single-thread slice")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision-form measurement (64 parameter sets, both tiers)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving-form measurement (Poisson proposal streams)")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-form measurement (256 sets x 4 uneven samples)")
    ap.add_argument("--no-bincentre", action="store_true",
                    help="skip the bin-centre measurement (template + binning effect)")
    ap.add_argument("--no-layered", action="store_true",
                    help="skip the layered-matter measurement (5-layer Earth path)")
    ap.add_argument("--tier", choices=("fp64", "mixed"), default=None,
                    help="precision tier of the timed step (profiling runs; the benchmark "
                         "line is FP64) or of --batch-schedule (FP32-mixed by default)")
    ap.add_argument("--computed-bins", action="store_true",
                    help="time osc_fill_pdf (bins computed per call) as the step")
    ap.add_argument("--batch-schedule", type=int, choices=(0, 1, 2), default=None,
                    help="only run the 256-set x 4-sample batched form with this schedule "
                         "(0 dynamic queue, 1 static stride, 2 one workgroup per tile), "
                         "--sets-per-item sets per work item, --steps launches; for "
                         "per-schedule profiles")
    ap.add_argument("--sets-per-item", type=int, default=8)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run torch device-to-device copies of MIB MiB (HBM counter "
                         "calibration under rocprofv3) and exit")
    return ap.parse_args()


def copy_calibration(mib, reps=5):
    """Plain device copies of a known size: the HBM byte counters of these
    dispatches calibrate the counters of the kernels above."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_MiB": mib, "bytes_read_per_copy": n * 8,
                      "bytes_written_per_copy": n * 8, "reps": reps}), flush=True)


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic():
    """HBM bytes per launch from the committed counter readings, or None if
    the kernel sources changed since they were taken."""
    if COUNTER_TRAFFIC is None or COUNTER_TRAFFIC["source_sha256"] != kernel_sources_sha256():
        return None
    c = COUNTER_TRAFFIC
    return 1024.0 * (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"])


def host_cores():
    """Physical cores of the host (distinct (socket, core) pairs of
    /proc/cpuinfo), and the logical CPUs this process may run on."""
    pairs, phys = set(), None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "physical id":
                    phys = val
                elif key == "core id":
                    pairs.add((phys, val))
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count()
    return (len(pairs) or None), allowed


def cpu_baseline(sample, n_all, n_one, reps=5):
    """The oracle (P per event and the contract histogram, fill_pdf with P
    written) timed on the host: the unchanged source built at -O3
    -march=native for this host, the median of `reps` passes over the first
    n_all events with every OpenMP thread and over the first n_one events
    with one thread.  The portable -O2 build the tests use is timed the
    same way and reported beside it."""
    import numpy as np
    import oracle
    from paper_1311_7579_amd import workload

    def rate(n):
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.fill_pdf(workload.TABLE1, sample.L_km, sample.rho_gcc, sample.Ye,
                            sample.e_true[:n], sample.flags[:n], sample.weight[:n],
                            sample.e_reco[:n], NBINS, LO, HI, want_p=True)
            times.append(time.perf_counter() - t0)
        return n / float(np.median(times)), float(np.sum(times))

    def both():
        threads = oracle.num_threads()
        all_rate, all_s = rate(n_all)
        oracle.set_num_threads(1)
        one_rate, one_s = rate(n_one)
        oracle.set_num_threads(threads)
        return threads, all_rate, all_s, one_rate, one_s

    portable = both()
    oracle.use_native_build()
    threads, all_rate, all_s, one_rate, one_s = both()
    physical, allowed = host_cores()
    return {
        "value": all_rate, "unit": "evals/s", "cores": threads, "kind": "oracle",
        "sample": f"median of {reps} passes over the first {n_all} events of the 1e7-event "
                  f"workload (fill_pdf with P written), {threads} OpenMP threads; oracle source "
                  f"built with gcc -O3 -march=native -ffp-contract=off on this host "
                  f"({all_s:.1f} s wall in all, about {all_s * threads:.0f} thread-seconds)",
        "single_core_value": one_rate,
        "single_core_sample": f"median of {reps} passes over the first {n_one} events, "
                              f"1 thread ({one_s:.1f} s in all)",
        "threads_used": threads, "host_physical_cores": physical,
        "logical_cpus_available": allowed,
        "portable_O2_build": {"value": portable[1], "single_core_value": portable[3]},
    }


# The paper's own timing comparison (Sec. 2.2 and its hardware statement):
# context for the speed-ups this benchmark measures, not a target.
PAPER_CONTEXT = {
    "gpu_speedup_vs_one_cpu_core": 132,
    "at_calculations": 1.45e6,
    "gpu": "NVIDIA Tesla M2070 (448 CUDA cores at 1.15 GHz), CUDA 5, FP64",
    "cpu": "Intel Xeon E5640 (4 cores at 2.67 GHz), one core, gcc 4.6.3 -O2, FP64",
    "openmp_speedup_vs_one_core": "2-3x with 4 threads",
    "headline": "about two orders of magnitude over a single CPU core",
}


def precision_form(osc, ctx, ds, binned, n_sets=64, set_seed=3, n_oracle=100_000):
    """The 1e7 events under 64 parameter sets, once per tier (binned
    sample, P written): throughput of each tier, and for every set the
    largest |P_mixed - P_fp64| over all events (on the device) and the
    largest |P - P_oracle| of each tier over the first n_oracle events."""
    import numpy as np
    import torch
    import oracle
    from paper_1311_7579_amd import workload
    sets = workload.make_param_sets(n_sets, set_seed)
    ctx.osc_set_params(sets)
    n = ds.n
    h = torch.empty(NBINS + 2, dtype=torch.float64, device="cuda")
    p64 = torch.empty(n, dtype=torch.float64, device="cuda")
    pmx = torch.empty(n, dtype=torch.float64, device="cuda")
    out = {}
    for name, prec, buf in (("fp64", osc.OSC_FP64, p64), ("fp32_mixed", osc.OSC_FP32_MIXED, pmx)):
        for k in range(2):   # warm-up
            ctx.osc_fill_pdf_binned(binned, k, h, buf, precision=prec)
        torch.cuda.synchronize()
        ctx.osc_profile_enable(True)
        t0 = time.perf_counter()
        for k in range(n_sets):
            ctx.osc_fill_pdf_binned(binned, k, h, buf, precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ev_ms, ev_n, merge_ms, merge_n = ctx.osc_profile_read()
        ctx.osc_profile_enable(False)
        out[name] = {"evals_per_s": n * n_sets / dt, "kernel_ms": ev_ms / max(ev_n, 1),
                     "merge_ms": merge_ms / max(merge_n, 1)}
    e = ds.e_true[:n_oracle].cpu().numpy()
    f = ds.flags[:n_oracle].cpu().numpy()
    rows = []
    for k in range(n_sets):
        ctx.osc_fill_pdf_binned(binned, k, h, p64, precision=osc.OSC_FP64)
        ctx.osc_fill_pdf_binned(binned, k, h, pmx, precision=osc.OSC_FP32_MIXED)
        d_all = float((pmx - p64).abs().max())
        po = oracle.prob_batch(sets[k], ds.L_km, ds.rho_gcc, ds.Ye, e, f)
        d_mx = float(np.abs(pmx[:n_oracle].cpu().numpy() - po).max())
        d_64 = float(np.abs(p64[:n_oracle].cpu().numpy() - po).max())
        rows.append([k, d_all, d_mx, d_64])
    arr = np.array(rows)
    out["per_set_error"] = {
        "columns": ["set", "max_abs_dP_mixed_vs_fp64_all_events",
                    f"max_abs_dP_mixed_vs_oracle_first_{n_oracle}",
                    f"max_abs_dP_fp64_vs_oracle_first_{n_oracle}"],
        "rows": rows}
    out["max_abs_dP_mixed_vs_fp64"] = float(arr[:, 1].max())
    out["max_abs_dP_mixed_vs_oracle"] = float(arr[:, 2].max())
    out["max_abs_dP_fp64_vs_oracle"] = float(arr[:, 3].max())
    out["config"] = (f"{n} events x {n_sets} parameter sets (seed {set_seed}), P written, "
                     f"bins cached; oracle on the first {n_oracle} events of every set")
    ctx.osc_set_params([workload.TABLE1])
    return out


def settle(fn, seconds=SETTLE_S * 3):
    """Untimed calls of fn for `seconds` (the engine clock ramps up again
    after the host-side set-up of a form)."""
    import torch
    t = time.perf_counter()
    while time.perf_counter() - t < seconds:
        fn()
        torch.cuda.synchronize()


def bincentre_form(osc, ctx, s, ds, ebe_ms, calls=200):
    """Sec. 1.1.1's approximate alternative on the same events: a migration
    template over 200 true-energy bins (0.1-10.1 GeV) and the 50 reco bins,
    then one PDF per call from P at the 18 x 200 bin centres.  Reports the
    build and per-call times, the PDF's deviation from event-by-event, and
    the binning effect of the paper's 25 MeV example bin for two synthetic
    fluxes."""
    import numpy as np
    import torch
    from paper_1311_7579_amd import workload
    nt, lo_t, hi_t = 200, 0.1, 10.1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tp = osc.Template(ctx, ds, nt, lo_t, hi_t, NBINS, LO, HI)
    build_ms = (time.perf_counter() - t0) * 1e3
    h = torch.empty(NBINS + 2, dtype=torch.float64, device="cuda")
    settle(lambda: tp.fill_pdf(0, h))
    t0 = time.perf_counter()
    for _ in range(calls):
        tp.fill_pdf(0, h)
    torch.cuda.synchronize()
    call_ms = (time.perf_counter() - t0) * 1e3 / calls
    hb = h.cpu().numpy()
    he = torch.empty(NBINS + 2, dtype=torch.float64, device="cuda")
    ctx.osc_fill_pdf(ds, 0, NBINS, LO, HI, he)
    he = he.cpu().numpy()
    full = he[:NBINS] > 0.01 * he[:NBINS].max()
    dev = np.abs(hb[:NBINS][full] / he[:NBINS][full] - 1.0)
    tp.close()

    def effect(e, w):
        f = workload.make_flags(np.ones(e.size, int), np.ones(e.size, int), np.zeros(e.size, bool))
        es = workload.Sample(e, f, w, e.copy(), L_km=295.0, rho_gcc=2.6)
        d = osc.DeviceSample.from_host(es)
        h1 = torch.empty(3, dtype=torch.float64, device="cuda")
        ctx.osc_fill_pdf(d, 0, 1, 0.600, 0.625, h1)
        t1 = osc.Template(ctx, d, 1, 0.600, 0.625, 1, 0.600, 0.625)
        h2 = torch.empty(3, dtype=torch.float64, device="cuda")
        t1.fill_pdf(0, h2)
        r = float(h1[0].item() / h2[0].item() - 1.0)
        t1.close()
        return r

    n = 200_000
    e = 0.600 + (np.arange(n) + 0.5) * (0.025 / n)
    flat = effect(e, np.ones(n))
    peaked = effect(e, e ** 2 * np.exp(-e / 0.3))   # spectrum E^2 exp(-E / 0.3 GeV), peak 0.6 GeV
    return {
        "config": "template of the 1e7-event workload: 200 true bins on [0.1, 10.1] GeV x 18 "
                  "channels x 52 reco rows; per call P at 3600 bin centres + contraction",
        "template_build_ms": build_ms, "ms_per_call": call_ms,
        "speedup_vs_event_by_event": ebe_ms / call_ms,
        "pdf_rel_dev_vs_event_by_event": {"max": float(dev.max()), "median": float(np.median(dev))},
        "binning_effect_0.600_0.625_GeV": {
            "flat_flux": flat, "flux_E2_exp(-E/0.3)": peaked,
            "note": "event-by-event / bin-centre - 1 for nu_mu -> nu_mu at 295 km, Table 1; "
                    "the paper quotes 2.6 % for its (unpublished) beam flux"},
    }


def layered_form(osc, ctx, n=10_000_000, reps=20):
    """Piecewise-constant matter: a five-layer path through the Earth
    (crust, mantle, core, mantle, crust; 11600 km) for an atmospheric-like
    sample of 1e7 events, E log-uniform on [0.5, 20] GeV, every channel,
    40 % antineutrinos; fused FP64 reweight + 50-bin PDF on [0, 20] GeV."""
    import numpy as np
    import torch
    from paper_1311_7579_amd import workload
    earth = [(700.0, 3.3, 0.5), (3500.0, 5.0, 0.495), (3200.0, 11.5, 0.466),
             (3500.0, 5.0, 0.495), (700.0, 3.3, 0.5)]
    rng = np.random.default_rng(61)
    e = 10 ** rng.uniform(np.log10(0.5), np.log10(20.0), n)
    f = workload.make_flags(rng.integers(0, 3, n), rng.integers(0, 3, n), rng.random(n) < 0.4)
    w = rng.uniform(0.5, 1.5, n)
    x = np.maximum(e * rng.normal(1.0, 0.1, n), 1e-12)
    ds = osc.DeviceSample.from_host(workload.Sample(e, f, w, x))
    h = torch.empty(52, dtype=torch.float64, device="cuda")
    settle(lambda: ctx.osc_fill_pdf_layered(ds, earth, 0, 50, 0.0, 20.0, h))
    ctx.osc_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.osc_fill_pdf_layered(ds, earth, 0, 50, 0.0, 20.0, h)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / reps
    ev_ms, ev_n, _, _ = ctx.osc_profile_read()
    ctx.osc_profile_enable(False)
    kernel_ms = ev_ms / max(ev_n, 1)
    flops = layered_flops_per_event(len(earth))
    tflops = flops * n / (kernel_ms * 1e-3) / 1e12
    return {"config": "5-layer Earth path (11600 km), 1e7 events, E log-uniform 0.5-20 GeV, "
                      "all channels, FP64, 50 bins",
            "layers": 5, "ms_per_call": wall_ms, "kernel_ms": kernel_ms,
            "evals_per_s": n / (wall_ms * 1e-3), "layer_evals_per_s": 5 * n / (kernel_ms * 1e-3),
            "roofline": {"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": tflops / FP64_PEAK_TFLOPS,
                         "flops_per_event": flops, "kernel": "layered_tile_kernel<kPdf, no P>"}}


def batched_form(osc, ctx, reps=5):
    """256 parameter sets x 4 samples of 1e5, 5e5, 2e6 and 5e6 events (295,
    810, 1300, 2500 km; densities U(2.4, 3.0)), mixed tier, one batched
    launch per step after autotuning."""
    import torch
    from paper_1311_7579_amd import workload
    samples = workload.make_batched_samples()
    ds = [osc.DeviceSample.from_host(s) for s in samples]
    sets = workload.make_param_sets(256, 4)
    evals = sum(s.n for s in samples) * len(sets)
    out = {"config": "256 sets x 4 samples (1e5, 5e5, 2e6, 5e6 events), FP32-mixed tier, "
                     "50 bins, hipGraph replay", "evals_per_launch": evals}
    batch = osc.Batch(ctx, ds, NBINS, LO, HI, precision=osc.OSC_FP32_MIXED, max_sets=256)
    try:
        t0 = time.perf_counter()
        out["tune_best_ms"] = batch.tune(sets)
        out["tune_s"] = time.perf_counter() - t0
        out["tuned_config"] = batch.config.as_dict()
        hist = torch.empty((256, 4, NBINS + 2), dtype=torch.float64, device="cuda")
        batch.run(sets, hist)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            batch.run(sets, hist)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out["ms_per_launch"] = dt * 1e3
        out["evals_per_s"] = evals / dt
    finally:
        batch.close()
    return out


def batch_schedule_run(osc, ctx, args):
    """The batched form (256 sets x 4 samples, FP32-mixed unless --tier
    fp64) in one fixed configuration, launched --steps times after --warmup
    launches: for kernel traces and counters per schedule."""
    import torch
    from paper_1311_7579_amd import workload
    samples = workload.make_batched_samples()
    ds = [osc.DeviceSample.from_host(s) for s in samples]
    sets = workload.make_param_sets(256, 4)
    prec = osc.OSC_FP64 if args.tier == "fp64" else osc.OSC_FP32_MIXED
    batch = osc.Batch(ctx, ds, NBINS, LO, HI, precision=prec, max_sets=256)
    try:
        batch.config = dict(sets_per_item=args.sets_per_item, schedule=args.batch_schedule,
                            waves_per_cu=0, use_graph=1)
        hist = torch.empty((256, 4, NBINS + 2), dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            batch.run(sets, hist)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            batch.run(sets, hist)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / max(args.steps, 1)
    finally:
        batch.close()
    evals = sum(s.n for s in samples) * len(sets)
    return {"batch_schedule": args.batch_schedule, "sets_per_item": args.sets_per_item,
            "tier": "fp64" if prec == osc.OSC_FP64 else "fp32_mixed",
            "ms_per_launch": dt * 1e3, "evals_per_s": evals / dt}


SERVE_BUDGET = 24 << 20    # device scratch shared by requests in flight


def serving_form(osc, ctx, n_requests):
    """8 resident samples of 1e4 .. 2e7 events, MCMC-style proposals (1 %
    steps, half in each precision tier) on 8 slots with a 24 MiB scratch
    budget: saturation throughput from a burst, then Poisson streams at
    0.5, 0.8 and 0.95 of it with p50/p99 latency."""
    from paper_1311_7579_amd import serving, workload
    samples = workload.make_serving_samples()
    ds = [osc.DeviceSample.from_host(s) for s in samples]
    ev = [s.n for s in samples]
    out = {"config": "8 samples (1e4..2e7 events, 3.02e7 total), 8 slots, 24 MiB scratch "
                     "budget, 50 % FP64 / 50 % FP32-mixed, 1 % MCMC steps",
           "requests_per_run": n_requests}
    server = osc.Server(ctx, ds, NBINS, LO, HI, slots=8, scratch_budget_bytes=SERVE_BUDGET)
    try:
        warm = workload.make_proposal_stream(64, 500, len(ds))
        serving.run_stream(server, warm, [0.0] * len(warm), ev)
        reqs = workload.make_proposal_stream(n_requests, 501, len(ds))
        server.reset_stats()
        _, sat = serving.run_stream(server, reqs, [0.0] * n_requests, ev)
        sat_rate = n_requests / sat["wall_s"]
        st = sat["stats"]
        out["saturation"] = {"requests_per_s": sat_rate, "evals_per_s": sat["evals_per_s"],
                             "p50_ms": sat["p50_ms"], "p99_ms": sat["p99_ms"],
                             **{k2: st[k2] for k2 in ("max_in_flight", "max_queued", "budget_waits",
                                                      "peak_scratch_bytes", "completed")}}
        for k, frac in enumerate((0.5, 0.8, 0.95)):
            reqs = workload.make_proposal_stream(n_requests, 510 + k, len(ds))
            arr = workload.poisson_arrivals(n_requests, frac * sat_rate, 520 + k)
            server.reset_stats()   # this stream's own counters and maxima
            _, summ = serving.run_stream(server, reqs, arr, ev)
            st = summ.pop("stats")
            summ.update({k2: st[k2] for k2 in ("max_in_flight", "max_queued", "budget_waits",
                                               "peak_scratch_bytes", "completed")})
            out[f"rate_{frac}"] = summ
        out["mcmc"] = serving_mcmc(osc, ctx, server, ds)
    finally:
        server.close()
    return out


def serving_mcmc(osc, ctx, server, ds, n_chains=8, n_steps=250):
    """Sec. 2.2's fit as served requests: fake data drawn (Poisson, seed 81)
    from every sample's PDF at Table 1, scaled to 3000 expected events in
    the 1e6-event sample's regular bins; 8 Metropolis chains over
    (sin^2 theta23, dm2_32) on that sample, FP64, each proposal one request
    whose -2 ln L (Eq. 2) is computed on the device."""
    import numpy as np
    import torch
    from paper_1311_7579_amd import serving, workload
    truth = workload.TABLE1
    ctx.osc_set_params([truth])
    h = torch.empty((len(ds), NBINS + 2), dtype=torch.float64, device="cuda")
    for k, d in enumerate(ds):
        ctx.osc_fill_pdf(d, 0, NBINS, LO, HI, h[k])
    pdf = h.cpu().numpy()[:, :NBINS]
    target = int(np.argmin([abs(d.n - 1_000_000) for d in ds]))
    mu_scale = 3000.0 / pdf[target].sum()
    data = np.random.default_rng(81).poisson(mu_scale * pdf).astype(float)
    server.set_data(data, mu_scale)
    try:
        r = serving.run_mcmc(server, start=dict(truth, sin2_th23=0.43, dm2_32=2.3e-3),
                             free=("sin2_th23", "dm2_32"), sigmas=(0.015, 2.5e-5),
                             bounds=((0.3, 0.7), (2.0e-3, 2.8e-3)), n_chains=n_chains,
                             n_steps=n_steps, seed=82, sample=target, tier=osc.OSC_FP64)
    finally:
        server.set_data(None)
    tail = r["chains"][:, n_steps // 2:, :].reshape(-1, 2)
    return {"config": f"{n_chains} chains x {n_steps} steps on the {ds[target].n}-event sample, "
                      "3000 expected events, free (sin2_th23, dm2_32), Table 1 truth",
            "acceptance": r["acceptance"], "steps_per_s": r["steps_per_s"],
            "evals_per_s": r["steps_per_s"] * ds[target].n,
            "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
            "posterior_second_half": {"sin2_th23": [float(tail[:, 0].mean()), float(tail[:, 0].std())],
                                      "dm2_32": [float(tail[:, 1].mean()), float(tail[:, 1].std())]}}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by events or parameter sets, see the design notes)", flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1311_7579_amd import osc, workload

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", flush=True)
        sys.exit(1)

    s = workload.make_sample(N_EVENTS, SEED)
    ctx = osc.Context(0)
    ctx.osc_set_params([workload.TABLE1])
    ds = osc.DeviceSample.from_host(s)
    binned = ctx.osc_binned_create(ds, NBINS, LO, HI)
    hist = torch.empty(NBINS + 2, dtype=torch.float64, device="cuda")
    p_out = torch.empty(N_EVENTS, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    tier = osc.OSC_FP32_MIXED if args.tier == "mixed" else osc.OSC_FP64

    if args.batch_schedule is not None:
        print(json.dumps(batch_schedule_run(osc, ctx, args)), flush=True)
        return

    def step_binned():
        ctx.osc_fill_pdf_binned(binned, 0, hist, p_out, precision=tier, stream=stream)

    def step_computed():
        ctx.osc_fill_pdf(ds, 0, NBINS, LO, HI, hist, p_out, precision=tier, stream=stream)

    step = step_computed if args.computed_bins else step_binned

    # The GPU's clocks take tens of milliseconds of load to settle: untimed
    # steps for at least SETTLE_S seconds, then the W warm-up steps, then the
    # K timed ones (a short cold run reads up to 15 % slower per step).
    settle_steps, t_settle = 0, time.perf_counter()
    while time.perf_counter() - t_settle < SETTLE_S:
        for _ in range(10):
            step()
        torch.cuda.synchronize()
        settle_steps += 10
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = N_EVENTS / (ms_per_step * 1e-3)

    # end-to-end latency of single calls: launch -> histogram on the host
    lat = []
    host_hist = torch.empty(NBINS + 2, dtype=torch.float64, pin_memory=True)
    for _ in range(args.latency_calls):
        a = time.perf_counter()
        step()
        host_hist.copy_(hist, non_blocking=False)
        lat.append(time.perf_counter() - a)
    lat = np.array(lat if lat else [float("nan")]) * 1e3
    # per-kernel device time, after the latency calls have kept the GPU busy:
    # the fused kernel's own dispatch records its begin and end in hipEvents
    # on the launch stream
    ctx.osc_profile_enable(True)
    for _ in range(max(args.steps, 50)):
        step()
    ev_ms, ev_n, merge_ms, merge_n = ctx.osc_profile_read()
    ctx.osc_profile_enable(False)
    kernel_ms = ev_ms / max(ev_n, 1)
    waves_per_cu = ctx.osc_occupancy(NBINS, True)
    merge_avg_ms = merge_ms / max(merge_n, 1)
    # the same step with the bin of every event computed per call
    other = step_binned if args.computed_bins else step_computed
    for _ in range(args.warmup):
        other()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        other()
    torch.cuda.synchronize()
    other_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ctx.osc_profile_enable(True)
    for _ in range(max(args.steps, 50)):
        other()
    o_ms, o_n, _, _ = ctx.osc_profile_read()
    ctx.osc_profile_enable(False)
    flops_ev = FLOPS_PER_EVENT_COMPUTED_BINS if args.computed_bins else FLOPS_PER_EVENT
    bytes_ev = BYTES_PER_EVENT_COMPUTED_BINS if args.computed_bins else BYTES_PER_EVENT

    # The fused kernel is bound by VALU issue (FP64 arithmetic), not by HBM:
    # roofline against the FP64 vector peak, HBM position alongside.
    achieved_gbs = bytes_ev * N_EVENTS / (kernel_ms * 1e-3) / 1e9
    fp64_tflops = flops_ev * N_EVENTS / (kernel_ms * 1e-3) / 1e12
    plain = not args.computed_bins and tier == osc.OSC_FP64
    traffic = counter_traffic() if plain else None
    mode = "kPdf" if args.computed_bins else "kPdfBinned"
    roofline = {
        "bound": "alu", "achieved": fp64_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": fp64_tflops / FP64_PEAK_TFLOPS, "traffic": traffic,
        "kernel": f"tile_kernel<{mode}, write P, {'FP32-mixed' if tier else 'FP64'}>",
        "kernel_ms": kernel_ms, "flops_per_event": flops_ev, "events_per_launch": N_EVENTS,
        "hbm": {"achieved_GBs": achieved_gbs, "peak_GBs": HBM_PEAK_GBS,
                "frac": achieved_gbs / HBM_PEAK_GBS,
                "algorithmic_bytes_per_event": bytes_ev,
                "traffic_over_algorithmic": (traffic / (bytes_ev * N_EVENTS)
                                             if traffic else None)},
        "merge_kernel_ms": merge_avg_ms,
        "resident_waves_per_cu": waves_per_cu,
        "valu_issue": valu_issue(kernel_ms, flops_ev) if plain else None,
    }

    result = {
        "metric": "oscillation-prob evals/sec (events x param sets) at 1 GPU + p50/p99 reweight latency",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "settle_steps": settle_steps,
        "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "plain FP64 reweight + 50-bin reco-E PDF, 1e7 events x 1 parameter "
                               "set (Table 1, 295 km, 2.6 g/cm^3), per-event P written, reco-E "
                               "bins cached at upload",
                   "events": N_EVENTS, "param_sets": 1, "nbins": NBINS, "range_GeV": [LO, HI],
                   "seed": SEED, "parallelism": "single GPU",
                   "tier": "fp32_mixed" if tier else "fp64",
                   "bins": "computed per call" if args.computed_bins else "cached"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "calls": args.latency_calls},
        "roofline": roofline,
        ("cached_bins" if args.computed_bins else "computed_bins"): {
            "ms_per_step": other_ms, "kernel_ms": o_ms / max(o_n, 1),
            "evals_per_s": N_EVENTS / (other_ms * 1e-3),
            "note": "the same step through " + ("osc_fill_pdf_binned" if args.computed_bins
                                                else "osc_fill_pdf (bin of every event "
                                                     "computed per call)")},
    }
    if not args.no_forms:
        result["precision_form"] = precision_form(osc, ctx, ds, binned)
    if not args.no_batch:
        result["batched_form"] = batched_form(osc, ctx)
    if not args.no_bincentre:
        result["bincentre_form"] = bincentre_form(osc, ctx, s, ds, ms_per_step)
    if not args.no_layered:
        result["layered_form"] = layered_form(osc, ctx)
    if not args.no_serve:
        result["serving_form"] = serving_form(osc, ctx, args.serve_requests)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(s, args.cpu_events, args.cpu_events_1t)
        cb = result["cpu_baseline"]
        result["speedup_vs_cpu_all_cores"] = value / cb["value"]
        result["speedup_vs_cpu_one_core"] = value / cb["single_core_value"]
        result["paper_context"] = dict(
            PAPER_CONTEXT,
            this_run={"gpu_speedup_vs_one_cpu_core": value / cb["single_core_value"],
                      "gpu_speedup_vs_all_threads": value / cb["value"],
                      "openmp_speedup_vs_one_core": cb["value"] / cb["single_core_value"],
                      "openmp_threads": cb["threads_used"],
                      "gpu": "one AMD Instinct MI355X (gfx950)",
                      "cpu": f"{cb['threads_used']} OpenMP threads on a host with "
                             f"{cb['host_physical_cores']} physical cores"})
    binned.close()
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
