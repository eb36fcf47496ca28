"""Throughput and latency of the plain FP64 reweight + binned PDF on one GPU.

Workload: 1e7 synthetic Monte Carlo events (true E log-uniform on
[0.1, 10] GeV, nu_mu -> nu_mu / nu_mu -> nu_e at 50 % each, 20 %
antineutrinos, weights U(0.5, 1.5), reco E = true E x N(1, 0.1)), Table 1
parameters, 295 km at 2.6 g/cm^3, 50 reco-E bins on [0, 3] GeV, per-event
P written out.  One step = one osc_fill_pdf call on the resident sample.

Prints one JSON line: evals/s over the timed steps, p50/p99 latency of
single calls measured on the host (launch to histogram on the host), the
roofline position of the per-event kernel timed with hipEvents on its own
stream, and the CPU oracle timed on a bounded slice of the same events.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_EVENTS = 10_000_000
SEED = 1
NBINS, LO, HI = 50, 0.0, 3.0

# Algorithmic HBM bytes per event of the fused kernel: read E (8), flags (1),
# weight (8), reco E (8); write P (8).  Histogram partials add
# (nbins + 2) * 8 B per 1024-event tile (0.4 B/event) and are left out.
BYTES_PER_EVENT = 33
HBM_PEAK_GBS = 8000.0
SETTLE_S = 0.1   # untimed load before the warm-up steps (clock settle)
# Algorithmic FP64 flops per event of the formulation the kernel follows
# (an FMA counts two, a reciprocal estimate one): matter term and amplitude
# inputs 9, cubic coefficients 12, trigonometric seeds (scaling in FP64) 6,
# one Halley and one Newton step on two roots 72, third root 2,
# differences, 1/(E Q) and the phase scale 16, coefficients of the
# projectors X1 and X2 6, two sin and cos - 1 of the phase differences 54
# (the phase products sit inside their reduction FMAs), numerators of X1
# and X2 16, amplitude sum 15, |S|^2 3, bin and weighted add 6.
FLOPS_PER_EVENT = 217
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz.
FP64_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# HBM traffic of one launch of the fused kernel on this workload, read with
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch) and scaled by
# what the same counters read for a plain device copy of known size.  Valid
# only for the kernel sources and build flags it was taken on (sha256 over
# KERNEL_SOURCES); reported as null once they change.
KERNEL_SOURCES = ("paper_1311_7579_amd/csrc/osc_device.h",
                  "paper_1311_7579_amd/csrc/osc_internal.h",
                  "paper_1311_7579_amd/csrc/osc_kernels.hip",
                  "paper_1311_7579_amd/build.py")
COUNTER_TRAFFIC = {
    "fetch_kib": 122169.5, "fetch_scale": 2.0,    # copy of 512 MiB: FETCH_SIZE 262158 KiB
    "write_kib": 82825.0, "write_scale": 1.0,     # copy of 512 MiB: WRITE_SIZE 524288 KiB
    # SQ_INSTS_VALU per event (wave instructions x 64 / events) and the
    # quarter-rate transcendentals among them, from the same run
    "valu_per_event": 195.9, "trans_per_event": 8,
    "source_sha256": "62f73101d553860446d2ddcf66c4a199e9aab1c6e8ffb584b9afc572c46906d8",
}
# VALU issue: one wave instruction per SIMD every 4 cycles (a quarter-rate
# transcendental takes 16), 1024 SIMDs at the 2.4 GHz peak engine clock.
VALU_SIMDS = 1024
CLOCK_HZ = 2.4e9


def valu_issue(kernel_ms):
    """Fraction of the kernel's duration the SIMDs need just to issue its
    VALU instructions (counter figures of the current sources, else None)."""
    if kernel_sources_sha256() != COUNTER_TRAFFIC["source_sha256"]:
        return None
    per_event = COUNTER_TRAFFIC["valu_per_event"]
    trans = COUNTER_TRAFFIC["trans_per_event"]
    cycles = (per_event * 4 + trans * 12) * (N_EVENTS / 64) / VALU_SIMDS
    need_ms = cycles / CLOCK_HZ * 1e3
    return {"valu_insts_per_event": per_event, "transcendentals_per_event": trans,
            "issue_ms_at_peak_clock": need_ms, "frac": need_ms / kernel_ms}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--latency-calls", type=int, default=1000)
    ap.add_argument("--cpu-events", type=int, default=10_000_000,
                    help="events of the oracle's timed slice (all host threads)")
    ap.add_argument("--cpu-events-1t", type=int, default=2_000_000,
                    help="events of the oracle's single-thread slice")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum wall time of the oracle's all-thread passes")
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


def cpu_baseline(sample, n_all, n_one, min_seconds):
    """The oracle (P per event, contract histogram) on the host: whole passes
    over the first n_all events with every OpenMP thread until min_seconds
    have passed, then one single-thread pass over the first n_one."""
    import oracle
    from paper_1311_7579_amd import workload

    def run(n):
        t0 = time.perf_counter()
        oracle.fill_pdf(workload.TABLE1, sample.L_km, sample.rho_gcc, sample.Ye,
                        sample.e_true[:n], sample.flags[:n], sample.weight[:n],
                        sample.e_reco[:n], NBINS, LO, HI, want_p=True)
        return time.perf_counter() - t0

    threads = oracle.num_threads()
    t_all, passes = 0.0, 0
    while passes == 0 or t_all < min_seconds:
        t_all += run(n_all)
        passes += 1
    oracle.set_num_threads(1)
    t_one = run(n_one)
    oracle.set_num_threads(threads)
    return {
        "value": passes * n_all / t_all, "unit": "evals/s", "cores": threads, "kind": "oracle",
        "sample": f"{passes} passes over the first {n_all} events of the 1e7-event workload "
                  f"(fill_pdf with P written), {threads} OpenMP threads, {t_all:.1f} s wall",
        "single_core_value": n_one / t_one,
        "single_core_sample": f"first {n_one} events, 1 thread ({t_one:.2f} s)",
    }


def precision_form(osc, ctx, ds, n_sets=64, set_seed=3):
    """The 1e7 events under 64 parameter sets, once per tier: throughput of
    each tier and the largest |P_mixed - P_fp64| over all events and sets."""
    import torch
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
            ctx.osc_fill_pdf(ds, k, NBINS, LO, HI, h, buf, precision=prec)
        torch.cuda.synchronize()
        ctx.osc_profile_enable(True)
        t0 = time.perf_counter()
        for k in range(n_sets):
            ctx.osc_fill_pdf(ds, k, NBINS, LO, HI, h, buf, precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ev_ms, ev_n, merge_ms, merge_n = ctx.osc_profile_read()
        ctx.osc_profile_enable(False)
        out[name] = {"evals_per_s": n * n_sets / dt, "kernel_ms": ev_ms / max(ev_n, 1),
                     "merge_ms": merge_ms / max(merge_n, 1)}
    worst = 0.0
    for k in range(n_sets):
        ctx.osc_fill_pdf(ds, k, NBINS, LO, HI, h, p64, precision=osc.OSC_FP64)
        ctx.osc_fill_pdf(ds, k, NBINS, LO, HI, h, pmx, precision=osc.OSC_FP32_MIXED)
        worst = max(worst, float((pmx - p64).abs().max()))
    out["max_abs_dP_mixed_vs_fp64"] = worst
    out["config"] = f"{n} events x {n_sets} parameter sets (seed {set_seed}), P written"
    ctx.osc_set_params([workload.TABLE1])
    return out


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
    for _ in range(10):
        tp.fill_pdf(0, h)
    torch.cuda.synchronize()
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


def layered_form(osc, ctx, n=10_000_000, reps=10):
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
    for _ in range(2):
        ctx.osc_fill_pdf_layered(ds, earth, 0, 50, 0.0, 20.0, h)
    torch.cuda.synchronize()
    ctx.osc_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.osc_fill_pdf_layered(ds, earth, 0, 50, 0.0, 20.0, h)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / reps
    ev_ms, ev_n, _, _ = ctx.osc_profile_read()
    ctx.osc_profile_enable(False)
    kernel_ms = ev_ms / max(ev_n, 1)
    return {"config": "5-layer Earth path (11600 km), 1e7 events, E log-uniform 0.5-20 GeV, "
                      "all channels, FP64, 50 bins",
            "layers": 5, "ms_per_call": wall_ms, "kernel_ms": kernel_ms,
            "evals_per_s": n / (wall_ms * 1e-3), "layer_evals_per_s": 5 * n / (kernel_ms * 1e-3)}


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
    hist = torch.empty(NBINS + 2, dtype=torch.float64, device="cuda")
    p_out = torch.empty(N_EVENTS, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        ctx.osc_fill_pdf(ds, 0, NBINS, LO, HI, hist, p_out, stream=stream)

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

    # The fused kernel is bound by VALU issue (FP64 arithmetic), not by HBM:
    # roofline against the FP64 vector peak, HBM position alongside.
    achieved_gbs = BYTES_PER_EVENT * N_EVENTS / (kernel_ms * 1e-3) / 1e9
    fp64_tflops = FLOPS_PER_EVENT * N_EVENTS / (kernel_ms * 1e-3) / 1e12
    traffic = counter_traffic()
    roofline = {
        "bound": "alu", "achieved": fp64_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": fp64_tflops / FP64_PEAK_TFLOPS, "traffic": traffic,
        "kernel": "tile_kernel<kPdf, write P, FP64>", "kernel_ms": kernel_ms,
        "flops_per_event": FLOPS_PER_EVENT, "events_per_launch": N_EVENTS,
        "hbm": {"achieved_GBs": achieved_gbs, "peak_GBs": HBM_PEAK_GBS,
                "frac": achieved_gbs / HBM_PEAK_GBS,
                "algorithmic_bytes_per_event": BYTES_PER_EVENT,
                "traffic_over_algorithmic": (traffic / (BYTES_PER_EVENT * N_EVENTS)
                                             if traffic else None)},
        "merge_kernel_ms": merge_avg_ms,
        "resident_waves_per_cu": waves_per_cu,
        "valu_issue": valu_issue(kernel_ms),
    }

    result = {
        "metric": "oscillation-prob evals/sec (events x param sets) at 1 GPU + p50/p99 reweight latency",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "settle_steps": settle_steps,
        "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "plain FP64 reweight + 50-bin reco-E PDF, 1e7 events x 1 parameter "
                               "set (Table 1, 295 km, 2.6 g/cm^3), per-event P written",
                   "events": N_EVENTS, "param_sets": 1, "nbins": NBINS, "range_GeV": [LO, HI],
                   "seed": SEED, "parallelism": "single GPU"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "calls": args.latency_calls},
        "roofline": roofline,
    }
    if not args.no_forms:
        result["precision_form"] = precision_form(osc, ctx, ds)
    if not args.no_batch:
        result["batched_form"] = batched_form(osc, ctx)
    if not args.no_bincentre:
        result["bincentre_form"] = bincentre_form(osc, ctx, s, ds, ms_per_step)
    if not args.no_layered:
        result["layered_form"] = layered_form(osc, ctx)
    if not args.no_serve:
        result["serving_form"] = serving_form(osc, ctx, args.serve_requests)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(s, args.cpu_events, args.cpu_events_1t,
                                              args.cpu_seconds)
        result["speedup_vs_cpu_all_cores"] = value / result["cpu_baseline"]["value"]
        result["speedup_vs_cpu_one_core"] = value / result["cpu_baseline"]["single_core_value"]
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
