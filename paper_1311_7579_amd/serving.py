"""Drive an osc_server with a timed request stream and summarise it.

Host-side plumbing only: requests are submitted at their arrival times
and the results collected; all computation runs in libosc.
"""
import time

import numpy as np


def run_stream(server, requests, arrivals_s, events_per_sample):
    """Submit requests[k] = (params, sample, tier) at arrivals_s[k] seconds
    after the start, wait for every result, and return the results and a
    summary (latency percentiles from submission to histogram on the host,
    throughput in evaluations per second, server statistics)."""
    t0 = time.perf_counter()
    tickets = []
    for (params, sample, tier), ta in zip(requests, arrivals_s):
        while True:
            dt = ta - (time.perf_counter() - t0)
            if dt <= 0:
                break
            if dt > 3e-4:
                time.sleep(dt - 2e-4)
        tickets.append(server.submit(params, sample, tier))
    t_sub = time.perf_counter() - t0
    results, lat, queue = [], [], []
    for t in tickets:
        h, la, q = server.wait(t)
        results.append(h)
        lat.append(la)
        queue.append(q)
    t_end = time.perf_counter() - t0
    lat = np.array(lat) * 1e3
    evals = sum(events_per_sample[s] for _, s, _ in requests)
    summary = {
        "requests": len(requests),
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "mean_queue_ms": float(np.mean(queue) * 1e3),
        "evals_per_s": evals / t_end, "wall_s": t_end, "submit_s": t_sub,
        "offered_rate_hz": len(requests) / max(arrivals_s[-1], 1e-9) if len(requests) else 0.0,
        "stats": server.stats(),
    }
    return results, summary
