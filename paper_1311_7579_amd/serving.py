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
        h, la, q, _ = server.wait(t)
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


def run_mcmc(server, start, free, sigmas, bounds, n_chains, n_steps, seed, sample=0,
             tier=0, poll_sleep_s=2e-5):
    """Metropolis chains of the fitter (Sec. 2.2) on a server with data set
    (``server.set_data``): each proposal is one request, and its -2 ln L comes back
    with its histogram.  ``free`` names the varied parameters (Gaussian steps
    of ``sigmas``, flat priors on ``bounds``); the others stay at ``start``.
    A proposal with -2 ln L' is accepted with probability
    min(1, exp(-(nll' - nll) / 2)).  The chains run concurrently, one
    request in flight each.  Returns the chains (n_chains, n_steps + 1,
    len(free)), their -2 ln L traces, the acceptance rate and timings."""
    rng = [np.random.default_rng([seed, c]) for c in range(n_chains)]
    sig = np.asarray(sigmas, dtype=np.float64)
    lo = np.array([b[0] for b in bounds], dtype=np.float64)
    hi = np.array([b[1] for b in bounds], dtype=np.float64)
    x0 = np.array([start[k] for k in free], dtype=np.float64)

    def params_of(x):
        p = dict(start)
        p.update({k: float(v) for k, v in zip(free, x)})
        return p

    chains = np.zeros((n_chains, n_steps + 1, len(free)))
    nlls = np.zeros((n_chains, n_steps + 1))
    cur = [x0.copy() for _ in range(n_chains)]
    cur_nll = [None] * n_chains
    step = [0] * n_chains
    pending = {}          # chain -> (ticket, proposal)
    accepted = 0
    lat = []
    t0 = time.perf_counter()
    for c in range(n_chains):
        pending[c] = (server.submit(params_of(cur[c]), sample, tier), cur[c].copy())
    while pending:
        for c in list(pending):
            ticket, prop = pending[c]
            r = server.poll(ticket)
            if r is None:
                continue
            del pending[c]
            lat.append(r.latency_s)
            if cur_nll[c] is None:                     # the starting point
                cur_nll[c] = r.nll
                chains[c, 0], nlls[c, 0] = cur[c], r.nll
            else:
                if np.log(rng[c].random()) < -0.5 * (r.nll - cur_nll[c]):
                    cur[c], cur_nll[c] = prop, r.nll
                    accepted += 1
                step[c] += 1
                chains[c, step[c]], nlls[c, step[c]] = cur[c], cur_nll[c]
            while step[c] < n_steps:
                prop = cur[c] + sig * rng[c].standard_normal(len(free))
                if np.all(prop > lo) and np.all(prop < hi):
                    pending[c] = (server.submit(params_of(prop), sample, tier), prop)
                    break
                step[c] += 1                           # outside the prior: rejected
                chains[c, step[c]], nlls[c, step[c]] = cur[c], cur_nll[c]
        if pending:
            time.sleep(poll_sleep_s)
    wall = time.perf_counter() - t0
    lat = np.array(lat) * 1e3
    evaluated = len(lat)
    return {
        "chains": chains, "nll": nlls,
        "acceptance": accepted / max(1, n_chains * n_steps),
        "requests": evaluated, "wall_s": wall, "steps_per_s": n_chains * n_steps / wall,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
    }
