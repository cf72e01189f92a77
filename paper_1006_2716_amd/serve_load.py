"""Client side of the serving engine: replays a request stream against a
context and reports latency percentiles and throughput.

Each site runs `n_iter` simulated DMFT iterations.  Its first request arrives
at its Poisson time; iteration j+1 is submitted as soon as result j has come
back (its Weiss function and RNG offset change, its fields and G stay on the
device).  Latency of a request = completion (poll returned) - arrival.
"""
from __future__ import annotations

import time

import numpy as np


def site_request(site: dict, it: int, weiss, sweeps: int, warm_first: int, warm_next: int, n_bins: int = 32) -> dict:
    """Problem dict of iteration `it` of a site (see workloads.serving_requests).
    A site with "n_chains" > 1 runs that many chains, each with the full
    warm-up and a share of the measured sweeps."""
    nw = warm_first if it == 0 else warm_next
    return dict(L=site["L"], beta=site["beta"], U=site["U"], weiss=weiss(site, it), n_warmup=nw,
                n_measure=sweeps - nw, recompute_every=50, n_bins=n_bins, seed=site["seed"], site=site["site"],
                sweep_offset=it * sweeps, delay=0, n_chains=site.get("n_chains", 1))


def replay(ctx, sites, arrivals, weiss, n_iter: int = 10, sweeps: int = 5000, warm_first: int = 500,
           warm_next: int = 100, n_bins: int = 32, poll_sleep: float = 2e-4, timeout_s: float = 600.0,
           progress=None) -> dict:
    """Drive `ctx` (a hfqmc.Context with a pool attached) with the stream.

    Returns latency percentiles (ms), throughput (proposals/s over the
    makespan), per-L latency medians and the per-request results."""
    handles = [ctx.site(s["L"], n_bins=n_bins, n_chains=s.get("n_chains", 1)) for s in sites]
    n = len(sites)
    it = [0] * n
    due = list(np.asarray(arrivals, dtype=float))
    arrive = [None] * n        # arrival time of the site's current request
    ticket = [None] * n
    step0 = [0] * n            # engine step count when the request was queued
    steps_per_request = []
    lat, lat_L, results = [], {}, {}
    proposals = 0
    t0 = time.perf_counter()
    last_report = t0
    remaining = n * n_iter
    try:
        while remaining:
            now = time.perf_counter() - t0
            if now > timeout_s:
                raise TimeoutError(f"serving replay exceeded {timeout_s} s with {remaining} requests left")
            for i in range(n):
                if ticket[i] is None and it[i] < n_iter and due[i] <= now:
                    if arrive[i] is None:
                        arrive[i] = due[i]
                    t = ctx.submit(handles[i], site_request(sites[i], it[i], weiss, sweeps, warm_first, warm_next,
                                                            n_bins))
                    if t is not None:
                        ticket[i] = t
                        step0[i] = ctx.serve_stats()["steps"]
            for i in range(n):
                if ticket[i] is None:
                    continue
                r = ctx.poll(ticket[i])
                if r is None:
                    continue
                done = time.perf_counter() - t0
                steps_per_request.append(ctx.serve_stats()["steps"] - step0[i])
                ms = (done - arrive[i]) * 1e3
                lat.append(ms)
                lat_L.setdefault(sites[i]["L"], []).append(ms)
                results[(i, it[i])] = r
                proposals += r["proposals"]
                ticket[i] = None
                arrive[i] = None
                it[i] += 1
                due[i] = done  # the next iteration arrives with this result
                remaining -= 1
            if progress and time.perf_counter() - last_report > 5.0:
                last_report = time.perf_counter()
                progress(f"serving: {n * n_iter - remaining}/{n * n_iter} requests done")
            time.sleep(poll_sleep)
        makespan = time.perf_counter() - t0
    finally:
        for i in range(n):
            if ticket[i] is not None:
                try:
                    ctx.cancel(ticket[i])
                except Exception:
                    pass
        # sites with requests still in flight stay open until the context closes
        for h in handles:
            try:
                h.close()
            except Exception:
                pass
    lat = np.asarray(lat)
    return dict(p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                max_ms=float(lat.max()), requests=int(lat.size), makespan_s=makespan,
                proposals=int(proposals), proposals_per_s=proposals / makespan,
                p50_ms_by_L={int(k): float(np.median(v)) for k, v in sorted(lat_L.items())},
                steps_per_request_p50=float(np.median(steps_per_request)),
                results=results)
