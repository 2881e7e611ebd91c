"""Serving loop over the continuous-batching engine: requests arrive as a
Poisson process, are submitted at their arrival time, and leave when the
engine reports them done; the latency of a request is its completion time
minus its arrival time.  Inputs are resident on the device before the clock
starts (the serving path under test is the quantizer, not the upload)."""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import cq


@dataclass
class Request:
    arrival_s: float
    job: cq.BatchJob


def poisson_arrivals(n: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of n requests with exponential gaps of mean 1 / rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def run(engine: cq.Engine, requests: list[Request], iters_per_step: int = 8) -> dict:
    """Drives the engine until every request has finished; returns latency
    percentiles (ms), throughput and occupancy figures."""
    import torch

    reqs = sorted(requests, key=lambda r: r.arrival_s)
    n = len(reqs)
    arrival, latency = {}, {}
    running_sum = steps = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i = 0
    while len(latency) < n:
        now = time.perf_counter() - t0
        while i < n and reqs[i].arrival_s <= now:
            arrival[engine.submit(reqs[i].job)] = reqs[i].arrival_s
            i += 1
        queued, running, _ = engine.pending()
        if queued + running == 0:
            time.sleep(max(0.0, reqs[i].arrival_s - now))  # idle until the next arrival
            continue
        done = engine.step(iters_per_step)
        steps += 1
        running_sum += engine.pending()[1] + len(done)
        t_done = time.perf_counter() - t0
        for ticket, _, st in done:
            if st["status"] != cq.CQ_OK:
                raise RuntimeError(f"request {ticket} failed with status {st['status']}")
            latency[ticket] = t_done - arrival[ticket]
    makespan = time.perf_counter() - t0
    lat_ms = 1e3 * np.array(sorted(latency.values()))
    return {
        "requests": n,
        "offered_rate_per_s": n / reqs[-1].arrival_s if reqs[-1].arrival_s > 0 else None,
        "throughput_per_s": n / makespan,
        "latency_ms_p50": float(np.percentile(lat_ms, 50)),
        "latency_ms_p90": float(np.percentile(lat_ms, 90)),
        "latency_ms_p99": float(np.percentile(lat_ms, 99)),
        "latency_ms_max": float(lat_ms[-1]),
        "steps": steps,
        "mean_jobs_in_flight": running_sum / max(1, steps),
        "iters_per_step": iters_per_step,
    }
