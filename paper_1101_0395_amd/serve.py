"""Serving loop over the continuous-batching engine: requests arrive as a
Poisson process, are submitted at their arrival time, and leave when the
engine reports them done; the latency of a request is its completion time
minus its arrival time.

A request's image is either already on the device, or sits in pinned host
memory and is copied to the device at arrival; with host I/O its palette,
index image and RGB image are also copied back to pinned host memory before
it counts as done, so the latency runs from arrival to the result on the
host."""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import cq


@dataclass
class Request:
    arrival_s: float
    job: cq.BatchJob
    host_img: torch.Tensor | None = None  # pinned; copied into job.img at arrival
    host_out: tuple | None = None         # pinned (palette, idx, rgb) receiving the results


def poisson_arrivals(n: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of n requests with exponential gaps of mean 1 / rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def make_request(arrival_s: float, img: torch.Tensor, K: int, seed: int, max_iters: int, tol: float,
                 device, host_io: bool) -> Request:
    """A k-means++ sort-means request for `img` (a host tensor if host_io,
    else a device tensor)."""
    if not host_io:
        return Request(arrival_s, cq.BatchJob(img, K, cq.INIT_KMEANSPP, seed, max_iters, tol, True))
    host = img if img.is_pinned() else img.pin_memory()
    dev_img = torch.empty(host.shape, dtype=torch.uint8, device=device)
    job = cq.BatchJob(dev_img, K, cq.INIT_KMEANSPP, seed, max_iters, tol, True)
    outs = tuple(torch.empty(t.shape, dtype=torch.uint8).pin_memory() for t in (job.palette, job.idx, job.rgb))
    return Request(arrival_s, job, host, outs)


def run(engine: cq.Engine, requests: list[Request], iters_per_step: int = 8) -> dict:
    """Drives the engine until every request has finished; returns latency
    percentiles (ms), throughput and occupancy figures."""
    reqs = sorted(requests, key=lambda r: r.arrival_s)
    n = len(reqs)
    by_ticket, latency = {}, {}
    running_sum = steps = 0
    stream = torch.cuda.current_stream(engine.device)
    torch.cuda.synchronize(engine.device)
    t0 = time.perf_counter()
    i = 0
    while len(latency) < n:
        now = time.perf_counter() - t0
        while i < n and reqs[i].arrival_s <= now:
            r = reqs[i]
            if r.host_img is not None:
                r.job.img.copy_(r.host_img, non_blocking=True)  # ordered before the engine's kernels
            by_ticket[engine.submit(r.job)] = r
            i += 1
        queued, running, _ = engine.pending()
        if queued + running == 0:
            time.sleep(max(0.0, reqs[i].arrival_s - now))  # idle until the next arrival
            continue
        done = engine.step(iters_per_step)
        steps += 1
        running_sum += engine.pending()[1] + len(done)
        copied = False
        for ticket, job, st in done:
            if st["status"] != cq.CQ_OK:
                raise RuntimeError(f"request {ticket} failed with status {st['status']}")
            r = by_ticket[ticket]
            if r.host_out is not None:
                for dst, src in zip(r.host_out, (job.palette, job.idx, job.rgb)):
                    dst.copy_(src, non_blocking=True)
                copied = True
        if copied:
            stream.synchronize()
        t_done = time.perf_counter() - t0
        for ticket, _, _ in done:
            latency[ticket] = t_done - by_ticket[ticket].arrival_s
    makespan = time.perf_counter() - t0
    lat_ms = 1e3 * np.array(sorted(latency.values()))
    last = reqs[-1].arrival_s
    return {
        "requests": n,
        "offered_rate_per_s": n / last if last > 0 else None,
        "throughput_per_s": n / makespan,
        "latency_ms_p50": float(np.percentile(lat_ms, 50)),
        "latency_ms_p90": float(np.percentile(lat_ms, 90)),
        "latency_ms_p99": float(np.percentile(lat_ms, 99)),
        "latency_ms_max": float(lat_ms[-1]),
        "steps": steps,
        "mean_jobs_in_flight": running_sum / max(1, steps),
        "iters_per_step": iters_per_step,
    }
