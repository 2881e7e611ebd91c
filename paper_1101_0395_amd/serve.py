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


def poisson_window(rate_per_s: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate over
    [0, duration_s): exponential gaps of mean 1 / rate, drawn in order."""
    rng = np.random.default_rng(seed)
    n = int(rate_per_s * duration_s * 1.2) + 64
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
    while t[-1] < duration_s:  # (never for the sizes used here)
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))])
    return t[t < duration_s]


class _Slot:
    """Device input and output buffers of one request in flight, and pinned
    host buffers for its results (sized for the largest image of the pool)."""

    def __init__(self, max_px: int, device):
        self.img = torch.empty(3 * max_px, dtype=torch.uint8, device=device)
        self.pal = torch.empty(3 * 256, dtype=torch.uint8, device=device)
        self.idx = torch.empty(max_px, dtype=torch.uint8, device=device)
        self.rgb = torch.empty(3 * max_px, dtype=torch.uint8, device=device)
        self.h_pal = torch.empty(3 * 256, dtype=torch.uint8).pin_memory()
        self.h_idx = torch.empty(max_px, dtype=torch.uint8).pin_memory()
        self.h_rgb = torch.empty(3 * max_px, dtype=torch.uint8).pin_memory()


def run_stream(engine: cq.Engine, pool: list[torch.Tensor], arrivals: np.ndarray, pick: np.ndarray,
               ks: np.ndarray, seeds: np.ndarray, slots: int, max_iters: int, tol: float,
               iters_per_step: int = 8) -> dict:
    """Open-loop serving of requests that arrive at `arrivals` (s, sorted):
    request r quantizes the pinned host image pool[pick[r]] with K = ks[r]
    (k-means++ seeded seeds[r], sort-means).  At most `slots` requests hold
    device buffers at once; a request that arrives while all are taken waits
    in a host backlog (it is "deferred": counted when the requests already
    waiting take every free slot).  A request is copied to the device
    when it gets a slot, submitted to the engine (which admits it when its
    pool range is free), and done once its palette, index image and RGB image
    are back in pinned host memory; its latency runs from its arrival to
    then.  Runs until every request is done, however long that takes."""
    from collections import deque

    n = len(arrivals)
    device = engine.device
    max_px = max(int(t.shape[0]) * int(t.shape[1]) for t in pool)
    free = [_Slot(max_px, device) for _ in range(slots)]
    stream = torch.cuda.current_stream(device)
    backlog: deque = deque()
    inflight = {}
    latency = np.full(n, np.nan)
    deferred = 0
    max_backlog = max_queued = 0
    running_sum = steps = 0
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    i = done_n = 0
    while done_n < n:
        now = time.perf_counter() - t0
        while i < n and arrivals[i] <= now:
            if len(backlog) >= len(free):  # every free slot is already spoken for
                deferred += 1
            backlog.append(i)
            i += 1
        max_backlog = max(max_backlog, len(backlog))
        while backlog and free:
            r = backlog.popleft()
            s = free.pop()
            src = pool[pick[r]]
            H, W = int(src.shape[0]), int(src.shape[1])
            K = int(ks[r])
            img = s.img[: 3 * H * W].view(H, W, 3)
            img.copy_(src, non_blocking=True)  # ordered before the engine's kernels on this stream
            job = cq.BatchJob(img, K, cq.INIT_KMEANSPP, int(seeds[r]), max_iters, tol, True,
                              palette=s.pal[: 3 * K].view(K, 3), idx=s.idx[: H * W].view(H, W),
                              rgb=s.rgb[: 3 * H * W].view(H, W, 3))
            inflight[engine.submit(job)] = (r, s, H * W, K)
        queued, running, _ = engine.pending()
        max_queued = max(max_queued, queued)
        if queued + running == 0:
            if i < n:
                time.sleep(max(0.0, arrivals[i] - (time.perf_counter() - t0)))
            continue
        done = engine.step(iters_per_step)
        steps += 1
        running_sum += engine.pending()[1] + len(done)
        for ticket, _, st in done:
            if st["status"] != cq.CQ_OK:
                raise RuntimeError(f"request {ticket} failed with status {st['status']}")
            r, s, px, K = inflight[ticket]
            s.h_pal[: 3 * K].copy_(s.pal[: 3 * K], non_blocking=True)
            s.h_idx[:px].copy_(s.idx[:px], non_blocking=True)
            s.h_rgb[: 3 * px].copy_(s.rgb[: 3 * px], non_blocking=True)
        if done:
            stream.synchronize()
            t_done = time.perf_counter() - t0
            for ticket, _, _ in done:
                r, s, _, _ = inflight.pop(ticket)
                latency[r] = t_done - arrivals[r]
                free.append(s)
                done_n += 1
    makespan = time.perf_counter() - t0
    lat_ms = 1e3 * np.sort(latency)
    return {
        "requests": n,
        "window_s": float(arrivals[-1]) if n else 0.0,
        "offered_rate_per_s": n / float(arrivals[-1]) if n else None,
        "makespan_s": makespan,
        "throughput_per_s": n / makespan,
        "latency_ms_p50": float(np.percentile(lat_ms, 50)),
        "latency_ms_p90": float(np.percentile(lat_ms, 90)),
        "latency_ms_p99": float(np.percentile(lat_ms, 99)),
        "latency_ms_max": float(lat_ms[-1]),
        "admitted_on_arrival": n - deferred,
        "deferred": deferred,
        "max_host_backlog": max_backlog,
        "max_engine_queue": max_queued,
        "request_slots": slots,
        "steps": steps,
        "mean_jobs_in_flight": running_sum / max(1, steps),
        "iters_per_step": iters_per_step,
    }
