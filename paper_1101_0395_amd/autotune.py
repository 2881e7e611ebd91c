"""Autotuner of the iteration schedule (``cq_schedule`` in include/cq.h).

How the Lloyd iterations are tiled changes no result, only the speed: the
colours each assignment block takes and how often a pruned run regroups its
colours by (cluster, distance bucket).  The best choice depends on how many
colours one call iterates over (a small batch leaves the GPU waiting on
latency; a large one is bound by its memory traffic), so the tuner times every
candidate schedule on batches of several sizes, checks that every candidate
gives the same palettes, images and statistics, and derives a table keyed by
the number of colours: each measured size's best schedule applies from the
geometric mean of its colour count and the next smaller one's.

    python -m paper_1101_0395_amd.autotune [--out schedule.json]

writes the measurements and the table (``paper_1101_0395_amd/schedule.json``
by default).  The library's built-in table is that file's ``table``; a test
checks that the two agree.  ``apply(path)`` loads a table into the library.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "schedule.json")
CHUNKS = (1024, 2048, 4096, 8192, 16384)
PERIODS = (1, 2, 3, 4)
MAX_ITERS, TOL = 100, 1e-4


def workloads(synth):
    """(name, shapes) of the tuning batches: shapes as (H, W, K, seed)."""
    c2 = [(512, 512, 256, s) for s in range(1, 9)]
    return [
        ("1 x 512x512, K=256", c2[:1]),
        ("8 x 512x512, K=256", c2),
        ("64 mixed-size images, K=256", [(h, w, 256, s) for h, w, _, s in synth.batch_shapes(64)]),
        ("512 mixed-size images, K=256", [(h, w, 256, s) for h, w, _, s in synth.batch_shapes(512)]),
    ]


def _images(synth, shapes, workers):
    mixed = [x for x in shapes if x[3] >= 1_000_000]
    imgs = {}
    if mixed:
        for x, im in zip(mixed, synth.batch_images(mixed, workers)):
            imgs[x] = im
    for x in shapes:
        if x not in imgs:
            imgs[x] = synth.smooth_field_blobs(x[0], x[1], x[3])
    return [imgs[x] for x in shapes]


def time_schedule(cq, torch, jobs, bws, chunk, period, reps):
    """Mean ms per batched call under the one-entry schedule (chunk, period),
    and the results of the last call."""
    cq.set_schedule([(0, chunk, period)])
    try:
        cq.cq_quantize_batch(jobs, bws)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            stats = cq.cq_quantize_batch(jobs, bws)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
    finally:
        cq.set_schedule([])
    outs = [(j.palette.clone(), j.idx.clone(), j.rgb.clone()) for j in jobs]
    return ms, stats, outs


def tune(cq, torch, imgs, shapes, dev, reps=3, chunks=CHUNKS, periods=PERIODS):
    """Times every (chunk, period) on one batch; raises if any two candidates
    disagree on a result.  Returns (colours, {"chunk,period": ms}, best)."""
    jobs = [cq.BatchJob(torch.from_numpy(im).to(dev), K, cq.INIT_KMEANSPP, seed, MAX_ITERS, TOL, True)
            for im, (_, _, K, seed) in zip(imgs, shapes)]
    bws = cq.BatchWorkspace(jobs, dev)
    ref = None
    times = {}
    colours = 0
    for chunk in chunks:
        for period in periods:
            ms, stats, outs = time_schedule(cq, torch, jobs, bws, chunk, period, reps)
            if ref is None:
                ref = (stats, outs)
                colours = sum(s["n_unique"] for s, (_, _, K, _) in zip(stats, shapes) if s["n_unique"] > K)
            elif stats != ref[0] or not all(all(torch.equal(a, b) for a, b in zip(x, y))
                                            for x, y in zip(outs, ref[1])):
                raise RuntimeError(f"schedule ({chunk}, {period}) changed a result")
            times[f"{chunk},{period}"] = ms
            print(f"[tune]   chunk {chunk:5d} period {period}: {ms:8.2f} ms", file=sys.stderr, flush=True)
    best = min(times, key=times.get)
    return colours, times, tuple(int(v) for v in best.split(","))


def table_from(measured):
    """Schedule table from [(colours, (chunk, period)), ...]: each size's best
    applies from the geometric mean of its colour count and the previous
    size's."""
    measured = sorted(measured)
    table = []
    for i, (colours, (chunk, period)) in enumerate(measured):
        start = 0 if i == 0 else int(math.sqrt(measured[i - 1][0] * colours))
        if table and (table[-1][1], table[-1][2]) == (chunk, period):
            continue
        table.append((start, chunk, period))
    return table


def apply(path: str = DEFAULT_PATH):
    """Loads the table of a tuning file into the library."""
    from paper_1101_0395_amd import cq
    with open(path) as f:
        cq.set_schedule([tuple(e) for e in json.load(f)["table"]])


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    from paper_1101_0395_amd import synth
    loads = workloads(synth)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    host = [_images(synth, shapes, workers) for _, shapes in loads]  # before the GPU is touched
    import torch

    from paper_1101_0395_amd import cq
    dev = torch.device("cuda:0")
    cq.lib()
    results, measured = [], []
    for (name, shapes), imgs in zip(loads, host):
        print(f"[tune] {name}", file=sys.stderr, flush=True)
        colours, times, best = tune(cq, torch, imgs, shapes, dev, reps=args.reps)
        results.append({"workload": name, "images": len(shapes), "colours": colours, "ms": times,
                        "best": list(best)})
        measured.append((colours, best))
        torch.cuda.empty_cache()
    out = {"device": torch.cuda.get_device_name(dev), "candidates": {"assign_chunk": list(CHUNKS),
                                                                    "regroup_period": list(PERIODS)},
           "settings": "k-means++, sort-means, tol 1e-4, at most 100 iterations, full map",
           "results": results, "table": [list(e) for e in table_from(measured)]}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["table"]))


if __name__ == "__main__":
    main()
