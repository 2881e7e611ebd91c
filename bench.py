"""Benchmark: exact weighted sort-means colour quantization on one MI355X.

Headline workload: the mixed batch of 512 natural-image stand-ins (long side
log-uniform in 64-2048, aspect 1-2, seeds 1,000,000 + i) with K = 256 for every
image, k-means++ initialization, sort-means pruning, tol 1e-4, at most 100
iterations, full pixel map (index and RGB images).  One step quantizes all 512
images end to end (histogram, init, iterations, palette, map) from
device-resident inputs with one batched call; the same images quantized one
call per image (the plain path) are timed beside it.  The same batch with each
image's own K (drawn from {16, ..., 256}) and the eight 512 x 512 stand-ins
are reported as extra keys.

Prints one JSON line: images/s, the distance-evaluation rates, the MSE
relative error against the CPU oracle on a sample, a roofline entry for the
dominant kernel (timed live with HIP events on the launch stream) and the
oracle's own throughput on the host CPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

H = W = 512
K = 256
SEEDS = list(range(1, 9))
MAX_ITERS = 100
TOL = 1e-4
C4_IMAGES = 512                # the mixed batch: seeds 1,000,000 + i

PEAK_FP64_VALU_TFLOPS = 78.6   # MI355X vector FP64
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
FLOP_PER_EVAL = 8              # 3 sub, 3 mul, 2 add per FP64 squared distance
# Algorithmic bytes of one colour in one sort-means pass: its 8-byte record
# (key, count, previous cluster, distance bucket) read, and written back with
# the new cluster.  At 8 FLOP x ~3.4 evaluations per colour that is under 2
# FLOP per byte, far below the FP64 ridge (78.6 TFLOP/s / 8 TB/s), so HBM is
# the roof: the mixed batch's 99 M records (0.8 GB) do not stay in the
# 256 MiB MALL from one pass to the next.
WALK_BYTES_PER_COLOUR = 16
ROOFLINE_KERNEL = "k_assign_walk"  # sort-means nearest-centre passes
TIMER_EVERY = 8                    # HIP-event bracket on every 8th launch of it


def measure_large(cq, synth, torch, dev, reps=5):
    """Histogram and pixel-map bandwidth on one 4096 x 4096 stand-in (seed 42),
    K = 256: each kernel timed with HIP events over `reps` calls; the bytes
    are the algorithmic ones (image read; colours and counts or index and
    RGB images written)."""
    H4 = W4 = 4096
    img = torch.from_numpy(synth.smooth_field_blobs(H4, W4, 42)).to(dev)
    ws = cq.Workspace(H4, W4, K, dev)
    keys, counts = cq.cq_histogram(img, ws)  # warm-up
    n = int(keys.numel())

    per_kernel = {}

    def timed(names, fn):
        total = 0.0
        for name in names:
            t = cq.KernelTimer(name, reps)
            t.enable()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            launches, ms = t.read()
            t.disable()
            per_kernel[name] = 1e3 * ms / max(1, launches)
            total += ms / max(1, launches)
        if total <= 0.0:
            raise RuntimeError(f"no launches of {names} were timed")
        return total

    hist_names = ["k_hist_part", "k_hist_count", "k_hist_emit"]
    hist_ms = timed(hist_names, lambda: cq.cq_histogram(img, ws))
    full_kernels = dict(per_kernel)
    keys_s, _ = cq.cq_histogram(img, ws, subsample=True)
    n_sub = int(keys_s.numel())
    sub_ms = timed(hist_names, lambda: cq.cq_histogram(img, ws, subsample=True))
    sub_kernels = {k: per_kernel[k] for k in hist_names}
    per_kernel.update(full_kernels)
    centers, _ = cq.cq_init(keys, counts, K, cq.INIT_KMEANSPP, 42, ws)
    km = cq.cq_kmeans(keys, counts, centers, 3, TOL, True, ws)  # a palette to map to
    cq.cq_map(img, keys, counts, km.palette, ws)
    map_ms = timed(["k_map"], lambda: cq.cq_map(img, keys, counts, km.palette, ws))
    lut_ms = timed(["k_lut"], lambda: cq.cq_map(img, keys, counts, km.palette, ws))
    hist_bytes = 3 * H4 * W4 + 8 * n
    map_bytes = 3 * H4 * W4 + H4 * W4 + 3 * H4 * W4
    hist_gbs = hist_bytes / (hist_ms * 1e-3) / 1e9
    map_gbs = map_bytes / (map_ms * 1e-3) / 1e9
    return {
        "workload": "one 4096x4096 stand-in (seed 42), K=256",
        "unique_colours": n,
        "histogram": {"us": 1e3 * hist_ms, "bytes": hist_bytes, "GB/s": hist_gbs,
                      "frac_of_hbm_peak": hist_gbs / PEAK_HBM_GBS},
        "pixel_map": {"us": 1e3 * map_ms, "bytes": map_bytes, "GB/s": map_gbs,
                      "frac_of_hbm_peak": map_gbs / PEAK_HBM_GBS},
        "colour_table_us": 1e3 * lut_ms,
        "kernel_us": per_kernel,
        # 2:1 subsampling: a quarter of the pixels are counted; the even rows
        # are still read whole, so the bytes are those rows plus the output
        "histogram_subsampled": {"us": 1e3 * sub_ms, "unique_colours": n_sub,
                                 "bytes_even_rows": 3 * ((H4 + 1) // 2) * W4 + 8 * n_sub,
                                 "GB/s_even_rows": (3 * ((H4 + 1) // 2) * W4 + 8 * n_sub) / (sub_ms * 1e-3) / 1e9,
                                 "speedup_vs_full": hist_ms / sub_ms,
                                 "kernel_us": sub_kernels},
    }


def measure_serving(cq, torch, synth, imgs, dev, host_c4, workers, seconds):
    """Continuous batching under Poisson arrivals (the serving engine).

    - "512x512_device_inputs": 96 requests for the eight 512 x 512 images in
      turn (request r uses k-means++ seed 1000 + r), K = 256, offered at
      500/s; inputs already on the device; at most 16 jobs in flight.
    - "poisson_2000_per_s": Poisson arrivals at 2000 requests/s for `seconds`
      (60 by default); request r takes an image drawn uniformly (rng seed 7)
      from a pool of 1024 mixed-size stand-ins (the batch shapes of seeds
      1,000,000 + i, i < 1024; the first 512 are the mixed batch) and its own
      K drawn from {16, 32, 64, 128, 256}.  Images start in pinned host
      memory and are copied in when a request gets device buffers; results go
      back to pinned host memory before a request counts as done.  At most 192
      requests hold device buffers, at most 128 are in flight in the engine,
      whose slot pool has 24 GiB; requests beyond that wait (deferred).
    Every request: sort-means, tol 1e-4, at most 100 iterations, full map."""
    import numpy as np

    from paper_1101_0395_amd import serve

    out = {}
    eng = cq.Engine(16, 16 * cq.engine_job_bytes(H, W), dev)
    arrivals = serve.poisson_arrivals(96, 500.0, seed=7)

    def homogeneous(arr):
        return [serve.make_request(float(t), imgs[r % len(imgs)], K, 1000 + r, MAX_ITERS, TOL, dev, False)
                for r, t in enumerate(arr)]

    serve.run(eng, homogeneous(arrivals[:16]))  # warm-up
    res = serve.run(eng, homogeneous(arrivals))
    eng.close()
    res["workload"] = ("96 requests, Poisson arrivals at 500/s, 512x512 stand-ins (seeds 1-8), K=256, "
                       "inputs on the device, 16 jobs in flight, 8 iterations per step")
    out["512x512_device_inputs"] = res

    shapes = synth.batch_shapes(1024)
    more = synth.batch_images(shapes[len(host_c4):], workers)
    pool = [torch.from_numpy(im).pin_memory() for im in list(host_c4) + more]
    rng = np.random.default_rng(7)
    rate = 2000.0
    arrivals = serve.poisson_window(rate, seconds, seed=8)
    n = len(arrivals)
    pick = rng.integers(0, len(pool), n)
    ks = rng.choice(np.array([16, 32, 64, 128, 256]), n)
    seeds = 3_000_000 + np.arange(n)
    eng = cq.Engine(128, 24 << 30, dev)
    warm = serve.poisson_window(rate, 0.1, seed=9)
    serve.run_stream(eng, pool, warm, pick, ks, seeds, 192, MAX_ITERS, TOL)  # warm-up
    res = serve.run_stream(eng, pool, arrivals, pick, ks, seeds, 192, MAX_ITERS, TOL)
    eng.close()
    res["mean_pixels"] = float(np.mean([pool[p].shape[0] * pool[p].shape[1] for p in pick]))
    res["workload"] = (f"Poisson arrivals at {rate:.0f}/s for {seconds:.0f} s ({n} requests); images drawn "
                       "from a pool of 1024 mixed-size stand-ins (long side 64-2048) in pinned host memory, "
                       "each request with its own K in {16..256}; host-to-device input and device-to-host "
                       "results inside the latency; 192 request slots, 128 jobs in flight, 24 GiB slot pool, "
                       "8 iterations per step")
    out["poisson_2000_per_s"] = res
    return out


def lbg_init_ms(cq, torch, jobs, dev):
    ws = cq.Workspace(H, W, K, dev)
    total = 0.0
    for i, job in enumerate(jobs):
        keys, counts = cq.cq_histogram(job.img, ws)
        cq.cq_init(keys, counts, K, cq.INIT_LBG, SEEDS[i], ws)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cq.cq_init(keys, counts, K, cq.INIT_LBG, SEEDS[i], ws)
        torch.cuda.synchronize()
        total += 1e3 * (time.perf_counter() - t0)
    return total


def measure_init_schemes(cq, torch, imgs, dev, reps=3):
    """The headline batch (eight 512 x 512 stand-ins, K = 256, sort-means, tol
    1e-4) with each initialization scheme: step time, the time of the scheme's
    own kernels (HIP events), mean iterations and mean MSE of the mapped
    images."""
    import numpy as np

    kernels = {cq.INIT_FORGY: ["k_forgy"], cq.INIT_MAXMIN: ["k_init_coop"], cq.INIT_KMEANSPP: ["k_init_coop"],
               cq.INIT_VAR: ["k_var_tiles", "k_var_pick", "k_var_find"], cq.INIT_SFF: ["k_sff"],
               cq.INIT_WU: ["k_wu_clear", "k_wu_accum", "k_wu_prefix", "k_wu_split"], cq.INIT_LBG: None,
               cq.INIT_DEN: ["k_den_tiles", "k_den_pick", "k_den_find"]}
    names = {cq.INIT_FORGY: "FGY", cq.INIT_MAXMIN: "MMX", cq.INIT_KMEANSPP: "KPP", cq.INIT_VAR: "VAR",
             cq.INIT_SFF: "SFF", cq.INIT_WU: "WU", cq.INIT_LBG: "LBG", cq.INIT_DEN: "DEN"}
    out = {}
    for scheme, kern in kernels.items():
        jobs = [cq.BatchJob(img, K, scheme, SEEDS[i], MAX_ITERS, TOL, True) for i, img in enumerate(imgs)]
        bws = cq.BatchWorkspace(jobs, dev)
        cq.cq_quantize_batch(jobs, bws)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st = cq.cq_quantize_batch(jobs, bws)
        torch.cuda.synchronize()
        step_ms = 1e3 * (time.perf_counter() - t0) / reps
        # LBG's stages run the k-means kernels themselves: its initialization
        # is the time of cq_init on the batch's histograms, one call per image
        init_ms = 0.0 if kern is not None else lbg_init_ms(cq, torch, jobs, dev)
        for name in kern or []:
            t = cq.KernelTimer(name, reps * 4)
            t.enable()
            for _ in range(reps):
                cq.cq_quantize_batch(jobs, bws)
            torch.cuda.synchronize()
            launches, ms = t.read()
            t.disable()
            init_ms += ms / reps
        out[names[scheme]] = {"step_ms": step_ms, "init_ms": init_ms,
                              "mean_iters": float(np.mean([x["iters"] for x in st])),
                              "mean_mse": float(np.mean([x["mse_img"] for x in st]))}
    return out


def measure_subsample(cq, torch, imgs, dev, reps=3):
    """The headline batch with the 2:1 subsampling of Section 2.2 (item 1)
    before the histogram, against the same batch without it: step time, mean
    unique colours and iterations, and mean MSE of the mapped (full) images."""
    import numpy as np

    out = {}
    for label, sub in (("full", False), ("subsampled", True)):
        jobs = [cq.BatchJob(img, K, cq.INIT_KMEANSPP, SEEDS[i], MAX_ITERS, TOL, True, subsample=sub)
                for i, img in enumerate(imgs)]
        bws = cq.BatchWorkspace(jobs, dev)
        cq.cq_quantize_batch(jobs, bws)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st = cq.cq_quantize_batch(jobs, bws)
        torch.cuda.synchronize()
        step_ms = 1e3 * (time.perf_counter() - t0) / reps
        kern_us = {}
        for name in ("k_hist_part", "k_hist_count", "k_hist_emit", "k_lut", "k_map"):
            t = cq.KernelTimer(name, reps)
            t.enable()
            for _ in range(reps):
                cq.cq_quantize_batch(jobs, bws)
            torch.cuda.synchronize()
            launches, ms = t.read()
            t.disable()
            kern_us[name] = 1e3 * ms / launches if launches else 0.0
        out[label] = {"step_ms": step_ms,
                      "mean_unique_colours": float(np.mean([x["n_unique"] for x in st])),
                      "mean_iters": float(np.mean([x["iters"] for x in st])),
                      "mean_mse": float(np.mean([x["mse_img"] for x in st])),
                      "kernel_us_per_launch": kern_us}
    out["speedup"] = out["full"]["step_ms"] / out["subsampled"]["step_ms"]
    out["mse_ratio"] = out["subsampled"]["mean_mse"] / out["full"]["mean_mse"]
    return out


def measure_km_vs_wsm(cq, torch, imgs, dev, Ks=(32, 64, 128, 256), iters=20):
    """The comparison of Section 3.2 on the eight stand-ins: plain KM (full
    search over every pixel) against WSM (sort-means on the weighted
    histogram), both from the same FGY centres and run for at most 20
    iterations (tol 0: a run ends early only once its SSE stops falling, and
    then both end together).  Per K: distance calculations per point and
    iteration (KM: K; WSM: over the unique colours), and the k-means time of
    each (one call per image, mean over the images)."""
    import numpy as np

    ws = cq.Workspace(H, W, max(Ks), dev)
    data = []
    for i, img in enumerate(imgs):
        hk, hc = cq.cq_histogram(img, ws)
        hk, hc = hk.clone(), hc.clone()
        pk, pc = cq.cq_pixel_keys(img)
        data.append((hk, hc, pk, pc))
    out = {}
    for K in Ks:
        km_ms, wsm_ms, km_ndc, wsm_ndc, same = [], [], [], [], True
        for i, (hk, hc, pk, pc) in enumerate(data):
            c0, _ = cq.cq_init(hk, hc, K, cq.INIT_FORGY, SEEDS[i], ws)
            c0 = c0.clone()
            res = {}
            for label, keys, counts, prune, acc in (("wsm", hk, hc, True, wsm_ms), ("km", pk, pc, False, km_ms)):
                cq.cq_kmeans(keys, counts, c0.clone(), iters, 0.0, prune, ws)  # warm-up
                c = c0.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = cq.cq_kmeans(keys, counts, c, iters, 0.0, prune, ws)
                acc.append(1e3 * (time.perf_counter() - t0))
                res[label] = r
            w, k = res["wsm"], res["km"]
            same = same and torch.equal(w.centers, k.centers) and w.sse_trace == k.sse_trace
            wsm_ndc.append(w.stats["ndc_total"] / (w.stats["n_unique"] * max(1, w.stats["iters"])))
            km_ndc.append(k.stats["ndc_total"] / (k.stats["n_unique"] * max(1, k.stats["iters"])))
        out[str(K)] = {"ndc_per_point_iter": {"km": float(np.mean(km_ndc)), "wsm": float(np.mean(wsm_ndc)),
                                              "km_over_wsm": float(np.mean(km_ndc) / np.mean(wsm_ndc))},
                       "kmeans_ms_per_image": {"km": float(np.mean(km_ms)), "wsm": float(np.mean(wsm_ms)),
                                               "km_over_wsm": float(np.mean(km_ms) / np.mean(wsm_ms))},
                       "identical_results": bool(same)}
    return out


def measure_k_sweep(cq, torch, imgs, dev, iters=20):
    """WSM time against K = 2..256 (the figure of Section 3.2) in the setting
    of the comparison table: FGY centres, at most 20 iterations (tol 0),
    sort-means; the whole quantization (histogram to pixel map) per image, mean
    over the eight stand-ins."""
    ws = cq.Workspace(H, W, 256, dev)
    pal = torch.zeros((256, 3), dtype=torch.uint8, device=dev)
    oidx = torch.empty((H, W), dtype=torch.uint8, device=dev)
    orgb = torch.empty((H, W, 3), dtype=torch.uint8, device=dev)
    ms = []
    for k in range(2, 257):
        cq.cq_quantize(imgs[0], k, cq.INIT_FORGY, 1, iters, 0.0, True, ws, palette=pal[:k], out_idx=oidx,
                       out_rgb=orgb)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, img in enumerate(imgs):
            cq.cq_quantize(img, k, cq.INIT_FORGY, SEEDS[i], iters, 0.0, True, ws, palette=pal[:k], out_idx=oidx,
                           out_rgb=orgb)
        torch.cuda.synchronize()
        ms.append(1e3 * (time.perf_counter() - t0) / len(imgs))
    at = {k: ms[k - 2] for k in (2, 16, 32, 64, 128, 256)}
    return {"ms_per_image_at": at, "ratio_256_over_16": at[256] / at[16], "ms_per_image_k2_to_256": ms}


def recorded_traffic():
    """HBM bytes per launch of the sort-means pass from the committed counter
    summary, if it was measured on the kernel source as it is now; else None."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "k_assign_walk_traffic_mixed_batch.md")
    try:
        text = open(path).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        src = open(os.path.join(ROOT, "paper_1101_0395_amd", "csrc", "kmeans.hip"), "rb").read()
    except (OSError, AttributeError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("source_sha256_16"):
        return None
    return rec.get("traffic_bytes_per_launch")


def cpu_info():
    """CPU model and logical CPU count of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def worker_count():
    """Host processes or threads for input generation and the oracle sample:
    the CPUs this process may run on, at most 16 (one GPU's share of a host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def make_jobs(cq, imgs, shapes, k_of, dev):
    return [cq.BatchJob(img, k_of(i), cq.INIT_KMEANSPP, shapes[i][3], MAX_ITERS, TOL, True)
            for i, img in enumerate(imgs)]


def time_batched(cq, torch, jobs, bws, steps, warmup, timer=None):
    """Warm-up steps, then `steps` timed batched calls bracketed by device
    synchronizations; returns (seconds, stats of the last step, all stats)."""
    for _ in range(warmup):
        cq.cq_quantize_batch(jobs, bws)
    torch.cuda.synchronize()
    if timer is not None:
        timer.enable()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(steps):
        stats.append(cq.cq_quantize_batch(jobs, bws))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, stats[-1], stats


def time_plain(cq, torch, jobs, dev, warm=8):
    """The plain path: one cq_quantize call per image (each synchronizes), over
    one workspace sized for the largest image; returns images/s."""
    big = max(jobs, key=lambda j: j.img.shape[0] * j.img.shape[1])
    ws = cq.Workspace(big.img.shape[0], big.img.shape[1], 256, dev)

    def one(j):
        cq.cq_quantize(j.img, j.palette.shape[0], cq.INIT_KMEANSPP, j.c.seed, MAX_ITERS, TOL, True, ws,
                       palette=j.palette, out_idx=j.idx, out_rgb=j.rgb)

    for j in jobs[:warm]:
        one(j)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in jobs:
        one(j)
    torch.cuda.synchronize()
    return len(jobs) / (time.perf_counter() - t0)


def oracle_sample(host_imgs, shapes, k_of, budget_s, workers):
    """The oracle on images of the batch in order, `workers` at a time (the
    C library releases the GIL, so threads run it side by side), until about
    `budget_s` seconds have passed; returns (results by image, seconds)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor, FIRST_COMPLETED, wait

    res = {}
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=workers) as pool:
        pending = {}
        nxt = 0

        def submit(i):
            h, w, _, seed = shapes[i]
            return pool.submit(oracle.quantize, host_imgs[i], k_of(i), oracle.INIT_KMEANSPP, seed, MAX_ITERS,
                               TOL, True, False)

        while nxt < len(host_imgs) and len(pending) < workers:
            pending[submit(nxt)] = nxt
            nxt += 1
        while pending:
            done, _ = wait(pending, return_when=FIRST_COMPLETED)
            for f in done:
                res[pending.pop(f)] = f.result()[3]
            if nxt < len(host_imgs) and time.perf_counter() - t0 < budget_s:
                pending[submit(nxt)] = nxt
                nxt += 1
    return res, time.perf_counter() - t0


def oracle_stages(host_imgs, shapes, k_of, n=4):
    """Single-threaded oracle time per stage (histogram, init, iterations,
    map) on the first n images of the batch, in ms summed over them."""
    import numpy as np

    import oracle
    out = {"histogram_ms": 0.0, "init_ms": 0.0, "kmeans_ms": 0.0, "map_ms": 0.0, "images": n, "pixels": 0}
    for i in range(n):
        img = host_imgs[i]
        _, _, _, seed = shapes[i]
        t = time.perf_counter()
        keys, counts = oracle.histogram(img)
        t1 = time.perf_counter()
        c0, _ = oracle.init(keys, counts, k_of(i), oracle.INIT_KMEANSPP, seed)
        t2 = time.perf_counter()
        km = oracle.kmeans(keys, counts, c0, MAX_ITERS, TOL, True)
        t3 = time.perf_counter()
        oracle.map_image(img, km.palette)
        t4 = time.perf_counter()
        out["histogram_ms"] += 1e3 * (t1 - t)
        out["init_ms"] += 1e3 * (t2 - t1)
        out["kmeans_ms"] += 1e3 * (t3 - t2)
        out["map_ms"] += 1e3 * (t4 - t3)
        out["pixels"] += int(np.prod(img.shape[:2]))
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--images", type=int, default=C4_IMAGES,
                    help="images of the mixed batch (the workload is defined at 512)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-call-per-image timings")
    ap.add_argument("--no-drawn-k", action="store_true", help="skip the mixed batch with each image's own K")
    ap.add_argument("--no-8x512", action="store_true", help="skip the eight 512x512 stand-ins")
    ap.add_argument("--no-large", action="store_true", help="skip the 4096x4096 histogram/map bandwidth figures")
    ap.add_argument("--no-serving", action="store_true", help="skip the continuous-batching latency figures")
    ap.add_argument("--no-init-schemes", action="store_true", help="skip the per-initialization figures")
    ap.add_argument("--no-subsample", action="store_true", help="skip the 2:1 subsampling figures")
    ap.add_argument("--no-km-vs-wsm", action="store_true", help="skip the KM against WSM comparison")
    ap.add_argument("--no-k-sweep", action="store_true", help="skip the WSM time against K = 2..256")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="finish with plain device-to-device copies of this many MiB (a known-size kernel "
                         "for scaling memory counters)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson arrival window of the serving figure")
    ap.add_argument("--gen-threads", action="store_true",
                    help="generate the inputs on threads instead of child processes (for runs under a profiler, "
                         "which would follow every child process)")
    ap.add_argument("--cpu-budget-s", type=float, default=20.0,
                    help="approximate wall seconds for the oracle baseline sample")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(images are independent, see the sharding notes in the design document)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np

    from paper_1101_0395_amd import synth

    workers = worker_count()
    shapes = synth.batch_shapes(args.images)
    t_gen = time.perf_counter()
    host_c4 = synth.batch_images(shapes, workers, threads=args.gen_threads)  # before the GPU is touched
    gen_s = time.perf_counter() - t_gen
    print(f"[bench] {len(host_c4)} images generated in {gen_s:.1f} s by {workers} processes", file=sys.stderr,
          flush=True)

    import torch

    from paper_1101_0395_amd import cq

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cq.lib()
    imgs_c4 = [torch.from_numpy(im).to(dev) for im in host_c4]
    n_pix = sum(int(im.shape[0]) * int(im.shape[1]) for im in host_c4)
    k256 = lambda i: K  # noqa: E731
    kdrawn = lambda i: shapes[i][2]  # noqa: E731

    # ---- headline: the mixed batch with K = 256 for every image
    jobs = make_jobs(cq, imgs_c4, shapes, k256, dev)
    bws = cq.BatchWorkspace(jobs, dev)
    # every TIMER_EVERY-th launch of the roofline kernel is bracketed with HIP
    # events on its stream (bracketing all of them would slow the step itself)
    timer = cq.KernelTimer(ROOFLINE_KERNEL, max_launches=args.steps * (MAX_ITERS + 16), every=TIMER_EVERY)
    elapsed, last, all_stats = time_batched(cq, torch, jobs, bws, args.steps, args.warmup, timer)
    timed, timed_ms = timer.read()
    launches = timer.seen
    timer.disable()
    if timed == 0:
        raise RuntimeError(f"no launch of {ROOFLINE_KERNEL} was timed")
    print(f"[bench] headline: {1e3 * elapsed / args.steps:.1f} ms per step", file=sys.stderr, flush=True)
    avg_launch_ms = timed_ms / timed
    kern_ms = avg_launch_ms * launches  # all launches of the kernel in the timed region
    stats = [s for st in all_stats for s in st]
    n_img = len(stats)
    ndc = sum(s["ndc_total"] for s in stats)
    dense = sum(s["n_unique"] * K * s["iters"] for s in stats)
    # distance evaluations of the sort-means passes: all but the first
    # iteration, which is a full search over the K centres (jobs with N' <= K
    # run no iteration)
    walk_ndc = sum(s["ndc_total"] - s["n_unique"] * K for s in stats if s["iters"] >= 1)
    achieved_tflops = FLOP_PER_EVAL * walk_ndc / (kern_ms * 1e-3) / 1e12 if kern_ms > 0 else 0.0
    # colours the sort-means passes read: every colour of a job in each of its
    # iterations after the first
    walk_colours = sum(s["n_unique"] * (s["iters"] - 1) for s in stats if s["iters"] >= 2)
    walk_bytes_per_launch = WALK_BYTES_PER_COLOUR * walk_colours / max(1, launches)
    achieved_gbs = walk_bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    batched_ips = n_img / elapsed

    plain_ips = None if args.no_plain else time_plain(cq, torch, jobs, dev)
    line = {
        "metric": "images/sec (mixed batch of 512 RGB images, long side 64-2048, K=256, k-means++, "
                  "sort-means, full map)",
        "value": batched_ips,
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "dtype_detail": "f64 distances and centres; u32/u64 integer histogram counts and cluster sums",
        "data": "synthetic (seeded natural-image stand-ins)",
        "config": {"workload": f"{args.images} images uint8 HxWx3, long side log-uniform in [64, 2048], aspect "
                               "U[1, 2], seeds 1,000,000 + i, per step one batched call, K=256 for every "
                               "image, k-means++ init, sort-means pruned, tol 1e-4, max 100 iters, full "
                               "pixel map (index and RGB)",
                   "images_per_step": len(jobs), "K": K, "pixels_per_step": n_pix,
                   "total_unique_colours": int(sum(s["n_unique"] for s in last)),
                   "mean_iters": float(np.mean([s["iters"] for s in last])),
                   "max_iters_run": int(max(s["iters"] for s in last))},
        "plain_images_per_s": plain_ips,
        "batched_vs_plain": batched_ips / plain_ips if plain_ips else None,
        "pixels_per_s": n_pix * args.steps / elapsed,
        "evals_per_s_assign": walk_ndc / (kern_ms * 1e-3) if kern_ms > 0 else None,
        "evals_per_s_wall": ndc / elapsed,
        "dense_equiv_evals_per_s_wall": dense / elapsed,
        "ndc_per_colour_iter": ndc / max(1, sum(s["n_unique"] * s["iters"] for s in stats)),
        "roofline": {
            "kernel": ROOFLINE_KERNEL,
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / PEAK_HBM_GBS,
            "traffic": recorded_traffic(),
            "algorithmic_bytes_per_launch": walk_bytes_per_launch,
            "launches": launches,
            "timed_launches": timed,
            "avg_launch_us": 1e3 * avg_launch_ms,
            # the same launches against the FP64 vector peak (8 FLOP per
            # evaluated distance)
            "fp64_view": {"achieved_tflops": achieved_tflops, "peak_tflops": PEAK_FP64_VALU_TFLOPS,
                          "frac": achieved_tflops / PEAK_FP64_VALU_TFLOPS},
        },
        "input_generation_s": gen_s,
    }
    headline_stats = last
    del bws, jobs
    torch.cuda.empty_cache()

    if not args.no_drawn_k:
        jobs = make_jobs(cq, imgs_c4, shapes, kdrawn, dev)
        bws = cq.BatchWorkspace(jobs, dev)
        sec, st, _ = time_batched(cq, torch, jobs, bws, max(1, min(args.steps, 3)), 1)
        reps = max(1, min(args.steps, 3))
        d = {"workload": "the same mixed batch, each image with its own K drawn from {16, 32, 64, 128, 256}",
             "images_per_s": len(jobs) * reps / sec, "ms_per_step": 1e3 * sec / reps,
             "evals_per_s_wall": sum(s["ndc_total"] for s in st) * reps / sec,
             "total_unique_colours": int(sum(s["n_unique"] for s in st)),
             "mean_iters": float(np.mean([s["iters"] for s in st]))}
        if not args.no_plain:
            p = time_plain(cq, torch, jobs, dev)
            d["plain_images_per_s"] = p
            d["batched_vs_plain"] = d["images_per_s"] / p
        line["mixed_batch_drawn_k"] = d
        del bws, jobs
        torch.cuda.empty_cache()

    host_imgs = [synth.smooth_field_blobs(H, W, s) for s in SEEDS]
    imgs = [torch.from_numpy(im).to(dev) for im in host_imgs]
    if not args.no_8x512:
        jobs = [cq.BatchJob(img, K, cq.INIT_KMEANSPP, SEEDS[i], MAX_ITERS, TOL, True) for i, img in enumerate(imgs)]
        bws = cq.BatchWorkspace(jobs, dev)
        sec, st, _ = time_batched(cq, torch, jobs, bws, 20, 3)
        d = {"workload": "8 images 512x512x3 (seeds 1-8), one batched call per step, K=256, k-means++, "
                         "sort-means, tol 1e-4, max 100 iters, full map",
             "images_per_s": len(jobs) * 20 / sec, "ms_per_step": 1e3 * sec / 20,
             "mean_unique_colours": float(np.mean([s["n_unique"] for s in st])),
             "mean_iters": float(np.mean([s["iters"] for s in st]))}
        if not args.no_plain:
            p = time_plain(cq, torch, jobs, dev)
            d["plain_images_per_s"] = p
            d["batched_vs_plain"] = d["images_per_s"] / p
        line["batch_8x512"] = d

    if not args.no_large:
        line["hbm_bound_steps_4096"] = measure_large(cq, synth, torch, dev)
    if not args.no_serving:
        line["serving"] = measure_serving(cq, torch, synth, imgs, dev, host_c4, workers, args.serve_seconds)
    if not args.no_init_schemes:
        line["init_schemes_8x512"] = measure_init_schemes(cq, torch, imgs, dev)
    if not args.no_subsample:
        line["subsample_8x512"] = measure_subsample(cq, torch, imgs, dev)
    if not args.no_km_vs_wsm:
        line["km_vs_wsm_8x512"] = measure_km_vs_wsm(cq, torch, imgs, dev)
    if not args.no_k_sweep:
        line["wsm_time_vs_k_8x512"] = measure_k_sweep(cq, torch, imgs, dev)

    if not args.no_cpu_baseline:
        res, cpu_s = oracle_sample(host_c4, shapes, k256, args.cpu_budget_s, workers)
        mse_err = []
        for i, rs in res.items():
            g = headline_stats[i]
            mse_err.append(abs(g["mse_img"] - rs["mse_img"]) / rs["mse_img"] if rs["mse_img"] else
                           abs(g["mse_img"]))
        model, ncpu = cpu_info()
        sample_px = sum(int(host_c4[i].shape[0]) * int(host_c4[i].shape[1]) for i in res)
        line["cpu_baseline"] = {
            "value": len(res) / cpu_s,
            "unit": "images/s",
            "cores": workers,
            "kind": "oracle",
            "sample": f"the first {len(res)} images of the mixed batch (K=256, same settings, {sample_px} pixels), "
                      f"the single-threaded C oracle run on {workers} threads at once, one image each",
            "cpu_model": model,
            "host_cpus": ncpu,
            "pixels_per_s": sample_px / cpu_s,
            "stages_1_core": oracle_stages(host_c4, shapes, k256),
        }
        line["mse_rel_err_max"] = max(mse_err)
        line["mse_rel_err_mean"] = float(np.mean(mse_err))
        line["mse_rel_err_images"] = len(mse_err)
    print(json.dumps(line), flush=True)

    if args.calibration_copy_mib > 0:
        src = torch.ones(args.calibration_copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
