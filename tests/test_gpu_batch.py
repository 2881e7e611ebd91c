"""GPU parity of the batch entry point: every job of a mixed batch (sizes,
palette sizes, schemes, pruning, stopping settings) equals the CPU oracle and
the same image quantized alone, bit for bit."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1101_0395_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def cqm(dev):
    from paper_1101_0395_amd import cq
    cq.lib()
    return cq


MIXED = [
    # (H, W, K, scheme, seed, prune, max_iters, tol)
    (64, 64, 16, oracle.INIT_MAXMIN, 0, False, 50, 1e-4),
    (1, 1, 4, oracle.INIT_KMEANSPP, 1, True, 20, 1e-4),
    (7, 13, 2, oracle.INIT_FORGY, 2, True, 30, 0.0),
    (300, 200, 256, oracle.INIT_KMEANSPP, 3, True, 100, 1e-4),
    (128, 96, 37, oracle.INIT_FORGY, 4, False, 40, 1e-3),
    (512, 512, 64, oracle.INIT_KMEANSPP, 5, True, 100, 1e-4),
    (33, 65, 1, oracle.INIT_MAXMIN, 6, True, 10, 1e-4),
    (200, 301, 128, oracle.INIT_MAXMIN, 7, True, 5, 1e-4),
    (5, 3, 8, oracle.INIT_KMEANSPP, 8, True, 20, 1e-4),
    (257, 129, 256, oracle.INIT_KMEANSPP, 9, False, 15, 1e-4),
    (240, 180, 64, oracle.INIT_VAR, 10, True, 100, 1e-4),
    (150, 90, 32, oracle.INIT_SFF, 11, True, 100, 1e-4),
    (6, 6, 16, oracle.INIT_VAR, 12, True, 10, 1e-4),  # N' <= K
]


def _image(H, W, seed):
    if H * W < 64:
        return np.array(np.random.default_rng(seed).integers(0, 3, (H, W, 3)) * 80, np.uint8)
    return synth.smooth_field_blobs(H, W, seed) if H * W > 20000 else synth.blobs_on_gradient(H, W, seed)


def test_mixed_batch_matches_oracle_and_solo(cqm, dev):
    _say("batch of %d mixed jobs" % len(MIXED))
    imgs = [_image(H, W, seed) for (H, W, _, _, seed, _, _, _) in MIXED]
    jobs = [cqm.BatchJob(torch.from_numpy(im).to(dev), K, scheme, seed, mi, tol, prune)
            for im, (H, W, K, scheme, seed, prune, mi, tol) in zip(imgs, MIXED)]
    ws = cqm.BatchWorkspace(jobs, dev)
    stats = cqm.cq_quantize_batch(jobs, ws)
    solo_ws = cqm.Workspace(512, 512, 256, dev)
    for job, im, st, (H, W, K, scheme, seed, prune, mi, tol) in zip(jobs, imgs, stats, MIXED):
        _say(f"  job {H}x{W} K={K} scheme={scheme} prune={prune}")
        rp, ri, rr, rs = oracle.quantize(im, K, scheme, seed, mi, tol, prune=prune)
        assert np.array_equal(job.palette.cpu().numpy(), rp)
        assert np.array_equal(job.idx.cpu().numpy(), ri)
        assert np.array_equal(job.rgb.cpu().numpy(), rr)
        for key in ("iters", "converged", "k_used", "n_unique", "ndc_total", "near_ties", "sse_final",
                    "mse_float", "mse_img"):
            assert st[key] == rs[key], key
        sp, si, sr, ss = cqm.cq_quantize(job.img, K, scheme, seed, mi, tol, prune, solo_ws)
        assert torch.equal(sp, job.palette) and torch.equal(sr, job.rgb) and ss == st


def test_largest_batch_matches_oracle(cqm, dev):
    """The largest batch accepted, 4096 jobs, in one call: small images of
    ragged sizes (1 x 1 to 24 x 24, few distinct channel values, so N' is
    often at most K), K from 1 to 64, every initialization scheme, pruned and
    unpruned, some subsampled, different stopping settings; every job bit for
    bit against the oracle."""
    n_jobs = 4096
    _say(f"largest batch: {n_jobs} jobs")
    schemes = (oracle.INIT_FORGY, oracle.INIT_MAXMIN, oracle.INIT_KMEANSPP, oracle.INIT_VAR, oracle.INIT_SFF,
               oracle.INIT_WU, oracle.INIT_LBG, oracle.INIT_DEN)
    rng = np.random.default_rng(2024)
    specs, imgs = [], []
    for i in range(n_jobs):
        H, W = int(rng.integers(1, 25)), int(rng.integers(1, 25))
        K = int(rng.integers(1, 65))
        specs.append((K, schemes[i % len(schemes)], 100 + i, bool(i % 2), (1, 5, 20)[i % 3],
                      (1e-4, 0.0)[i % 4 == 3], i % 5 == 4))
        imgs.append(np.array(rng.integers(0, 6, (H, W, 3)) * 51, np.uint8))
    jobs = [cqm.BatchJob(torch.from_numpy(im).to(dev), K, sc, seed, mi, tol, prune, subsample=sub)
            for im, (K, sc, seed, prune, mi, tol, sub) in zip(imgs, specs)]
    ws = cqm.BatchWorkspace(jobs, dev)
    stats = cqm.cq_quantize_batch(jobs, ws)

    # the oracle's C calls release the interpreter lock and share no state,
    # so a thread pool runs them side by side (each call clears its own
    # 2^24-entry tables, about 35 ms)
    def reference(a):
        im, (K, sc, seed, prune, mi, tol, sub) = a
        return oracle.quantize(im, K, sc, seed, mi, tol, prune=prune, subsample=sub)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as pool:
        refs = list(pool.map(reference, zip(imgs, specs)))
    for i, (job, im, st, (K, sc, seed, prune, mi, tol, sub), ref) in enumerate(
            zip(jobs, imgs, stats, specs, refs)):
        rp, ri, rr, rs = ref
        what = f"job {i}: {im.shape[0]}x{im.shape[1]} K={K} scheme={sc} prune={prune} subsample={sub}"
        assert np.array_equal(job.palette.cpu().numpy(), rp), what
        assert np.array_equal(job.idx.cpu().numpy(), ri), what
        assert np.array_equal(job.rgb.cpu().numpy(), rr), what
        for key in ("iters", "converged", "k_used", "n_unique", "ndc_total", "near_ties", "sse_final",
                    "mse_float", "mse_img"):
            assert st[key] == rs[key], (what, key)


def test_batch_rerun_is_deterministic(cqm, dev):
    _say("batch rerun")
    imgs = [synth.smooth_field_blobs(256, 256, s) for s in range(3)]
    jobs = [cqm.BatchJob(torch.from_numpy(im).to(dev), 256, oracle.INIT_KMEANSPP, s, 100, 1e-4)
            for s, im in enumerate(imgs)]
    ws = cqm.BatchWorkspace(jobs, dev)
    a = cqm.cq_quantize_batch(jobs, ws)
    pals = [j.palette.clone() for j in jobs]
    b = cqm.cq_quantize_batch(jobs, ws)
    assert a == b
    assert all(torch.equal(p, j.palette) for p, j in zip(pals, jobs))


def test_batch_rejects_bad_job(cqm, dev):
    _say("batch argument check")
    img = torch.zeros((4, 4, 3), dtype=torch.uint8, device=dev)
    good = cqm.BatchJob(img, 4, oracle.INIT_KMEANSPP, 0, 10, 1e-4)
    bad = cqm.BatchJob(img, 4, oracle.INIT_KMEANSPP, 0, 10, 1e-4)
    bad.c.K = 0
    ws = cqm.BatchWorkspace([good, good], dev)
    with pytest.raises(cqm.CqError) as e:
        cqm.cq_quantize_batch([good, bad], ws)
    assert e.value.code == cqm.CQ_EINVAL and "job 1" in str(e.value)


def test_benchmark_batch_matches_oracle(cqm, dev):
    """The batch the benchmark times (eight 512 x 512 stand-ins, seeds 1-8,
    K = 256, k-means++, sort-means, tol 1e-4, at most 100 iterations, full map),
    in one batched call as the benchmark makes it: every image bit for bit
    against the oracle."""
    import bench

    _say("benchmark batch: 8 x 512x512, K=256")
    host = [synth.smooth_field_blobs(bench.H, bench.W, s) for s in bench.SEEDS]
    jobs = [cqm.BatchJob(torch.from_numpy(im).to(dev), bench.K, cqm.INIT_KMEANSPP, s, bench.MAX_ITERS, bench.TOL,
                         True) for im, s in zip(host, bench.SEEDS)]
    stats = cqm.cq_quantize_batch(jobs, cqm.BatchWorkspace(jobs, dev))
    for im, s, job, st in zip(host, bench.SEEDS, jobs, stats):
        rp, ri, rr, rs = oracle.quantize(im, bench.K, oracle.INIT_KMEANSPP, s, bench.MAX_ITERS, bench.TOL, prune=True)
        assert np.array_equal(job.palette.cpu().numpy(), rp), s
        assert np.array_equal(job.idx.cpu().numpy(), ri) and np.array_equal(job.rgb.cpu().numpy(), rr), s
        for key in ("iters", "converged", "k_used", "n_unique", "ndc_total", "near_ties", "sse_final", "mse_float",
                    "mse_img"):
            assert st[key] == rs[key], (s, key)


def test_init_launch_shares_cus_between_teams_and_single_blocks(cqm, dev):
    """k-means++ and max-min jobs of more than 32768 colours (teams of
    several blocks) and of fewer (one block each) in one batch: the launch
    plan puts the single-block jobs into the CUs the teams leave, so they run
    in the teams' launch.  Every job equals the oracle bit for bit."""
    _say("init launch of teams and single-block jobs")
    specs = [(300, 260, 64, oracle.INIT_KMEANSPP, 21), (280, 300, 64, oracle.INIT_MAXMIN, 22),
             (320, 320, 256, oracle.INIT_KMEANSPP, 23)]
    specs += [(40 + 7 * i, 50 + 5 * i, 16 if i % 2 else 64,
               oracle.INIT_MAXMIN if i % 3 == 0 else oracle.INIT_KMEANSPP, 30 + i) for i in range(20)]
    imgs = [_image(H, W, seed) for H, W, _, _, seed in specs]
    jobs = [cqm.BatchJob(torch.from_numpy(im).to(dev), K, scheme, seed, 3, 1e-4, True)
            for im, (H, W, K, scheme, seed) in zip(imgs, specs)]
    ws = cqm.BatchWorkspace(jobs, dev)
    stats = cqm.cq_quantize_batch(jobs, ws)
    sizes = []
    for job, im, st, (H, W, K, scheme, seed) in zip(jobs, imgs, stats, specs):
        rp, ri, rr, rs = oracle.quantize(im, K, scheme, seed, 3, 1e-4, prune=True)
        sizes.append(rs["n_unique"])
        assert np.array_equal(job.palette.cpu().numpy(), rp), (H, W)
        assert np.array_equal(job.idx.cpu().numpy(), ri), (H, W)
        for key in ("iters", "k_used", "n_unique", "ndc_total", "near_ties", "sse_final"):
            assert st[key] == rs[key], (H, W, key)
    assert all(n > 32768 for n in sizes[:3]) and all(n <= 32768 for n in sizes[3:]), sizes
