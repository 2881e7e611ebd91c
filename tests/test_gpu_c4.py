"""GPU parity at the real shapes of the mixed batch (long side log-uniform in
64-2048, aspect 1-2, seeds 1,000,000 + i, K drawn from {16, ..., 256}) and of
the converged 4096 x 4096 run: every image of one batched call, and its solo
run, equal to the CPU oracle bit for bit (palette, index and RGB images,
iterations, distance and near-tie counts, SSE and both MSEs)."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1101_0395_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STAT_KEYS = ("iters", "converged", "k_used", "n_unique", "ndc_total", "near_ties", "sse_final", "mse_float",
             "mse_img")


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


def _subset():
    """Indices into the 512-image batch: the four largest images (long side
    1900-2048) and eight more drawn by a seeded generator among the rest, so
    that small, middle and large sizes and every K appear."""
    shapes = synth.batch_shapes(512)
    order = sorted(range(512), key=lambda i: -shapes[i][0] * shapes[i][1])
    big = order[:4]
    rest = [i for i in range(512) if i not in big]
    pick = sorted(np.random.default_rng(5).choice(rest, 8, replace=False).tolist())
    return [(i,) + shapes[i] for i in sorted(big + pick)]


@pytest.fixture(scope="module")
def subset():
    sub = _subset()
    imgs = synth.batch_images([(H, W, K, seed) for _, H, W, K, seed in sub], min(16, os.cpu_count() or 1))
    return sub, imgs


def _run_and_compare(cqm, dev, sub, imgs, k_of):
    jobs = [cqm.BatchJob(torch.from_numpy(im).to(dev), k_of(K), cqm.INIT_KMEANSPP, seed, 100, 1e-4, True)
            for im, (_, H, W, K, seed) in zip(imgs, sub)]
    _say("  batched call of %d images, %d pixels" % (len(jobs), sum(im.shape[0] * im.shape[1] for im in imgs)))
    stats = cqm.cq_quantize_batch(jobs, cqm.BatchWorkspace(jobs, dev))

    def reference(a):
        im, (_, H, W, K, seed) = a
        return oracle.quantize(im, k_of(K), oracle.INIT_KMEANSPP, seed, 100, 1e-4, prune=True)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as pool:
        refs = list(pool.map(reference, zip(imgs, sub)))
    big = max(sub, key=lambda s: s[1] * s[2])
    solo_ws = cqm.Workspace(big[1], big[2], 256, dev)
    for job, im, st, (i, H, W, K, seed), (rp, ri, rr, rs) in zip(jobs, imgs, stats, sub, refs):
        what = f"image {i}: {H}x{W} K={k_of(K)} N'={rs['n_unique']} iters={rs['iters']}"
        _say("  " + what)
        assert np.array_equal(job.palette.cpu().numpy(), rp), what
        assert np.array_equal(job.idx.cpu().numpy(), ri), what
        assert np.array_equal(job.rgb.cpu().numpy(), rr), what
        for key in STAT_KEYS:
            assert st[key] == rs[key], (what, key)
        sp, si, sr, ss = cqm.cq_quantize(job.img, k_of(K), cqm.INIT_KMEANSPP, seed, 100, 1e-4, True, solo_ws)
        assert torch.equal(sp, job.palette) and torch.equal(si, job.idx) and torch.equal(sr, job.rgb), what
        assert ss == st, what


def test_mixed_batch_subset_drawn_k(cqm, dev, subset):
    """Twelve images of the mixed batch with their own K, one batched call."""
    _say("mixed batch subset, drawn K")
    sub, imgs = subset
    assert max(max(H, W) for _, H, W, _, _ in sub) >= 1900
    assert {K for _, _, _, K, _ in sub} == {16, 32, 64, 128, 256}
    _run_and_compare(cqm, dev, sub, imgs, lambda K: K)


def test_mixed_batch_subset_k256(cqm, dev, subset):
    """The same twelve images with K = 256 for every image (the setting of
    the batched against one-call-per-image comparison)."""
    _say("mixed batch subset, K = 256")
    sub, imgs = subset
    _run_and_compare(cqm, dev, sub, imgs, lambda K: 256)


def test_converged_4096(cqm, dev):
    """The 4096 x 4096 stand-in (seed 42) quantized end to end, K = 256,
    k-means++, sort-means, tol 1e-4, at most 100 iterations, until the
    stopping rule fires: palette, index and RGB images and every statistic
    equal to the oracle's."""
    _say("converged 4096x4096, K=256")
    img = synth.smooth_field_blobs(4096, 4096, 42)
    ws = cqm.Workspace(4096, 4096, 256, dev)
    pal, gi, gr, st = cqm.cq_quantize(torch.from_numpy(img).to(dev), 256, cqm.INIT_KMEANSPP, 42, 100, 1e-4, True,
                                      ws)
    rp, ri, rr, rs = oracle.quantize(img, 256, oracle.INIT_KMEANSPP, 42, 100, 1e-4, prune=True)
    _say(f"  N'={rs['n_unique']} iters={rs['iters']} converged={rs['converged']} mse={rs['mse_img']}")
    assert rs["converged"] == 1 and rs["iters"] < 100
    assert np.array_equal(pal.cpu().numpy(), rp)
    assert np.array_equal(gi.cpu().numpy(), ri)
    assert np.array_equal(gr.cpu().numpy(), rr)
    for key in STAT_KEYS:
        assert st[key] == rs[key], key
