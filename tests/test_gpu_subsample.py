"""GPU parity of the optional 2:1 subsampling of Section 2.2 (item 1): the
histogram then counts only the pixels at even row and even column, the
clustering runs on those colours, and the pixel map and its MSE still cover
every pixel.  Every result equals the CPU oracle bit for bit, through the
single-image, batch and serving entry points."""
import sys

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


@pytest.fixture(scope="module")
def ws(cqm, dev):
    return cqm.Workspace(1024, 1024, 256, dev)


def _to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _image(H, W, seed):
    if H * W < 64:
        return np.array(np.random.default_rng(seed).integers(0, 3, (H, W, 3)) * 80, np.uint8)
    return synth.smooth_field_blobs(H, W, seed) if H * W > 20000 else synth.blobs_on_gradient(H, W, seed)


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (2, 2), (3, 5), (7, 13), (33, 65), (64, 64), (127, 129),
                                   (512, 512), (1024, 1023)])
def test_subsampled_histogram_parity(cqm, dev, ws, shape):
    H, W = shape
    _say(f"subsampled histogram {H}x{W}")
    img = synth.smooth_field_blobs(H, W, H * 1000 + W + 7)
    keys, counts = cqm.cq_histogram(_to_dev(img, dev), ws, subsample=True)
    rk, rc = oracle.histogram(img, subsample=True)
    assert np.array_equal(_u32(keys), rk) and np.array_equal(_u32(counts), rc)
    assert int(rc.sum()) == ((H + 1) // 2) * ((W + 1) // 2)


def test_subsampled_histogram_strided_and_odd_pixels_ignored(cqm, dev, ws):
    _say("subsampled histogram, strided rows, colours only at odd positions")
    rng = np.random.default_rng(5)
    H, W = 45, 39
    base = np.zeros((H, W, 3), np.uint8)
    base[0::2, 0::2] = rng.integers(0, 4, ((H + 1) // 2, (W + 1) // 2, 3)) * 60
    base[1::2, :] = rng.integers(0, 256, (H // 2, W, 3))   # odd rows: never counted
    base[0::2, 1::2] = rng.integers(0, 256, ((H + 1) // 2, W // 2, 3))  # odd columns: never counted
    padded = torch.zeros((H, W * 3 + 9), dtype=torch.uint8, device=dev)
    padded[:, : W * 3] = _to_dev(base.reshape(H, W * 3), dev)
    view = padded.as_strided((H, W, 3), (W * 3 + 9, 3, 1))
    keys, counts = cqm.cq_histogram(view, ws, subsample=True)
    rk, rc = oracle.histogram(base, subsample=True)
    assert np.array_equal(_u32(keys), rk) and np.array_equal(_u32(counts), rc)
    assert len(rk) <= 64
    # the same view without subsampling still counts every pixel
    keys, counts = cqm.cq_histogram(view, ws)
    rk, rc = oracle.histogram(base)
    assert np.array_equal(_u32(keys), rk) and np.array_equal(_u32(counts), rc)


QUANT = [
    # (H, W, K, scheme, seed, prune, max_iters, tol)
    (512, 512, 256, oracle.INIT_KMEANSPP, 1, True, 100, 1e-4),
    (301, 199, 64, oracle.INIT_MAXMIN, 2, False, 60, 1e-4),
    (255, 257, 32, oracle.INIT_FORGY, 3, True, 100, 0.0),
    (200, 120, 48, oracle.INIT_VAR, 4, True, 100, 1e-4),
    (160, 240, 64, oracle.INIT_SFF, 5, True, 100, 1e-4),
    (5, 3, 16, oracle.INIT_KMEANSPP, 6, True, 20, 1e-4),  # 6 pixels counted, N' <= K
    (1, 1, 4, oracle.INIT_MAXMIN, 7, True, 20, 1e-4),
]


@pytest.mark.parametrize("spec", QUANT)
def test_subsampled_quantize_parity(cqm, dev, ws, spec):
    H, W, K, scheme, seed, prune, mi, tol = spec
    _say(f"subsampled quantize {H}x{W} K={K} scheme={scheme} prune={prune}")
    img = _image(H, W, seed)
    pal, idx, rgb, st = cqm.cq_quantize(_to_dev(img, dev), K, scheme, seed, mi, tol, prune, ws, subsample=True)
    rp, ri, rr, rs = oracle.quantize(img, K, scheme, seed, mi, tol, prune=prune, subsample=True)
    assert np.array_equal(pal.cpu().numpy(), rp)
    assert np.array_equal(idx.cpu().numpy(), ri)
    assert np.array_equal(rgb.cpu().numpy(), rr)
    for key in STAT_KEYS:
        assert st[key] == rs[key], key


def test_subsampled_quantize_1024_strided(cqm, dev, ws):
    _say("subsampled quantize 1024x1000 strided")
    H, W = 1024, 1000
    img = synth.smooth_field_blobs(H, W, 77)
    padded = torch.zeros((H, W * 3 + 32), dtype=torch.uint8, device=dev)
    padded[:, : W * 3] = _to_dev(img.reshape(H, W * 3), dev)
    view = padded.as_strided((H, W, 3), (W * 3 + 32, 3, 1))
    pal, idx, rgb, st = cqm.cq_quantize(view, 256, oracle.INIT_KMEANSPP, 9, 100, 1e-4, True, ws, subsample=True)
    rp, ri, rr, rs = oracle.quantize(img, 256, oracle.INIT_KMEANSPP, 9, 100, 1e-4, prune=True, subsample=True)
    assert np.array_equal(pal.cpu().numpy(), rp) and np.array_equal(idx.cpu().numpy(), ri)
    assert np.array_equal(rgb.cpu().numpy(), rr)
    for key in STAT_KEYS:
        assert st[key] == rs[key], key


def test_batch_and_engine_mix_subsampled_and_full_jobs(cqm, dev):
    """The same images with and without subsampling in one batch and through
    the serving engine: every job equals the oracle with its own setting."""
    specs = [(256, 256, 128, oracle.INIT_KMEANSPP, 21, True), (97, 131, 32, oracle.INIT_MAXMIN, 22, False),
             (3, 5, 8, oracle.INIT_FORGY, 23, True), (300, 200, 64, oracle.INIT_SFF, 24, True)]
    imgs = [_image(H, W, s) for (H, W, _, _, s, _) in specs]
    cases = [(i, sub) for i in range(len(specs)) for sub in (True, False)]

    def make_jobs():
        return [cqm.BatchJob(_to_dev(imgs[i], dev), specs[i][2], specs[i][3], specs[i][4], 100, 1e-4, specs[i][5],
                             subsample=sub) for i, sub in cases]

    def check(job, st, i, sub):
        H, W, K, scheme, seed, prune = specs[i]
        rp, ri, rr, rs = oracle.quantize(imgs[i], K, scheme, seed, 100, 1e-4, prune=prune, subsample=sub)
        assert np.array_equal(job.palette.cpu().numpy(), rp)
        assert np.array_equal(job.idx.cpu().numpy(), ri) and np.array_equal(job.rgb.cpu().numpy(), rr)
        for key in STAT_KEYS:
            assert st[key] == rs[key], key

    _say("batch: %d jobs, subsampled and full" % len(cases))
    jobs = make_jobs()
    stats = cqm.cq_quantize_batch(jobs, cqm.BatchWorkspace(jobs, dev))
    for job, st, (i, sub) in zip(jobs, stats, cases):
        check(job, st, i, sub)

    _say("engine: %d jobs, subsampled and full" % len(cases))
    jobs = make_jobs()
    eng = cqm.Engine(max_jobs=3, pool_bytes=3 * cqm.engine_job_bytes(300, 200), device=dev)
    tickets, done = {}, {}
    for k, job in enumerate(jobs[:5]):
        tickets[eng.submit(job)] = k
    for k, job in enumerate(jobs[5:], start=5):
        for t, _, st in eng.step(3):
            done[t] = st
        tickets[eng.submit(job)] = k
    while len(done) < len(jobs):
        for t, _, st in eng.step(8):
            done[t] = st
    for t, k in tickets.items():
        assert done[t]["status"] == cqm.CQ_OK
        check(jobs[k], done[t], *cases[k])
    eng.close()
