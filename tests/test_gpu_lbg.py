"""GPU parity of the LBG initialization (Section 2.3: the centroid, then
doubling stages c -/+ eps, each refined by k-means with the paper's threshold
of Section 3.3): initial centres bit-exact against the oracle for powers of
two and other K, a lone colour whose empty half keeps c + eps, and whole
quantizations with LBG through the single-image, batch and engine entry
points (jobs doubling at different stages share launches)."""
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
    return cqm.Workspace(512, 512, 256, dev)


def _dev_u32(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(dev)


@pytest.mark.parametrize("K", [1, 2, 3, 6, 7, 33, 128])
def test_lbg_init_parity(cqm, dev, ws, K):
    _say(f"LBG init K={K}")
    img = synth.smooth_field_blobs(160, 200, K + 5)
    keys, counts = oracle.histogram(img)
    ref, ref_used = oracle.init(keys, counts, K, oracle.INIT_LBG, 0)
    got, used = cqm.cq_init(_dev_u32(keys, dev), _dev_u32(counts, dev), K, oracle.INIT_LBG, 0, ws)
    assert used == ref_used
    assert np.array_equal(got.cpu().numpy(), ref)


def test_lbg_lone_colour_keeps_the_perturbed_centre(cqm, dev, ws):
    _say("LBG init: lone colour")
    group = [(40 + i, 60 + j, 50) for i in range(4) for j in range(4)]
    ks = np.array(sorted((r << 16) | (g << 8) | b for r, g, b in group + [(230, 230, 230)]), np.uint32)
    cs = np.ones(len(ks), np.uint32)
    ref, _ = oracle.init(ks, cs, 4, oracle.INIT_LBG, 0)
    got, _ = cqm.cq_init(_dev_u32(ks, dev), _dev_u32(cs, dev), 4, oracle.INIT_LBG, 0, ws)
    assert np.array_equal(got.cpu().numpy(), ref)
    assert [231.0, 231.0, 231.0] in ref.tolist()


@pytest.mark.parametrize("spec", [(256, 256, 256, 1, True), (150, 210, 48, 2, False), (5, 3, 16, 3, True)])
def test_lbg_quantize_parity(cqm, dev, ws, spec):
    H, W, K, seed, prune = spec
    _say(f"LBG quantize {H}x{W} K={K} prune={prune}")
    if H * W < 64:
        img = np.array(np.random.default_rng(seed).integers(0, 3, (H, W, 3)) * 80, np.uint8)
    else:
        img = synth.smooth_field_blobs(H, W, seed)
    pal, idx, rgb, st = cqm.cq_quantize(torch.from_numpy(img).to(dev), K, oracle.INIT_LBG, seed, 100, 1e-4, prune,
                                        ws)
    rp, ri, rr, rs = oracle.quantize(img, K, oracle.INIT_LBG, seed, 100, 1e-4, prune=prune)
    assert np.array_equal(pal.cpu().numpy(), rp) and np.array_equal(idx.cpu().numpy(), ri)
    assert np.array_equal(rgb.cpu().numpy(), rr)
    for key in STAT_KEYS:
        assert st[key] == rs[key], key


def test_lbg_in_batch_and_engine(cqm, dev):
    specs = [(200, 160, 64, oracle.INIT_LBG), (120, 90, 5, oracle.INIT_LBG), (150, 100, 32, oracle.INIT_KMEANSPP),
             (90, 90, 20, oracle.INIT_LBG), (4, 4, 16, oracle.INIT_LBG)]
    imgs = [synth.smooth_field_blobs(H, W, 60 + i) if H * W > 64 else
            np.array(np.random.default_rng(i).integers(0, 3, (H, W, 3)) * 80, np.uint8)
            for i, (H, W, _, _) in enumerate(specs)]

    def jobs():
        return [cqm.BatchJob(torch.from_numpy(im).to(dev), K, sc, 7, 100, 1e-4, True)
                for im, (H, W, K, sc) in zip(imgs, specs)]

    def check(job, st, i):
        H, W, K, sc = specs[i]
        rp, ri, rr, rs = oracle.quantize(imgs[i], K, sc, 7, 100, 1e-4, prune=True)
        assert np.array_equal(job.palette.cpu().numpy(), rp) and np.array_equal(job.idx.cpu().numpy(), ri)
        for key in STAT_KEYS:
            assert st[key] == rs[key], key

    _say("LBG in a batch")
    bj = jobs()
    for i, (job, st) in enumerate(zip(bj, cqm.cq_quantize_batch(bj, cqm.BatchWorkspace(bj, dev)))):
        check(job, st, i)
    _say("LBG through the engine")
    ej = jobs()
    eng = cqm.Engine(max_jobs=3, pool_bytes=3 * cqm.engine_job_bytes(200, 160), device=dev)
    tickets = {}
    for i, j in enumerate(ej):
        tickets[eng.submit(j)] = i
    done = {}
    while len(done) < len(ej):
        for t, _, st in eng.step(6):
            done[t] = st
    for t, i in tickets.items():
        assert done[t]["status"] == cqm.CQ_OK
        check(ej[i], done[t], i)
    eng.close()
