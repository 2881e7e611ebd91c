"""Launch schedules (cq_schedule) change no result: one mixed batch run under
the built-in table, under extreme single-entry tables (the smallest and the
largest assignment blocks, regrouping every iteration and almost never) and
under a table whose entry switches inside the batch's size range gives the
same palettes, index and RGB images and statistics, all equal to the oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_1101_0395_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SCHEDULES = [
    [],                                      # the built-in table
    [(0, 256, 1)],
    [(0, 32768, 1)],
    [(0, 1024, 1000)],
    [(0, 8192, 3)],
    [(0, 512, 2), (100_000, 2048, 5)],
]


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


def test_schedules_give_identical_results(cqm, dev):
    shapes = [(h, w, k, s) for h, w, k, s in synth.batch_shapes(40) if h * w <= 400_000][:10]
    imgs = [synth.batch_image(h, w, s) for h, w, _, s in shapes]
    jobs = [cqm.BatchJob(torch.from_numpy(im).to(dev), K, cqm.INIT_KMEANSPP, seed, 100, 1e-4, bool(i % 4))
            for i, (im, (_, _, K, seed)) in enumerate(zip(imgs, shapes))]
    ws = cqm.BatchWorkspace(jobs, dev)
    ref = None
    try:
        for table in SCHEDULES:
            _say(f"schedule {table or 'built-in'}")
            cqm.set_schedule(table)
            stats = cqm.cq_quantize_batch(jobs, ws)
            outs = [(j.palette.cpu().numpy(), j.idx.cpu().numpy(), j.rgb.cpu().numpy()) for j in jobs]
            if ref is None:
                ref = (stats, outs)
                for i, (im, (_, _, K, seed), st, (p, x, r)) in enumerate(zip(imgs, shapes, stats, outs)):
                    rp, ri, rr, rs = oracle.quantize(im, K, oracle.INIT_KMEANSPP, seed, 100, 1e-4, prune=bool(i % 4))
                    assert np.array_equal(p, rp) and np.array_equal(x, ri) and np.array_equal(r, rr), i
                    for key in ("iters", "ndc_total", "near_ties", "sse_final", "mse_img"):
                        assert st[key] == rs[key], (i, key)
            else:
                assert stats == ref[0]
                for (p, x, r), (q, y, s) in zip(outs, ref[1]):
                    assert np.array_equal(p, q) and np.array_equal(x, y) and np.array_equal(r, s)
    finally:
        cqm.set_schedule([])
