"""GPU parity of the serving engine (continuous batching): jobs submitted in
waves join and leave the set in flight between steps, at different iteration
counts, through a pool too small to hold them all; every job's outputs and
statistics equal the CPU oracle and the same image quantized alone, bit for
bit."""
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


STREAM = [
    # (H, W, K, scheme, seed, prune, max_iters, tol)
    (256, 256, 256, oracle.INIT_KMEANSPP, 11, True, 100, 1e-4),
    (64, 64, 16, oracle.INIT_MAXMIN, 12, False, 50, 1e-4),
    (300, 200, 64, oracle.INIT_FORGY, 13, True, 100, 1e-4),
    (5, 3, 16, oracle.INIT_KMEANSPP, 14, True, 20, 1e-4),       # N' <= 15 < K: no iteration
    (512, 512, 256, oracle.INIT_KMEANSPP, 15, True, 100, 1e-4),
    (128, 96, 37, oracle.INIT_FORGY, 16, False, 40, 1e-3),
    (200, 301, 128, oracle.INIT_MAXMIN, 17, True, 5, 1e-4),     # stops at max_iters
    (33, 65, 1, oracle.INIT_MAXMIN, 18, True, 10, 1e-4),
    (257, 129, 256, oracle.INIT_KMEANSPP, 19, True, 100, 0.0),  # runs until SSE stops falling
    (96, 160, 200, oracle.INIT_KMEANSPP, 20, True, 100, 1e-4),
    (400, 300, 32, oracle.INIT_KMEANSPP, 21, True, 100, 1e-4),
    (7, 13, 2, oracle.INIT_FORGY, 22, True, 30, 0.0),
]
# (jobs submitted before the step, iterations in the step)
SCHEDULE = [(4, 3), (0, 1), (3, 2), (0, 8), (5, 3), (0, 1)]


def _image(H, W, seed):
    if H * W < 64:
        return np.array(np.random.default_rng(seed).integers(0, 3, (H, W, 3)) * 80, np.uint8)
    return synth.smooth_field_blobs(H, W, seed) if H * W > 20000 else synth.blobs_on_gradient(H, W, seed)


def _run_stream(cqm, dev, eng, spec):
    imgs = [_image(H, W, seed) for (H, W, _, _, seed, _, _, _) in spec]
    jobs = [cqm.BatchJob(torch.from_numpy(im).to(dev), K, scheme, seed, mi, tol, prune)
            for im, (H, W, K, scheme, seed, prune, mi, tol) in zip(imgs, spec)]
    tickets, finished = {}, {}
    waited = False
    nxt = 0
    sched = list(SCHEDULE)
    while len(finished) < len(jobs):
        n_sub, iters = sched.pop(0) if sched else (0, 8)
        for _ in range(n_sub):
            if nxt < len(jobs):
                tickets[eng.submit(jobs[nxt])] = nxt
                nxt += 1
        if not sched:
            while nxt < len(jobs):
                tickets[eng.submit(jobs[nxt])] = nxt
                nxt += 1
        queued, running, _ = eng.pending()
        for ticket, job, st in eng.step(iters):
            i = tickets[ticket]
            assert ticket not in finished and job is jobs[i]
            assert st["status"] == cqm.CQ_OK
            finished[ticket] = st
        q2, r2, _ = eng.pending()
        waited = waited or q2 > 0  # a job stayed queued after a step: admission was limited
        assert r2 <= eng.max_jobs
    assert eng.pending() == (0, 0, 0)
    return imgs, jobs, tickets, finished, waited


def test_engine_stream_matches_oracle_and_solo(cqm, dev):
    big = cqm.engine_job_bytes(512, 512)
    # room for the largest job plus a few small ones, never for all of them
    eng = cqm.Engine(max_jobs=5, pool_bytes=big + 3 * cqm.engine_job_bytes(300, 200), device=dev)
    _say("engine stream of %d jobs" % len(STREAM))
    imgs, jobs, tickets, finished, waited = _run_stream(cqm, dev, eng, STREAM)
    assert waited
    solo_ws = cqm.Workspace(512, 512, 256, dev)
    for ticket, i in sorted(tickets.items()):
        H, W, K, scheme, seed, prune, mi, tol = STREAM[i]
        _say(f"  job {i}: {H}x{W} K={K} scheme={scheme} prune={prune}")
        st, job = finished[ticket], jobs[i]
        rp, ri, rr, rs = oracle.quantize(imgs[i], K, scheme, seed, mi, tol, prune=prune)
        assert np.array_equal(job.palette.cpu().numpy(), rp)
        assert np.array_equal(job.idx.cpu().numpy(), ri)
        assert np.array_equal(job.rgb.cpu().numpy(), rr)
        for key in STAT_KEYS:
            assert st[key] == rs[key], key
        sp, si, sr, ss = cqm.cq_quantize(job.img, K, scheme, seed, mi, tol, prune, solo_ws)
        assert torch.equal(sp, job.palette) and torch.equal(si, job.idx) and torch.equal(sr, job.rgb)
        assert all(ss[key] == st[key] for key in STAT_KEYS)
    eng.close()


def test_engine_reuses_slots_and_repeats_results(cqm, dev):
    """The same stream twice through one engine (slots reused with stale
    contents, different admission interleavings): identical results."""
    eng = cqm.Engine(max_jobs=3, pool_bytes=3 * cqm.engine_job_bytes(400, 300), device=dev)
    spec = [s for s in STREAM if s[0] * s[1] <= 400 * 300]
    _say("engine reuse: %d jobs twice" % len(spec))
    _, jobs1, t1, f1, _ = _run_stream(cqm, dev, eng, spec)
    _, jobs2, t2, f2, _ = _run_stream(cqm, dev, eng, list(reversed(spec)))
    by_job1 = {t1[t]: (jobs1[t1[t]], f1[t]) for t in f1}
    by_job2 = {len(spec) - 1 - t2[t]: (jobs2[t2[t]], f2[t]) for t in f2}
    for i in range(len(spec)):
        (a, sa), (b, sb) = by_job1[i], by_job2[i]
        assert torch.equal(a.palette, b.palette) and torch.equal(a.idx, b.idx) and torch.equal(a.rgb, b.rgb)
        assert all(sa[key] == sb[key] for key in STAT_KEYS)
    eng.close()


def test_engine_zero_iteration_step_finishes_few_colour_jobs(cqm, dev):
    eng = cqm.Engine(max_jobs=2, pool_bytes=2 * cqm.engine_job_bytes(64, 64), device=dev)
    img = torch.from_numpy(_image(5, 3, 3)).to(dev)
    many = torch.from_numpy(_image(64, 64, 4)).to(dev)
    j_few = cqm.BatchJob(img, 16, oracle.INIT_KMEANSPP, 1, 10, 1e-4, True)  # 15 pixels: N' <= K
    j_many = cqm.BatchJob(many, 16, oracle.INIT_KMEANSPP, 1, 10, 1e-4, True)
    t_few, t_many = eng.submit(j_few), eng.submit(j_many)
    out = eng.step(0)
    assert [t for t, _, _ in out] == [t_few]  # no iteration ran: only the N' <= K job is done
    assert eng.pending()[1] == 1
    rest = []
    while not rest:
        rest = eng.step(4)
    assert [t for t, _, _ in rest] == [t_many]
    ws = cqm.Workspace(64, 64, 16, dev)
    for job, st in ((j_few, out[0][2]), (j_many, rest[0][2])):
        sp, si, sr, ss = cqm.cq_quantize(job.img, job.palette.shape[0], oracle.INIT_KMEANSPP, 1, 10, 1e-4, True, ws)
        assert torch.equal(sp, job.palette) and torch.equal(si, job.idx) and torch.equal(sr, job.rgb)
        assert all(ss[key] == st[key] for key in STAT_KEYS)
    eng.close()
