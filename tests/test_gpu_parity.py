"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every comparison is bit-exact: histogram keys and counts, initial centres,
memberships, FP64 centres, the SSE trace, iteration and distance counts, the
palette, the mapped image and its integer squared-error sum.  The relative MSE
error bound of 1e-6 is therefore met with zero error.
"""
import sys

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


@pytest.fixture(scope="module")
def ws_small(cqm, dev):
    return cqm.Workspace(1024, 1024, 256, dev)


def _to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


RAGGED = [(1, 1), (1, 7), (3, 5), (7, 13), (33, 65), (64, 64), (127, 129), (512, 512)]


@pytest.mark.parametrize("shape", RAGGED)
def test_histogram_parity(cqm, dev, ws_small, shape):
    H, W = shape
    _say(f"histogram {H}x{W}")
    img = synth.smooth_field_blobs(H, W, H * 1000 + W)
    keys, counts = cqm.cq_histogram(_to_dev(img, dev), ws_small)
    rk, rc = oracle.histogram(img)
    assert np.array_equal(_u32(keys), rk)
    assert np.array_equal(_u32(counts), rc)


def test_histogram_strided_rows_and_capacity(cqm, dev, ws_small):
    _say("histogram strided + capacity")
    rng = np.random.default_rng(3)
    base = rng.integers(0, 6, (37, 41, 3)).astype(np.uint8)
    padded = torch.zeros((37, 41 * 3 + 5), dtype=torch.uint8, device=dev)
    padded[:, :123] = _to_dev(base.reshape(37, 123), dev)
    view = padded.as_strided((37, 41, 3), (128, 3, 1))
    keys, counts = cqm.cq_histogram(view, ws_small)
    rk, rc = oracle.histogram(base)
    assert np.array_equal(_u32(keys), rk) and np.array_equal(_u32(counts), rc)
    with pytest.raises(cqm.CqError) as e:
        cqm.cq_histogram(view, ws_small, capacity=len(rk) - 1)
    assert e.value.code == cqm.CQ_ECAPACITY
    # the table was left clean: a second run still matches
    keys, counts = cqm.cq_histogram(view, ws_small)
    assert np.array_equal(_u32(keys), rk) and np.array_equal(_u32(counts), rc)


def test_histogram_single_colour_and_all_distinct(cqm, dev, ws_small):
    _say("histogram single colour / all distinct")
    img = np.full((50, 70, 3), 77, np.uint8)
    keys, counts = cqm.cq_histogram(_to_dev(img, dev), ws_small)
    assert _u32(keys).tolist() == [(77 << 16) | (77 << 8) | 77] and _u32(counts).tolist() == [3500]
    ks = np.random.default_rng(0).permutation(1 << 24)[: 300 * 300].astype(np.uint32)
    img = np.stack([(ks >> 16) & 255, (ks >> 8) & 255, ks & 255], 1).astype(np.uint8).reshape(300, 300, 3)
    keys, counts = cqm.cq_histogram(_to_dev(img, dev), ws_small)
    assert np.array_equal(_u32(keys), np.sort(ks)) and (_u32(counts) == 1).all()


def _hist_pair(img, cqm, dev, ws):
    rk, rc = oracle.histogram(img)
    return rk, rc, _to_dev(rk.view(np.int32), dev), _to_dev(rc.view(np.int32), dev)


@pytest.mark.parametrize("scheme", [oracle.INIT_FORGY, oracle.INIT_MAXMIN, oracle.INIT_KMEANSPP, oracle.INIT_VAR,
                                    oracle.INIT_SFF, oracle.INIT_WU, oracle.INIT_LBG, oracle.INIT_DEN])
@pytest.mark.parametrize("K,seed", [(16, 0), (64, 3), (256, 1)])
def test_init_parity(cqm, dev, ws_small, scheme, K, seed):
    _say(f"init scheme={scheme} K={K} seed={seed}")
    img = synth.smooth_field_blobs(200, 300, seed)
    rk, rc, dk, dc = _hist_pair(img, cqm, dev, ws_small)
    ref, ref_used = oracle.init(rk, rc, K, scheme, seed)
    got, used = cqm.cq_init(dk, dc, K, scheme, seed, ws_small)
    assert used == ref_used
    assert np.array_equal(got.cpu().numpy(), ref)


@pytest.mark.parametrize("n", [4096, 4097, 16384, 24577, 32768, 32769, 65537, 262145])
def test_cooperative_init_at_capacity_boundaries(cqm, dev, ws_small, n):
    """k-means++ and max-min on colour sets at the sizes where the
    initialization changes the colours per thread a block holds (4096 to
    32768 colours per block) or grows a team of blocks: bit-identical centres,
    with counts from 1 up to 10^5 so that the draws' weights vary widely."""
    _say(f"cooperative init n={n}")
    rng = np.random.default_rng(n)
    rk = np.sort(rng.choice(1 << 24, n, replace=False)).astype(np.uint32)
    rc = np.minimum(rng.pareto(1.2, n) * 3 + 1, 1e5).astype(np.uint32)
    dk, dc = _to_dev(rk.view(np.int32), dev), _to_dev(rc.view(np.int32), dev)
    for scheme in (oracle.INIT_KMEANSPP, oracle.INIT_MAXMIN):
        ref, ref_used = oracle.init(rk, rc, 256, scheme, n)
        got, used = cqm.cq_init(dk, dc, 256, scheme, n, ws_small)
        assert used == ref_used
        assert np.array_equal(got.cpu().numpy(), ref), scheme


def test_var_weighted_duplicates_and_sff_small_sets(cqm, dev, ws_small):
    """VAR where one colour's pixels span several groups (repeated centres),
    and SFF on sets smaller than its subset size (the subset is every colour)."""
    _say("init VAR heavy colour / SFF small set")
    rng = np.random.default_rng(31)
    img = rng.integers(0, 256, (64, 96, 3)).astype(np.uint8)
    img[:40] = (200, 10, 90)  # 2560 of 6144 pixels share one colour
    rk, rc, dk, dc = _hist_pair(img, cqm, dev, ws_small)
    for K in (5, 16, 64):
        ref, _ = oracle.init(rk, rc, K, oracle.INIT_VAR, 0)
        got, _ = cqm.cq_init(dk, dc, K, oracle.INIT_VAR, 0, ws_small)
        assert np.array_equal(got.cpu().numpy(), ref), K
    small = rng.integers(0, 256, (10, 12, 3)).astype(np.uint8)
    rk, rc, dk, dc = _hist_pair(small, cqm, dev, ws_small)
    for K in (8, 40, 100):  # subsets 34, 296 and 921 capped at the ~120 colours
        for seed in (1, 2):
            ref, _ = oracle.init(rk, rc, K, oracle.INIT_SFF, seed)
            got, _ = cqm.cq_init(dk, dc, K, oracle.INIT_SFF, seed, ws_small)
            assert np.array_equal(got.cpu().numpy(), ref), (K, seed)


def test_sff_sequential_draws_match(cqm, dev, ws_small, monkeypatch):
    """The one-at-a-time draws SFF falls back to when a draw is rejected give
    the same centres as the parallel draws (forced by CQ_SFF_SEQUENTIAL)."""
    _say("init SFF sequential draws")
    img = synth.smooth_field_blobs(200, 300, 4)
    rk, rc, dk, dc = _hist_pair(img, cqm, dev, ws_small)
    for K in (16, 256):
        ref, _ = oracle.init(rk, rc, K, oracle.INIT_SFF, K)
        monkeypatch.setenv("CQ_SFF_SEQUENTIAL", "1")
        seq, _ = cqm.cq_init(dk, dc, K, oracle.INIT_SFF, K, ws_small)
        monkeypatch.delenv("CQ_SFF_SEQUENTIAL")
        par, _ = cqm.cq_init(dk, dc, K, oracle.INIT_SFF, K, ws_small)
        assert np.array_equal(seq.cpu().numpy(), ref) and np.array_equal(par.cpu().numpy(), ref), K


def test_init_fewer_colours_than_k(cqm, dev, ws_small):
    _say("init N' <= K")
    img = np.array([[[1, 2, 3], [1, 2, 3], [9, 9, 9]]], np.uint8)
    rk, rc, dk, dc = _hist_pair(img, cqm, dev, ws_small)
    for scheme in (0, 1, 2):
        got, used = cqm.cq_init(dk, dc, 4, scheme, 0, ws_small)
        ref, ref_used = oracle.init(rk, rc, 4, scheme, 0)
        assert used == ref_used == 2 and np.array_equal(got.cpu().numpy(), ref)


def _compare_kmeans(g, r):
    assert np.array_equal(g.assign.cpu().numpy(), r.assign)
    assert np.array_equal(g.centers.cpu().numpy(), r.centers)
    assert np.array_equal(np.array(g.sse_trace), r.sse_trace)
    assert np.array_equal(g.palette.cpu().numpy(), r.palette)
    for key in ("iters", "converged", "k_used", "ndc_total", "near_ties", "sse_final", "mse_float"):
        assert g.stats[key] == r.stats[key], key


@pytest.mark.parametrize("prune", [False, True])
@pytest.mark.parametrize("K,seed,scheme", [(1, 5, 2), (2, 4, 1), (16, 0, 1), (37, 2, 0), (64, 3, 2),
                                          (256, 1, 2)])
def test_kmeans_parity(cqm, dev, ws_small, prune, K, seed, scheme):
    _say(f"kmeans K={K} seed={seed} scheme={scheme} prune={prune}")
    img = synth.smooth_field_blobs(160, 224, seed) if K > 16 else synth.blobs_on_gradient(64, 64, seed)
    rk, rc, dk, dc = _hist_pair(img, cqm, dev, ws_small)
    c0, _ = oracle.init(rk, rc, K, scheme, seed)
    r = oracle.kmeans(rk, rc, c0, 100, 1e-4, prune)
    g = cqm.cq_kmeans(dk, dc, _to_dev(c0, dev), 100, 1e-4, prune, ws_small)
    _compare_kmeans(g, r)


def test_kmeans_coincident_user_centres(cqm, dev, ws_small):
    _say("kmeans coincident centres")
    img = synth.smooth_field_blobs(96, 128, 11)
    rk, rc, dk, dc = _hist_pair(img, cqm, dev, ws_small)
    c0, _ = oracle.init(rk, rc, 24, oracle.INIT_KMEANSPP, 11)
    c0[23] = c0[0]
    c0[22] = c0[5]
    for prune in (False, True):
        r = oracle.kmeans(rk, rc, c0, 40, 0.0, prune)
        g = cqm.cq_kmeans(dk, dc, _to_dev(c0, dev), 40, 0.0, prune, ws_small)
        _compare_kmeans(g, r)


def test_kmeans_empty_clusters_keep_their_centres(cqm, dev, ws_small):
    """Two centres far outside the colour cube are nearest to no colour in any
    iteration: their clusters stay empty and they keep their position (their
    palette entries clamped to the cube); everything else equals the oracle,
    pruned and unpruned."""
    _say("kmeans empty clusters")
    img = synth.smooth_field_blobs(96, 128, 5)
    rk, rc, dk, dc = _hist_pair(img, cqm, dev, ws_small)
    c0, _ = oracle.init(rk, rc, 20, oracle.INIT_KMEANSPP, 5)
    c0[4] = (-300.0, 400.0, -300.0)
    c0[17] = (1000.5, 1000.25, -1000.0)
    for prune in (False, True):
        r = oracle.kmeans(rk, rc, c0, 60, 0.0, prune)
        g = cqm.cq_kmeans(dk, dc, _to_dev(c0, dev), 60, 0.0, prune, ws_small)
        _compare_kmeans(g, r)
        centres = g.centers.cpu().numpy()
        assert np.array_equal(centres[4], c0[4]) and np.array_equal(centres[17], c0[17])
        assert not np.any(g.assign.cpu().numpy() == 4) and not np.any(g.assign.cpu().numpy() == 17)


def _key(r, g, b):
    return (r << 16) | (g << 8) | b


# Colours and start centres whose first update puts the centres where a colour
# of the second iteration (a sort-means pass) lies at exactly the same distance
# from two of them (the centre positions are worked out in the comments).
EXACT_TIES = [
    # one channel: colours 0 (x3), 10, 15, 20, 30 and centres 6, 25 become
    # centres 5, 25; colour 15 (cluster 0) is 10 from both and stays in 0
    ([(0, 0, 0, 3), (10, 0, 0, 1), (15, 0, 0, 1), (20, 0, 0, 1), (30, 0, 0, 1)],
     [(6.0, 0.0, 0.0), (25.0, 0.0, 0.0)]),
    # three centres: the first update gives (15,5,0), (5,15,0), (14,16,11);
    # colour (15,15,0), in cluster 2, is at squared distance 100 from centres
    # 0 and 1, which row 2 lists as centre 1 (203) before centre 0 (243): the
    # pass meets centre 1 first and must end at centre 0
    ([(5, 15, 0, 1), (13, 17, 22, 1), (15, 5, 0, 1), (15, 15, 0, 1)],
     [(15.0, 5.0, 0.0), (5.0, 15.0, 0.0), (14.0, 16.0, 8.0)]),
]


@pytest.mark.parametrize("case", range(len(EXACT_TIES)))
def test_kmeans_exact_ties_in_sort_means_passes(cqm, dev, ws_small, case):
    """Exact distance ties met by the sort-means passes: the lower centre
    index wins (also when the pass meets the higher one first), and the
    distance and near-tie counts equal the oracle's, pruned and unpruned."""
    _say(f"kmeans exact ties case {case}")
    colours, c0 = EXACT_TIES[case]
    rk = np.array([_key(r, g, b) for r, g, b, _ in colours], np.uint32)
    rc = np.array([n for *_, n in colours], np.uint32)
    assert np.all(np.diff(rk.astype(np.int64)) > 0)
    c0 = np.array(c0, np.float64)
    dk, dc = _to_dev(rk.view(np.int32), dev), _to_dev(rc.view(np.int32), dev)
    for prune in (False, True):
        r = oracle.kmeans(rk, rc, c0, 6, 0.0, prune)
        g = cqm.cq_kmeans(dk, dc, _to_dev(c0, dev), 6, 0.0, prune, ws_small)
        _compare_kmeans(g, r)
        assert r.stats["iters"] >= 2 and r.stats["near_ties"] >= 1


def test_kmeans_max_iters_one_and_nonfinite_start(cqm, dev, ws_small):
    _say("kmeans max_iters=1 / non-finite start")
    img = synth.blobs_on_gradient(64, 64, 7)
    rk, rc, dk, dc = _hist_pair(img, cqm, dev, ws_small)
    c0, _ = oracle.init(rk, rc, 16, oracle.INIT_MAXMIN, 7)
    r = oracle.kmeans(rk, rc, c0, 1, 1e-4, True)
    g = cqm.cq_kmeans(dk, dc, _to_dev(c0, dev), 1, 1e-4, True, ws_small)
    _compare_kmeans(g, r)
    bad = c0.copy()
    bad[3, 1] = np.nan
    with pytest.raises(cqm.CqError) as e:
        cqm.cq_kmeans(dk, dc, _to_dev(bad, dev), 5, 1e-4, True, ws_small)
    assert e.value.code == cqm.CQ_EINVAL


def test_kmeans_rejects_keys_and_counts_out_of_range(cqm, dev, ws_small):
    """Caller-supplied colours: a key of 2^24 or more, or counts summing to
    more than 2^28, are refused with CQ_EINVAL before any iteration, pruned
    or not; the same colours within range run (and match the oracle)."""
    _say("kmeans argument range on the device")
    img = synth.blobs_on_gradient(64, 64, 11)
    rk, rc, dk, dc = _hist_pair(img, cqm, dev, ws_small)
    c0, _ = oracle.init(rk, rc, 16, oracle.INIT_MAXMIN, 11)
    for prune in (False, True):
        bad_keys = dk.clone()
        bad_keys[len(rk) // 2] = 1 << 24
        with pytest.raises(cqm.CqError) as e:
            cqm.cq_kmeans(bad_keys, dc, _to_dev(c0, dev), 5, 1e-4, prune, ws_small)
        assert e.value.code == cqm.CQ_EINVAL and "2^24" in str(e.value)
        heavy = dc.clone()
        heavy[0] = (1 << 28) - int(rc[1:].sum()) + 1  # total 2^28 + 1
        with pytest.raises(cqm.CqError) as e:
            cqm.cq_kmeans(dk, heavy, _to_dev(c0, dev), 5, 1e-4, prune, ws_small)
        assert e.value.code == cqm.CQ_EINVAL and "2^28" in str(e.value)
        edge = dc.clone()
        edge[0] = (1 << 28) - int(rc[1:].sum())  # total exactly 2^28: accepted
        hk = rc.copy()
        hk[0] = (1 << 28) - int(rc[1:].sum())
        r = oracle.kmeans(rk, hk, c0, 5, 1e-4, prune)
        g = cqm.cq_kmeans(dk, edge, _to_dev(c0, dev), 5, 1e-4, prune, ws_small)
        _compare_kmeans(g, r)


@pytest.mark.parametrize("K", [1, 5, 16, 255, 256])
def test_map_parity(cqm, dev, ws_small, K):
    _say(f"map K={K}")
    img = synth.smooth_field_blobs(123, 77, K)
    rk, rc, dk, dc = _hist_pair(img, cqm, dev, ws_small)
    pal = np.random.default_rng(K).integers(0, 256, (K, 3)).astype(np.uint8)
    if K > 4:
        pal[K - 1] = pal[1]  # duplicate entry: lowest index wins
    idx, rgb, err = cqm.cq_map(_to_dev(img, dev), dk, dc, _to_dev(pal, dev), ws_small)
    ridx, rrgb, rerr = oracle.map_image(img, pal)
    assert np.array_equal(idx.cpu().numpy(), ridx)
    assert np.array_equal(rgb.cpu().numpy(), rrgb)
    assert err == rerr


def _compare_quantize(g, r, img):
    gp, gi, gr, gs = g
    rp, ri, rr, rs = r
    assert np.array_equal(gp.cpu().numpy(), rp)
    assert np.array_equal(gi.cpu().numpy(), ri)
    assert np.array_equal(gr.cpu().numpy(), rr)
    for key in ("iters", "converged", "k_used", "n_unique", "ndc_total", "near_ties", "sse_final",
                "mse_float", "mse_img"):
        assert gs[key] == rs[key], key
    mse = ((img.astype(np.float64) - gr.cpu().numpy().astype(np.float64)) ** 2).sum(-1).mean()
    assert gs["mse_img"] == pytest.approx(mse, rel=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_quantize_small_config(cqm, dev, ws_small, seed):
    _say(f"quantize 64x64 K=16 MMX plain seed={seed}")
    img = synth.blobs_on_gradient(64, 64, seed)
    r = oracle.quantize(img, 16, oracle.INIT_MAXMIN, seed, 50, 1e-4, prune=False)
    g = cqm.cq_quantize(_to_dev(img, dev), 16, oracle.INIT_MAXMIN, seed, 50, 1e-4, False, ws_small)
    _compare_quantize(g, r, img)


@pytest.mark.parametrize("K", [32, 64, 128, 256])
def test_quantize_512_config(cqm, dev, ws_small, K):
    _say(f"quantize 512x512 K={K} KPP pruned seed=1")
    img = synth.smooth_field_blobs(512, 512, 1)
    r = oracle.quantize(img, K, oracle.INIT_KMEANSPP, 1, 100, 1e-4, prune=True)
    g = cqm.cq_quantize(_to_dev(img, dev), K, oracle.INIT_KMEANSPP, 1, 100, 1e-4, True, ws_small)
    _compare_quantize(g, r, img)


def test_quantize_fewer_colours_than_k_and_ragged(cqm, dev, ws_small):
    _say("quantize N' <= K, ragged 5x3")
    img = np.array([[[5, 6, 7], [200, 100, 0], [5, 6, 7]]] * 5, np.uint8)
    r = oracle.quantize(img, 8, oracle.INIT_KMEANSPP, 0, 20, 1e-4)
    g = cqm.cq_quantize(_to_dev(img, dev), 8, oracle.INIT_KMEANSPP, 0, 20, 1e-4, True, ws_small)
    _compare_quantize(g, r, img)


def test_deterministic_repeat(cqm, dev, ws_small):
    _say("determinism")
    img = _to_dev(synth.smooth_field_blobs(300, 200, 9), dev)
    a = cqm.cq_quantize(img, 128, oracle.INIT_KMEANSPP, 9, 100, 1e-4, True, ws_small)
    b = cqm.cq_quantize(img, 128, oracle.INIT_KMEANSPP, 9, 100, 1e-4, True, ws_small)
    assert torch.equal(a[0], b[0]) and torch.equal(a[2], b[2]) and a[3] == b[3]


def test_full_size_4096(cqm, dev):
    """4096 x 4096 (16.7M pixels): histogram and map bit-exact against the
    oracle, three k-means iterations bit-exact, and the end-to-end run's
    image checked against its palette pixel by pixel on a sample."""
    _say("full size 4096x4096")
    H = W = 4096
    img = synth.smooth_field_blobs(H, W, 42)
    ws = cqm.Workspace(H, W, 256, dev)
    dimg = _to_dev(img, dev)
    keys, counts = cqm.cq_histogram(dimg, ws)
    rk, rc = oracle.histogram(img)
    assert np.array_equal(_u32(keys), rk) and np.array_equal(_u32(counts), rc)
    _say(f"  N' = {len(rk)}")
    c0, _ = oracle.init(rk, rc, 256, oracle.INIT_KMEANSPP, 42)
    g0, _ = cqm.cq_init(keys, counts, 256, oracle.INIT_KMEANSPP, 42, ws)
    assert np.array_equal(g0.cpu().numpy(), c0)
    # more colours than the blocks of a team keep in LDS: runs read from memory
    m0, _ = oracle.init(rk, rc, 64, oracle.INIT_MAXMIN, 5)
    gm, _ = cqm.cq_init(keys, counts, 64, oracle.INIT_MAXMIN, 5, ws)
    assert np.array_equal(gm.cpu().numpy(), m0)
    # VAR over thousands of tiles (several rounds of the tile scan), and SFF
    v0, _ = oracle.init(rk, rc, 256, oracle.INIT_VAR, 0)
    gv, _ = cqm.cq_init(keys, counts, 256, oracle.INIT_VAR, 0, ws)
    assert np.array_equal(gv.cpu().numpy(), v0)
    f0, _ = oracle.init(rk, rc, 256, oracle.INIT_SFF, 9)
    gf, _ = cqm.cq_init(keys, counts, 256, oracle.INIT_SFF, 9, ws)
    assert np.array_equal(gf.cpu().numpy(), f0)
    r = oracle.kmeans(rk, rc, c0, 3, 1e-4, True)
    g = cqm.cq_kmeans(keys, counts, _to_dev(c0, dev), 3, 1e-4, True, ws)
    _compare_kmeans(g, r)
    idx, rgb, err = cqm.cq_map(dimg, keys, counts, g.palette, ws)
    ridx, rrgb, rerr = oracle.map_image(img, r.palette)
    assert np.array_equal(idx.cpu().numpy(), ridx) and np.array_equal(rgb.cpu().numpy(), rrgb)
    assert err == rerr
    pal, gi, gr, st = cqm.cq_quantize(dimg, 256, oracle.INIT_KMEANSPP, 42, 100, 1e-4, True, ws)
    P = pal.cpu().numpy().astype(np.int64)
    rng = np.random.default_rng(0)
    ys, xs = rng.integers(0, H, 20000), rng.integers(0, W, 20000)
    X = img[ys, xs].astype(np.int64)
    D = ((X[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    assert np.array_equal(gi.cpu().numpy()[ys, xs], np.argmin(D, axis=1))
    mse = ((img.astype(np.float64) - gr.cpu().numpy().astype(np.float64)) ** 2).sum(-1).mean()
    assert st["mse_img"] == pytest.approx(mse, rel=1e-12)
    assert st["converged"] == 1


@pytest.mark.gpu
def test_every_colour_once(cqm, dev):
    """The largest histogram there is: a 4096 x 4096 image holding each of the
    2^24 colours once (a seeded permutation).  Histogram bit-exact (every key,
    count 1), cooperative inits with runs read from memory, three pruned
    k-means iterations bit-exact, and the map checked pixel by pixel on a
    sample against the palette."""
    _say("every 24-bit colour once (4096x4096)")
    H = W = 4096
    perm = np.random.default_rng(7).permutation(1 << 24).astype(np.uint32)
    img = np.stack([(perm >> 16) & 255, (perm >> 8) & 255, perm & 255], -1).astype(np.uint8).reshape(H, W, 3)
    ws = cqm.Workspace(H, W, 256, dev)
    dimg = _to_dev(img, dev)
    keys, counts = cqm.cq_histogram(dimg, ws)
    gk, gc = _u32(keys), _u32(counts)
    assert np.array_equal(gk, np.arange(1 << 24, dtype=np.uint32)) and np.all(gc == 1)
    rk, rc = oracle.histogram(img)
    assert np.array_equal(gk, rk) and np.array_equal(gc, rc)
    for scheme, seed in ((oracle.INIT_KMEANSPP, 3), (oracle.INIT_MAXMIN, 4)):
        c, _ = oracle.init(rk, rc, 16, scheme, seed)
        g, _ = cqm.cq_init(keys, counts, 16, scheme, seed, ws)
        assert np.array_equal(g.cpu().numpy(), c), scheme
    c0, _ = oracle.init(rk, rc, 256, oracle.INIT_FORGY, 3)
    g0, _ = cqm.cq_init(keys, counts, 256, oracle.INIT_FORGY, 3, ws)
    assert np.array_equal(g0.cpu().numpy(), c0)
    r = oracle.kmeans(rk, rc, c0, 3, 1e-4, True)
    g = cqm.cq_kmeans(keys, counts, _to_dev(c0, dev), 3, 1e-4, True, ws)
    _compare_kmeans(g, r)
    idx, rgb, err = cqm.cq_map(dimg, keys, counts, g.palette, ws)
    P = r.palette.astype(np.int64)
    rng = np.random.default_rng(1)
    ys, xs = rng.integers(0, H, 20000), rng.integers(0, W, 20000)
    X = img[ys, xs].astype(np.int64)
    D = ((X[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    want = np.argmin(D, axis=1)
    assert np.array_equal(idx.cpu().numpy()[ys, xs], want)
    assert np.array_equal(rgb.cpu().numpy()[ys, xs], r.palette[want])
    sq = ((img.astype(np.int64) - rgb.cpu().numpy().astype(np.int64)) ** 2).sum()
    assert err == sq


@pytest.mark.gpu
def test_largest_image(cqm, dev):
    """The largest image accepted, 2^28 pixels (16384 x 16384): a 4096 x 4096
    stand-in tiled 4 x 4, so every colour's count is 16 times its count in the
    tile.  Histogram bit-exact; FGY init and three pruned iterations bit-exact
    against the oracle on that histogram; the map equal to the tile's map
    repeated, and its squared-error sum 16 times the tile's."""
    _say("largest image 16384x16384 (2^28 pixels)")
    base = synth.smooth_field_blobs(4096, 4096, 42)
    img = np.tile(base, (4, 4, 1))
    H, W = img.shape[:2]
    assert H * W == 1 << 28
    ws = cqm.Workspace(H, W, 256, dev)
    dimg = _to_dev(img, dev)
    keys, counts = cqm.cq_histogram(dimg, ws)
    bk, bc = oracle.histogram(base)
    rk, rc = oracle.histogram(img)
    assert np.array_equal(rk, bk) and np.array_equal(rc, bc * np.uint32(16))
    assert np.array_equal(_u32(keys), rk) and np.array_equal(_u32(counts), rc)
    _say(f"  N' = {len(bk)}")
    c0, _ = oracle.init(bk, rc, 256, oracle.INIT_FORGY, 5)
    g0, _ = cqm.cq_init(keys, counts, 256, oracle.INIT_FORGY, 5, ws)
    assert np.array_equal(g0.cpu().numpy(), c0)
    r = oracle.kmeans(bk, rc, c0, 3, 1e-4, True)
    g = cqm.cq_kmeans(keys, counts, _to_dev(c0, dev), 3, 1e-4, True, ws)
    _compare_kmeans(g, r)
    # FGY ignores the counts and every weighted sum scales by 16: the run on
    # the tile alone reaches the same centres with 16 times smaller SSE terms
    rb = oracle.kmeans(bk, bc, c0, 3, 1e-4, True)
    assert np.array_equal(rb.centers, r.centers)
    assert np.array_equal(np.array(rb.sse_trace) * 16.0, np.array(r.sse_trace))
    idx, rgb, err = cqm.cq_map(dimg, keys, counts, g.palette, ws)
    ridx, rrgb, rerr = oracle.map_image(base, r.palette)
    gi = idx.cpu().numpy()
    del idx
    assert np.array_equal(gi, np.tile(ridx, (4, 4)))
    del gi
    gr = rgb.cpu().numpy()
    del rgb
    assert np.array_equal(gr, np.tile(rrgb, (4, 4, 1)))
    assert err == 16 * rerr
