"""Pins of the CPU oracle against the paper and against mathematics.

Every test here is CPU-only.  None of them re-types the oracle's own formulas:
they check published values, closed forms, library routines (numpy.unique,
numpy argmin over a brute-force distance matrix, scikit-learn's Lloyd),
invariants and brute force on tiny inputs.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1101_0395_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows[parts[0]] = parts[1:]
    return rows


def _keys_of(img):
    img = np.asarray(img)
    return ((img[..., 0].astype(np.uint32) << 16) | (img[..., 1].astype(np.uint32) << 8)
            | img[..., 2].astype(np.uint32))


def _rgb_of(keys):
    keys = np.asarray(keys, np.int64)
    return np.stack([(keys >> 16) & 255, (keys >> 8) & 255, keys & 255], axis=1)


def _random_small_image(rng, H, W, n_colors):
    base = rng.integers(0, 256, (n_colors, 3))
    pick = rng.integers(0, n_colors, H * W)
    return base[pick].reshape(H, W, 3).astype(np.uint8)


# --------------------------------------------------------------------------- RNG

def test_splitmix64_published_sequence():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) as f:
        expect = [int(x) for x in f.read().split("\n") if x and not x.startswith("#")]
    assert oracle.splitmix64(1234567, len(expect)) == expect


def test_uniform_below_range_and_uniformity():
    draws = np.array(oracle.uniform_below(99, 7, 70_000))
    assert draws.min() >= 0 and draws.max() <= 6
    obs = np.bincount(draws, minlength=7)
    chi2 = (((obs - 10_000) ** 2) / 10_000).sum()
    assert chi2 < 30.0  # 6 dof: P(chi2 > 30) ~ 4e-5
    assert oracle.uniform_below(5, 1, 10) == [0] * 10
    big = (1 << 63) + 1  # more than half of all outputs fall in the rejected band
    assert all(v < big for v in oracle.uniform_below(3, big, 200))


# --------------------------------------------------------------------- histogram

@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (17, 33), (64, 64)])
def test_histogram_matches_numpy_unique(shape):
    rng = np.random.default_rng(shape[0] * 100 + shape[1])
    img = _random_small_image(rng, shape[0], shape[1], 40)
    keys, counts = oracle.histogram(img)
    u, c = np.unique(img.reshape(-1, 3), axis=0, return_counts=True)
    # lexicographic (R, G, B) order is ascending 0xRRGGBB order
    assert np.array_equal(_rgb_of(keys), u)
    assert np.array_equal(counts, c)
    assert int(counts.sum()) == shape[0] * shape[1]


def test_histogram_brute_force_dict_and_stride():
    rng = np.random.default_rng(5)
    img = rng.integers(0, 4, (9, 11, 3)).astype(np.uint8)
    padded = np.zeros((9, 11 * 3 + 7), np.uint8)  # rows with 7 bytes of padding
    padded[:, : 33] = img.reshape(9, 33)
    view = np.lib.stride_tricks.as_strided(padded, shape=(9, 11, 3), strides=(40, 3, 1))
    keys, counts = oracle.histogram(view)
    ref = {}
    for px in img.reshape(-1, 3):
        k = (int(px[0]) << 16) | (int(px[1]) << 8) | int(px[2])
        ref[k] = ref.get(k, 0) + 1
    assert list(keys) == sorted(ref)
    assert [int(c) for c in counts] == [ref[k] for k in sorted(ref)]


def test_histogram_capacity_error():
    img = np.arange(30, dtype=np.uint8).reshape(1, 10, 3)
    with pytest.raises(oracle.OracleError) as e:
        oracle.histogram(img, capacity=3)
    assert e.value.code == oracle.ECAPACITY


# -------------------------------------------------------------------------- init

def _hist_small(seed, n_colors=60, H=24, W=24):
    rng = np.random.default_rng(seed)
    img = _random_small_image(rng, H, W, n_colors)
    return oracle.histogram(img)


def test_forgy_picks_distinct_colours():
    keys, counts = _hist_small(1)
    C, k_used = oracle.init(keys, counts, 16, oracle.INIT_FORGY, 7)
    assert k_used == 16
    rgb = _rgb_of(keys)
    picked = [int(np.flatnonzero((rgb == c).all(1))[0]) for c in C.astype(np.int64)]
    assert len(set(picked)) == 16


def test_maxmin_is_farthest_first():
    keys, counts = _hist_small(2)
    X = _rgb_of(keys).astype(np.int64)
    for seed in range(5):
        C, _ = oracle.init(keys, counts, 12, oracle.INIT_MAXMIN, seed)
        C = C.astype(np.int64)
        # first centre: colour number U(N') of the seed's stream
        first = oracle.uniform_below(seed, len(keys), 1)[0]
        assert np.array_equal(C[0], X[first])
        for j in range(1, 12):
            d = ((X[:, None, :] - C[None, :j, :]) ** 2).sum(-1).min(1)
            best = int(np.argmax(d))  # numpy: first index of the maximum
            assert np.array_equal(C[j], X[best])


def test_kmeanspp_sampling_distribution():
    # 5 colours with uneven counts; the second centre must follow n_i D_i^2.
    img = np.zeros((1, 20, 3), np.uint8)
    cols = [(0, 0, 0), (10, 0, 0), (0, 30, 0), (0, 0, 50), (40, 40, 40)]
    reps = [8, 5, 3, 2, 2]
    px = [c for c, r in zip(cols, reps) for _ in range(r)]
    img[0] = np.array(px, np.uint8)
    keys, counts = oracle.histogram(img)
    X = _rgb_of(keys).astype(np.int64)
    n_trials = 4000
    first_hits = np.zeros(len(keys))
    second_hits = {}
    for seed in range(n_trials):
        C, _ = oracle.init(keys, counts, 2, oracle.INIT_KMEANSPP, seed)
        i0 = int(np.flatnonzero((X == C[0].astype(np.int64)).all(1))[0])
        i1 = int(np.flatnonzero((X == C[1].astype(np.int64)).all(1))[0])
        first_hits[i0] += 1
        second_hits.setdefault(i0, np.zeros(len(keys)))[i1] += 1
    p0 = counts / counts.sum()
    chi2 = (((first_hits - n_trials * p0) ** 2) / (n_trials * p0)).sum()
    assert chi2 < 25.0  # 4 dof
    for i0, hits in second_hits.items():
        d2 = ((X - X[i0]) ** 2).sum(1)
        w = counts * d2
        p = w / w.sum()
        m = hits.sum()
        mask = p > 0
        assert hits[~mask].sum() == 0  # zero-weight colours are never drawn
        chi2 = (((hits[mask] - m * p[mask]) ** 2) / (m * p[mask])).sum()
        assert chi2 < 30.0


def test_init_with_fewer_colours_than_k():
    img = np.array([[[1, 2, 3], [1, 2, 3], [9, 9, 9]]], np.uint8)
    keys, counts = oracle.histogram(img)
    for scheme in (oracle.INIT_FORGY, oracle.INIT_MAXMIN, oracle.INIT_KMEANSPP):
        C, k_used = oracle.init(keys, counts, 4, scheme, 0)
        assert k_used == 2
        assert np.array_equal(C[:2], [[1, 2, 3], [9, 9, 9]])
        assert np.array_equal(C[2:], np.zeros((2, 3)))


# ---------------------------------------------------------------- k-means steps

def test_worked_example():
    g = _read_golden("worked_example_k2.txt")
    img = np.array([[[0, 0, 0], [0, 0, 0], [10, 0, 0], [100, 0, 0]]], np.uint8)
    keys, counts = oracle.histogram(img)
    assert list(keys) == [int(v) for v in g["keys"]]
    assert list(counts) == [int(v) for v in g["counts"]]
    res = oracle.kmeans(keys, counts, [[0, 0, 0], [100, 0, 0]], 10, 1e-4, prune=True)
    assert list(res.assign) == [int(v) for v in g["assign"]]
    assert res.stats["iters"] == int(g["iters"][0]) and res.stats["converged"] == 1
    assert res.centers[0, 0] == 10 / 3 and res.centers[1, 0] == 100.0
    assert res.sse_trace[-1] == pytest.approx(int(g["sse_numerator_over_9"][0]) / 9, rel=1e-15)
    assert list(res.palette.reshape(-1)) == [int(v) for v in g["palette"]]
    idx, rgb, err = oracle.map_image(img, res.palette)
    assert list(idx.reshape(-1)) == [int(v) for v in g["idx"]]
    assert err == int(g["sq_err_sum"][0])


def test_first_assignment_is_bruteforce_argmin_with_lowest_index_ties():
    rng = np.random.default_rng(11)
    for trial in range(20):
        keys, counts = _hist_small(100 + trial, n_colors=50)
        X = _rgb_of(keys).astype(np.int64)
        K = 9
        # integer-valued centres with deliberate duplicates -> exact distance ties
        C = rng.integers(0, 256, (K, 3))
        C[5] = C[2]
        C[8] = C[0]
        res = oracle.kmeans(keys, counts, C.astype(np.float64), 1, 0.0, prune=False)
        D = ((X[:, None, :] - C[None, :, :]) ** 2).sum(-1)
        assert np.array_equal(res.assign, np.argmin(D, axis=1))  # first minimum


@pytest.mark.parametrize("seed", range(12))
def test_pruned_equals_unpruned(seed):
    """Section 2.2: with the same initial centres WSM equals plain k-means."""
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(8, 48)), int(rng.integers(8, 48))
    img = synth.blobs_on_gradient(H, W, seed)
    keys, counts = oracle.histogram(img)
    K = int(rng.choice([2, 3, 5, 16, 40]))
    scheme = int(rng.choice([oracle.INIT_FORGY, oracle.INIT_MAXMIN, oracle.INIT_KMEANSPP]))
    C, _ = oracle.init(keys, counts, K, scheme, seed)
    if seed % 3 == 0 and K >= 3:
        C[K - 1] = C[0]  # coincident centres exercise the tie rules of the sorted rows
    a = oracle.kmeans(keys, counts, C, 60, 0.0, prune=False)
    b = oracle.kmeans(keys, counts, C, 60, 0.0, prune=True)
    assert np.array_equal(a.assign, b.assign)
    assert np.array_equal(a.centers, b.centers)
    assert np.array_equal(a.sse_trace, b.sse_trace)
    assert a.stats["iters"] == b.stats["iters"]
    if len(keys) > K:
        assert b.stats["ndc_total"] <= a.stats["ndc_total"]
        assert a.stats["ndc_total"] == a.stats["iters"] * len(keys) * K


def _pixel_lloyd(pixels, C, iters):
    """Unweighted Lloyd on every pixel (Algo. 1), numpy brute force."""
    C = C.copy()
    P = pixels.astype(np.float64)
    for _ in range(iters):
        D = ((P[:, None, :] - C[None, :, :]) ** 2).sum(-1)
        m = np.argmin(D, axis=1)
        for k in range(C.shape[0]):
            sel = m == k
            if sel.any():
                C[k] = P[sel].mean(axis=0)
    return C, m


@pytest.mark.parametrize("seed", range(4))
def test_weighted_histogram_lloyd_equals_pixel_lloyd(seed):
    """Weighting unique colours by frequency (Section 2.2, item 2) reproduces
    Lloyd on all pixels."""
    img = synth.blobs_on_gradient(20, 24, seed)
    keys, counts = oracle.histogram(img)
    C0, _ = oracle.init(keys, counts, 6, oracle.INIT_KMEANSPP, seed)
    for iters in (1, 2, 5):
        res = oracle.kmeans(keys, counts, C0, iters, 0.0, prune=True)
        if res.stats["iters"] < iters:
            continue
        Cp, mp = _pixel_lloyd(img.reshape(-1, 3), C0, iters)
        np.testing.assert_allclose(res.centers, Cp, rtol=0, atol=1e-12)
        # per-pixel membership equals the membership of the pixel's colour
        pix_keys = _keys_of(img).reshape(-1)
        lut = dict(zip(keys.tolist(), res.assign.tolist()))
        assert np.array_equal(np.array([lut[k] for k in pix_keys.tolist()]), mp)


def test_sse_identity_and_monotone():
    img = synth.smooth_field_blobs(96, 80, 3)
    keys, counts = oracle.histogram(img)
    X = _rgb_of(keys).astype(np.float64)
    C0, _ = oracle.init(keys, counts, 24, oracle.INIT_KMEANSPP, 3)
    trace = []
    C = C0
    for it in range(1, 9):
        res = oracle.kmeans(keys, counts, C0, it, 0.0, prune=True)
        if res.stats["iters"] < it:
            break
        direct = (counts * ((X - res.centers[res.assign]) ** 2).sum(1)).sum()
        assert res.sse_trace[-1] == pytest.approx(direct, rel=1e-12)
        trace = res.sse_trace
        C = res.centers
    assert len(trace) >= 4
    assert all(trace[i + 1] <= trace[i] * (1 + 1e-12) for i in range(len(trace) - 1))
    del C


def test_k1_closed_form():
    img = synth.blobs_on_gradient(16, 16, 9)
    keys, counts = oracle.histogram(img)
    X = _rgb_of(keys)
    res = oracle.kmeans(keys, counts, [[1.0, 2.0, 3.0]], 10, 1e-4, prune=True)
    N = int(counts.sum())
    S = [int((counts.astype(object) * X[:, c].astype(object)).sum()) for c in range(3)]
    Q = int((counts.astype(object) * (X.astype(object) ** 2).sum(1)).sum())
    for c in range(3):
        assert res.centers[0, c] == S[c] / N
    from fractions import Fraction
    sse = Fraction(Q) - Fraction(sum(s * s for s in S), N)
    assert res.sse_trace[0] == pytest.approx(float(sse), rel=1e-14)
    assert res.stats["iters"] == 2 and res.stats["converged"] == 1


def test_fewer_colours_than_k_gives_exact_palette():
    img = np.array([[[5, 6, 7], [200, 100, 0], [5, 6, 7]]], np.uint8)
    pal, idx, rgb, st = oracle.quantize(img, 8, oracle.INIT_KMEANSPP, 0, 20, 1e-4)
    assert st["k_used"] == 2 and st["mse_img"] == 0.0 and st["iters"] == 0
    assert np.array_equal(rgb, img)
    assert np.array_equal(pal[:2], [[5, 6, 7], [200, 100, 0]])


def test_two_separated_clusters_converge_to_cluster_means():
    rng = np.random.default_rng(4)
    a = rng.integers(0, 20, (200, 3))
    b = rng.integers(230, 256, (300, 3))
    img = np.concatenate([a, b]).reshape(20, 25, 3).astype(np.uint8)
    keys, counts = oracle.histogram(img)
    res = oracle.kmeans(keys, counts, [[0.0, 0.0, 0.0], [255.0, 255.0, 255.0]], 20, 0.0, True)
    np.testing.assert_array_equal(res.centers[0], a.mean(0))
    np.testing.assert_array_equal(res.centers[1], b.mean(0))


def test_matches_scikit_learn_lloyd_on_separated_data():
    sklearn_cluster = pytest.importorskip("sklearn.cluster")
    rng = np.random.default_rng(8)
    mus = np.array([[20, 30, 40], [200, 40, 60], [60, 210, 90], [100, 100, 230], [240, 240, 20]])
    pts = np.concatenate([np.clip(np.rint(m + 6 * rng.standard_normal((400, 3))), 0, 255)
                          for m in mus]).astype(np.uint8)
    keys, counts = oracle.histogram(pts.reshape(1, -1, 3))
    X = _rgb_of(keys).astype(np.float64)
    C0 = mus.astype(np.float64) + 3.0
    res = oracle.kmeans(keys, counts, C0, 3, 0.0, prune=True)
    km = sklearn_cluster.KMeans(n_clusters=5, init=C0, n_init=1, algorithm="lloyd",
                                max_iter=3, tol=0.0).fit(X, sample_weight=counts.astype(np.float64))
    np.testing.assert_allclose(res.centers, km.cluster_centers_, rtol=0, atol=1e-9)


def test_stopping_rule():
    img = synth.blobs_on_gradient(32, 32, 1)
    keys, counts = oracle.histogram(img)
    C0, _ = oracle.init(keys, counts, 8, oracle.INIT_MAXMIN, 1)
    one = oracle.kmeans(keys, counts, C0, 1, 1e-4, True)
    assert one.stats["iters"] == 1 and one.stats["converged"] == 0
    loose = oracle.kmeans(keys, counts, C0, 50, 1e9, True)
    assert loose.stats["iters"] == 2 and loose.stats["converged"] == 1
    tight = oracle.kmeans(keys, counts, C0, 500, 1e-4, True)
    tr = tight.sse_trace
    t = tight.stats["iters"]
    assert tight.stats["converged"] == 1
    assert (tr[t - 2] - tr[t - 1]) / tr[t - 1] <= 1e-4
    assert all((tr[i - 1] - tr[i]) / tr[i] > 1e-4 for i in range(1, t - 1))


def test_empty_cluster_keeps_centre():
    img = np.array([[[0, 0, 0], [2, 0, 0], [4, 0, 0]]], np.uint8)
    keys, counts = oracle.histogram(img)
    res = oracle.kmeans(keys, counts, [[2.0, 0, 0], [250.0, 250.0, 250.0]], 5, 0.0, True)
    assert np.array_equal(res.centers[1], [250.0, 250.0, 250.0])
    assert np.array_equal(res.assign, [0, 0, 0])


# ------------------------------------------------------------------------- map

def test_map_is_nearest_palette_entry_and_mse():
    img = synth.smooth_field_blobs(40, 56, 2)
    rng = np.random.default_rng(0)
    pal = rng.integers(0, 256, (20, 3)).astype(np.uint8)
    pal[7] = pal[3]  # duplicate entry: ties go to the lower index
    idx, rgb, err = oracle.map_image(img, pal)
    P = pal.astype(np.int64)
    X = img.reshape(-1, 3).astype(np.int64)
    D = ((X[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    assert np.array_equal(idx.reshape(-1), np.argmin(D, axis=1))
    assert np.array_equal(rgb, pal[idx])
    mse = ((img.astype(np.float64) - rgb.astype(np.float64)) ** 2).sum(-1).mean()  # Section 3.1
    assert err / (40 * 56) == pytest.approx(mse, rel=1e-15)


def test_quantize_end_to_end_small_config():
    img = synth.blobs_on_gradient(64, 64, 0)
    pal, idx, rgb, st = oracle.quantize(img, 16, oracle.INIT_MAXMIN, 0, 50, 1e-4, prune=False)
    assert st["k_used"] == 16 and 1 <= st["iters"] <= 50
    assert st["n_unique"] == len(np.unique(_keys_of(img)))
    mse = ((img.astype(np.float64) - rgb.astype(np.float64)) ** 2).sum(-1).mean()
    assert st["mse_img"] == pytest.approx(mse, rel=1e-15)
    psnr = 20 * math.log10(255 / math.sqrt(st["mse_img"]))
    assert 10 < psnr < 60
    again = oracle.quantize(img, 16, oracle.INIT_MAXMIN, 0, 50, 1e-4, prune=True)
    assert np.array_equal(again[0], pal) and again[3]["sse_final"] == st["sse_final"]


# ---------------------------------------------------------------- VAR and SFF
def _rand_colours(rng, n, max_count=5):
    keys = np.sort(rng.choice(1 << 24, size=n, replace=False)).astype(np.uint32)
    counts = rng.integers(1, max_count + 1, size=n).astype(np.uint32)
    return keys, counts


def _var_brute(keys, counts, K):
    """VAR of Section 2.3 on the expanded pixel list, in plain Python."""
    px = np.repeat(keys.astype(np.int64), counts.astype(np.int64))
    ch = [(px >> 16) & 255, (px >> 8) & 255, px & 255]
    N = len(px)
    scores = [N * int((c * c).sum()) - int(c.sum()) ** 2 for c in ch]
    c = max(range(3), key=lambda i: (scores[i], -i))  # largest; ties to the lower channel
    order = np.lexsort((px, ch[c]))  # by channel value, then key
    out = []
    for g in range(K):
        lo, hi = g * N // K, (g + 1) * N // K
        k = int(px[order[lo + (hi - lo - 1) // 2]])
        out.append([(k >> 16) & 255, (k >> 8) & 255, k & 255])
    return np.array(out, dtype=np.float64)


@pytest.mark.parametrize("seed", range(6))
def test_var_matches_pixel_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    keys, counts = _rand_colours(rng, 60)
    for K in (1, 2, 5, 7, 16, 59):
        got, used = oracle.init(keys, counts, K, oracle.INIT_VAR, 0)
        assert used == K
        assert np.array_equal(got, _var_brute(keys, counts, K)), K


def test_var_closed_form_single_channel():
    # R = 0..99 once each, G = B = 0: the groups of 25 pixels have lower
    # medians at R = 12, 37, 62, 87
    keys = (np.arange(100, dtype=np.uint32) << 16)
    counts = np.ones(100, dtype=np.uint32)
    got, _ = oracle.init(keys, counts, 4, oracle.INIT_VAR, 0)
    assert got[:, 0].tolist() == [12, 37, 62, 87] and not got[:, 1:].any()
    # weights move the medians: R = 0 holding 300 of 399 pixels takes 3 groups
    counts2 = counts.copy()
    counts2[0] = 300
    got2, _ = oracle.init(keys, counts2, 4, oracle.INIT_VAR, 0)
    assert got2[:, 0].tolist() == [0, 0, 0, 49]


def test_var_picks_the_widest_channel():
    rng = np.random.default_rng(5)
    r = rng.integers(0, 256, 200)
    g = rng.integers(100, 110, 200)
    b = rng.integers(50, 60, 200)
    keys, counts = np.unique((r << 16) | (g << 8) | b, return_counts=True)
    got, _ = oracle.init(keys.astype(np.uint32), counts.astype(np.uint32), 8, oracle.INIT_VAR, 0)
    assert np.all(np.diff(got[:, 0]) >= 0)  # the centres ascend along R


def test_sff_subset_size():
    for K in range(1, 257):
        want = max(K, math.ceil(2 * K * math.log(K)))
        assert oracle.sff_subset(K, 1 << 28) == want
        assert oracle.sff_subset(K, 50) == min(want, 50)
        # no 2 K ln K lies near an integer, so the ceiling does not depend on
        # the last bit of the logarithm
        v = 2 * K * math.log(K)
        assert K == 1 or abs(v - round(v)) > 1e-9


class _Stream:
    """The oracle's splitmix64 stream (pinned to the published sequence)."""

    def __init__(self, seed):
        import ctypes
        self.s = ctypes.c_uint64(seed)
        self.ctypes = ctypes

    def below(self, T):
        return int(oracle.lib().cqref_uniform_below(self.ctypes.byref(self.s), T))


def _sff_brute(keys, K, seed):
    n = len(keys)
    L = min(max(K, math.ceil(2 * K * math.log(K))), n)
    st = _Stream(seed)
    perm = list(range(n))
    for j in range(L):
        r = j + st.below(n - j)
        perm[j], perm[r] = perm[r], perm[j]
    sub = [int(keys[perm[s]]) for s in range(L)]
    rgb = [((k >> 16) & 255, (k >> 8) & 255, k & 255) for k in sub]
    d2 = [None] * L
    pick = st.below(L)
    out = []
    for j in range(K):
        if j > 0:
            best = max(d2)
            pick = d2.index(best)  # lowest subset position among the farthest
        out.append(list(rgb[pick]))
        for s in range(L):
            d = sum((a - b) ** 2 for a, b in zip(rgb[s], rgb[pick]))
            d2[s] = d if d2[s] is None else min(d2[s], d)
    return np.array(out, dtype=np.float64)


@pytest.mark.parametrize("seed", range(5))
def test_sff_matches_brute_force(seed):
    rng = np.random.default_rng(2000 + seed)
    keys, counts = _rand_colours(rng, 300)
    for K in (1, 2, 3, 8, 20):  # subsets of 1, 4, 7, 34 and 120 colours
        got, _ = oracle.init(keys, counts, K, oracle.INIT_SFF, 77 + seed)
        assert np.array_equal(got, _sff_brute(keys, K, 77 + seed)), K


def test_sff_centres_are_distinct_subset_colours():
    rng = np.random.default_rng(9)
    keys, counts = _rand_colours(rng, 5000)
    got, _ = oracle.init(keys, counts, 64, oracle.INIT_SFF, 3)
    ks = (got[:, 0].astype(np.int64) << 16) | (got[:, 1].astype(np.int64) << 8) | got[:, 2].astype(np.int64)
    assert len(set(ks.tolist())) == 64 and set(ks.tolist()) <= set(keys.tolist())


@pytest.mark.parametrize("seed", range(4))
def test_sff_ties_go_to_the_lowest_subset_position(seed):
    # a 3 x 3 x 3 lattice: farthest-first meets equal distances at every step
    v = np.array([0, 100, 200])
    keys = np.sort(((v[:, None, None] << 16) | (v[None, :, None] << 8) | v[None, None, :]).ravel()).astype(np.uint32)
    counts = np.ones(len(keys), dtype=np.uint32)
    for K in (4, 6):  # subsets of 12 and 22 of the 27 colours
        got, _ = oracle.init(keys, counts, K, oracle.INIT_SFF, seed)
        assert np.array_equal(got, _sff_brute(keys, K, seed)), K


# ---------------------------------------------------------------- 2:1 subsampling
@pytest.mark.parametrize("shape", [(7, 9), (8, 10), (1, 5), (33, 2)])
def test_subsampled_histogram_is_the_even_pixels(shape):
    rng = np.random.default_rng(sum(shape))
    img = rng.integers(0, 4, (shape[0], shape[1] + 3, 3)).astype(np.uint8) * 60  # padded rows
    view = img[:, : shape[1]]
    keys, counts = oracle.histogram(view, subsample=True)
    sub = view[::2, ::2].reshape(-1, 3).astype(np.int64)
    uk, uc = np.unique((sub[:, 0] << 16) | (sub[:, 1] << 8) | sub[:, 2], return_counts=True)
    assert np.array_equal(keys, uk) and np.array_equal(counts, uc)


def test_subsampled_quantize_clusters_the_even_pixels_and_maps_all():
    img = synth.blobs_on_gradient(41, 37, 2)
    pal, idx, rgb, st = oracle.quantize(img, 16, oracle.INIT_KMEANSPP, 5, 50, 1e-4, subsample=True)
    # the same clustering from the even pixels taken by slicing
    k2, c2 = oracle.histogram(np.ascontiguousarray(img[::2, ::2]))
    cen, _ = oracle.init(k2, c2, 16, oracle.INIT_KMEANSPP, 5)
    km = oracle.kmeans(k2, c2, cen, 50, 1e-4, True)
    assert np.array_equal(pal, km.palette)
    assert st["n_unique"] == len(k2) and st["iters"] == km.stats["iters"]
    # every pixel of the full image is mapped to its nearest palette entry
    X = img.reshape(-1, 3).astype(np.int64)
    D = ((X[:, None, :] - pal.astype(np.int64)[None, :, :]) ** 2).sum(-1)
    assert np.array_equal(idx.reshape(-1), np.argmin(D, axis=1))
    assert st["mse_img"] == pytest.approx(D.min(axis=1).mean(), rel=1e-12)


# ---------------------------------------------------------------- WU (greedy orthogonal bipartitioning)
def _cells_of(keys):
    k = keys.astype(np.int64)
    return np.stack([(k >> 19) & 31, (k >> 11) & 31, (k >> 3) & 31], 1)  # value >> 3 per channel


def _in_box(cells, box):
    lo, hi = np.asarray(box[:3]), np.asarray(box[3:])
    return np.all((cells >= lo) & (cells <= hi), axis=1)


def _sse_exact(keys, counts, mask):
    """Sum over the pixels of the squared distance to their weighted mean,
    as an exact fraction (the definition, from the colour list)."""
    from fractions import Fraction

    w = int(counts[mask].sum())
    if w == 0:
        return Fraction(0)
    rgb = _rgb_of(keys[mask]).astype(np.int64)
    n = counts[mask].astype(np.int64)
    mean = [Fraction(int((n * rgb[:, c]).sum()), w) for c in range(3)]
    return sum(int(ni) * sum((int(x[c]) - mean[c]) ** 2 for c in range(3)) for ni, x in zip(n, rgb))


def _cuts(box):
    for a in range(3):
        for c in range(box[a], box[3 + a]):
            lower, upper = list(box), list(box)
            lower[3 + a] = c
            upper[a] = c + 1
            yield lower, upper


def _wu_data(seed, n=160):
    rng = np.random.default_rng(seed)
    # clustered colours so that boxes differ clearly in spread
    centres = rng.integers(20, 236, size=(5, 3))
    pts = centres[rng.integers(0, 5, n)] + rng.normal(0, 18, (n, 3))
    pts = np.clip(np.rint(pts), 0, 255).astype(np.uint32)
    keys = np.unique((pts[:, 0] << 16) | (pts[:, 1] << 8) | pts[:, 2]).astype(np.uint32)
    counts = rng.integers(1, 6, len(keys)).astype(np.uint32)
    return keys, counts


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_wu_each_step_splits_the_worst_box_at_its_best_cut(seed):
    """Wu's greedy step from K to K + 1 boxes, checked with exact squared
    errors computed from the colours: the box that is split has the largest
    error among the boxes with an allowed cut, the lower part keeps its index
    and the upper part is appended, and the cut minimises the summed error of
    the two parts over every plane along every channel."""
    from fractions import Fraction

    keys, counts = _wu_data(seed)
    cells = _cells_of(keys)
    tol = Fraction(1, 10 ** 12)
    prev = oracle.wu_boxes(keys, counts, 1)
    assert prev.tolist() == [[0, 0, 0, 31, 31, 31]]
    for K in range(2, 14):
        cur = oracle.wu_boxes(keys, counts, K)
        assert len(cur) == len(prev) + 1
        changed = [j for j in range(len(prev)) if not np.array_equal(cur[j], prev[j])]
        assert len(changed) == 1
        j = changed[0]
        parent, lower, upper = prev[j].tolist(), cur[j].tolist(), cur[-1].tolist()
        assert (lower, upper) in [(lo, up) for lo, up in _cuts(parent)]
        # the split box: largest error among boxes that have an allowed cut
        def cuttable(box):
            return any(counts[_in_box(cells, lo)].sum() > 0 and counts[_in_box(cells, up)].sum() > 0
                       for lo, up in _cuts(box))
        errs = [_sse_exact(keys, counts, _in_box(cells, b)) if cuttable(b.tolist()) else Fraction(-1)
                for b in prev]
        assert errs[j] >= max(errs) * (1 - tol)
        # the cut: least summed error over all allowed cuts of the parent
        options = []
        for lo, up in _cuts(parent):
            ml, mu = _in_box(cells, lo), _in_box(cells, up)
            if counts[ml].sum() > 0 and counts[mu].sum() > 0:
                options.append(_sse_exact(keys, counts, ml) + _sse_exact(keys, counts, mu))
        got = _sse_exact(keys, counts, _in_box(cells, lower)) + _sse_exact(keys, counts, _in_box(cells, upper))
        assert got <= min(options) * (1 + tol)
        prev = cur


def test_wu_boxes_partition_the_grid_and_centres_are_box_means():
    from fractions import Fraction

    keys, counts = _wu_data(7, n=400)
    K = 24
    boxes = oracle.wu_boxes(keys, counts, K)
    assert len(boxes) == K
    grid = np.zeros((32, 32, 32), np.int32)
    for b in boxes:
        grid[b[0]:b[3] + 1, b[1]:b[4] + 1, b[2]:b[5] + 1] += 1
    assert (grid == 1).all()  # disjoint and covering
    cen, k_used = oracle.init(keys, counts, K, oracle.INIT_WU, 0)
    assert k_used == K
    cells = _cells_of(keys)
    rgb = _rgb_of(keys).astype(np.int64)
    for k, b in enumerate(boxes):
        m = _in_box(cells, b)
        w = int(counts[m].sum())
        assert w > 0
        for c in range(3):
            assert cen[k, c] == float(Fraction(int((counts[m].astype(np.int64) * rgb[m, c]).sum()), w))


def test_wu_one_box_is_the_weighted_mean_and_two_clusters_are_found():
    from fractions import Fraction

    keys, counts = _wu_data(3)
    cen, _ = oracle.init(keys, counts, 1, oracle.INIT_WU, 0)
    rgb = _rgb_of(keys).astype(np.int64)
    w = int(counts.sum())
    assert cen[0].tolist() == [float(Fraction(int((counts * rgb[:, c]).sum()), w)) for c in range(3)]
    # two tight, far-apart groups (more colours than K): K = 2 gives their means
    a = [(10 + i, 20, 30 + j) for i in range(3) for j in range(3)]
    b = [(200, 180 + i, 90 + j) for i in range(3) for j in range(3)]
    ks = np.array(sorted((r << 16) | (g << 8) | bl for r, g, bl in a + b), np.uint32)
    cs = np.ones(len(ks), np.uint32)
    cen, _ = oracle.init(ks, cs, 2, oracle.INIT_WU, 0)
    got = sorted(map(tuple, cen.tolist()))
    assert got == [(11.0, 20.0, 31.0), (200.0, 181.0, 91.0)]


def test_wu_with_fewer_occupied_cells_than_k_repeats_the_first_mean():
    # 12 colours in three cells (each cell's colours differ only below bit 3)
    ks = np.array(sorted(((8 * c) << 16) | (i << 8) | j for c in (1, 9, 20) for i in range(2) for j in range(2)),
                  np.uint32)
    cs = np.arange(1, len(ks) + 1, dtype=np.uint32)
    boxes = oracle.wu_boxes(ks, cs, 8)
    assert len(boxes) == 3
    cen, k_used = oracle.init(ks, cs, 8, oracle.INIT_WU, 0)
    assert k_used == 8
    assert all(cen[k].tolist() == cen[0].tolist() for k in range(3, 8))
    assert len({tuple(c) for c in cen[:3].tolist()}) == 3


def test_wu_ties_go_to_the_lower_channel_and_the_first_plane():
    # two colours mirrored in R and B: every plane between them along R or B
    # splits them with the same value (an exact tie in FP64: the same integer
    # sums), and G offers no cut
    ks = np.array(sorted([(40 << 16) | (100 << 8) | 200, (200 << 16) | (100 << 8) | 40]), np.uint32)
    cs = np.array([3, 3], np.uint32)
    boxes = oracle.wu_boxes(ks, cs, 2)
    assert boxes.tolist() == [[0, 0, 0, 5, 31, 31], [6, 0, 0, 31, 31, 31]]
    # G and B mirrored: G wins
    ks = np.array(sorted([(100 << 16) | (40 << 8) | 200, (100 << 16) | (200 << 8) | 40]), np.uint32)
    boxes = oracle.wu_boxes(ks, cs, 2)
    assert boxes.tolist() == [[0, 0, 0, 31, 5, 31], [0, 6, 0, 31, 31, 31]]
    # R and G mirrored: R wins
    ks = np.array(sorted([(40 << 16) | (200 << 8) | 100, (200 << 16) | (40 << 8) | 100]), np.uint32)
    boxes = oracle.wu_boxes(ks, cs, 2)
    assert boxes.tolist() == [[0, 0, 0, 5, 31, 31], [6, 0, 0, 31, 31, 31]]


# ---------------------------------------------------------------- LBG (splitting)
def _lbg_brute(keys, counts, K, eps=1.0, tol=0.001, max_iters=100):
    """LBG of Section 2.3 in plain Python: the centroid, then stages that
    split centre j into c_j - eps (kept) and c_j + eps (appended), each
    followed by weighted Lloyd iterations (FP64 centres S / n, nearest centre by
    FP64 distance with the lowest index on ties, empty clusters kept) until the
    relative SSE decrease, computed exactly, is at most tol."""
    from fractions import Fraction

    rgb = [tuple(int(v) for v in x) for x in _rgb_of(keys)]
    n = [int(c) for c in counts]
    N = sum(n)
    C = [[float(sum(w * x[c] for w, x in zip(n, rgb))) / float(N) for c in range(3)]]
    m = 1
    while m < K:
        split = m if 2 * m <= K else K - m
        for j in range(split):
            C.append([v + eps for v in C[j]])
            C[j] = [v - eps for v in C[j]]
        m += split
        prev = None
        for it in range(1, max_iters + 1):
            S = [[0, 0, 0] for _ in range(m)]
            Q = [0] * m
            W = [0] * m
            for w, x in zip(n, rgb):
                best, bd = 0, None
                for k in range(m):
                    dx, dy, dz = x[0] - C[k][0], x[1] - C[k][1], x[2] - C[k][2]
                    d = (dx * dx + dy * dy) + dz * dz
                    if bd is None or d < bd:
                        best, bd = k, d
                W[best] += w
                Q[best] += w * (x[0] ** 2 + x[1] ** 2 + x[2] ** 2)
                for c in range(3):
                    S[best][c] += w * x[c]
            for k in range(m):
                if W[k]:
                    C[k] = [float(S[k][c]) / float(W[k]) for c in range(3)]
            sse = sum(Fraction(W[k] * Q[k] - sum(v * v for v in S[k]), W[k]) for k in range(m) if W[k])
            if sse == 0 or (prev is not None and prev - sse <= Fraction(tol) * sse):
                break
            prev = sse
    return np.array(C, np.float64)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lbg_matches_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    keys, counts = _rand_colours(rng, 40, max_count=7)
    for K in (1, 2, 3, 5, 6, 7, 8):
        got, k_used = oracle.init(keys, counts, K, oracle.INIT_LBG, 0)
        assert k_used == K
        assert np.array_equal(got, _lbg_brute(keys, counts, K)), K


def test_lbg_one_centre_is_the_centroid_and_four_groups_are_found():
    from fractions import Fraction

    rng = np.random.default_rng(9)
    keys, counts = _rand_colours(rng, 30)
    got, _ = oracle.init(keys, counts, 1, oracle.INIT_LBG, 0)
    rgb = _rgb_of(keys).astype(np.int64)
    w = int(counts.sum())
    assert got[0].tolist() == [float(Fraction(int((counts * rgb[:, c]).sum()), w)) for c in range(3)]
    # four tight groups along the grey axis: the splits along (1, 1, 1) find them
    pts = [(v + i, v + j, v) for v in (20, 90, 160, 230) for i in range(2) for j in range(2)]
    ks = np.array(sorted((r << 16) | (g << 8) | b for r, g, b in pts), np.uint32)
    got, _ = oracle.init(ks, np.ones(len(ks), np.uint32), 4, oracle.INIT_LBG, 0)
    assert sorted(map(tuple, got.tolist())) == [(v + 0.5, v + 0.5, float(v)) for v in (20, 90, 160, 230)]


def test_lbg_split_of_a_single_colour_keeps_the_perturbed_centre():
    # an isolated colour forms its own cluster after the first stage; at the
    # second stage its two halves are equidistant from it, the kept half
    # (lower index) takes it and the appended half c + eps stays empty
    group = [(40 + i, 60 + j, 50) for i in range(4) for j in range(4)]
    lone = (230, 230, 230)
    ks = np.array(sorted((r << 16) | (g << 8) | b for r, g, b in group + [lone]), np.uint32)
    cs = np.ones(len(ks), np.uint32)
    got, _ = oracle.init(ks, cs, 4, oracle.INIT_LBG, 0)
    assert [231.0, 231.0, 231.0] in got.tolist()
    assert [230.0, 230.0, 230.0] in got.tolist()
    assert np.array_equal(got, _lbg_brute(ks, cs, 4))


# ---------------------------------------------------------------- DEN (density-based)
def _den_cell(k):
    k = int(k)
    return ((k >> 21) & 7) * 64 + ((k >> 13) & 7) * 8 + ((k >> 5) & 7)


def _den_brute(keys, K, seed):
    """DEN in plain Python: exact largest-remainder quotas over the 512 cells
    (unique colours as the points), then per cell in index order a partial
    Fisher-Yates over the cell's colours in key order."""
    from fractions import Fraction

    n = len(keys)
    cells = [[] for _ in range(512)]
    for k in keys:
        cells[_den_cell(k)].append(int(k))
    share = [Fraction(K * len(c), n) for c in cells]
    quota = [int(s) for s in share]  # floor
    left = K - sum(quota)
    order = sorted(range(512), key=lambda c: (-(share[c] - quota[c]), c))
    for c in order[:left]:
        quota[c] += 1
    st = _Stream(seed)
    out = []
    for c in range(512):
        lst = list(cells[c])
        for j in range(quota[c]):
            r = j + st.below(len(lst) - j)
            lst[j], lst[r] = lst[r], lst[j]
            out.append([(lst[j] >> 16) & 255, (lst[j] >> 8) & 255, lst[j] & 255])
    return np.array(out, np.float64), np.array(quota)


@pytest.mark.parametrize("seed", range(4))
def test_den_matches_brute_force(seed):
    rng = np.random.default_rng(200 + seed)
    keys, counts = _rand_colours(rng, 700)
    for K in (1, 7, 64, 256):
        got, k_used = oracle.init(keys, counts, K, oracle.INIT_DEN, seed)
        want, quota = _den_brute(keys, K, seed)
        assert k_used == K
        assert np.array_equal(oracle.den_quotas(keys, K), quota)
        assert np.array_equal(got, want), K


def test_den_quotas_follow_the_cell_populations():
    # colours in three cells holding 60 %, 30 % and 10 % of them
    rng = np.random.default_rng(5)
    ks = []
    for base, m in (((10, 10, 10), 60), ((200, 40, 40), 30), ((90, 220, 150), 10)):
        while sum(1 for k in ks if _den_cell(k) == _den_cell((base[0] << 16) | (base[1] << 8) | base[2])) < m:
            r, g, b = (int(v) for v in np.array(base) + rng.integers(0, 20, 3))
            k = (r << 16) | (g << 8) | b
            if k not in ks and _den_cell(k) == _den_cell((base[0] << 16) | (base[1] << 8) | base[2]):
                ks.append(k)
    keys = np.array(sorted(ks), np.uint32)
    q = oracle.den_quotas(keys, 10)
    assert sorted(q[q > 0].tolist()) == [1, 3, 6] and q.sum() == 10
    # 7 centres: shares 4.2, 2.1, 0.7 -> floors 4, 2, 0 and the one left to the
    # largest remainder (0.7)
    q = oracle.den_quotas(keys, 7)
    assert sorted(q[q > 0].tolist()) == [1, 2, 4]
    cen, _ = oracle.init(keys, np.ones(len(keys), np.uint32), 7, oracle.INIT_DEN, 3)
    assert len({tuple(c) for c in cen.tolist()}) == 7  # distinct colours
    ckeys = [(int(r) << 16) | (int(g) << 8) | int(b) for r, g, b in cen]
    assert all(k in set(keys.tolist()) for k in ckeys)


def test_scaling_every_count_by_a_power_of_two_scales_only_the_sse():
    """Section 2.2's weighted means do not change when every pixel count is
    multiplied by the same factor, and each SSE term is multiplied by it.  With
    a factor of 16 the scaling is exact in floating point, so an image tiled
    4 x 4 gives the same centres, memberships, NDC and near ties as the tile,
    an SSE trace exactly 16 times larger, and the same stopping iteration."""
    base = synth.smooth_field_blobs(48, 40, 3)
    bk, bc = oracle.histogram(base)
    tk, tc = oracle.histogram(np.tile(base, (4, 4, 1)))
    assert np.array_equal(tk, bk) and np.array_equal(tc, bc * np.uint32(16))
    c0, _ = oracle.init(bk, bc, 24, oracle.INIT_FORGY, 1)
    for prune in (False, True):
        a = oracle.kmeans(bk, bc, c0, 100, 1e-4, prune)
        b = oracle.kmeans(tk, tc, c0, 100, 1e-4, prune)
        assert np.array_equal(a.centers, b.centers) and np.array_equal(a.assign, b.assign)
        assert np.array_equal(np.array(a.sse_trace) * 16.0, np.array(b.sse_trace))
        for key in ("iters", "converged", "ndc_total", "near_ties", "mse_float"):
            assert a.stats[key] == b.stats[key], key


def _sq_dist(a, b):
    """Squared FP64 distances between the rows of a and b, (dx dx + dy dy) + dz dz."""
    d = a[:, None, :] - b[None, :, :]
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


@pytest.mark.parametrize("seed,K", [(0, 8), (1, 16), (2, 32), (3, 12)])
def test_sort_means_ndc_is_the_count_of_centres_within_twice_the_distance(seed, K):
    """Section 2.2 counts, per colour and sort-means iteration, the centres
    that are no more than twice as far from the colour's previous centre as
    the colour itself (that centre included); the first iteration compares
    every colour with all K centres.  A separate dense Lloyd in numpy (argmin
    with the lowest index on ties, weighted means from integer sums, empty
    clusters kept) gives the same memberships and centres as the oracle's
    pruned run, and those counts, with the bound's 1e-12 relative slack, sum
    to its NDC."""
    img = synth.blobs_on_gradient(40, 48, seed)
    keys, counts = oracle.histogram(img)
    c0, _ = oracle.init(keys, counts, K, oracle.INIT_KMEANSPP, seed)
    c0 = np.array(c0, np.float64).reshape(-1, 3)
    if seed == 3:
        c0[K - 1] = c0[0]  # coincident centres: distance 0 in the table
    r = oracle.kmeans(keys, counts, c0, 12, 0.0, True)
    X = np.stack([(keys >> 16) & 255, (keys >> 8) & 255, keys & 255], -1).astype(np.float64)
    w = counts.astype(np.int64)
    C = c0.copy()
    prev_assign = None
    ndc = 0
    for it in range(1, r.stats["iters"] + 1):
        D = _sq_dist(X, C)
        A = np.argmin(D, axis=1)
        if it == 1:
            ndc += len(keys) * K
        else:
            prev = D[np.arange(len(keys)), prev_assign]
            limit = 4.0 * prev * (1.0 + 1e-12)
            DC = _sq_dist(C, C)
            within = DC[prev_assign] <= limit[:, None]
            within[np.arange(len(keys)), prev_assign] = False
            ndc += int((1 + within.sum(axis=1)).sum())
        Xi = X.astype(np.int64)
        for k in range(K):
            m = A == k
            n = int(w[m].sum())
            if n:
                C[k] = (w[m][:, None] * Xi[m]).sum(axis=0).astype(np.float64) / float(n)
        prev_assign = A
    assert np.array_equal(A, r.assign)
    assert np.array_equal(C, r.centers)
    assert ndc == r.stats["ndc_total"]
    assert ndc < r.stats["iters"] * len(keys) * K


# ---------------------------------------------------------------- near ties

def _near_tie_count(evaluated):
    """Rows of evaluated distances (inf where not evaluated): a row is a near
    tie when it has two finite entries or more and its two smallest (of the
    multiset, so an exact repeat counts) differ by at most 1e-5 of the
    second."""
    s = np.sort(evaluated, axis=1)
    d1, d2 = s[:, 0], s[:, 1]
    return int(((d2 != np.inf) & ((d2 - d1) <= 1e-5 * d2)).sum())


def _lattice_image(seed, H=40, W=48, step=64):
    """60 colours on a lattice of spacing `step` per channel, each moved by
    at most 1 per channel: many colours sit exactly half-way between two
    lattice colours, so the first full search meets exact distance ties."""
    rng = np.random.default_rng(seed)
    base = rng.choice(np.arange(0, 256, step), size=(60, 3))
    img = base[rng.integers(0, 60, H * W)] + rng.integers(-1, 2, (H * W, 3))
    return np.clip(img, 0, 255).reshape(H, W, 3).astype(np.uint8)


@pytest.mark.parametrize("seed,K,prune,lattice", [(0, 8, True, True), (1, 16, True, True), (2, 16, False, True),
                                                  (3, 8, False, True), (4, 24, True, False),
                                                  (5, 12, True, False)])
def test_near_tie_count_matches_brute_force(seed, K, prune, lattice):
    """The near-tie count is, per colour and iteration, whether the two
    smallest distances the search evaluated differ by at most 1e-5 relative:
    all K in a full search, and in a sort-means pass the previous centre and
    every centre within twice its distance (the evaluated set of Section 2.2,
    counted as in the NDC pin below).  A separate dense numpy Lloyd supplies
    the centres of every iteration; the count is recomputed from the sorted
    rows of evaluated distances."""
    img = _lattice_image(seed) if lattice else synth.blobs_on_gradient(40, 48, seed)
    keys, counts = oracle.histogram(img)
    c0, _ = oracle.init(keys, counts, K, oracle.INIT_KMEANSPP, seed)
    c0 = np.array(c0, np.float64).reshape(-1, 3)
    if not lattice:
        c0[K - 1] = c0[0]  # coincident centres: an exact tie in every first-iteration row
    r = oracle.kmeans(keys, counts, c0, 12, 0.0, prune)
    X = np.stack([(keys >> 16) & 255, (keys >> 8) & 255, keys & 255], -1).astype(np.float64)
    Xi = X.astype(np.int64)
    w = counts.astype(np.int64)
    C = c0.copy()
    prev_assign = None
    ties = 0
    rows = np.arange(len(keys))
    for it in range(1, r.stats["iters"] + 1):
        D = _sq_dist(X, C)
        A = np.argmin(D, axis=1)
        if it == 1 or not prune:
            ties += _near_tie_count(D)
        else:
            prev = D[rows, prev_assign]
            within = _sq_dist(C, C)[prev_assign] <= (4.0 * prev * (1.0 + 1e-12))[:, None]
            within[rows, prev_assign] = True
            ties += _near_tie_count(np.where(within, D, np.inf))
        for k in range(K):
            m = A == k
            n = int(w[m].sum())
            if n:
                C[k] = (w[m][:, None] * Xi[m]).sum(axis=0).astype(np.float64) / float(n)
        prev_assign = A
    assert np.array_equal(A, r.assign) and np.array_equal(C, r.centers)
    assert ties > 0  # the pin must see near ties to mean anything
    assert ties == r.stats["near_ties"]


def test_near_tie_in_a_sort_means_pass_at_a_fixed_point():
    """Centres at red 40 and 120 are the means of their clusters (colours 0
    and 80 once each and 40 ten times; 120 ten times), so they never move.
    Colour 80 is at distance 1600 from both: an exact tie in the full first
    iteration, and again in the sort-means pass of iteration 2, whose bound
    4 x 1600 admits centre 1 (at 6400 from centre 0).  The run stops at
    iteration 2 (no SSE drop, tol 0), with one near tie per iteration."""
    keys = np.array([0, 40 << 16, 80 << 16, 120 << 16], np.uint32)
    counts = np.array([1, 10, 1, 10], np.uint32)
    for prune in (False, True):
        r = oracle.kmeans(keys, counts, [[40, 0, 0], [120, 0, 0]], 10, 0.0, prune)
        assert list(r.assign) == [0, 0, 0, 1] and r.stats["iters"] == 2
        assert np.array_equal(r.centers, [[40, 0, 0], [120, 0, 0]])
        assert r.stats["near_ties"] == 2
        # iteration 2: colours 0 and 80 also evaluate centre 1 (6400 <= 4 x 1600)
        assert r.stats["ndc_total"] == (8 + 2 + 1 + 2 + 1 if prune else 16)


def test_near_ties_of_exact_ties_and_a_lone_centre():
    """Closed cases: a colour equidistant from two centres is a near tie in
    every full search; with K = 1 no second distance exists, so none is."""
    keys = np.array([0x000000, 0x0A0000, 0x140000], np.uint32)  # r = 0, 10, 20
    counts = np.array([1, 5, 1], np.uint32)
    # centres 0 and 20: colour 10 is at 100 from both, the others at 0 and 400
    r = oracle.kmeans(keys, counts, [[0, 0, 0], [20, 0, 0]], 1, 0.0, prune=False)
    assert r.stats["near_ties"] == 1 and list(r.assign) == [0, 0, 1]
    r1 = oracle.kmeans(keys, counts, [[10, 0, 0]], 5, 0.0, prune=True)
    assert r1.stats["near_ties"] == 0


# ------------------------------------------------------------ palette rounding

def test_palette_rounds_exact_halves_up():
    """The palette is floor(c + 0.5): a centre exactly half-way between two
    integers goes up (round half to even would send 0.5, 2.5, ... down).  Two
    colours (v, v, v) and (v + 1, v + 1, v + 1) with equal counts have the
    exact mean v + 0.5 under K = 1."""
    for v in range(0, 255):
        keys = np.array([v * 0x010101, (v + 1) * 0x010101], np.uint32)
        counts = np.array([3, 3], np.uint32)
        r = oracle.kmeans(keys, counts, [[0, 0, 0]], 2, 0.0, prune=False)
        assert r.centers[0, 0] == v + 0.5
        assert list(r.palette[0]) == [v + 1] * 3, v
    # just below a half stays down: (v, v + 1) with counts 2 : 1 is v + 1/3
    keys = np.array([0x020202, 0x030303], np.uint32)
    r = oracle.kmeans(keys, np.array([2, 1], np.uint32), [[0, 0, 0]], 2, 0.0, prune=False)
    assert list(r.palette[0]) == [2, 2, 2]
    # through the whole quantizer: a 1 x 2 image of those two colours, K = 1
    img = np.array([[[4, 4, 4], [5, 5, 5]]], np.uint8)
    pal, idx, _, st = oracle.quantize(img, 1, oracle.INIT_FORGY, 0, 5, 0.0, prune=False)
    assert list(pal[0]) == [5, 5, 5] and st["mse_img"] == 0.5 * 3


# --------------------------------------------------------- rejection sampling

def _uniform_below_reference(raw, T):
    """Rejection sampling from its definition with Python integers: the 2^64
    raw outputs split into floor(2^64 / T) whole copies of [0, T) from the
    top, and the 2^64 mod T lowest outputs are redrawn.  Yields (value, raw
    outputs consumed) per draw."""
    reject_below = (1 << 64) % T
    used = 0
    for r in raw:
        used += 1
        if r >= reject_below:
            yield r % T, used
            used = 0


@pytest.mark.parametrize("T", [(1 << 63) + 1, (1 << 63) + 12345, 3 << 62, (1 << 64) - 1, 7, 1000003])
def test_uniform_below_rejects_exactly_the_low_band(T):
    """Values of uniform_below on the pinned splitmix64 stream equal
    rejection sampling computed from the published raw outputs.  Above 2^63
    almost half of the outputs are redrawn, so a plain r mod T (or a wrong
    threshold) gives a different sequence after the first rejection."""
    seed, n = 99, 400
    raw = oracle.splitmix64(seed, 4 * n)
    ref = list(_uniform_below_reference(raw, T))[:n]
    assert len(ref) == n
    got = oracle.uniform_below(seed, T, n)
    assert got == [v for v, _ in ref]
    rejected = sum(u - 1 for _, u in ref)
    if T > (1 << 63) and T < (1 << 64) - 1:
        assert rejected > n // 4  # the band is large: many redraws happened
        assert got != [r % T for r in raw[:n]]
