"""The allocation-free entry point cq_quantize_noalloc, through the C ABI,
against cq_quantize on a caller workspace: two calls in a row, the second on a
smaller image (the fixed scratch keeps the first call's contents), each equal
to cq_quantize bit for bit; and an image above its 2^20-pixel limit refused."""
import numpy as np
import pytest

from paper_1101_0395_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _one(cqm, dev, H, W, K, scheme, seed):
    print(f"noalloc {H}x{W} K={K} scheme={scheme}", flush=True)
    img = torch.from_numpy(synth.smooth_field_blobs(H, W, seed)).to(dev)
    ws = cqm.Workspace(H, W, K, dev)
    rp, ri, rr, rs = cqm.cq_quantize(img, K, scheme, seed, 100, 1e-4, True, ws)
    pal = torch.zeros((K, 3), dtype=torch.uint8, device=dev)
    idx = torch.empty((H, W), dtype=torch.uint8, device=dev)
    rgb = torch.empty((H, W, 3), dtype=torch.uint8, device=dev)
    st = cqm.cq_quantize_noalloc(img, K, scheme, seed, 100, 1e-4, True, pal, idx, rgb)
    assert torch.equal(pal, rp) and torch.equal(idx, ri) and torch.equal(rgb, rr)
    assert st == rs


def test_noalloc_matches_quantize_twice_second_smaller(cqm, dev):
    _one(cqm, dev, 1024, 1024, 256, cqm.INIT_KMEANSPP, 3)   # the largest image it takes
    _one(cqm, dev, 300, 211, 64, cqm.INIT_MAXMIN, 4)        # then a smaller one over the same scratch
    _one(cqm, dev, 97, 13, 16, cqm.INIT_LBG, 5)             # LBG stages stage through the same host area


def test_noalloc_rejects_images_beyond_its_scratch(cqm, dev):
    img = torch.zeros((1025, 1024, 3), dtype=torch.uint8, device=dev)
    pal = torch.zeros((16, 3), dtype=torch.uint8, device=dev)
    with pytest.raises(cqm.CqError) as e:
        cqm.cq_quantize_noalloc(img, 16, cqm.INIT_KMEANSPP, 0, 10, 1e-4, True, pal, None, None)
    assert e.value.code == cqm.CQ_EINVAL and "pixels" in str(e.value)
