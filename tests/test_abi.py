"""CPU-side checks of the C-ABI library: it loads, exports every entry point
declared in include/cq.h, sizes workspaces, and rejects invalid arguments
before touching a device."""
import ctypes
import os
import re

import pytest

from paper_1101_0395_amd import cq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "cq.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(cq_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = cq.lib()
    names = _declared()
    assert set(names) == set(cq.EXPORTS)
    for name in names:
        assert hasattr(L, name), name


def test_workspace_bytes():
    L = cq.lib()
    small = L.cq_workspace_bytes(64, 64, 16)
    big = L.cq_workspace_bytes(4096, 4096, 256)
    assert small > (1 << 24)  # the 2^24-entry byte colour table
    assert big > small
    # per pixel: a work region of two 8-byte records per colour (it also holds
    # the histogram's 6 bytes per pixel) plus keys, counts and memberships (9)
    assert big - small >= 24 * (4096 * 4096 - 64 * 64)
    for bad in [(0, 5, 16), (5, 0, 16), (5, 5, 0), (5, 5, 257), (1 << 15, 1 << 14, 16)]:
        assert L.cq_workspace_bytes(*bad) == 0


def _status(fn, *args):
    rc = fn(*args)
    return rc, cq.lib().cq_last_error().decode()


def test_invalid_arguments_are_rejected_without_a_device():
    L = cq.lib()
    fake = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first
    n = ctypes.c_int64(0)
    # null image
    rc, msg = _status(L.cq_histogram, None, 4, 4, 12, fake, fake, 16, ctypes.byref(n), fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL and "img" in msg
    # stride below 3 W
    rc, msg = _status(L.cq_histogram, fake, 4, 4, 11, fake, fake, 16, ctypes.byref(n), fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL and "stride" in msg
    # workspace too small / misaligned / null
    rc, msg = _status(L.cq_histogram, fake, 4, 4, 12, fake, fake, 16, ctypes.byref(n), fake, 1024, None)
    assert rc == cq.CQ_EWORKSPACE
    rc, msg = _status(L.cq_histogram, fake, 4, 4, 12, fake, fake, 16, ctypes.byref(n),
                      ctypes.c_void_p(0x10001), 1 << 30, None)
    assert rc == cq.CQ_EWORKSPACE and "aligned" in msg
    rc, msg = _status(L.cq_workspace_prepare, None, 1 << 30, None)
    assert rc == cq.CQ_EWORKSPACE
    # K out of range
    k_used = ctypes.c_int32(0)
    for K in (0, 257):
        rc, msg = _status(L.cq_init, fake, fake, 10, K, 2, 0, fake, ctypes.byref(k_used), fake, 1 << 30, None)
        assert rc == cq.CQ_EINVAL and "K" in msg
    # unknown init scheme
    rc, msg = _status(L.cq_init, fake, fake, 10, 4, 9, 0, fake, ctypes.byref(k_used), fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL
    # k-means: bad tol, bad max_iters, null assign
    st = cq.CqStats()
    rc, _ = _status(L.cq_kmeans, fake, fake, 10, 4, fake, 10, -1.0, 1, fake, None, None, ctypes.byref(st),
                    fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL
    rc, _ = _status(L.cq_kmeans, fake, fake, 10, 4, fake, 10, float("nan"), 1, fake, None, None,
                    ctypes.byref(st), fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL
    rc, _ = _status(L.cq_kmeans, fake, fake, 10, 4, fake, 0, 1e-4, 1, fake, None, None, ctypes.byref(st),
                    fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL
    rc, _ = _status(L.cq_kmeans, fake, fake, 10, 4, fake, 10, 1e-4, 1, None, None, None, ctypes.byref(st),
                    fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL
    # map: squared error requested without counts
    err = ctypes.c_uint64(0)
    rc, msg = _status(L.cq_map, fake, 4, 4, 12, fake, None, 3, fake, 4, fake, None, ctypes.byref(err),
                      fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL and "counts" in msg
    # quantize: user init is not a quantize scheme; oversize image
    rc, _ = _status(L.cq_quantize, fake, 4, 4, 12, 4, 3, 0, 10, 1e-4, 1, fake, None, None,
                    ctypes.byref(st), fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL
    rc, _ = _status(L.cq_quantize, fake, 1 << 15, 1 << 14, 3 << 14, 4, 2, 0, 10, 1e-4, 1, fake, None,
                    None, ctypes.byref(st), fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1101_0395_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                with open(os.path.join(dirpath, f)) as fh:
                    text = fh.read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "cqref" not in text, f
