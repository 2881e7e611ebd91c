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
    rc, msg = _status(L.cq_histogram, None, 4, 4, 12, 0, fake, fake, 16, ctypes.byref(n), fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL and "img" in msg
    # stride below 3 W
    rc, msg = _status(L.cq_histogram, fake, 4, 4, 11, 0, fake, fake, 16, ctypes.byref(n), fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL and "stride" in msg
    # workspace too small / misaligned / null
    rc, msg = _status(L.cq_histogram, fake, 4, 4, 12, 0, fake, fake, 16, ctypes.byref(n), fake, 1024, None)
    assert rc == cq.CQ_EWORKSPACE
    rc, msg = _status(L.cq_histogram, fake, 4, 4, 12, 0, fake, fake, 16, ctypes.byref(n),
                      ctypes.c_void_p(0x10001), 1 << 30, None)
    assert rc == cq.CQ_EWORKSPACE and "aligned" in msg
    # subsample flag other than 0 or 1
    rc, msg = _status(L.cq_histogram, fake, 4, 4, 12, 2, fake, fake, 16, ctypes.byref(n), fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL and "subsample" in msg
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
    rc, _ = _status(L.cq_quantize, fake, 4, 4, 12, 0, 4, 3, 0, 10, 1e-4, 1, fake, None, None,
                    ctypes.byref(st), fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL
    rc, _ = _status(L.cq_quantize, fake, 1 << 15, 1 << 14, 3 << 14, 0, 4, 2, 0, 10, 1e-4, 1, fake, None,
                    None, ctypes.byref(st), fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL


def test_empty_inputs_are_rejected_without_a_device():
    """An image with no pixels, a histogram with no colours and a batch with
    no jobs are argument errors, reported before any device work."""
    L = cq.lib()
    fake = ctypes.c_void_p(0x10000)
    n = ctypes.c_int64(0)
    st = cq.CqStats()
    k_used = ctypes.c_int32(0)
    err = ctypes.c_uint64(0)
    for H, W in ((0, 4), (4, 0), (-1, 4)):
        rc, msg = _status(L.cq_histogram, fake, H, W, 12, 0, fake, fake, 16, ctypes.byref(n), fake, 1 << 30, None)
        assert rc == cq.CQ_EINVAL and "positive" in msg, (H, W, msg)
        rc, _ = _status(L.cq_pixel_keys, fake, H, W, 12, fake, fake, None)
        assert rc == cq.CQ_EINVAL, (H, W)
        rc, _ = _status(L.cq_map, fake, H, W, 12, fake, fake, 3, fake, 4, fake, None, ctypes.byref(err),
                        fake, 1 << 30, None)
        assert rc == cq.CQ_EINVAL, (H, W)
        rc, _ = _status(L.cq_quantize, fake, H, W, 12, 0, 4, 2, 0, 10, 1e-4, 1, fake, None, None,
                        ctypes.byref(st), fake, 1 << 30, None)
        assert rc == cq.CQ_EINVAL, (H, W)
    rc, msg = _status(L.cq_init, fake, fake, 0, 4, 2, 0, fake, ctypes.byref(k_used), fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL and "n_unique" in msg
    rc, msg = _status(L.cq_kmeans, fake, fake, 0, 4, fake, 10, 1e-4, 1, fake, None, None, ctypes.byref(st),
                      fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL and "n_unique" in msg
    rc, msg = _status(L.cq_quantize_batch, None, 0, None, fake, 1 << 30, None)
    assert rc == cq.CQ_EINVAL and "n_jobs" in msg


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1101_0395_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                with open(os.path.join(dirpath, f)) as fh:
                    text = fh.read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "cqref" not in text, f


def test_engine_sizes_and_argument_checks_without_a_device():
    """Engine calls that do no device work: sizing, creation over a workspace
    that is never dereferenced, submission checks, step argument checks."""
    L = cq.lib()
    job_small = L.cq_engine_job_bytes(64, 64)
    job_big = L.cq_engine_job_bytes(512, 512)
    assert job_small % 256 == 0 and job_big > job_small > (1 << 24)
    assert L.cq_engine_job_bytes(0, 4) == 0 and L.cq_engine_job_bytes(1 << 15, 1 << 14) == 0
    head = L.cq_engine_workspace_bytes(4, 0)
    assert head > 0 and L.cq_engine_workspace_bytes(4, 1000) == head + 1024
    assert L.cq_engine_workspace_bytes(0, 0) == 0 and L.cq_engine_workspace_bytes(4097, 0) == 0

    ws = ctypes.c_void_p(1 << 40)  # aligned, never dereferenced by these calls
    h = ctypes.c_void_p()
    rc, msg = _status(L.cq_engine_create, 4, ws, head - 1, None, ctypes.byref(h))
    assert rc == cq.CQ_EWORKSPACE
    rc, msg = _status(L.cq_engine_create, 0, ws, head, None, ctypes.byref(h))
    assert rc == cq.CQ_EINVAL
    pool = 2 * job_small + job_small // 2  # room for two 64x64 jobs
    rc, msg = _status(L.cq_engine_create, 4, ws, head + pool, None, ctypes.byref(h))
    assert rc == cq.CQ_OK and h.value
    try:
        fake = ctypes.c_void_p(0x10000)
        job = cq.CqJob(fake, 64, 64, 192, 16, cq.INIT_KMEANSPP, 1, 10, 1e-4, 1, fake, None, None)
        t = ctypes.c_int64()
        for expect in (1, 2, 3):
            assert L.cq_engine_submit(h, ctypes.byref(job), ctypes.byref(t)) == cq.CQ_OK
            assert t.value == expect
        big = cq.CqJob(fake, 2048, 2048, 6144, 16, cq.INIT_KMEANSPP, 1, 10, 1e-4, 1, fake, None, None)
        rc, msg = _status(L.cq_engine_submit, h, ctypes.byref(big), ctypes.byref(t))
        assert rc == cq.CQ_ECAPACITY and "pool" in msg
        bad = cq.CqJob(fake, 64, 64, 192, 300, cq.INIT_KMEANSPP, 1, 10, 1e-4, 1, fake, None, None)
        rc, msg = _status(L.cq_engine_submit, h, ctypes.byref(bad), ctypes.byref(t))
        assert rc == cq.CQ_EINVAL and "K" in msg
        bad = cq.CqJob(fake, 64, 64, 192, 16, cq.INIT_KMEANSPP, 1, 10, 1e-4, 1, fake, None, None, -1)
        rc, msg = _status(L.cq_engine_submit, h, ctypes.byref(bad), ctypes.byref(t))
        assert rc == cq.CQ_EINVAL and "subsample" in msg
        q, r, u = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        assert L.cq_engine_pending(h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(u)) == cq.CQ_OK
        assert (q.value, r.value, u.value) == (3, 0, 0)  # admission happens in a step
        done = (cq.CqEngineDone * 4)()
        n = ctypes.c_int32()
        rc, msg = _status(L.cq_engine_step, h, 8, done, 3, ctypes.byref(n))
        assert rc == cq.CQ_EINVAL and "capacity" in msg
        rc, msg = _status(L.cq_engine_step, h, -1, done, 4, ctypes.byref(n))
        assert rc == cq.CQ_EINVAL and "iters" in msg
    finally:
        L.cq_engine_destroy(h)
    L.cq_engine_destroy(None)


def test_schedule_table_round_trip_and_checks_without_a_device():
    """cq_set_schedule / cq_get_schedule: a valid table is stored as given, an
    invalid one is refused and leaves the table as it was, and n = 0
    restores the built-in table."""
    builtin = cq.get_schedule()
    assert builtin[0][0] == 0 and all(a[0] < b[0] for a, b in zip(builtin, builtin[1:]))
    try:
        cq.set_schedule([(0, 512, 3), (1000, 8192, 1)])
        assert cq.get_schedule() == [(0, 512, 3), (1000, 8192, 1)]
        for bad in ([(5, 1024, 1)],                      # first entry not at 0
                    [(0, 1024, 1), (0, 2048, 1)],        # not increasing
                    [(0, 1000, 1)],                      # not a multiple of 256
                    [(0, 65536, 1)],                     # above 32768
                    [(0, 1024, 0)]):                     # period below 1
            with pytest.raises(cq.CqError) as e:
                cq.set_schedule(bad)
            assert e.value.code == cq.CQ_EINVAL
            assert cq.get_schedule() == [(0, 512, 3), (1000, 8192, 1)]
    finally:
        cq.set_schedule([])
    assert cq.get_schedule() == builtin


def test_builtin_schedule_is_the_tuned_table():
    """The library's built-in schedule is the table the autotuner wrote
    (paper_1101_0395_amd/schedule.json), and every tuned workload's
    measured best is the entry that its colour count selects."""
    import json
    with open(os.path.join(ROOT, "paper_1101_0395_amd", "schedule.json")) as f:
        tuned = json.load(f)
    cq.set_schedule([])
    table = [tuple(e) for e in tuned["table"]]
    assert cq.get_schedule() == table
    for r in tuned["results"]:
        chosen = [e for e in table if e[0] <= r["colours"]][-1]
        best = min(r["ms"], key=r["ms"].get)
        assert (chosen[1], chosen[2]) == tuple(int(v) for v in best.split(",")), r["workload"]
