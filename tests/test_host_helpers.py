"""Host-side checks of arithmetic helpers shared by the HIP kernels (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1101_0395_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_mod_u64_matches_integer_remainder(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    exe = tmp_path / "mod_check"
    src = os.path.join(ROOT, "tests", "host", "mod_u64_check.cpp")
    subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-std=c++17", "-O2", "-I", CSRC, src, "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 mismatches" in out.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_engine_pool_allocator_matches_byte_map_model(tmp_path):
    exe = tmp_path / "pool_check"
    src = os.path.join(ROOT, "tests", "host", "pool_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O2", "-I", CSRC, src, "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert " 0 mismatches" in out.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_cooperative_init_launch_plan(tmp_path):
    exe = tmp_path / "coop_plan_check"
    src = os.path.join(ROOT, "tests", "host", "coop_plan_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O2", "-I", CSRC, src, "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_public_structs_match_binding_layout(tmp_path):
    import ctypes

    from paper_1101_0395_amd import cq

    exe = tmp_path / "struct_layout"
    src = os.path.join(ROOT, "tests", "host", "struct_layout.c")
    subprocess.run(["gcc", "-std=c11", "-O0", "-I", os.path.join(ROOT, "include"), src, "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60, check=True).stdout
    py = {"cq_job": cq.CqJob, "cq_stats": cq.CqStats, "cq_engine_done": cq.CqEngineDone,
          "cq_schedule": cq.CqSchedule}
    seen = 0
    for line in out.splitlines():
        name, field, value = line.split()
        want = ctypes.sizeof(py[name]) if field == "size" else getattr(py[name], field).offset
        assert int(value) == want, line
        seen += 1
    assert seen == 24
