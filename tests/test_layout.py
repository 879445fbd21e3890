"""The bricked mesh layout and the walk's dilated-integer cell steps, checked on
the host: tests/layout/dilated_steps.cpp is compiled against the library's own
qrt_walk.h (host side of its __host__ __device__ helpers) and run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2406_15632_amd", "csrc")


def test_dilated_steps_match_brick_index(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc):
        pytest.fail("hipcc is needed to compile the layout check")
    exe = tmp_path / "dilated_steps"
    cmd = [hipcc, "-x", "hip", "--offload-host-only", "-O1", "-I", CSRC,
           os.path.join(ROOT, "tests", "layout", "dilated_steps.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok "), out.stdout
    assert int(out.stdout.split()[1]) > 100000


def test_walk_block_order_is_a_block_preserving_bijection(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc):
        pytest.fail("hipcc is needed to compile the block-order check")
    exe = tmp_path / "block_order"
    cmd = [hipcc, "-x", "hip", "--offload-host-only", "-O1", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "layout", "block_order.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok 14", out.stdout
