"""CPU check of the batch planner's device layout (no device needed).

Compiles tests/batch_layout_harness.cpp against the built library and runs it:
every table and packed-mask region of a batch must lie inside the buffer the
plan sizes, including for batches with many work items (a plan once omitted
the work-item table from its size, so the masks ran past the allocation).
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1810_02612_amd")


def test_batch_layout_stays_inside_its_buffer(tmp_path):
    lib = os.path.join(PKG, "liblbl.so")
    if not os.path.exists(lib):
        pytest.skip("library not built")
    exe = str(tmp_path / "harness")
    cmd = ["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           os.path.join(ROOT, "tests", "batch_layout_harness.cpp"), "-L", PKG, "-llbl",
           f"-Wl,-rpath,{PKG}", "-o", exe]
    subprocess.check_call(cmd)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "batch layout OK" in r.stdout
