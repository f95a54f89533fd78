"""The GPE workspace is allocated all or nothing (csrc/alloc_group.h): after an allocation that
fails part-way no buffer stays allocated and no pointer stays set, so the next GPE call allocates
again instead of launching kernels on missing buffers.  Checked on the CPU with an allocator that
fails at each call in turn (tests/host/alloc_group_check.cpp, built with g++)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "alloc_group_check.cpp")


def test_alloc_group_all_or_nothing(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "alloc_group_check")
    r = subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        SRC, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


def test_gpe_workspace_uses_the_group_allocation():
    """ensure_gpe allocates its six buffers through alloc_group, not one by one."""
    src = open(os.path.join(ROOT, "paper_1504_02897_amd", "csrc", "capi.cpp")).read()
    body = src[src.index("ddi_status ensure_gpe"):src.index("ddi_status ts_step_impl")]
    assert "alloc_group(" in body and "hipMalloc(p, b)" in body
    assert body.count("hipMalloc") == 1
