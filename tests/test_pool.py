"""The serving engines' arena allocator (paper_2508_14568_amd/csrc/pool.h),
built with the host compiler and checked against a model of every 256-byte
unit (tests/pool_check.cpp): no overlap, first fit, full merging on release,
and any request of at most total() bytes fitting an empty pool (no CPU
fallback of anything: the allocator only hands out offsets)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2508_14568_amd", "csrc")


def test_pool_against_unit_model(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "pool_check"
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC, os.path.join(HERE, "pool_check.cpp"),
                    "-o", str(exe)], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=False, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
