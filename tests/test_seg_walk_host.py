"""The walk segmentation's closed form (segment start state from exact
integer division at major-axis crossings) checked on the host: the library's
own header code, compiled for the CPU, must reproduce the canonical exact walk
voxel for voxel for every segment length, and never produce a key outside the
map.  Covers ties (exact diagonals), axis-parallel, zero-length, clipped and
long rays (past the 32-level cap)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "seg_walk_check.hip")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("segchk") / "seg_walk_check")
    subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2206_06079_amd", "csrc"), SRC, "-o", exe], check=True,
                   capture_output=True)
    return exe


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_segments_reproduce_canonical_walk(checker, seed):
    out = subprocess.run([checker, str(seed), "100000"], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok 100000")
