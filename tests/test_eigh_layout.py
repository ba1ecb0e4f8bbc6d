"""Host-only bounds check of the block eigensolver's workspace layout (no GPU).

tests/eigh_layout_check.cpp is built with g++ and AddressSanitizer from the
geometry header the kernels use (eigh_geometry.h: launch constants, workgroup
counts, workspace layout); it replays the single-block launch sequence and
checks every launch's index ranges against the layout.  Sizes: the cfg3 T1u
block (n = 10080, FP32 and FP64 working storage, with and without refinement),
the blocks of the tile-form tests (4501, 8400), the first block above the
tile switch (2050), the LDS tail boundary (97), the smallest blocks, and the two-stage reduction
(full -> band -> tridiagonal) on the cfg3 block and the large test blocks, with and
without refinement.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_eigh_layout_in_bounds(tmp_path):
    exe = str(tmp_path / "eigh_layout_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I",
                    os.path.join(ROOT, "paper_2603_24860_amd", "csrc"),
                    os.path.join(ROOT, "tests", "eigh_layout_check.cpp"), "-o", exe],
                   check=True, timeout=300)
    cases = ["10080 0 0", "10080 1 0", "10080 0 100", "4501 0 0", "8400 0 0", "2050 0 0",
             "2160 1 100", "97 1 0", "96 0 0", "1 0 0", "2 1 1",
             # the two-stage reduction (K = -1): cfg3 T1u block, large test blocks, one ragged panel
             "10080 0 -1", "10080 1 -1", "4500 1 -1", "8400 0 -1", "600 0 -1", "33 1 -1",
             # with refinement of k (K = -1 - k): cfg3 T1u block with 100, small blocks
             "10080 0 -101", "4500 1 -21", "600 0 -21", "33 1 -3", "34 0 -2", "2 0 -3",
             "65 0 -66", "10241 0 -101"]
    args = " ".join(cases).split()
    r = subprocess.run([exe] + args, capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count("in bounds") == len(cases), r.stdout
