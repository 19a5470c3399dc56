"""Partial-sum workspace of the Krylov multi-dot kernels (no GPU): the
allocation rules in csrc/blas_sizes.h cover the largest call each buffer
serves, for the 4^4, 16^4, 16^3x32 and 32^3x64 shapes and coarse restarts
1, 5, 30 and 64.  The setup's test-vector norms (12 V elements, N_tv
vectors) have a buffer of their own; sharing the coarse GMRES buffer, sized
from the much shorter coarse vectors, overflowed it on the 16^4 workload."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_partial_sum_buffers_cover_every_call(tmp_path):
    exe = str(tmp_path / "part_sizing")
    src = os.path.join(ROOT, "tests", "cpp", "part_sizing.cpp")
    inc = os.path.join(ROOT, "paper_1512_04506_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", inc, src, "-o", exe], check=True)
    p = subprocess.run([exe], capture_output=True, text=True)
    print(p.stdout)
    assert p.returncode == 0, p.stdout
    assert "FAIL" not in p.stdout
    # c2 was one of the shapes that overflowed the shared buffer
    n = int(p.stdout.strip().splitlines()[-1].split(":")[-1])
    assert n >= 4
