"""Host checks of the launch schedules, compiled from the library's own
schedule source with the host compiler: the first launch's task order (a
permutation of items and row blocks, proportional per XCD range, no item in
a range's tail), per-process row blocks (cover, never span two processes,
respect the entry and row limits) and the gather-order sort of off-process
blocks (sorted in the order the kernel's loads visit positions, plain or
laid out by runs of 2, 4 and 8 entries per lane; slots a permutation
pointing at each entry's stored position; long single-row blocks, single
rows whose aligned span exceeds the capacity, and blocks flagged to keep
their order left in stored order), the vector loads of the run kernels
(inside the padded arrays, every entry of a block used exactly once, LDS
indices below the block capacity, aligned spans within the capacity for
blocks cut at capacity - 7), and, on saddle-point matrices whose zero block
starts at a process boundary, that every column the on-process product's
runs use to read v is the block's own process's."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1612_08060_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_schedules(tmp_path):
    exe = str(tmp_path / "schedule_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-fopenmp", "-I", CSRC,
                    os.path.join(ROOT, "tests", "native", "schedule_check.cpp"),
                    os.path.join(CSRC, "schedule.cpp"), "-o", exe], check=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0 and res.stdout.strip() == "ok", res.stdout + res.stderr
