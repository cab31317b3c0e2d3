"""Host logic of the row-marching pass: the task layout (paper_2605_07954_amd/csrc/march_layout.h,
the same header the kernels include) covers every row of every band exactly once and every column,
keeps the bands that start or end at the grid's sides inside it, and keeps a zoned layout's middle
segments out of the edge zones -- over several thousand grid shapes, depths, lane widths, device
sizes and segment minimums.  Compiled for the host with hipcc; no GPU is needed."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not found")
def test_march_task_layout_covers_the_grid(tmp_path):
    exe = str(tmp_path / "march_layout_check")
    hipcc = HIPCC if os.path.exists(HIPCC) else shutil.which("hipcc")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", os.path.join(HERE, "march_layout_check.cpp"),
                        "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr
