"""Host build of the FFT split planning (csrc/fft_splits.h): the candidate
schedules the autotuner may time are valid splits of the grid length, the
default split is among them, tiles are 2^12 (and 2^13 for FP32 grids), and
splits with an extra pass appear only for grids of at most 2^20 cells."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "fft_splits_test.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC),
                    reason="hipcc not available")
def test_fft_splits_host(tmp_path):
    exe = str(tmp_path / "fft_splits_test")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", SRC, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and "ALL OK" in out.stdout, out.stdout + out.stderr
