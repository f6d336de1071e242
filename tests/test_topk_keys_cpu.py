"""Host build of the top-K key order and rank merge (csrc/topk_keys.h).

The fused significance kernels rank candidates by (ln p, bin) and merge the
sorted per-wave lists by rank.  This test compiles the shared header into a
host program (no kernel runs) and checks, against a plain sort: ties in ln p,
+-inf and NaN scores (NaN ranks as +inf, never as a candidate), ln Q at its
limits, and the defensive path for keys that are not distinct (an unfilled
slot reads as empty).
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "topk_keys_test.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC),
                    reason="hipcc not available")
def test_topk_keys_host(tmp_path):
    exe = str(tmp_path / "topk_keys_test")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", SRC, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and "ALL OK" in out.stdout, out.stdout + out.stderr
