"""Occupancy of the FFT pass kernels, read from the compiler's resource report
(a device-code build of csrc/fft.hip for gfx950 with the library's flags, no
GPU needed).  An FP32 pass tile of 8192 elements is a workgroup of eight
waves with 72-78 KB of LDS, so two fit a CU (160 KB) only if each wave keeps
to 128 registers (four waves per SIMD); an FP64 tile of 4096 elements must
keep its LDS within 80 KB for the same two workgroups.  Either regression
halves the passes' occupancy without changing any result, so no parity test
would see it."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_0901_1913_amd", "csrc", "fft.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _report(tmp_path):
    from paper_0901_1913_amd import build
    cmd = [HIPCC, *build.FLAGS, "-Rpass-analysis=kernel-resource-usage", "-c", SRC,
           "-o", str(tmp_path / "fft.o")]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs|AGPRs|LDS Size \[bytes/block\]): (\d+)", line)
        if m and cur is not None:
            kernels[cur][m.group(1).split(" ")[0]] = int(m.group(2))
    return kernels


def _pass_kernels(kernels):
    """(type, log2 rows, log2 columns, fused) -> resource report."""
    out = {}
    for name, res in kernels.items():
        m = re.search(r"k_fft_passI([fd])Li(\d+)ELi(\d+)ELb([01])E", name)
        if m:
            out[(m.group(1), int(m.group(2)), int(m.group(3)), m.group(4) == "1")] = res
    return out


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC),
                    reason="hipcc not available")
def test_fft_pass_kernels_keep_two_workgroups_per_cu(tmp_path):
    passes = _pass_kernels(_report(tmp_path))
    assert passes, "no FFT pass kernel in the resource report"
    big_fp32 = {k: v for k, v in passes.items() if k[0] == "f" and not k[3] and k[1] + k[2] == 13}
    fp64_multi = {k: v for k, v in passes.items() if k[0] == "d" and k[2] > 0}
    assert len(big_fp32) >= 6 and len(fp64_multi) >= 5, (sorted(big_fp32), sorted(fp64_multi))
    for k, v in big_fp32.items():
        regs = v["VGPRs"] + v.get("AGPRs", 0)
        assert regs <= 128, (k, v)
        assert 2 * v["LDS"] <= 160 * 1024, (k, v)
    for k, v in fp64_multi.items():
        assert 2 * v["LDS"] <= 160 * 1024, (k, v)
