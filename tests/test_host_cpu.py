"""Host-side behaviour that needs no GPU: the benchmark's one-GPU contract and
the absence of any CPU fallback in the product path."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          cwd=ROOT, capture_output=True, text=True, timeout=300)


def test_bench_refuses_more_than_one_gpu():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _has_gpu():
    import torch
    return torch.cuda.is_available()


@pytest.mark.skipif(_has_gpu(), reason="checks the behaviour on a machine without a GPU")
def test_no_gpu_means_an_error_not_a_fallback():
    from paper_0901_1913_amd import fchi2 as F
    from paper_0901_1913_amd import synth
    cur = synth.make("plain")
    with pytest.raises(F.FChi2Error):
        F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="fp64")
    r = _bench("--steps", "1", "--warmup", "0")
    assert r.returncode != 0 and r.stdout == ""
    assert "needs a GPU" in r.stderr
