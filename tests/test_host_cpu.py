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


def test_time_order_sorts_within_each_curve():
    """The autograd wrapper's per-curve time order (a host-side tensor helper):
    stable within each CSR range, curves keep their ranges, empty curves and
    ties included."""
    import numpy as np
    import torch
    from paper_0901_1913_amd import fchi2 as F
    rng = np.random.default_rng(2)
    off = np.array([0, 7, 7, 20, 21, 40])
    t = torch.from_numpy(np.round(rng.uniform(0, 5, off[-1]), 1))  # many ties
    p = F.time_order(off, t).numpy()
    assert sorted(p.tolist()) == list(range(off[-1]))
    tn = t.numpy()
    for a, b in zip(off[:-1], off[1:]):
        seg = p[a:b]
        assert ((seg >= a) & (seg < b)).all()
        want = a + np.argsort(tn[a:b], kind="stable")
        assert np.array_equal(seg, want)
