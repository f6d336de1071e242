"""Gridding error against the spreading kernel's width.

The exponential-of-semicircle kernel (beta = 2.3 w, upsampling 2) has a
truncation error that falls about geometrically with its width w.  Measured
against the FP64 oracle on the same bins, the search's error must therefore
fall as w grows, until it reaches the rounding floor of the grid's storage
type (FP64 grids: ~1e-12 here; FP32 grids: ~1e-6).  Every width the plan
accepts (4..16, odd ones included) is run; this also pins the FP32-grid
kernel evaluation at every width.
"""
import numpy as np
import pytest

from oracle import fchi2_oracle as ora
from paper_0901_1913_amd import synth
from tests.gpu_util import note, run_search, sample_bins

pytestmark = pytest.mark.gpu

KAPPA = {"mixed": 1e2, "fp64": 1e6}


def _errors(precision, widths):
    cur = synth.make("plain", n_freq=2 ** 12, f_max=2.5)
    bins = sample_bins(cur.n_freq, 400, 77)
    freqs = bins * (cur.f_max / cur.n_freq)
    t, x, s = cur.curve(0)
    ref = ora.dchi2(t, x, s, freqs, cur.H)
    gate = ora.gate_mask(ref, freqs, KAPPA[precision])
    assert gate.sum() > 0.5 * len(bins)
    out = {}
    for w in widths:
        note(f"plain {precision} kernel_width={w}")
        d, _, _, _ = run_search(cur, precision, kernel_width=w)
        out[w] = float(ora.rel_err(d[0][:, bins], ref["dchi2"])[:, gate].max())
    print(f"{precision} gated max rel err by width: "
          + ", ".join(f"w={w}: {e:.2e}" for w, e in out.items()), flush=True)
    return out


def test_fp64_error_falls_with_width():
    e = _errors("fp64", [4, 6, 8, 10, 12, 14, 16])
    ws = sorted(e)
    for a, b in zip(ws, ws[1:]):
        # two more taps: at least 4x smaller, until the FP64 floor
        assert e[b] <= max(e[a] / 4.0, 1e-10), (a, b, e)
    assert e[4] > 1e-6  # the narrow kernel's truncation error is visible
    assert e[14] <= 1e-10 and e[16] <= 1e-10


def test_mixed_error_falls_with_width_odd_widths_included():
    e = _errors("mixed", [4, 5, 6, 7, 8, 9, 10, 12, 16])
    assert e[6] <= e[4] / 4.0 and e[8] <= max(e[6] / 4.0, 3e-6), e
    for w in (5, 7, 9):  # one more tap is never worse (up to the floor)
        assert e[w] <= max(e[w - 1], 3e-6), (w, e)
    for w in (8, 9, 10, 12, 16):  # the 1e-5 target from w = 8 on
        assert e[w] <= 1e-5, (w, e)
