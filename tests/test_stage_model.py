"""CPU check of the fast method's stage conventions against the oracle.

The numpy stage model (kernel spreading, +i FFT, deconvolution, product-to-sum
assembly of Section 2, prefix Cholesky) must reproduce the oracle's direct
least squares, with an error that falls as the spreading kernel widens.
"""
import numpy as np

from oracle import fchi2_oracle as ora
from paper_0901_1913_amd import synth
from tests import stage_model as sm


def test_stage_model_matches_oracle_and_converges():
    c = synth.make("plain", n=300, n_freq=2 ** 12)
    t, x, s = c.curve(0)
    bins = np.array([5, 100, 172, 1000, 2047, 4000])
    ref = ora.dchi2(t, x, s, bins * c.f_max / c.n_freq, c.H)["dchi2"]
    errs = []
    for w in (8, 10, 14):
        got = sm.dchi2(t, x, s, c.f_max, c.H, c.n_freq, w=w, bins=bins)
        errs.append(np.max(ora.rel_err(got, ref)))
    assert errs[0] < 5e-6
    assert errs[1] < errs[0] / 10
    assert errs[2] < 1e-10
