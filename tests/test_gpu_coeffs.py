"""Coefficients of the H-harmonic fit from the search (fchi2_search_coeffs,
eq. eqcoeffs with the weighted mean added back to A_0) against the oracle's
coefficients (with_coeffs=True) on gated bins, and the search rows they come
with identical to fchi2_search's.

The coefficient error is measured relative to the size of the fitted
variation: |A_gpu - A_ora| / max(|A_ora[1:]|, sqrt(2 H' / W)), where
sqrt(2 H / W) is the amplitude scale of a fit to pure noise (the null mean of
Delta chi2 is 2H, and Delta chi2 ~ W |A|^2 / 2 for a sinusoid), so that bins
without signal are not judged on noise-sized coefficients.
"""
import numpy as np
import pytest

from oracle import fchi2_oracle as ora
from paper_0901_1913_amd import fchi2 as F
from paper_0901_1913_amd import synth
from tests.gpu_util import note, sample_bins, to_dev

pytestmark = pytest.mark.gpu

KAPPA = {"mixed": 1e2, "fp64": 1e6}
TOL = {"fp64": 1e-9, "mixed": 5e-6}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_coefficients_match_oracle(precision):
    import torch
    cur = synth.make("plain", n=800, n_freq=2 ** 12, f_max=2.5, precision=precision)
    note(f"coefficients {precision}")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=precision)
    t, x, s = to_dev(cur)
    d, c0, fl, A = plan.search_coeffs(t, x, s)
    d2, _, fl2 = plan.search(t, x, s)
    torch.cuda.synchronize()
    assert torch.equal(d, d2) and torch.equal(fl, fl2)
    A = A.double().cpu().numpy()[0]
    k0 = int(round(cur.n_freq / cur.f_max / 2.37))
    bins = np.unique(np.concatenate([sample_bins(cur.n_freq, 300, 4), [k0 - 1, k0, k0 + 1]]))
    fr = bins * (cur.f_max / cur.n_freq)
    r = ora.dchi2(cur.t, cur.x, cur.sigma, fr, cur.H, with_coeffs=True)
    gate = ora.gate_mask(r, fr, KAPPA[precision])
    ref = r["coeffs"]                      # [bins, 2H+1]
    got = A[:, bins].T
    scale = np.maximum(np.linalg.norm(ref[:, 1:], axis=1), np.sqrt(2.0 * cur.H / r["W"]))
    err = np.abs(got - ref).max(axis=1) / scale
    print(f"coeffs {precision}: gated max {err[gate].max():.3e} median "
          f"{np.median(err[gate]):.3e}; at the signal bin {err[bins == k0][0]:.3e}", flush=True)
    assert err[gate].max() <= TOL[precision]
    # The signal bin recovers the injected amplitudes: 0.5 sin + 0.2 cos(2x).
    j = np.nonzero(bins == k0)[0][0]
    amp1 = np.hypot(got[j, 1], got[j, 2])
    assert abs(amp1 - 0.5) < 0.05, amp1
    # Bin 0: the mean only.
    assert A[0, 0] == pytest.approx(r["xbar"], rel=1e-6) and not A[1:, 0].any()
