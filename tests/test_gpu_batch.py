"""Batched execution: sub-range searches, the autotuner and its cache."""
import os

import numpy as np
import pytest

from oracle import fchi2_oracle as ora
from paper_0901_1913_amd import fchi2 as F
from paper_0901_1913_amd import synth
from tests.gpu_util import note, sample_bins, to_dev

pytestmark = pytest.mark.gpu


def _small_batch():
    return synth.batch(n_curves=40, n_lo=30, n_hi=3000, span_lo=30.0, span_hi=300.0,
                       n_freq=2 ** 13, f_max=3.0)


def test_search_curves_equals_full_search():
    import torch
    cur = _small_batch()
    note("search_curves vs full search")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed",
                  curves_per_wave=7)
    t, x, s = to_dev(cur)
    d, c0, fl = plan.search(t, x, s)
    d_ref, c0_ref, fl_ref = d.clone(), c0.clone(), fl.clone()
    d.fill_(-1.0)
    for first, count in [(0, 1), (1, 5), (6, 17), (23, 17)]:
        plan.search_curves(first, count, t, x, s, d, c0, fl)
    torch.cuda.synchronize()
    assert torch.equal(d, d_ref) and torch.equal(c0, c0_ref) and torch.equal(fl, fl_ref)
    with pytest.raises(F.FChi2Error):
        plan.search_curves(35, 10, t, x, s, d, c0, fl)


def test_autotune_and_cache(tmp_path):
    import torch
    cur = _small_batch()
    note("autotune")
    cache = str(tmp_path / "tune.txt")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
    t, x, s = to_dev(cur)
    before = plan.info()
    info = plan.autotune(t, x, s, cache_path=cache)
    assert os.path.exists(cache)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and "gfx950" in lines[0]
    print("tuned", before, "->", info, flush=True)
    d, _, _ = plan.search(t, x, s)
    torch.cuda.synchronize()
    dd = d.double().cpu().numpy()
    for c in (0, 13, 39):
        tt, xx, ss = cur.curve(c)
        bins = sample_bins(cur.n_freq, 150, 40 + c)
        fr = bins * cur.f_max / cur.n_freq
        r = ora.dchi2(tt, xx, ss, fr, cur.H)
        gate = ora.gate_mask(r, fr, 1e2)
        err = ora.rel_err(dd[c][:, bins], r["dchi2"])[:, gate]
        assert err.max() <= 1e-5, (c, err.max())
    # A second plan of the same shape takes the cached schedule.
    plan2 = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
    assert plan2.autotune(t, x, s, cache_path=cache) == info
    assert len(open(cache).read().strip().splitlines()) == 1
