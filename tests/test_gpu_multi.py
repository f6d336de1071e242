"""Shared-alpha search (Section 5): many sources at the same sampling times
with proportional errors reuse alpha's factor per frequency.

Source s is the ordinary curve (t, x[s], scale[s] * sigma); the oracle runs
it as such.  Checked: parity with the FP64 oracle on sampled bins (small FP64
and mixed cases, the full multi workload), agreement with the ordinary
batched search of the same sources, rejected sources, unsupported plans.
"""
import numpy as np
import pytest

from oracle import fchi2_oracle as ora
from paper_0901_1913_amd import fchi2 as F
from paper_0901_1913_amd import synth
from tests.gpu_util import note, sample_bins

pytestmark = pytest.mark.gpu

KAPPA = {"mixed": 1e2, "fp64": 1e6}
TOL = {"mixed": 1e-5, "fp64": 1e-8}


def _dev(src):
    import torch
    t = torch.from_numpy(src.t).cuda()
    sg = torch.from_numpy(src.sigma).cuda()
    x = torch.from_numpy(np.ascontiguousarray(src.x)).cuda()
    sc = torch.from_numpy(src.scale).cuda()
    return t, sg, x, sc


def _run(src, precision):
    import torch
    plan = F.Plan(src.offsets, src.f_max, src.H, src.n_freq, precision=precision)
    t, sg, x, sc = _dev(src)
    d, c0, fl = plan.search_multi(t, sg, x, sc)
    torch.cuda.synchronize()
    return d.double().cpu().numpy(), c0.cpu().numpy(), fl.cpu().numpy(), plan


def _check_sources(src, d, c0, sources, nbins, precision, seed):
    worst = 0.0
    freqs = np.arange(src.n_freq) * (src.f_max / src.n_freq)
    for s in sources:
        t, x, sg = src.source(int(s))
        bins = sample_bins(src.n_freq, nbins, seed + int(s))
        r = ora.dchi2(t, x, sg, freqs[bins], src.H)
        gate = ora.gate_mask(r, freqs[bins], KAPPA[precision])
        e = ora.rel_err(d[s][:, bins], r["dchi2"])[:, gate]
        if e.size:
            worst = max(worst, float(e.max()))
        assert c0[s] == pytest.approx(r["chi2_0"], rel=1e-12)
    return worst


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_small_matches_oracle(precision):
    src = synth.make("multi", n_sources=40, n=300, span=100.0, n_freq=1 << 12, f_max=5.0,
                     precision=precision)
    note(f"search_multi small {precision} (40 sources x 300 points, 2^12 bins)")
    d, c0, fl, _ = _run(src, precision)
    worst = _check_sources(src, d, c0, range(src.n_sources), 24, precision, 500)
    print(f"multi small {precision}: worst gated rel err {worst:.3e}", flush=True)
    assert worst <= TOL[precision]
    assert fl[0] & F.BIN_DC


def test_agrees_with_ordinary_batched_search():
    """The same sources as ordinary curves (t replicated, sigma scaled)."""
    import torch
    src = synth.make("multi", n_sources=64, n=500, span=200.0, n_freq=1 << 14, f_max=8.0,
                     precision="fp64")
    note("search_multi vs ordinary batched search, fp64, 64 sources")
    d, c0, fl, _ = _run(src, "fp64")
    n = src.t.shape[0]
    off = np.arange(src.n_sources + 1, dtype=np.int64) * n
    plan = F.Plan(off, src.f_max, src.H, src.n_freq, precision="fp64")
    tt = torch.from_numpy(np.tile(src.t, src.n_sources)).cuda()
    xx = torch.from_numpy(src.x.reshape(-1).copy()).cuda()
    ss = torch.from_numpy((src.scale[:, None] * src.sigma[None, :]).reshape(-1)).cuda()
    db, cb, fb = plan.search(tt, xx, ss)
    torch.cuda.synchronize()
    db = db.cpu().numpy()
    floor = (2.0 * np.arange(1, src.H + 1))[None, :, None]
    k = np.arange(src.n_freq)
    # well-conditioned bins only: f >= 2/span (alpha's conditioning blows up
    # rounding differences below 1/span, Section 3e) and no dropped pivot
    span = src.t[-1] - src.t[0]
    fbn = fb.cpu().numpy()[0]
    ok = (k * (src.f_max / src.n_freq) * span >= 2.0) & ((fbn & F.BIN_PIVOT) == 0)
    e = (np.abs(d - db) / np.maximum(db, floor))[:, :, ok]
    print(f"multi vs batched: max {e.max():.3e} over {ok.sum()} bins", flush=True)
    assert e.max() <= 1e-9
    np.testing.assert_allclose(c0, cb.cpu().numpy(), rtol=1e-12)


def test_full_multi_workload_sampled():
    src = synth.make("multi")
    note("search_multi full workload (2000 sources x 400 points, 2^16 bins, mixed)")
    d, c0, fl, _ = _run(src, "mixed")
    rng = np.random.default_rng(61)
    sources = rng.choice(src.n_sources, 12, replace=False)
    worst = _check_sources(src, d, c0, sources, 16, "mixed", 900)
    # the injected period of a periodic source is its best bin (H = 3 row)
    per = src.meta["periods"]
    hits = 0
    tried = 0
    for s in np.nonzero(np.isfinite(per))[0][:20]:
        f0 = 1.0 / per[s]
        if f0 >= src.f_max:
            continue
        tried += 1
        k0 = f0 / (src.f_max / src.n_freq)
        kk = int(np.argmax(d[s, src.H - 1, 1:])) + 1
        hits += abs(kk - k0) <= 2 or abs(kk - 2 * k0) <= 2 or abs(kk - k0 / 2) <= 2
    print(f"multi full: worst gated rel err {worst:.3e}; signal found in {hits}/{tried}",
          flush=True)
    assert worst <= 1e-5
    assert hits >= tried * 0.5


def test_rejected_sources_and_unsupported_plans():
    import torch
    src = synth.make("multi", n_sources=6, n=200, span=100.0, n_freq=1 << 12, f_max=5.0,
                     precision="fp64")
    x = src.x.copy()
    x[2, 17] = np.nan
    scale = src.scale.copy()
    scale[4] = -1.0
    plan = F.Plan(src.offsets, src.f_max, src.H, src.n_freq, precision="fp64")
    note("search_multi rejected sources and unsupported plans")
    t = torch.from_numpy(src.t).cuda()
    sg = torch.from_numpy(src.sigma).cuda()
    d, c0, fl = plan.search_multi(t, sg, torch.from_numpy(x).cuda(),
                                  torch.from_numpy(scale).cuda())
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    c0 = c0.cpu().numpy()
    assert np.all(np.isnan(d[2])) and np.all(np.isnan(d[4]))
    assert not (fl.cpu().numpy()[1:] & 0xF8).any()   # the time base itself is fine
    assert np.isnan(c0[2]) and np.isnan(c0[4])
    good = [0, 1, 3, 5]
    assert np.all(np.isfinite(d[good]))
    ref = ora.dchi2(*src.source(3), [0.37], src.H)
    k = int(round(0.37 / (src.f_max / src.n_freq)))
    r2 = ora.dchi2(*src.source(3), [k * src.f_max / src.n_freq], src.H)
    assert np.max(ora.rel_err(d[3][:, k:k + 1], r2["dchi2"])) <= 1e-8
    assert ref["chi2_0"] == pytest.approx(c0[3], rel=1e-12)
    with pytest.raises(F.FChi2Error):
        F.Plan(src.offsets, src.f_max, 6, src.n_freq, precision="fp64").search_multi(
            t, sg, torch.from_numpy(x).cuda(), torch.from_numpy(scale).cuda())
    with pytest.raises(ValueError):
        F.Plan([0, 100, 200], src.f_max, src.H, src.n_freq).search_multi(
            t, sg, torch.from_numpy(x).cuda(), torch.from_numpy(scale).cuda())
