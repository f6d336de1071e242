"""Parity at the full workload sizes, on bins the oracle evaluates one by one.

Each test runs the search as bench.py does (default plan for the workload,
autotuned before the search) and compares seeded samples of bins, plus the neighbourhood of the
injected signal, with the FP64 oracle under the gate of the target
(rel err <= 1e-5 on bins with k >= 1, f >= 1/span, kappa <= 1e2 mixed /
1e6 FP64).
"""
import numpy as np
import pytest

from oracle import fchi2_oracle as ora
from paper_0901_1913_amd import fchi2 as F
from paper_0901_1913_amd import synth
from tests.gpu_util import note, run_search, sample_bins, to_dev

pytestmark = pytest.mark.gpu

KAPPA = {"mixed": 1e2, "fp64": 1e6}


def _compare(cur, d, bins, precision, c=0, label="", r=None):
    t, x, s = cur.curve(c)
    fr = bins * (cur.f_max / cur.n_freq)
    if r is None:
        r = ora.dchi2(t, x, s, fr, cur.H)
    err = ora.rel_err(d[c][:, bins], r["dchi2"])
    gate = ora.gate_mask(r, fr, KAPPA[precision])
    e = err[:, gate]
    if e.size:
        print(f"{label}: {gate.sum()}/{len(bins)} gated bins, max {e.max():.3e}, "
              f"median {np.median(e):.3e}; ungated max {err.max():.3e}", flush=True)
    return e, r


def test_long_full_size():
    cur = synth.make("long")
    note("long full size (n=1e5, 2^22 bins, mixed)")
    d, _, _, _ = run_search(cur, tune=True)
    k0 = int(round(cur.n_freq / cur.f_max / 0.731))
    one = int(round(cur.n_freq / cur.f_max))  # 1 cycle/day alias region
    bins = np.unique(np.concatenate([sample_bins(cur.n_freq, 200, 2),
                                     np.arange(k0 - 3, k0 + 4), 2 * k0 + np.arange(-2, 3),
                                     one + np.arange(-4, 5)]))
    e, _ = _compare(cur, d, bins, "mixed", label="long full")
    assert e.max() <= 1e-5
    assert abs(int(np.argmax(d[0][cur.H - 1])) - k0) <= 1


def test_diff_full_size_forward_and_gradient():
    import torch
    cur = synth.make("diff")
    note("diff full size (n=2e4, 2^20 bins, mixed) + gradient")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed",
                  keep_for_backward=True)
    t, x, s = to_dev(cur)
    plan.autotune(t, x, s)
    dd, _, _ = plan.search(t, x, s)
    span = cur.t[-1] - cur.t[0]
    df = cur.f_max / cur.n_freq
    k_lo = int(np.ceil(1.0 / (span * df)))
    idx = plan.top_peaks(dd, cur.H - 1, k_lo, 16)
    g = torch.zeros_like(dd)
    g[0, cur.H - 1, idx[0]] = 1.0
    gx, gs = plan.backward(t, x, s, g)
    torch.cuda.synchronize()
    d = dd.double().cpu().numpy()
    idx = idx.cpu().numpy()[0]
    bins = np.unique(np.concatenate([sample_bins(cur.n_freq, 200, 4), idx]))
    e, _ = _compare(cur, d, bins, "mixed", label="diff full")
    assert e.max() <= 1e-5
    rx, rs = ora.grad(cur.t, cur.x, cur.sigma, [(float(k) * df, cur.H, 1.0) for k in idx])
    ex = np.linalg.norm(gx.cpu().numpy() - rx) / np.linalg.norm(rx)
    es = np.linalg.norm(gs.cpu().numpy() - rs) / np.linalg.norm(rs)
    print(f"diff full gradient: rel l2 dx {ex:.3e}, dsigma {es:.3e}", flush=True)
    assert ex <= 1e-5 and es <= 1e-5


def test_stress_full_size_three_way():
    """Precision stress: mixed vs all-FP64 GPU vs the oracle."""
    cur = synth.make("stress")
    note("stress full size (n=1e6, 2^24 bins, H=8) mixed")
    dm, _, flm, _ = run_search(cur, "mixed", tune=True)
    note("stress full size fp64")
    dd, _, _, _ = run_search(cur, "fp64")
    floor = (2.0 * np.arange(1, cur.H + 1))[:, None]
    k = np.arange(cur.n_freq)
    span = cur.t[-1] - cur.t[0]
    ok = (k >= 1) & (k * cur.f_max / cur.n_freq >= 1.0 / span) & ((flm[0] & F.BIN_PIVOT) == 0)
    gg = np.abs(dm[0] - dd[0])[:, ok] / np.maximum(dd[0], floor)[:, ok]
    print(f"stress mixed vs fp64 GPU over {ok.sum()} bins: max {gg.max():.3e}, "
          f"median {np.median(gg):.3e}, p99.99 {np.percentile(gg, 99.99):.3e}", flush=True)
    k0 = int(round(cur.n_freq / cur.f_max / 0.1234))
    bins = np.unique(np.concatenate([sample_bins(cur.n_freq, 16, 5), [k0 - 1, k0, k0 + 1]]))
    em, r = _compare(cur, dm, bins, "mixed", label="stress mixed vs oracle")
    ed, _ = _compare(cur, dd, bins, "fp64", label="stress fp64 vs oracle", r=r)
    assert em.max() <= 1e-5 and ed.max() <= 1e-8
    assert np.percentile(gg, 99.9) <= 1e-5


def test_batch_full_size_sampled_curves():
    import torch
    cur = synth.make("batch")
    note("batch full size (1e4 curves, 2^16 bins)")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed", graph=True)
    t, x, s = to_dev(cur)
    plan.autotune(t, x, s)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        d, _, _ = plan.search(t, x, s, want_flags=False)
        st.synchronize()
    d = d.double().cpu().numpy()
    rng = np.random.default_rng(33)
    worst = 0.0
    for c in rng.choice(cur.n_curves, 24, replace=False):
        bins = sample_bins(cur.n_freq, 12, 100 + int(c))
        e, _ = _compare(cur, d, bins, "mixed", c=int(c), label=f"batch curve {c}")
        if e.size:
            worst = max(worst, float(e.max()))
    assert worst <= 1e-5
