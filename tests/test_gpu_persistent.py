"""The persistent batched search (FCHI2_PERSISTENT, or the autotuner's
persistent schedule) runs every stage with the same tile code on the same
schedule as the staged search, one curve per workgroup claimed from a device
work queue, so its rows, chi2_0 and flags must be identical bit for bit to the
staged search's: checked on uneven batches with rejected, empty and short
curves, several H, forced FFT splits and spreading tiles, curve subsets,
repeated calls and graph replays, and against the oracle."""
import numpy as np
import pytest

from oracle import fchi2_oracle as ora
from paper_0901_1913_amd import fchi2 as F
from paper_0901_1913_amd import synth
from tests.gpu_util import note, sample_bins, to_dev
from tests.test_gpu_fused import same_bits

pytestmark = pytest.mark.gpu


def _with_edge_curves(cur):
    """cur plus an empty curve, a curve with a NaN value, a curve of four
    points (fewer than 2H + 1 for H >= 2) and an unsorted curve."""
    t, x, s = [], [], []
    for c in range(cur.n_curves):
        a, b, e = cur.curve(c)
        t.append(a), x.append(b), s.append(e)
    a, b, e = cur.curve(0)
    t.append(a[:0]), x.append(b[:0]), s.append(e[:0])
    bn = b.copy()
    bn[len(bn) // 2] = np.nan
    t.append(a), x.append(bn), s.append(e)
    t.append(a[:4]), x.append(b[:4]), s.append(e[:4])
    t.append(a[::-1].copy()), x.append(b), s.append(e)
    off = np.zeros(len(t) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(v) for v in t])
    return synth.Curves(t=np.concatenate(t), x=np.concatenate(x), sigma=np.concatenate(s),
                        offsets=off, H=cur.H, n_freq=cur.n_freq, f_max=cur.f_max,
                        precision=cur.precision, name=cur.name + "+edge", meta=cur.meta)


def _run(cur, persistent, precision="mixed", **kw):
    import torch
    t, x, s = to_dev(cur)
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=precision,
                  persistent=persistent, **kw)
    info = plan.info()
    d, c0, fl = plan.search(t, x, s)
    torch.cuda.synchronize()
    out = (d.cpu(), c0.cpu(), fl.cpu())
    plan.close()
    return out, info


@pytest.mark.parametrize("H", [1, 3, 5, 8])
def test_persistent_identical_uneven_batch(H):
    cur = _with_edge_curves(synth.make("batch", n_curves=37, n_freq=2 ** 14, f_max=6.0, H=H,
                                       n_lo=20, n_hi=4000, span_hi=150.0))
    note(f"persistent vs staged: uneven batch H={H}, {cur.n_curves} curves")
    a, ia = _run(cur, False)
    b, ib = _run(cur, True)
    assert not ia["persistent"] and ib["persistent"], (ia, ib)
    assert ia["fft_log_radices"] == ib["fft_log_radices"]
    for u, v in zip(a, b):
        assert same_bits(u, v)
    d = b[0].double().numpy()
    fl = b[2].numpy()
    n = cur.n_curves
    assert np.isfinite(d[0]).any()
    assert np.isnan(d[n - 4]).all() and np.isnan(d[n - 3]).all() and np.isnan(d[n - 1]).all()
    assert (fl[n - 4] & F.CURVE_EMPTY).all() and (fl[n - 3] & F.CURVE_NONFINITE).all()
    assert (fl[n - 1] & F.CURVE_UNSORTED).all()


def test_persistent_ignored_where_not_supported():
    """FP64 and band plans keep the staged search (the flag is ignored)."""
    cur = synth.make("batch", n_curves=5, n_freq=2 ** 13, f_max=4.0, n_lo=100, n_hi=800)
    note("persistent flag on an FP64 plan")
    a, ia = _run(cur, False, precision="fp64")
    b, ib = _run(cur, True, precision="fp64")
    assert not ib["persistent"]
    for u, v in zip(a, b):
        assert same_bits(u, v)


def test_persistent_curve_subset_repeat_and_graph():
    """search_curves on a subset (the queue covers only those curves), two
    searches in a row (the queue restarts), and graph replays."""
    import torch
    cur = synth.make("batch", n_curves=29, n_freq=2 ** 14, f_max=5.0, n_lo=30, n_hi=3000)
    t, x, s = to_dev(cur)
    ref, _ = _run(cur, False)
    note("persistent: subset of curves")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed",
                  persistent=True)
    assert plan.info()["persistent"]
    d = torch.full((cur.n_curves, cur.H, cur.n_freq), -1.0, dtype=torch.float32,
                   device="cuda")
    c0 = torch.full((cur.n_curves,), -1.0, dtype=torch.float64, device="cuda")
    fl = torch.zeros((cur.n_curves, cur.n_freq), dtype=torch.uint8, device="cuda")
    plan.search_curves(7, 11, t, x, s, d, c0, fl)
    torch.cuda.synchronize()
    dc = d.cpu()
    assert same_bits(dc[7:18], ref[0][7:18])
    assert same_bits(fl.cpu()[7:18], ref[2][7:18])
    assert (dc[:7] == -1.0).all() and (dc[18:] == -1.0).all()
    note("persistent: two searches in a row")
    for _ in range(2):
        dd, cc, ff = plan.search(t, x, s)
        torch.cuda.synchronize()
        for u, v in zip((dd.cpu(), cc.cpu(), ff.cpu()), ref):
            assert same_bits(u, v)
    plan.close()
    note("persistent: graph replays")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed",
                  persistent=True, graph=True)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        for rep in range(3):
            dd, cc, ff = plan.search(t, x, s)
            st.synchronize()
            for u, v in zip((dd.cpu(), cc.cpu(), ff.cpu()), ref):
                assert same_bits(u, v), rep
    plan.close()


# (n_freq, [(log2 radix of passes 1..np)]): every pass a 2^12-element tile.
SPLITS = [
    (2 ** 16, [(9, 9), (6, 6, 6)]),
    (2 ** 18, [(7, 7, 6), (6, 7, 7)]),
]


@pytest.mark.parametrize("n_freq,splits", SPLITS)
def test_persistent_forced_splits_and_oracle(tmp_path, n_freq, splits):
    """Schedules forced through the autotuner's cache, staged and persistent,
    both spreading tiles: identical bits, and the oracle agrees."""
    import torch
    cur = synth.make("batch", n_curves=9, n_freq=n_freq, f_max=10.0, n_lo=200, n_hi=3000)
    t, x, s = to_dev(cur)
    cache = tmp_path / "tune.txt"
    note("persistent splits: first autotune writes the shape key")
    F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed").autotune(
        t, x, s, cache_path=str(cache))
    key = open(cache).read().splitlines()[0].split(" | ")[0]
    bins = sample_bins(cur.n_freq, 120, 21)
    fr = bins * (cur.f_max / cur.n_freq)
    for ln in splits:
        np_ = len(ln)
        lnp = list(ln) + [0] * (4 - np_)
        lep = [12] * np_ + [0] * (4 - np_)
        for tile in (10, 11):
            res = []
            for ps in (0, 1):
                cache.write_text(f"{key} | np={np_} fft={','.join(map(str, lnp))} "
                                 f"le={','.join(map(str, lep))} tile={tile} wave=4 fused=0 "
                                 f"persist={ps} ms=0\n")
                note(f"split {ln} tile {tile} persist={ps}")
                plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
                info = plan.autotune(t, x, s, cache_path=str(cache))
                assert info["fft_log_radices"] == list(ln), info
                assert info["persistent"] == bool(ps) and info["spread_tile"] == 1 << tile, info
                d, c0, fl = plan.search(t, x, s)
                torch.cuda.synchronize()
                res.append((d.cpu(), c0.cpu(), fl.cpu()))
                plan.close()
            for u, v in zip(*res):
                assert same_bits(u, v), (ln, tile)
        d = res[1][0].double().numpy()
        for c in (0, 4, 8):
            ref = ora.dchi2(*cur.curve(c), fr, cur.H)
            gate = ora.gate_mask(ref, fr, 1e2)
            e = ora.rel_err(d[c][:, bins], ref["dchi2"])[:, gate]
            print(f"persistent split {ln} curve {c}: gated max {e.max():.3e} on "
                  f"{gate.sum()} bins", flush=True)
            assert e.max() <= 1e-5


def test_persistent_autotuned_against_oracle():
    """Whatever schedule the autotuner picks (staged, fused or persistent),
    the tuned search meets the oracle on the gated bins (schedules differ in
    their rounding, which ill-conditioned bins amplify, so the comparison is
    with the oracle under its gate, not between schedules)."""
    import torch
    cur = synth.make("batch", n_curves=64, n_freq=2 ** 16, f_max=10.0, n_lo=50, n_hi=5000)
    t, x, s = to_dev(cur)
    note("persistent: autotuned plan")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
    info = plan.autotune(t, x, s)
    print(f"autotuned: {info}", flush=True)
    d, c0, fl = plan.search(t, x, s)
    torch.cuda.synchronize()
    d = d.double().cpu().numpy()
    bins = sample_bins(cur.n_freq, 150, 23)
    fr = bins * (cur.f_max / cur.n_freq)
    for c in (0, 17, 40, 63):
        ref = ora.dchi2(*cur.curve(c), fr, cur.H)
        gate = ora.gate_mask(ref, fr, 1e2)
        e = ora.rel_err(d[c][:, bins], ref["dchi2"])[:, gate]
        print(f"autotuned curve {c}: gated max {e.max():.3e} on {gate.sum()} bins", flush=True)
        assert e.max() <= 1e-5
    plan.close()
