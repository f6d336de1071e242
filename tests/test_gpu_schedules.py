"""Every FFT schedule gives the same search: digit splits and, for FP32 grids,
the per-pass tile size (4096 or 8192 elements).

A schedule is forced through the autotuner's cache file: the library applies
a cached line for the plan's shape when it names one of its candidate
schedules.  Each forced schedule is checked against the FP64 oracle on
sampled bins, and where it differs most from the first schedule (over every
unflagged bin) both are checked against the oracle: a large difference is
allowed only where the normal matrix is ill-conditioned (outside the gate).
"""
import numpy as np
import pytest

from oracle import fchi2_oracle as ora
from paper_0901_1913_amd import fchi2 as F
from paper_0901_1913_amd import synth
from tests.gpu_util import note, sample_bins, to_dev

pytestmark = pytest.mark.gpu

# (log2 radix, log2 tile) of passes 1..np (pass 1 is the last one run), for
# L = 2^20: all 4096-element tiles, all 8192, the first pass on 4096 and the
# rest on 8192, other splits, and a four-pass split.
SCHEDULES = [
    ((7, 7, 6), (12, 12, 12)),
    ((7, 7, 6), (13, 13, 13)),
    ((7, 7, 6), (13, 13, 12)),
    ((6, 6, 8), (13, 13, 13)),
    ((5, 7, 8), (13, 13, 12)),
    ((8, 6, 6), (12, 12, 12)),
    ((4, 4, 4, 8), (12, 12, 12, 12)),
]


def test_every_schedule_matches_the_oracle(tmp_path):
    import torch
    cur = synth.make("long", n=5000, span=300.0, n_freq=2 ** 18, f_max=50.0)
    t, x, s = to_dev(cur)
    cache = tmp_path / "tune.txt"
    note("schedules: first autotune writes the shape key")
    F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed").autotune(
        t, x, s, cache_path=str(cache))
    key = open(cache).read().splitlines()[0].split(" | ")[0]
    bins = sample_bins(cur.n_freq, 160, 91)
    fr = bins * (cur.f_max / cur.n_freq)
    ref = ora.dchi2(*cur.curve(0), fr, cur.H)
    gate = ora.gate_mask(ref, fr, 1e2)
    assert gate.sum() > 100
    floor = (2.0 * np.arange(1, cur.H + 1))[:, None]
    first = None
    for ln, le in SCHEDULES:
        np_ = len(ln)
        lnp = list(ln) + [0] * (4 - np_)
        lep = list(le) + [0] * (4 - np_)
        cache.write_text(f"{key} | np={np_} fft={','.join(map(str, lnp))} "
                         f"le={','.join(map(str, lep))} tile=11 wave=1 ms=0\n")
        note(f"schedule radices {ln} tiles {le}")
        plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
        info = plan.autotune(t, x, s, cache_path=str(cache))
        assert info["fft_log_radices"] == list(ln) and info["fft_log_tiles"] == list(le), info
        d, _, fl = plan.search(t, x, s)
        torch.cuda.synchronize()
        d = d.double().cpu().numpy()[0]
        fl = fl.cpu().numpy()[0]
        e = ora.rel_err(d[:, bins], ref["dchi2"])[:, gate]
        print(f"radices {ln} tiles {le}: gated max rel err {e.max():.3e}", flush=True)
        assert e.max() <= 1e-5
        ok = (fl & (F.BIN_PIVOT | F.BIN_LOW_F | F.BIN_DC)) == 0
        if first is None:
            first = d
        else:
            diff = np.where(ok[None, :], np.abs(d - first) / np.maximum(first, floor), 0.0)
            worst = np.unique(np.argsort(diff.max(axis=0))[-8:])
            fw = worst * (cur.f_max / cur.n_freq)
            rw = ora.dchi2(*cur.curve(0), fw, cur.H)
            gw = ora.gate_mask(rw, fw, 1e2)
            print(f"  largest differences from the first schedule: "
                  f"{diff[:, worst].max():.3e} at bins {worst.tolist()}, gated {gw.tolist()}",
                  flush=True)
            for dd in (d, first):
                ew = ora.rel_err(dd[:, worst], rw["dchi2"])[:, gw]
                assert ew.size == 0 or ew.max() <= 1e-5, (ln, le, worst, ew.max())
        plan.close()


def test_tile_size_changes_no_bit_forward_or_adjoint(tmp_path):
    """The tile size only regroups the same per-column transforms: the search
    and the adjoint give identical bits on 4096- and 8192-element tiles."""
    import torch
    cur = synth.make("diff", n=3000, n_freq=2 ** 18, f_max=20.0)
    t, x, s = to_dev(cur)
    cache = tmp_path / "tune.txt"
    note("tile sizes: first autotune writes the shape key")
    F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed",
           keep_for_backward=True).autotune(t, x, s, cache_path=str(cache))
    key = open(cache).read().splitlines()[0].split(" | ")[0]
    span = float(cur.t[-1] - cur.t[0])
    k_lo = int(np.ceil(cur.n_freq / (span * cur.f_max)))
    outs = []
    for le in ((12, 12, 12), (13, 13, 13), (13, 13, 12)):
        cache.write_text(f"{key} | np=3 fft=7,7,6,0 le={le[0]},{le[1]},{le[2]},0 "
                         f"tile=11 wave=1 ms=0\n")
        note(f"tile sizes {le}: forward and adjoint")
        plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed",
                      keep_for_backward=True)
        info = plan.autotune(t, x, s, cache_path=str(cache))
        assert info["fft_log_tiles"] == list(le), info
        d, _, _ = plan.search(t, x, s)
        idx = plan.top_peaks(d, cur.H - 1, k_lo, 16)
        g = torch.zeros_like(d)
        g[0, cur.H - 1, idx[0]] = 1.0
        gx, gs = plan.backward(t, x, s, g)
        torch.cuda.synchronize()
        outs.append((d.cpu(), idx.cpu(), gx.cpu(), gs.cpu()))
        plan.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert torch.equal(a, b)


def test_set_schedule_reproduces_the_tuned_plan():
    """set_schedule applies a schedule as info() reports it: same results bit
    for bit as the tuned plan; schedules the plan does not build are refused."""
    import torch
    cur = synth.make("batch", n_curves=12, n_freq=2 ** 16, f_max=10.0, n_lo=100, n_hi=3000)
    t, x, s = to_dev(cur)
    note("set_schedule: tuned plan")
    a = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
    info = a.autotune(t, x, s)
    da, ca, fa = a.search(t, x, s)
    torch.cuda.synchronize()
    note(f"set_schedule: {info}")
    b = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
    assert b.set_schedule(info) == info
    db, cb, fb = b.search(t, x, s)
    torch.cuda.synchronize()
    assert torch.equal(da, db) and torch.equal(ca, cb) and torch.equal(fa, fb)
    for bad in (dict(info, fft_log_radices=[5, 5, 5, 3], fft_log_tiles=[12] * 4),
                dict(info, fft_log_tiles=[11] * len(info["fft_log_tiles"])),
                dict(info, curves_per_wave=10 ** 6), dict(info, spread_tile=512)):
        with pytest.raises(F.FChi2Error):
            b.set_schedule(bad)
    assert b.info() == info
    a.close()
    b.close()


def test_solve_sub_wave_identical():
    """The last FFT pass and the solve run on sub-waves (each sub-wave's solve
    right after its spectra are written): the same kernels per curve, so rows,
    chi2_0, flags, coefficients and the adjoint are identical bit for bit to
    the whole-wave schedule."""
    import torch
    from tests.test_gpu_fused import same_bits
    cur = synth.make("batch", n_curves=29, n_freq=2 ** 14, f_max=6.0, n_lo=20, n_hi=3000,
                     span_hi=150.0)
    t, x, s = to_dev(cur)
    outs = []
    for wave, sub in ((10, 0), (10, 3), (29, 7), (29, 0)):
        note(f"sub-wave: wave {wave}, last pass and solve on {sub or wave}")
        plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed",
                      keep_for_backward=True)
        info = plan.set_schedule(dict(plan.info(), curves_per_wave=wave, solve_sub_wave=sub))
        assert info["curves_per_wave"] == wave and info["solve_sub_wave"] == sub
        d, c0, fl, coef = plan.search_coeffs(t, x, s)
        d2, _, _ = plan.search(t, x, s)
        g = torch.zeros_like(d2)
        g[:, cur.H - 1, 100:110] = 1.0
        gx, gs = plan.backward(t, x, s, g)
        torch.cuda.synchronize()
        outs.append([v.cpu() for v in (d, c0, fl, coef, d2, gx, gs)])
        plan.close()
    for o in outs[1:]:
        for u, v in zip(outs[0], o):
            assert same_bits(u, v)
    with pytest.raises(F.FChi2Error):
        plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
        plan.set_schedule(dict(plan.info(), curves_per_wave=4, solve_sub_wave=5))
