"""The spreading fused into the first FFT pass (FCHI2_FUSED_SPREAD, or the
autotuner's fused schedule) computes every cell from the points with the same
kernel argument and in the same order as the standalone spreading kernel, so
the whole search, its flags and its adjoint must be identical bit for bit;
checked over precisions, FFT splits (two and three passes, both tile sizes),
uneven batches, floor gridding, and against the oracle."""
import numpy as np
import pytest

from oracle import fchi2_oracle as ora
from paper_0901_1913_amd import fchi2 as F
from paper_0901_1913_amd import synth
from tests.gpu_util import note, sample_bins, to_dev

pytestmark = pytest.mark.gpu


def same_bits(u, v):
    """Bitwise equality (NaN rows of rejected curves compare equal)."""
    import torch
    if u.dtype != v.dtype or u.shape != v.shape:
        return False
    if u.dtype.is_floating_point:
        it = {8: torch.int64, 4: torch.int32}[u.element_size()]
        return torch.equal(u.view(it), v.view(it))
    return torch.equal(u, v)


def _both(cur, precision, **kw):
    import torch
    t, x, s = to_dev(cur)
    outs = []
    for fused in (False, True):
        plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=precision,
                      fused_spread=fused, **kw)
        assert plan.info()["fused_spread"] == fused
        d, c0, fl = plan.search(t, x, s)
        torch.cuda.synchronize()
        outs.append((d.cpu(), c0.cpu(), fl.cpu()))
        plan.close()
    return outs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_identical_plain_and_batch(precision):
    import torch
    for label, cur in (
            ("plain", synth.make("plain", n=700, n_freq=2 ** 12, f_max=2.5)),
            ("batch", synth.make("batch", n_curves=24, n_freq=2 ** 13, f_max=4.0,
                                 span_hi=150.0)),
            ("long", synth.make("long", n=6000, span=300.0, n_freq=2 ** 16, f_max=20.0))):
        note(f"fused vs standalone spreading: {label} {precision}")
        a, b = _both(cur, precision)
        for u, v in zip(a, b):
            assert same_bits(u, v), label
        assert np.isfinite(a[0].double().numpy()).any()


def test_fused_identical_floor_gridding():
    import torch
    cur = synth.make("long", n=4000, span=300.0, n_freq=2 ** 14, f_max=5.0)
    note("fused vs standalone: floor gridding")
    a, b = _both(cur, "mixed", kernel_width=1)
    for u, v in zip(a, b):
        assert same_bits(u, v)


# (n_freq, [(log2 radix, log2 tile) of passes 1..np]): L = 4 n_freq cells.
SPLITS = [
    (2 ** 18, [((7, 7, 6), (12, 12, 12)), ((7, 7, 6), (13, 13, 13)), ((6, 6, 8), (13, 13, 12))]),
    (2 ** 16, [((9, 9), (12, 12)), ((9, 9), (13, 13)), ((6, 6, 6), (12, 12, 12))]),
]


@pytest.mark.parametrize("n_freq,splits", SPLITS)
def test_fused_every_split_and_oracle(tmp_path, n_freq, splits):
    """Forced schedules (through the autotuner's cache) with and without the
    fused first pass give identical bits, and match the oracle."""
    import torch
    cur = synth.make("batch", n_curves=6, n_freq=n_freq, f_max=10.0, n_lo=200, n_hi=3000)
    t, x, s = to_dev(cur)
    cache = tmp_path / "tune.txt"
    note("fused splits: first autotune writes the shape key")
    F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed").autotune(
        t, x, s, cache_path=str(cache))
    key = open(cache).read().splitlines()[0].split(" | ")[0]
    bins = sample_bins(cur.n_freq, 120, 17)
    fr = bins * (cur.f_max / cur.n_freq)
    for ln, le in splits:
        np_ = len(ln)
        lnp = list(ln) + [0] * (4 - np_)
        lep = list(le) + [0] * (4 - np_)
        res = []
        for fz in (0, 1):
            cache.write_text(f"{key} | np={np_} fft={','.join(map(str, lnp))} "
                             f"le={','.join(map(str, lep))} tile=11 wave=3 fused={fz} ms=0\n")
            note(f"split {ln} tiles {le} fused={fz}")
            plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
            info = plan.autotune(t, x, s, cache_path=str(cache))
            assert info["fft_log_radices"] == list(ln) and info["fused_spread"] == bool(fz), info
            d, c0, fl = plan.search(t, x, s)
            torch.cuda.synchronize()
            res.append((d.cpu(), c0.cpu(), fl.cpu()))
            plan.close()
        for u, v in zip(*res):
            assert same_bits(u, v), (ln, le)
        d = res[1][0].double().numpy()
        for c in (0, 3, 5):
            ref = ora.dchi2(*cur.curve(c), fr, cur.H)
            gate = ora.gate_mask(ref, fr, 1e2)
            e = ora.rel_err(d[c][:, bins], ref["dchi2"])[:, gate]
            print(f"split {ln} curve {c}: gated max {e.max():.3e} on {gate.sum()} bins",
                  flush=True)
            assert e.max() <= 1e-5


def test_fused_adjoint_identical():
    import torch
    cur = synth.make("diff", n=3000, n_freq=2 ** 16, f_max=20.0)
    t, x, s = to_dev(cur)
    outs = []
    for fused in (False, True):
        note(f"adjoint with fused={fused}")
        plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed",
                      keep_for_backward=True, fused_spread=fused)
        d, _, _ = plan.search(t, x, s)
        g = torch.zeros_like(d)
        g[0, cur.H - 1, 2000:2100] = 1.0
        gx, gs = plan.backward(t, x, s, g)
        torch.cuda.synchronize()
        outs.append((d.cpu(), gx.cpu(), gs.cpu()))
        plan.close()
    for u, v in zip(*outs):
        assert same_bits(u, v)
