"""Fine search on the ungridded data (Section 3e) vs the FP64 oracle.

fchi2_fine_search evaluates Delta chi2 directly from the points at R trial
frequencies around given centres (no gridding) and keeps the best trial with
its coefficients.  The oracle evaluates the plain definition at the same
trial frequencies, f_r = f_c + hw (2 r / (R - 1) - 1), computed here from the
test's own centres (signal frequencies of the workloads and fixed values).
"""
import numpy as np
import pytest

from oracle import fchi2_oracle as ora
from paper_0901_1913_amd import fchi2 as F
from paper_0901_1913_amd import synth
from tests.gpu_util import note, to_dev

pytestmark = pytest.mark.gpu


def _trials(fc, hw, R):
    r = np.arange(R, dtype=np.float64)
    return fc + hw * (2.0 * r / (R - 1) - 1.0) if R > 1 else np.array([fc])


def _centres(nc, values):
    import torch
    return torch.tensor(np.tile(np.asarray(values, dtype=np.float64), (nc, 1)),
                        dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("name,R", [("plain", 33), ("diff", 16)])
def test_rows_and_coefficients_match_oracle(name, R):
    import torch
    cur = synth.make(name)
    note(f"fine search {name} R={R} vs oracle at every trial")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=cur.precision)
    t, x, s = to_dev(cur)
    P = {"plain": 2.37, "diff": 3.3}[name]
    centres = [1.0 / P, 2.0 / P, 0.7731, 3.1]
    hw = cur.f_max / cur.n_freq
    res = plan.fine_search(t, x, s, _centres(1, centres), R=R, half_width=hw, want_rows=True)
    torch.cuda.synchronize()
    rows = res["rows"].cpu().numpy()[0]
    worst = 0.0
    for j, fc in enumerate(centres):
        fr = _trials(fc, hw, R)
        ref = ora.dchi2(cur.t, cur.x, cur.sigma, fr, cur.H, with_coeffs=True)
        gate = ora.gate_mask(ref, fr, 1e6)
        e = ora.rel_err(rows[j].T, ref["dchi2"])[:, gate]
        worst = max(worst, float(e.max()))
        # best trial of row H: the oracle's arg max, ties within the tolerance allowed
        d_ora = ref["dchi2"][cur.H - 1]
        fb = res["f_best"][0, j].item()
        rb = int(np.argmin(np.abs(fr - fb)))
        assert fr[rb] == pytest.approx(fb, rel=0, abs=1e-12 * fc)
        assert d_ora[rb] >= d_ora.max() - 1e-9 * max(d_ora.max(), 2 * cur.H)
        np.testing.assert_allclose(res["dchi2_best"][0, j].cpu().numpy(), rows[j, rb], rtol=0,
                                   atol=0)
        if gate[rb]:
            A = res["coef"][0, j].cpu().numpy()
            Ar = ref["coeffs"][rb]
            assert np.max(np.abs(A - Ar)) <= 1e-8 * np.max(np.abs(Ar)), (fc, A, Ar)
    print(f"fine {name}: worst gated rel err over {len(centres)}x{R} trials {worst:.3e}",
          flush=True)
    assert worst <= 1e-9


def test_refine_finds_the_local_optimum_long():
    """Three zoom levels around the sawtooth frequency of the long workload reach
    the optimum of an oracle scan of the same neighbourhood."""
    import torch
    cur = synth.make("long")
    note("fine refine long workload (n=1e5) vs oracle scan")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
    t, x, s = to_dev(cur)
    f0 = 1.0 / 0.731
    df = cur.f_max / cur.n_freq
    fc = round(f0 / df) * df              # the nearest grid bin, as a search would give
    res = plan.refine(t, x, s, _centres(1, [fc, 2 * fc]), levels=3, R=64)
    torch.cuda.synchronize()
    fb = res["f_best"][0, 0].item()
    db = res["dchi2_best"][0, 0].cpu().numpy()
    scan = np.linspace(fc - df, fc + df, 201)
    ref = ora.dchi2(cur.t, cur.x, cur.sigma, scan, cur.H)["dchi2"][cur.H - 1]
    step = scan[1] - scan[0]
    k = int(np.argmax(ref))
    print(f"refine: f_best {fb:.10f}, oracle scan optimum {scan[k]:.10f} (step {step:.2e}); "
          f"Delta {db[-1]:.6f} vs {ref[k]:.6f}", flush=True)
    assert abs(fb - scan[k]) <= step
    assert db[-1] >= ref[k] * (1 - 1e-9)  # at least as good as the finer scan's best
    one = ora.dchi2(cur.t, cur.x, cur.sigma, [fb], cur.H)["dchi2"][:, 0]
    assert np.max(ora.rel_err(db[:, None], one[:, None])) <= 1e-9


def test_batch_sampled_curves():
    import torch
    cur = synth.make("batch")
    note("fine search batch (1e4 curves, K=2, R=32) vs oracle samples")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
    t, x, s = to_dev(cur)
    centres = [0.5317, 1.7]
    hw = 4 * cur.f_max / cur.n_freq
    res = plan.fine_search(t, x, s, _centres(cur.n_curves, centres), R=32, half_width=hw,
                           want_rows=True)
    rows = res["rows"].cpu().numpy()
    rng = np.random.default_rng(91)
    worst = 0.0
    for c in rng.choice(cur.n_curves, 12, replace=False):
        tc, xc, sc = cur.curve(int(c))
        for j, fc in enumerate(centres):
            fr = _trials(fc, hw, 32)
            ref = ora.dchi2(tc, xc, sc, fr, cur.H)
            gate = ora.gate_mask(ref, fr, 1e6)
            if gate.any():
                worst = max(worst, float(ora.rel_err(rows[c, j].T, ref["dchi2"])[:, gate].max()))
    print(f"fine batch: worst gated rel err {worst:.3e}", flush=True)
    assert worst <= 1e-9


def test_edge_cases_and_determinism():
    import torch
    cur = synth.make("plain", n_freq=1 << 12, f_max=2.5)
    n = cur.t.shape[0]
    t2 = np.concatenate([cur.t, cur.t])
    x2 = np.concatenate([cur.x, cur.x])
    x2[n + 3] = np.inf
    s2 = np.concatenate([cur.sigma, cur.sigma])
    plan = F.Plan([0, n, 2 * n], cur.f_max, cur.H, cur.n_freq, precision="fp64")
    note("fine search edge cases: NaN centre, rejected curve, R=1, hw=0, repeat")
    tt, xx, ss = (torch.from_numpy(a).cuda() for a in (t2, x2, s2))
    fcs = torch.tensor([[0.42, float("nan"), -1.0], [0.42, 0.5, 0.6]], dtype=torch.float64,
                       device="cuda")
    r1 = plan.fine_search(tt, xx, ss, fcs, R=1)
    r2 = plan.fine_search(tt, xx, ss, fcs, R=17, half_width=0.0)
    a = plan.fine_search(tt, xx, ss, fcs, R=40)
    b = plan.fine_search(tt, xx, ss, fcs, R=40)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(torch.nan_to_num(a[k].double(), nan=-7.0),
                           torch.nan_to_num(b[k].double(), nan=-7.0)), k
    f1 = r1["f_best"].cpu().numpy()
    assert f1[0, 0] == 0.42 and np.isnan(f1[0, 1]) and np.isnan(f1[0, 2])
    assert np.all(np.isnan(f1[1]))
    assert r1["flags"][1, 0].item() & F.CURVE_NONFINITE
    assert r2["f_best"][0, 0].item() == 0.42
    torch.testing.assert_close(r1["dchi2_best"][0, 0], r2["dchi2_best"][0, 0], rtol=0, atol=0)
    ref = ora.dchi2(cur.t, cur.x, cur.sigma, [0.42], cur.H, with_coeffs=True)
    assert np.max(ora.rel_err(r1["dchi2_best"][0, 0].cpu().numpy()[:, None],
                              ref["dchi2"])) <= 1e-9
    with pytest.raises(F.FChi2Error):
        plan.fine_search(tt, xx, ss, fcs, R=5000)
    with pytest.raises(F.FChi2Error):
        plan.fine_search(tt, xx, ss, fcs, R=8, half_width=-1.0)
