"""Harmonic phases that wrap around the periodic grid.

With a coarse grid (2H * span * f_max / n_freq above 1) the phase m u of the
higher harmonics runs over several periods of the grid; the transforms at
integer bins do not change by whole periods (Section 2's Q and P at f_k), so
the search must still match the oracle.  Cases: three periods (t_span given,
the plan covers them), the paper's own density (os = 2, Section 3a, where the
top harmonic just passes one period with the kernel's reach), the standalone
and the fused spreading, both precisions, the adjoint, and the flag for a
curve that needs more periods than a plan without t_span covers (two)."""
import numpy as np
import pytest

from oracle import fchi2_oracle as ora
from paper_0901_1913_amd import fchi2 as F
from paper_0901_1913_amd import synth
from tests.gpu_util import note, sample_bins, to_dev

pytestmark = pytest.mark.gpu

KAPPA = {"mixed": 1e2, "fp64": 1e6}
TOL = {"mixed": 1e-5, "fp64": 1e-8}


def _parity(cur, d, label, precision, nb=160, seed=3):
    bins = sample_bins(cur.n_freq, nb, seed)
    fr = bins * (cur.f_max / cur.n_freq)
    r = ora.dchi2(cur.t, cur.x, cur.sigma, fr, cur.H)
    gate = ora.gate_mask(r, fr, KAPPA[precision])
    e = ora.rel_err(d[:, bins], r["dchi2"])[:, gate]
    print(f"{label}: gated {gate.sum()}/{len(bins)} max {e.max():.3e} median "
          f"{np.median(e):.3e}", flush=True)
    assert gate.sum() > 0.5 * len(bins) and e.max() <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("fused", [False, True])
def test_three_periods_match_oracle(precision, fused):
    import torch
    cur = synth.make("plain", n=700, n_freq=2 ** 11, f_max=10.0, precision=precision)
    span = float(cur.t[-1] - cur.t[0])
    reach = 2 * cur.H * span * cur.f_max / cur.n_freq
    note(f"wrap {reach:.2f} periods {precision} fused={fused}")
    assert reach > 2.5
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=precision,
                  t_span=[span], fused_spread=fused)
    t, x, s = to_dev(cur)
    d, c0, fl = plan.search(t, x, s)
    torch.cuda.synchronize()
    assert not (fl.cpu().numpy() & F.CURVE_WRAP).any()
    _parity(cur, d.double().cpu().numpy()[0], f"3 periods {precision} fused={fused}",
            precision)


def test_flagged_beyond_the_plans_periods():
    import torch
    cur = synth.make("plain", n=700, n_freq=2 ** 11, f_max=10.0, precision="mixed")
    note("wrap beyond two periods without t_span")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
    t, x, s = to_dev(cur)
    d, c0, fl = plan.search(t, x, s)
    torch.cuda.synchronize()
    assert (fl.cpu().numpy()[0] & F.CURVE_WRAP).all()
    assert torch.isnan(d).all() and torch.isnan(c0).all()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_papers_density(precision):
    """n_freq from os = 2: bin spacing 1/(2 H span) up to f_max, Section 3a."""
    import torch
    cur = synth.make("batch", n_curves=4, n_lo=300, n_hi=900, span_lo=200.0, span_hi=400.0,
                     precision=precision)
    spans = [float(cur.curve(c)[0][-1] - cur.curve(c)[0][0]) for c in range(cur.n_curves)]
    # f_max chosen so that os H span f_max lands just below 2^13: the grid is
    # then exactly as fine as the paper asks, and the top harmonic's phase
    # (plus the kernel's reach and the origin shift) passes one period.
    cur.f_max = 8191.9 / (2.0 * cur.H * max(spans))
    nf = F.auto_n_freq(cur.H, cur.f_max, 2.0, max(spans))
    assert nf == 2 ** 13
    L = 4 * nf
    w = 14 if precision == "fp64" else 10
    reach = 2 * cur.H * max(spans) * cur.f_max / nf * L + (w // 2 + 2) + w // 2 + 3
    assert reach > L
    note(f"paper's density: n_freq {nf} {precision}")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, 0, precision=precision, oversampling=2.0,
                  t_span=spans)
    assert plan.n_freq == nf
    t, x, s = to_dev(cur)
    d, c0, fl = plan.search(t, x, s)
    torch.cuda.synchronize()
    assert not (fl.cpu().numpy() & F.CURVE_WRAP).any()
    cur.n_freq = plan.n_freq
    dd = d.double().cpu().numpy()
    for c in range(cur.n_curves):
        one = synth.Curves(*[np.ascontiguousarray(a) for a in cur.curve(c)],
                           offsets=np.array([0, cur.curve(c)[0].shape[0]]), H=cur.H,
                           n_freq=cur.n_freq, f_max=cur.f_max, precision=precision)
        _parity(one, dd[c], f"os=2 curve {c} {precision}", precision, nb=60, seed=c)


def test_adjoint_with_wrap():
    """The adjoint gathers the periodic grid modulo its length."""
    import torch
    cur = synth.make("diff", n=1500, span=500.0, n_freq=2 ** 13, f_max=5.0, precision="fp64")
    span = float(cur.t[-1] - cur.t[0])
    reach = 2 * cur.H * span * cur.f_max / cur.n_freq
    note(f"adjoint with {reach:.2f} periods")
    assert reach > 1.2
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="fp64",
                  keep_for_backward=True, t_span=[span])
    t, x, s = to_dev(cur)
    d, _, _ = plan.search(t, x, s)
    idx = plan.top_peaks(d, cur.H - 1, int(np.ceil(cur.n_freq / (span * cur.f_max))), 8)
    g = torch.zeros_like(d)
    g[0, cur.H - 1, idx[0]] = 1.0
    gx, gs = plan.backward(t, x, s, g)
    torch.cuda.synchronize()
    df = cur.f_max / cur.n_freq
    terms = [(float(k) * df, cur.H, 1.0) for k in idx[0].cpu().numpy() if k >= 0]
    rx, rs = ora.grad(cur.t, cur.x, cur.sigma, terms)
    ex = np.linalg.norm(gx.cpu().numpy() - rx) / np.linalg.norm(rx)
    es = np.linalg.norm(gs.cpu().numpy() - rs) / np.linalg.norm(rs)
    print(f"adjoint with wrap: rel l2 dx {ex:.3e} dsigma {es:.3e}", flush=True)
    assert ex <= 1e-8 and es <= 1e-8
