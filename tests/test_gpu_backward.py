"""Adjoint (fchi2_backward / FChi2Fn) against the oracle's closed-form gradient
and central finite differences, and the top-K peak picker."""
import numpy as np
import pytest

from oracle import fchi2_oracle as ora
from paper_0901_1913_amd import fchi2 as F
from paper_0901_1913_amd import synth
from tests.gpu_util import note, to_dev

pytestmark = pytest.mark.gpu


def _diff_small(precision):
    return synth.make("diff", n=2000, span=500.0, n_freq=2 ** 14, f_max=4.0,
                      precision=precision)


def _peaks(plan, dchi2, cur, K=16):
    import torch
    span = cur.t[-1] - cur.t[0]
    df = cur.f_max / cur.n_freq
    k_lo = int(np.ceil(1.0 / (span * df)))
    idx = plan.top_peaks(dchi2, cur.H - 1, k_lo, K)
    torch.cuda.synchronize()
    return idx.cpu().numpy()[0], k_lo


def _check_peaks(d, idx, k_lo, K):
    """Peaks are strict local maxima, in descending order, and the top K."""
    row = d
    k = np.arange(k_lo, row.shape[0] - 1)
    is_max = (row[k] > row[k - 1]) & (row[k] >= row[k + 1])
    cand = k[is_max]
    order = np.lexsort((cand, -row[cand]))
    expect = cand[order][:K]
    assert np.array_equal(idx[: len(expect)], expect), (idx, expect)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-5)])
def test_backward_matches_closed_form(precision, tol):
    import torch
    cur = _diff_small(precision)
    note(f"backward {precision}")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=precision,
                  keep_for_backward=True)
    t, x, s = to_dev(cur)
    d, _, _ = plan.search(t, x, s)
    idx, k_lo = _peaks(plan, d, cur)
    _check_peaks(d.double().cpu().numpy()[0][cur.H - 1], idx, k_lo, 16)
    g = torch.zeros_like(d)
    # Loss: sum of Delta(H) over the top peaks, plus 0.5 * Delta(1) at a bin.
    g[0, cur.H - 1, torch.from_numpy(idx).cuda()] = 1.0
    kb = int(idx[3]) + 5
    g[0, 0, kb] = 0.5
    gx, gs = plan.backward(t, x, s, g)
    torch.cuda.synchronize()
    gx, gs = gx.cpu().numpy(), gs.cpu().numpy()
    df = cur.f_max / cur.n_freq
    terms = [(float(k) * df, cur.H, 1.0) for k in idx] + [(kb * df, 1, 0.5)]
    rx, rs = ora.grad(cur.t, cur.x, cur.sigma, terms)
    ex = np.linalg.norm(gx - rx) / np.linalg.norm(rx)
    es = np.linalg.norm(gs - rs) / np.linalg.norm(rs)
    print(f"backward {precision}: rel l2 dx {ex:.3e} dsigma {es:.3e}", flush=True)
    assert ex <= tol and es <= tol


def test_autograd_function_and_finite_differences():
    import torch
    cur = _diff_small("fp64")
    note("autograd + FD fp64")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="fp64",
                  keep_for_backward=True)
    t, x, s = to_dev(cur)
    d0, _, _ = plan.search(t, x, s)
    idx, _ = _peaks(plan, d0, cur)
    sel = torch.from_numpy(idx).cuda()
    xr = x.clone().requires_grad_(True)
    sr = s.clone().requires_grad_(True)
    Fn = F.fchi2_fn()
    loss = Fn.apply(t, xr, sr, plan)[0, cur.H - 1, sel].sum()
    loss.backward()
    gx = xr.grad.cpu().numpy()
    gs = sr.grad.cpu().numpy()

    def L(xx, ss):
        dd, _, _ = plan.search(t, xx, ss)
        return float(dd[0, cur.H - 1, sel].sum())

    for i in (0, 17, 999, 1999):
        h = 1e-3
        xp, xm = x.clone(), x.clone()
        xp[i] += h
        xm[i] -= h
        fd = (L(xp, s) - L(xm, s)) / (2 * h)
        assert abs(fd - gx[i]) <= 1e-6 * max(1.0, abs(gx[i])), (i, fd, gx[i])
        h = 1e-5 * float(s[i])
        sp, sm = s.clone(), s.clone()
        sp[i] += h
        sm[i] -= h
        fd = (L(x, sp) - L(x, sm)) / (2 * h)
        assert abs(fd - gs[i]) <= 1e-4 * max(1.0, abs(gs[i])), (i, fd, gs[i])


def test_backward_requires_keep_flag():
    import torch
    cur = _diff_small("mixed")
    note("backward without keep flag")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
    t, x, s = to_dev(cur)
    d, _, _ = plan.search(t, x, s)
    with pytest.raises(F.FChi2Error) as e:
        plan.backward(t, x, s, torch.zeros_like(d))
    assert e.value.status == F.ERR_STATE


def test_backward_of_an_older_forward_is_refused():
    """Two forwards on one plan, then the backward of the first: the workspace
    holds the second's spectra, so the gradient must be refused, not taken."""
    import torch
    cur = _diff_small("mixed")
    note("backward of an older forward")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed",
                  keep_for_backward=True)
    t, x, s = to_dev(cur)
    Fn = F.fchi2_fn()
    x1 = x.clone().requires_grad_(True)
    x2 = (1.5 * x).requires_grad_(True)
    d1 = Fn.apply(t, x1, s, plan)
    d2 = Fn.apply(t, x2, s, plan)
    with pytest.raises(F.FChi2Error) as e:
        d1[0, cur.H - 1, 100:200].sum().backward()
    assert e.value.status == F.ERR_STATE
    # The most recent forward still differentiates.
    d2[0, cur.H - 1, 100:200].sum().backward()
    torch.cuda.synchronize()
    assert torch.isfinite(x2.grad).all()


def test_autograd_sorts_each_curve_and_returns_gradients_in_caller_order():
    """FChi2Fn(..., sort=True) on points shuffled within each curve: the rows
    equal those of the time-ordered input bit for bit and the gradients come
    back in the caller's order; without the sort the shuffled curves are
    flagged and get NaN rows."""
    import torch
    cur = synth.make("batch", n_curves=3, n_freq=2 ** 13, f_max=4.0, n_lo=200, n_hi=800)
    note("autograd with per-curve time sort, 3 shuffled curves")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed",
                  keep_for_backward=True)
    t, x, s = to_dev(cur)
    rng = np.random.default_rng(5)
    off = cur.offsets
    perm = np.concatenate([a + rng.permutation(b - a) for a, b in zip(off[:-1], off[1:])])
    pt = torch.from_numpy(perm).cuda()
    Fn = F.fchi2_fn()
    xr, sr = x.clone().requires_grad_(True), s.clone().requires_grad_(True)
    d_ref = Fn.apply(t, xr, sr, plan)
    d_ref[:, cur.H - 1, 100:300].sum().backward()
    xq, sq = x[pt].clone().requires_grad_(True), s[pt].clone().requires_grad_(True)
    d = Fn.apply(t[pt], xq, sq, plan, True)
    d[:, cur.H - 1, 100:300].sum().backward()
    torch.cuda.synchronize()
    assert torch.equal(d.detach(), d_ref.detach())
    assert torch.isfinite(xr.grad).all() and torch.isfinite(sr.grad).all()
    assert torch.equal(xq.grad, xr.grad[pt]) and torch.equal(sq.grad, sr.grad[pt])
    d_bad, _, fl = plan.search(t[pt], x[pt], s[pt])
    torch.cuda.synchronize()
    assert torch.isnan(d_bad).all()
    assert (fl.cpu().numpy() & F.CURVE_UNSORTED).all()
