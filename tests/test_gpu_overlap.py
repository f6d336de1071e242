"""The overlapped wave schedule (FCHI2_TWO_STREAMS, waves of at most half the
buffers' capacity: the next wave's spreading on a second stream while the
current wave's FFT passes and solve run) launches the staged search's
kernels on the same curves, so every output is identical bit for bit to the
one-stream schedule: rows, chi2_0, flags, coefficients, the adjoint, curve
subsets, graph replays (captured across both streams), profiled runs and the
top-K epilogue."""
import numpy as np
import pytest

from paper_0901_1913_amd import fchi2 as F
from paper_0901_1913_amd import synth
from tests.gpu_util import note, to_dev
from tests.test_gpu_fused import same_bits

pytestmark = pytest.mark.gpu


def _cur():
    return synth.make("batch", n_curves=43, n_freq=2 ** 14, f_max=6.0, n_lo=20, n_hi=4000,
                      span_hi=150.0)


def test_overlap_identical_outputs_and_adjoint():
    import torch
    cur = _cur()
    t, x, s = to_dev(cur)
    outs = []
    for wave, sub, two in ((43, 0, True), (10, 0, True), (21, 5, True), (7, 0, True),
                           (10, 0, False)):
        note(f"overlap: wave {wave}, sub {sub}, two streams {two}")
        plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed",
                      keep_for_backward=True, two_streams=two)
        plan.set_schedule(dict(plan.info(), curves_per_wave=wave, solve_sub_wave=sub))
        d, c0, fl, coef = plan.search_coeffs(t, x, s)
        d2, _, fl2 = plan.search(t, x, s)
        g = torch.zeros_like(d2)
        g[:, cur.H - 1, 200:230] = 1.0
        gx, gs = plan.backward(t, x, s, g)
        torch.cuda.synchronize()
        outs.append([v.cpu() for v in (d, c0, fl, coef, d2, fl2, gx, gs)])
        plan.close()
    for o in outs[1:]:
        for u, v in zip(outs[0], o):
            assert same_bits(u, v)
    assert np.isfinite(outs[0][0].double().numpy()).any()


def test_overlap_subset_graph_and_profile():
    import torch
    cur = _cur()
    t, x, s = to_dev(cur)
    ref = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed")
    ref.set_schedule(dict(ref.info(), curves_per_wave=43))
    rd, rc, rf = ref.search(t, x, s)
    torch.cuda.synchronize()
    rd, rc, rf = rd.cpu(), rc.cpu(), rf.cpu()
    ref.close()
    note("overlap: curve subset")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed", graph=True,
                  two_streams=True)
    plan.set_schedule(dict(plan.info(), curves_per_wave=6))
    d = torch.full((cur.n_curves, cur.H, cur.n_freq), -1.0, dtype=torch.float32, device="cuda")
    c0 = torch.full((cur.n_curves,), -1.0, dtype=torch.float64, device="cuda")
    fl = torch.zeros((cur.n_curves, cur.n_freq), dtype=torch.uint8, device="cuda")
    plan.search_curves(5, 29, t, x, s, d, c0, fl)
    torch.cuda.synchronize()
    assert same_bits(d.cpu()[5:34], rd[5:34]) and same_bits(fl.cpu()[5:34], rf[5:34])
    assert (d.cpu()[:5] == -1.0).all() and (d.cpu()[34:] == -1.0).all()
    note("overlap: graph replays with eager searches between")
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        for rep in range(3):
            dd, cc, ff = plan.search(t, x, s, stream=st)
            st.synchronize()
            assert same_bits(dd.cpu(), rd) and same_bits(cc.cpu(), rc) and same_bits(ff.cpu(), rf)
            d2, _, _ = plan.search(t, x, s)  # eager (default stream, no graph)
            torch.cuda.synchronize()
            assert same_bits(d2.cpu(), rd)
    note("overlap: profiled search")
    plan.profile(True)
    dd, _, _ = plan.search(t, x, s)
    pr = plan.profile_read()
    plan.profile(False)
    torch.cuda.synchronize()
    assert same_bits(dd.cpu(), rd)
    waves = (cur.n_curves + 5) // 6
    assert pr["spread"][1] == waves and pr["fft_first"][1] == waves and pr["solve"][1] == waves
    plan.close()


def test_overlap_top_candidates_identical():
    """The search with the significance epilogue on overlapped waves selects
    the same candidates with the same values as on one wave."""
    import torch
    cur = _cur()
    t, x, s = to_dev(cur)
    outs = []
    for wave in (43, 10, 7):
        note(f"overlap: top-16 search, wave {wave}")
        plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision="mixed",
                      two_streams=True)
        plan.set_schedule(dict(plan.info(), curves_per_wave=wave))
        top = plan.search_top(t, x, s, K=16, k_lo=3)
        torch.cuda.synchronize()
        outs.append({k: v.cpu() for k, v in top.items()})
        plan.close()
    for o in outs[1:]:
        for k in outs[0]:
            assert same_bits(outs[0][k], o[k]), k
    assert (outs[0]["idx"] >= 0).any()
