"""Helpers for the GPU tests: run the HIP path through the C ABI binding."""
import os
import sys

import numpy as np

from paper_0901_1913_amd import fchi2 as F


def note(msg):
    """Name the case before a GPU step (flushed so a crash still shows it).
    With FCHI2_TEST_PROGRESS set to a file path, the line is also appended
    there (pytest holds a test's own output until the test ends)."""
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()
    path = os.environ.get("FCHI2_TEST_PROGRESS")
    if path:
        with open(path, "a") as fh:
            fh.write(f"[gpu] {msg}\n")


def to_dev(curves):
    import torch
    t = torch.from_numpy(curves.t).cuda()
    x = torch.from_numpy(curves.x).cuda()
    s = torch.from_numpy(curves.sigma).cuda()
    return t, x, s


def run_search(curves, precision=None, tune=False, **plan_kw):
    """Delta chi2 [n_curves, H, n_freq] (float64 numpy), chi2_0, flags, plan.

    tune=True runs the autotuner first, as bench.py does before timing.
    """
    import torch
    precision = precision or curves.precision
    plan = F.Plan(curves.offsets, curves.f_max, curves.H, curves.n_freq,
                  precision=precision, **plan_kw)
    t, x, s = to_dev(curves)
    if tune:
        print(f"[gpu] autotuned: {plan.autotune(t, x, s)}", flush=True)
    d, c0, fl = plan.search(t, x, s)
    torch.cuda.synchronize()
    return (d.double().cpu().numpy(), c0.cpu().numpy(), fl.cpu().numpy(), plan)


def sample_bins(n_freq, n, seed, k_min=1):
    rng = np.random.default_rng(seed)
    b = rng.choice(np.arange(k_min, n_freq), size=min(n, n_freq - k_min), replace=False)
    return np.sort(np.concatenate([b, [k_min, n_freq - 1]])).astype(np.int64)
