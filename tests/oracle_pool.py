"""Run the FP64 oracle over many (curve, bins) tasks on the host's CPU share
(at most 16 processes), for the full-size parity tests."""
import os

import numpy as np


def _task(args):
    t, x, s, freqs, H = args
    from threadpoolctl import threadpool_limits
    from oracle import fchi2_oracle as ora
    with threadpool_limits(1):
        r = ora.dchi2(t, x, s, freqs, H)
    return r


def pool_size():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def run(tasks):
    """tasks: list of (t, x, sigma, freqs, H); returns the oracle dicts (in
    task order), noting progress every tenth of the tasks."""
    import multiprocessing as mp
    from tests.gpu_util import note
    out = [None] * len(tasks)
    step = max(1, len(tasks) // 10)
    with mp.get_context("fork").Pool(pool_size()) as pool:
        for done, (i, r) in enumerate(pool.imap_unordered(_indexed, enumerate(tasks)), 1):
            out[i] = r
            if done % step == 0 or done == len(tasks):
                note(f"oracle: {done}/{len(tasks)} tasks done")
    return out


def _indexed(item):
    i, args = item
    return i, _task(args)


def split_bins(bins, parts):
    return [b for b in np.array_split(np.asarray(bins), max(1, parts)) if len(b)]
