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
    """tasks: list of (t, x, sigma, freqs, H); returns the oracle dicts."""
    import multiprocessing as mp
    with mp.get_context("fork").Pool(pool_size()) as pool:
        return pool.map(_task, tasks, chunksize=1)


def split_bins(bins, parts):
    return [b for b in np.array_split(np.asarray(bins), max(1, parts)) if len(b)]
