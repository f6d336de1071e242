#!/usr/bin/env python3
"""Throughput of the F-chi2 hot path on one MI355X.

The headline is the batched survey: one step is one fchi2_search over all
10^4 curves of the batch workload (moments, spreading, FFT passes, per-bin
assembly and Cholesky for every H'), replayed from a HIP graph, with the
inputs already resident in device memory; the value is trial frequencies x H
per second.  The same search run as a loop of single-curve calls (the plain
form, same kernels) is timed beside it.

Prints one JSON line.  Beside the throughput it reports the roofline of the
kernel that takes the most time (algorithmic bytes per launch: 3H real grids
of 4 or 8 bytes per cell, a full FFT pass reading and writing each once;
over its average launch duration measured with HIP events on the search
stream in a separate profiled pass), the same model for the gridding + FFT
stages and for the whole step, the FP64 solve rate, the FP64 CPU oracle
timed on a bounded sample of the batch (whose values double as a parity
check), one line per other workload (plain FP64, long curve,
differentiation, precision stress in mixed and FP64), and extras: the fused
top-16 search, shared-alpha sources, floor gridding and detrending, the
fine search around the long curve's peaks, and frequency-band shares.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
METRIC = ("trial freqs·H/sec for Δχ² (rel err ≤1e-5 vs FP64 oracle); "
          "batched vs plain")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def model_bytes(n, H, n_freq, b, o):
    """Algorithmic bytes per curve, by the byte model of the HBM-grid
    schedule (3H real grids of L = 4 n_freq cells of b bytes, a
    two-pass FFT with an output-pruned last pass, o-byte outputs):
    inputs 24 n; spreading writes L; FFT pass 1 reads and writes L; the last
    pass reads L and writes 2 n_freq; the assembly reads 2 n_freq; output
    H n_freq o.  A full read + write pass of the grids is 2 L per grid."""
    L = 4 * n_freq
    g = 3 * H * b
    return {"inputs": 24 * n, "spread": g * L, "full_pass": g * 2 * L,
            "last_pass": g * (L + 2 * n_freq), "solve": g * 2 * n_freq + H * n_freq * o,
            "gridding_fft": 24 * n + g * (4 * L + 2 * n_freq),
            "step": 24 * n + g * (4 * L + 4 * n_freq) + H * n_freq * o}


def solve_flops(H):
    """FP64 flops per bin of assembly + prefix Cholesky:
    d^3/3 + 2 d^2 + d (d + 1), d = 2H + 1."""
    d = 2 * H + 1
    return d ** 3 / 3 + 2 * d * d + d * (d + 1)


def stage_roofline(cur, stages, steps_profiled, b, o, schedule):
    """Per-stage bytes by the byte model and rates from a profiled
    pass: the dominant kernel's roofline, the gridding + FFT and whole-step
    effective bandwidths, and the solve's FP64 rate.  Each FFT pass is a full
    read and write of the grids (a schedule with more than two passes moves
    more than the two-pass model counts); with the spreading fused into the
    first pass, that pass is also charged the spreading's grid write; the
    persistent search (one launch for the whole chain) is charged the whole
    step's bytes."""
    H, nf, nc = cur.H, cur.n_freq, cur.n_curves
    n_tot = int(cur.t.shape[0])
    m = model_bytes(n_tot / nc, H, nf, b, o)
    n_pass = len(schedule["fft_log_radices"])
    per_stage_bytes = {  # per search, all curves
        "spread": nc * (m["spread"]) + 24 * n_tot,
        "fft_first": nc * m["full_pass"], "fft_mid": nc * m["full_pass"] * max(0, n_pass - 2),
        "fft_last": nc * m["last_pass"], "solve": nc * m["solve"]}
    if schedule.get("fused_spread"):
        per_stage_bytes["fft_first"] += nc * m["spread"]
        per_stage_bytes["spread"] = 24 * n_tot
    if schedule.get("persistent"):
        per_stage_bytes = {"persistent": nc * m["step"]}
    ms = {k: v[0] / steps_profiled for k, v in stages.items() if v[1]}
    launches = {k: v[1] / steps_profiled for k, v in stages.items() if v[1]}
    cand = {k: ms[k] for k in per_stage_bytes if k in ms}
    dom = max(cand, key=cand.get)
    avg_launch_ms = ms[dom] / launches[dom]
    bytes_launch = per_stage_bytes[dom] / launches[dom]
    achieved = bytes_launch / (avg_launch_ms * 1e-3) / 1e9
    fft_ms = sum(ms.get(k, 0.0) for k in ("spread", "fft_first", "fft_mid", "fft_last"))
    if "persistent" in ms:  # one launch: no separate gridding + FFT time
        fft_ms = step_ms = sum(ms.values())
    step_ms = sum(ms.values())
    grid_gb = nc * m["gridding_fft"] / 1e9
    step_gb = nc * m["step"] / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None, "bytes_per_launch": int(bytes_launch),
            "avg_launch_ms": round(avg_launch_ms, 5), "launches_per_step": launches[dom],
            "byte_model": "3H real grids x b bytes: a full pass reads and writes 2 L per grid"}
    sections = {
        "gridding_fft": {"gb_per_step_model": round(grid_gb, 2), "ms": round(fft_ms, 4),
                         "gbs": round(grid_gb / (fft_ms * 1e-3), 1),
                         "frac": round(grid_gb / (fft_ms * 1e-3) / HBM_PEAK_GBS, 4)},
        "whole_step": {"gb_per_step_model": round(step_gb, 2), "ms": round(step_ms, 4),
                       "gbs": round(step_gb / (step_ms * 1e-3), 1),
                       "frac": round(step_gb / (step_ms * 1e-3) / HBM_PEAK_GBS, 4)},
    }
    if "persistent" in ms:
        sections["gridding_fft"] = None
    if "solve" in ms:
        fl = solve_flops(H) * nf * nc
        tf = fl / (ms["solve"] * 1e-3) / 1e12
        sections["solve_fp64"] = {"tflops": round(tf, 2), "peak": FP64_PEAK_TFLOPS,
                                  "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                                  "flops_per_bin": round(solve_flops(H), 1)}
    stage_ms = {k: round(v, 5) for k, v in ms.items()}
    return roof, sections, stage_ms


# Source files of each stage's kernels: a stage's measured traffic is used
# only while the hash of these files matches the one stored with it.
_FFT_SRC = ["fft.hip", "fft_tile.h"]
STAGE_SOURCES = {
    "fft_first": _FFT_SRC, "fft_mid": _FFT_SRC, "fft_last": _FFT_SRC,
    "solve": ["solve.hip", "solve_bin.h"],
    "spread": ["spread.hip", "spread_tile.h", "es_kernel.h"],
    "persistent": ["persist.hip", "fft_tile.h", "spread_tile.h", "solve_bin.h"],
}


def stage_source_hash(stage):
    """First 16 hex digits of the sha256 of the stage's kernel sources, or
    None if the stage or a file is unknown."""
    import hashlib
    if stage not in STAGE_SOURCES:
        return None
    h = hashlib.sha256()
    for f in STAGE_SOURCES[stage]:
        fp = os.path.join(ROOT, "paper_0901_1913_amd", "csrc", f)
        if not os.path.isfile(fp):
            return None
        h.update(open(fp, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(name):
    """HBM bytes per curve of each stage's launch from a committed rocprofv3
    PMC summary (profiles/<name>_hbm_traffic.md: bytes per launch of
    curves_per_launch curves), or {} if there is none, or None for a stage
    whose kernel source changed since the counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", f"{name}_hbm_traffic.md")
    if not os.path.exists(path):
        return {}
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return {}
    meta = json.loads(m.group(1))
    out = {}
    per = max(1, int(meta.get("curves_per_launch", 1)))
    for st, nbytes in meta.get("bytes_per_launch", {}).items():
        hx = stage_source_hash(st)
        ok = hx is not None and hx == meta.get("source_sha256_16", {}).get(st)
        out[st] = (float(nbytes) / per) if ok else None
    return out


def _oracle_task(args):
    t, x, s, freqs, H = args
    from threadpoolctl import threadpool_limits
    from oracle import fchi2_oracle as ora
    with threadpool_limits(1):
        r = ora.dchi2(t, x, s, freqs, H)
    return r["dchi2"], r["kappa"], r["span"]


def pool_size():
    """Worker processes for the oracle: the CPUs this process may run on,
    capped at 16 (the host CPU share that goes with one GPU on the benchmark
    machines, whatever the host reports in all)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_pool(tasks):
    """Run oracle tasks on pool_size() processes; returns the results, the
    wall time and the number of processes."""
    import multiprocessing as mp
    cores = pool_size()
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_task, tasks, chunksize=1)
    return res, time.perf_counter() - t0, cores


BINS_EACH = 80  # oracle bins on every curve of the batch sample


def batch_sample(cur, seed=7, n_strat=32, bins_strat=96, bins_each=BINS_EACH):
    """The bounded oracle sample of the batch: 32 curves stratified by length
    and by signal / noise (8 length quartile x signal classes, 4 curves each)
    with bins_strat seeded random bins each, plus bins_each random bins on
    every curve.  Returns {curve: sorted bins}."""
    rng = np.random.default_rng(seed)
    nc = cur.n_curves
    n = np.diff(cur.offsets)
    sig = np.asarray(cur.meta.get("with_signal", np.zeros(nc, dtype=bool)), dtype=bool)
    q = np.searchsorted(np.quantile(n, [0.25, 0.5, 0.75]), n, side="right")
    pick = []
    for qq in range(4):
        for ss in (False, True):
            idx = np.nonzero((q == qq) & (sig == ss))[0]
            pick += list(rng.choice(idx, size=min(n_strat // 8, len(idx)), replace=False))
    sample = {}
    for c in range(nc):
        sample[c] = set(rng.choice(np.arange(1, cur.n_freq), size=bins_each, replace=False))
    for c in pick:
        sample[int(c)] |= set(rng.choice(np.arange(1, cur.n_freq), size=bins_strat,
                                         replace=False))
    return {c: np.array(sorted(b), dtype=np.int64) for c, b in sample.items()}, \
        [int(c) for c in pick]


def parity_summary(errs, gates):
    e = np.concatenate([x[:, g].ravel() for x, g in zip(errs, gates)])
    a = np.concatenate([x.ravel() for x in errs])
    return {"gated_values": int(e.size), "max_rel_err_gated": float(e.max()) if e.size else None,
            "median_rel_err_gated": float(np.median(e)) if e.size else None,
            "max_rel_err_all": float(a.max())}


_LAST_MEDIAN = {}


def time_search(plan, t, x, s, steps, warmup, stream, **kw):
    """Mean over `steps` searches after `warmup` (HIP events on the search
    stream, one between consecutive searches, none inside a search); the
    median of the per-search times is kept in _LAST_MEDIAN["ms"]."""
    import torch
    d = kw.pop("dchi2")
    for _ in range(warmup):
        plan.search(t, x, s, dchi2=d, stream=stream, **kw)
    stream.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    w0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        plan.search(t, x, s, dchi2=d, stream=stream, **kw)
        ev[i + 1].record(stream)
    stream.synchronize()
    wall = time.perf_counter() - w0
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    _LAST_MEDIAN["ms"] = float(np.median(per))
    return ev[0].elapsed_time(ev[steps]) / steps, 1e3 * wall / steps


def profiled_pass(plan, t, x, s, stream, reps=1, **kw):
    """Per-stage launch times from the library's event pairs (graph replay is
    bypassed while profiling): {stage: (total ms, launches)} over reps."""
    plan.profile(True)
    for _ in range(reps):
        plan.search(t, x, s, stream=stream, **kw)
    stream.synchronize()
    st = plan.profile_read()
    plan.profile(False)
    return st


_ORACLE_CACHE = {}
_BINS_CACHE = {}


def peak_and_low_bins(row, k_lo, n_peaks=32, halo=2, n_low=32):
    """The n_peaks highest strict local maxima of a Delta chi2 row (bins >= k_lo)
    +- halo and the n_low lowest bins from k_lo up: where the oracle is also
    evaluated (it computes its own values there)."""
    k = np.arange(max(k_lo, 1), row.shape[0] - 1)
    is_max = (row[k] > row[k - 1]) & (row[k] >= row[k + 1])
    pk = k[is_max][np.argsort(-row[k[is_max]], kind="stable")[:n_peaks]]
    around = (pk[:, None] + np.arange(-halo, halo + 1)[None, :]).ravel()
    return np.concatenate([around, np.arange(k_lo, k_lo + n_low)])


def workload_line(name, steps, warmup, precision=None, parity_bins=2048, seed=11,
                  extra_bins=None, schedule=None, tune_cache=None, full_grid=False,
                  parity=True):
    """Timing (autotuned, or on the given schedule), stage split, roofline and
    oracle parity of one single-curve workload: on every bin (full_grid), or
    on parity_bins seeded bins, the 32 highest local maxima of the H row +-2,
    the 32 lowest bins from f = 1/span up and the caller's extra bins."""
    import torch
    from paper_0901_1913_amd import fchi2 as F
    from paper_0901_1913_amd import synth
    cur = synth.make(name) if precision is None else synth.make(name, precision=precision)
    prec = cur.precision
    t = torch.from_numpy(cur.t).cuda()
    x = torch.from_numpy(cur.x).cuda()
    s = torch.from_numpy(cur.sigma).cuda()
    # Graph replay (one launch call per search) on a stream of its own, as for
    # the batch: a small search is otherwise limited by the host's calls.
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=prec, graph=True)
    ws = plan.workspace()
    t0 = time.perf_counter()
    if schedule is not None:
        schedule = plan.set_schedule(schedule)
    else:
        schedule = plan.autotune(t, x, s, cache_path=tune_cache)
    tune_s = time.perf_counter() - t0
    d = torch.empty((1, cur.H, cur.n_freq), dtype=plan.out_dtype, device="cuda")
    c0 = torch.empty(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        ms, wall = time_search(plan, t, x, s, steps, warmup, stream, dchi2=d, chi2_0=c0,
                               workspace=ws, want_flags=False)
        st = profiled_pass(plan, t, x, s, stream, reps=2, dchi2=d, chi2_0=c0, workspace=ws,
                           want_flags=False)
    b, o = (4, 4) if prec == "mixed" else (8, 8)
    roof, sections, stage_ms = stage_roofline(cur, st, 2, b, o, schedule)
    tr = measured_traffic(f"{name}_{prec}").get(roof["kernel"])
    roof["traffic"] = None if tr is None else int(round(tr))  # one curve per launch
    ms_median = _LAST_MEDIAN["ms"]
    units = cur.n_freq * cur.H
    line = {"workload": name, "n": int(cur.t.shape[0]), "H": cur.H, "n_freq": cur.n_freq,
            "f_max": cur.f_max, "precision": prec, "ms_per_search": round(ms, 5),
            "ms_median": round(ms_median, 5),
            "wall_ms_per_search": round(wall, 5), "value": round(units / (ms * 1e-3), 1),
            "unit": "freq*H/s", "schedule": schedule, "autotune_s": round(tune_s, 2),
            "stages_ms": stage_ms, "roofline": roof, "sections": sections}
    if not parity:  # profiling runs: the GPU part only
        plan.close()
        log(f"{name} {prec}: {ms:.4f} ms/search (no parity check)")
        return line
    # Parity bins (oracle on the host's CPU share).
    span = float(cur.t[-1] - cur.t[0])
    k_lo = int(np.ceil(cur.n_freq / (span * cur.f_max)))
    bkey = (name, full_grid, parity_bins, seed)
    if full_grid:
        bins = np.arange(1, cur.n_freq)
    elif bkey in _BINS_CACHE:  # the FP64 line of a workload reuses the mixed line's bins
        bins = _BINS_CACHE[bkey]
    else:
        rng = np.random.default_rng(seed)
        bins = rng.choice(np.arange(1, cur.n_freq), size=parity_bins, replace=False)
        row = d[0, cur.H - 1].double().cpu().numpy()
        bins = np.concatenate([bins, peak_and_low_bins(row, k_lo)])
        if extra_bins is not None:
            bins = np.concatenate([bins, extra_bins])
    bins = np.unique(bins[(bins >= 1) & (bins < cur.n_freq)])
    _BINS_CACHE[bkey] = bins
    dd = d.double().cpu().numpy()[0][:, bins]
    plan.close()
    key = (name, bins.tobytes())
    if key not in _ORACLE_CACHE:
        chunks = np.array_split(bins, max(1, min(len(bins), 4 * pool_size())))
        _ORACLE_CACHE[key] = oracle_pool([(cur.t, cur.x, cur.sigma,
                                           c * (cur.f_max / cur.n_freq), cur.H)
                                          for c in chunks if len(c)])
    res, el, cores = _ORACLE_CACHE[key]
    d_ora = np.concatenate([r[0] for r in res], axis=1)
    kappa = np.concatenate([r[1] for r in res])
    span = res[0][2]
    from oracle import fchi2_oracle as ora
    err = ora.rel_err(dd, d_ora)
    kmax = 1e2 if prec == "mixed" else 1e6
    fr = bins * (cur.f_max / cur.n_freq)
    gate = (fr >= 1.0 / span) & (kappa <= kmax)
    par = parity_summary([err], [gate])
    par.update({"bins": int(len(bins)), "gate": f"k >= 1, f >= 1/span, kappa <= {kmax:g}",
                "sample": ("every bin" if full_grid else
                           f"{parity_bins} seeded bins, the 32 highest local maxima of the "
                           f"H row +-2, the 32 lowest bins from 1/span"
                           + (", extra bins" if extra_bins is not None else ""))})
    log(f"{name} {prec}: {ms:.4f} ms/search, parity max {par['max_rel_err_gated']:.3e} "
        f"on {len(bins)} bins")
    return {**line, "parity": par,
            "oracle": {"value": round(len(bins) * cur.H / el, 2), "cores": cores,
                       "bins": int(len(bins)), "wall_s": round(el, 2),
                       "full_grid_s": (round(el, 2) if full_grid else
                                       round(units / (len(bins) * cur.H / el), 1)),
                       "full_grid_s_kind": "measured" if full_grid else "extrapolated"}}


def multi_vs_curves(steps):
    """Shared-alpha search of the multi workload vs the same sources run as
    ordinary curves (t replicated, errors scaled) through the batched search."""
    import torch
    from paper_0901_1913_amd import fchi2 as F
    from paper_0901_1913_amd import synth
    src = synth.make("multi")
    S, n = src.n_sources, src.t.shape[0]
    units = S * src.n_freq * src.H
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    plan = F.Plan(src.offsets, src.f_max, src.H, src.n_freq, precision=src.precision)
    t = torch.from_numpy(src.t).cuda()
    sg = torch.from_numpy(src.sigma).cuda()
    x = torch.from_numpy(np.ascontiguousarray(src.x)).cuda()
    sc = torch.from_numpy(src.scale).cuda()
    schedule_m = plan.autotune_multi(t, sg, x, sc)
    plan.search_multi(t, sg, x, sc)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        plan.search_multi(t, sg, x, sc)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_m = e0.elapsed_time(e1) / steps
    plan.close()
    off = np.arange(S + 1, dtype=np.int64) * n
    plan = F.Plan(off, src.f_max, src.H, src.n_freq, precision=src.precision, graph=True)
    tt = torch.from_numpy(np.tile(src.t, S)).cuda()
    ss = torch.from_numpy((src.scale[:, None] * src.sigma[None, :]).reshape(-1)).cuda()
    xx = x.reshape(-1)
    schedule = plan.autotune(tt, xx, ss)
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        d, c0, _ = plan.search(tt, xx, ss, want_flags=False, stream=side)
        e0.record(side)
        for _ in range(steps):
            plan.search(tt, xx, ss, dchi2=d, chi2_0=c0, want_flags=False, stream=side)
        e1.record(side)
        side.synchronize()
    ms_c = e0.elapsed_time(e1) / steps
    plan.close()
    log(f"multi: shared alpha {ms_m:.3f} ms, as curves {ms_c:.3f} ms")
    return {"workload": "multi", "n_sources": S, "n": n, "H": src.H, "n_freq": src.n_freq,
            "precision": src.precision, "shared_alpha_ms": round(ms_m, 4),
            "shared_alpha_schedule": schedule_m,
            "shared_alpha_value": round(units / (ms_m * 1e-3), 1),
            "as_curves_ms": round(ms_c, 4), "as_curves_value": round(units / (ms_c * 1e-3), 1),
            "as_curves_schedule": schedule, "speedup": round(ms_c / ms_m, 3),
            "unit": "freq*H/s"}


def gradient_timing(steps):
    """Adjoint of the search on the diff workload: forward with the spectra
    kept, top-16 strict local maxima of the H row frozen, then the gradient
    of the sum of their Delta chi2 with respect to x and sigma.  Forward and
    backward timed without per-launch events (the backward's stage split
    from a separate profiled pass); forward parity on 512 seeded bins, the
    32 highest local maxima +-2 and the 32 lowest bins; the gradient against
    the oracle's closed form (relative l2 and element-wise)."""
    import torch
    from paper_0901_1913_amd import fchi2 as F
    from paper_0901_1913_amd import synth
    from oracle import fchi2_oracle as ora
    cur = synth.make("diff")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=cur.precision,
                  keep_for_backward=True)
    t = torch.from_numpy(cur.t).cuda()
    x = torch.from_numpy(cur.x).cuda()
    s = torch.from_numpy(cur.sigma).cuda()
    schedule = plan.autotune(t, x, s)
    d, _, _ = plan.search(t, x, s)
    span = float(cur.t[-1] - cur.t[0])
    df = cur.f_max / cur.n_freq
    k_lo = int(np.ceil(1.0 / (span * df)))
    idx = plan.top_peaks(d, cur.H - 1, k_lo, 16)
    g = torch.zeros_like(d)
    g[0, cur.H - 1, idx[0]] = 1.0
    gx, gs = plan.backward(t, x, s, g)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.search(t, x, s, dchi2=d)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_f = e0.elapsed_time(e1) / steps
    e0.record(stream)
    for _ in range(steps):
        gx, gs = plan.backward(t, x, s, g)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1) / steps
    plan.profile(True)
    plan.backward(t, x, s, g)
    st = plan.profile_read()
    plan.profile(False)
    # Parity: forward on the sample, gradient against the closed form.
    row = d[0, cur.H - 1].double().cpu().numpy()
    dd = d[0].double().cpu().numpy()
    rng = np.random.default_rng(13)
    bins = np.unique(np.concatenate([rng.choice(np.arange(1, cur.n_freq), 512, replace=False),
                                     peak_and_low_bins(row, k_lo)]))
    bins = bins[(bins >= 1) & (bins < cur.n_freq)]
    chunks = np.array_split(bins, 4 * pool_size())
    res, el, cores = oracle_pool([(cur.t, cur.x, cur.sigma, c * df, cur.H) for c in chunks
                                  if len(c)])
    d_ora = np.concatenate([r[0] for r in res], axis=1)
    kappa = np.concatenate([r[1] for r in res])
    err = ora.rel_err(dd[:, bins], d_ora)
    gate = (bins * df >= 1.0 / span) & (kappa <= 1e2)
    par = parity_summary([err], [gate])
    pk = idx.cpu().numpy()[0]
    rx, rs = ora.grad(cur.t, cur.x, cur.sigma, [(float(k) * df, cur.H, 1.0) for k in pk])
    gxn, gsn = gx.cpu().numpy(), gs.cpu().numpy()
    par.update({"bins": int(len(bins)), "gate": "k >= 1, f >= 1/span, kappa <= 100",
                "grad_x_rel_l2": float(np.linalg.norm(gxn - rx) / np.linalg.norm(rx)),
                "grad_sigma_rel_l2": float(np.linalg.norm(gsn - rs) / np.linalg.norm(rs)),
                "grad_x_max_rel": float(np.abs(gxn - rx).max() / np.abs(rx).max()),
                "grad_sigma_max_rel": float(np.abs(gsn - rs).max() / np.abs(rs).max())})
    plan.close()
    units = cur.n_freq * cur.H
    log(f"gradient (diff): forward {ms_f:.4f} ms, backward {ms_b:.4f} ms, parity max "
        f"{par['max_rel_err_gated']:.3e}, grad l2 {par['grad_x_rel_l2']:.2e}")
    return {"workload": "diff", "n": int(cur.t.shape[0]), "H": cur.H, "n_freq": cur.n_freq,
            "precision": cur.precision, "forward_ms": round(ms_f, 5),
            "backward_ms": round(ms_b, 5),
            "backward_value": round(units / (ms_b * 1e-3), 1), "unit": "freq*H/s",
            "backward_stages_ms": {k: round(v[0], 5) for k, v in st.items()
                                   if v[1] and k.startswith("bwd")},
            "schedule": schedule, "parity": par,
            "oracle": {"cores": cores, "bins": int(len(bins)), "wall_s": round(el, 2)}}


def fine_timing(steps, K=16, R=64, levels=3, n_check=4):
    """Fine search on the ungridded data (Section 3e) around the long curve's
    K highest strict local maxima of the H row (fchi2_top_peaks on the
    search's rows): `levels` zoom levels of R direct-sum trials each, timed
    with events over the whole zoom; parity of the first level's rows against
    the oracle at the same trial frequencies for n_check of the centres, and
    of every centre's final best against the oracle at its frequency."""
    import torch
    from paper_0901_1913_amd import fchi2 as F
    from paper_0901_1913_amd import synth
    from oracle import fchi2_oracle as ora
    cur = synth.make("long")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=cur.precision)
    t = torch.from_numpy(cur.t).cuda()
    x = torch.from_numpy(cur.x).cuda()
    s = torch.from_numpy(cur.sigma).cuda()
    d, _, _ = plan.search(t, x, s)
    span = float(cur.t[-1] - cur.t[0])
    df = cur.f_max / cur.n_freq
    k_lo = int(np.ceil(1.0 / (span * df)))
    idx = plan.top_peaks(d, cur.H - 1, k_lo, K)
    fc = idx.double() * df
    res = plan.refine(t, x, s, fc, levels=levels, R=R)  # warm-up
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.top_peaks(d, cur.H - 1, k_lo, K, out=idx)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_peaks = e0.elapsed_time(e1) / steps
    e0.record(stream)
    for _ in range(steps):
        res = plan.refine(t, x, s, fc, levels=levels, R=R)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    lvl1 = plan.fine_search(t, x, s, fc, R=R, want_rows=True)
    rows = lvl1["rows"][0, :n_check].double().cpu().numpy()      # [n_check, R, H]
    fcn = fc[0].cpu().numpy()
    r = np.arange(R, dtype=np.float64)
    trials = np.concatenate([f + df * (2.0 * r / (R - 1) - 1.0) for f in fcn[:n_check]])
    fb = res["f_best"][0].cpu().numpy()
    db = res["dchi2_best"][0].cpu().numpy()                       # [K, H]
    freqs = np.concatenate([trials, fb])
    chunks = np.array_split(freqs, 4 * pool_size())
    out, el, cores = oracle_pool([(cur.t, cur.x, cur.sigma, c, cur.H) for c in chunks if len(c)])
    d_ora = np.concatenate([o[0] for o in out], axis=1)
    kappa = np.concatenate([o[1] for o in out])
    gpu = np.concatenate([rows.reshape(-1, cur.H).T, db.T], axis=1)
    err = ora.rel_err(gpu, d_ora)
    gate = (freqs >= 1.0 / span) & (kappa <= 1e6)
    par = parity_summary([err], [gate])
    par.update({"trials": int(len(trials)), "best": int(len(fb)),
                "gate": "f >= 1/span, kappa <= 1e6 (direct sums in FP64)"})
    plan.close()
    n_trials = K * R * levels
    log(f"fine search (long): {K} centres x {levels} levels x {R} trials in {ms:.4f} ms, "
        f"parity max {par['max_rel_err_gated']:.3e}")
    return {"workload": "long", "n": int(cur.t.shape[0]), "H": cur.H, "centres": K,
            "levels": levels, "trials_per_level": R, "ms": round(ms, 5),
            "top_peaks_ms": round(ms_peaks, 5),
            "value": round(n_trials * cur.H / (ms * 1e-3), 1), "unit": "trial freq*H/s",
            "parity": par, "oracle": {"cores": cores, "freqs": int(len(freqs)),
                                      "wall_s": round(el, 2)}}


def variants_timing(steps):
    """The paper-faithful variants on the long workload: the search with floor
    gridding (kernel_width = 1, Section 3b) and the cubic detrending."""
    import torch
    from paper_0901_1913_amd import fchi2 as F
    from paper_0901_1913_amd import synth
    cur = synth.make("long")
    t = torch.from_numpy(cur.t).cuda()
    x = torch.from_numpy(cur.x).cuda()
    s = torch.from_numpy(cur.sigma).cuda()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=cur.precision,
                  kernel_width=1)
    schedule = plan.autotune(t, x, s)
    d, c0, fl = plan.search(t, x, s)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        plan.search(t, x, s, dchi2=d, chi2_0=c0, flags=fl)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_floor = e0.elapsed_time(e1) / steps
    xr = plan.detrend(t, x, s, 3)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        plan.detrend(t, x, s, 3, x_out=xr)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_det = e0.elapsed_time(e1) / steps
    plan.close()
    units = cur.n_freq * cur.H
    log(f"variants (long): floor gridding {ms_floor:.4f} ms, cubic detrend {ms_det:.4f} ms")
    return {"workload": "long", "floor_gridding_ms": round(ms_floor, 5),
            "floor_gridding_value": round(units / (ms_floor * 1e-3), 1),
            "floor_gridding_schedule": schedule,
            "detrend_degree3_ms": round(ms_det, 5),
            "detrend_points_per_s": round(cur.t.shape[0] / (ms_det * 1e-3), 1),
            "unit": "freq*H/s"}


def band_share_timing(steps, G=8):
    """One device's share of the stress curve split into G frequency bands
    (same bin spacing, n_freq / G bins): the first band is an ordinary plan,
    any other band a band plan (first_bin > 0, modulated complex grids)."""
    import torch
    from paper_0901_1913_amd import fchi2 as F
    from paper_0901_1913_amd import synth
    cur = synth.make("stress")
    nb = cur.n_freq // G
    t = torch.from_numpy(cur.t).cuda()
    x = torch.from_numpy(cur.x).cuda()
    s = torch.from_numpy(cur.sigma).cuda()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    out = {"workload": "stress", "n": int(cur.t.shape[0]), "H": cur.H, "bands": G,
           "n_freq_per_band": nb, "precision": "mixed", "unit": "freq*H/s"}
    for g in (0, 1):
        plan = F.Plan(cur.offsets, cur.f_max / G, cur.H, nb, precision="mixed",
                      first_bin=g * nb)
        schedule = plan.autotune(t, x, s)
        d, c0, fl = plan.search(t, x, s)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            plan.search(t, x, s, dchi2=d, chi2_0=c0, flags=fl)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        plan.close()
        del d, c0, fl
        out[f"band{g}_ms"] = round(ms, 4)
        out[f"band{g}_value"] = round(nb * cur.H / (ms * 1e-3), 1)
        out[f"band{g}_schedule"] = schedule
        log(f"stress band {g} of {G}: {ms:.3f} ms")
    return out


def calibration_copy(mib):
    """One device copy of mib MiB: a kernel of known traffic against which the
    HBM counters of a profiled run are scaled."""
    import torch
    nel = mib * (1 << 20) // 4
    c_src = torch.ones(nel, dtype=torch.float32, device="cuda")
    c_dst = torch.empty_like(c_src)
    torch.cuda.synchronize()
    c_dst.copy_(c_src)
    torch.cuda.synchronize()
    log(f"calibration copy: {mib} MiB read + {mib} MiB written")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the single-curve loop beside the batched search")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the plain, long, diff and stress lines")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the shared-alpha, variants and band-share sections")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (one file serves every workload)")
    ap.add_argument("--schedule", default=None,
                    help="JSON schedule as Plan.info() reports it: applied instead of "
                         "autotuning (batched search, or the --workload-only line)")
    ap.add_argument("--workload-only", default=None,
                    choices=["plain", "long", "diff", "stress"],
                    help="run only this workload's line and print it (for profiling; "
                         "not the headline)")
    ap.add_argument("--no-parity", action="store_true",
                    help="--workload-only: time and profile the GPU search without the "
                         "oracle comparison (for profiler runs)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one device copy of this many MiB (a known-size kernel "
                         "against which HBM counters are scaled)")
    a = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(a.gpus, world)}); the search "
              "would shard by curves or frequency bands across GPUs, and no multi-GPU "
              "path is implemented.", file=sys.stderr)
        return 2

    import torch
    from paper_0901_1913_amd import fchi2 as F
    from paper_0901_1913_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    sched_arg = json.loads(a.schedule) if a.schedule else None
    if a.workload_only:
        if a.calib_copy_mb > 0:
            calibration_copy(a.calib_copy_mb)
        line = workload_line(a.workload_only, a.steps, a.warmup, schedule=sched_arg,
                             tune_cache=a.tune_cache, parity=not a.no_parity)
        print(json.dumps({"workload_only": line}), flush=True)
        return 0
    cur = synth.make("batch")
    n_tot = int(cur.t.shape[0])
    log(f"batch: {cur.n_curves} curves, {n_tot} points, H={cur.H}, n_freq={cur.n_freq}")
    t = torch.from_numpy(cur.t).cuda()
    x = torch.from_numpy(cur.x).cuda()
    s = torch.from_numpy(cur.sigma).cuda()
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=cur.precision,
                  graph=True, two_streams=True)
    ws = plan.workspace()
    t0 = time.perf_counter()
    if sched_arg is not None:
        schedule = plan.set_schedule(sched_arg)
    else:
        schedule = plan.autotune(t, x, s, cache_path=a.tune_cache)
    torch.cuda.synchronize()
    log(f"batch autotuned in {time.perf_counter() - t0:.1f} s (not timed): {schedule}")
    dchi2 = torch.empty((cur.n_curves, cur.H, cur.n_freq), dtype=plan.out_dtype, device="cuda")
    chi2_0 = torch.empty(cur.n_curves, dtype=torch.float64, device="cuda")
    if a.calib_copy_mb > 0:
        calibration_copy(a.calib_copy_mb)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    units = cur.n_curves * cur.n_freq * cur.H
    with torch.cuda.stream(stream):
        ms_step, wall_ms = time_search(plan, t, x, s, a.steps, a.warmup, stream, dchi2=dchi2,
                                       chi2_0=chi2_0, workspace=ws, want_flags=False)
        ms_median = _LAST_MEDIAN["ms"]
        log(f"batched (graph replay): {ms_step:.3f} ms/step over {a.steps} steps "
            f"(median {ms_median:.3f}, wall {wall_ms:.3f})")
        ref = dchi2.clone()
        # Stage split: a one-stream plan on the same schedule, so that each
        # kernel's launches are timed undisturbed (in the timed schedule the
        # next wave's spreading runs beside the current wave's passes).
        plan1 = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=cur.precision)
        plan1.set_schedule(schedule)
        ws1 = plan1.workspace()
        plan1.search(t, x, s, dchi2=dchi2, chi2_0=chi2_0, workspace=ws1, want_flags=False,
                     stream=stream)
        st = profiled_pass(plan1, t, x, s, stream, dchi2=dchi2, chi2_0=chi2_0, workspace=ws1,
                           want_flags=False)
        plan1.close()
        del ws1
        ms_plain, same = None, None
        if not a.no_plain:
            # Plain form: the same kernels and schedule, one curve per call, no graph.
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for c in range(cur.n_curves):
                plan.search_curves(c, 1, t, x, s, dchi2, chi2_0, workspace=ws, stream=stream)
            e1.record(stream)
            stream.synchronize()
            ms_plain = e0.elapsed_time(e1)
            same = bool(torch.equal(ref, dchi2))
            log(f"plain loop: {ms_plain:.3f} ms per pass (identical outputs: {same})")
        # Significance epilogue: K candidates per curve instead of the rows.
        K = 16
        plan.search_top(t, x, s, K=K, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(a.steps):
            top = plan.search_top(t, x, s, K=K, stream=stream)
        e1.record(stream)
        stream.synchronize()
        ms_top = e0.elapsed_time(e1) / a.steps
        log(f"fused top-{K}: {ms_top:.3f} ms/step")
    roof, sections, stage_ms = stage_roofline(cur, st, 1, 4, 4, schedule)
    tr = measured_traffic("batch_mixed").get(roof["kernel"])
    waves = st["solve"][1] if st.get("solve", (0, 0))[1] else None  # one solve per wave
    roof["traffic"] = None if (tr is None or not waves) else int(round(
        tr * cur.n_curves / waves))
    roof["stage_split"] = "one-stream plan on the timed schedule (kernels undisturbed)"
    # The whole step on the timed search itself (its spreading overlaps the
    # passes, so the stages' sum exceeds it).
    ws_gb = sections["whole_step"]["gb_per_step_model"]
    sections["whole_step"].update({
        "ms": round(ms_step, 4), "gbs": round(ws_gb / (ms_step * 1e-3), 1),
        "frac": round(ws_gb / (ms_step * 1e-3) / HBM_PEAK_GBS, 4),
        "stage_sum_ms": round(sum(stage_ms.values()), 4)})
    out = {
        "metric": METRIC, "value": round(units / (ms_step * 1e-3), 1), "unit": "freq*H/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 4),
        "ms_median": round(ms_median, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "batch", "n_curves": cur.n_curves, "n_total": n_tot,
                   "H": cur.H, "n_freq": cur.n_freq, "f_max": cur.f_max,
                   "precision": cur.precision, "form": "one graph-replayed search",
                   "schedule": schedule},
        "roofline": roof, "sections": sections, "stages_ms_per_step": stage_ms,
        "plain": None if ms_plain is None else {
            "ms_per_pass": round(ms_plain, 3), "value": round(units / (ms_plain * 1e-3), 1),
            "speedup_batched_over_plain": round(ms_plain / ms_step, 3),
            "identical_outputs": same},
        "fused_top16": {"ms_per_step": round(ms_top, 4),
                        "value": round(units / (ms_top * 1e-3), 1),
                        "rows_bytes": int(cur.n_curves * cur.H * cur.n_freq * 4),
                        "top16_bytes": int(sum(v.numel() * v.element_size()
                                               for v in top.values()))},
    }
    # Oracle on a bounded, stratified sample of the batch: CPU baseline and parity.
    if not a.no_cpu_baseline:
        from oracle import fchi2_oracle as ora
        sample, strat = batch_sample(cur)
        tasks, order = [], []
        df = cur.f_max / cur.n_freq
        for c, bins in sample.items():
            tt, xx, ss = cur.curve(c)
            # the stratified curves' bins split across tasks to balance the pool
            for part in np.array_split(bins, max(1, len(bins) // 16)):
                tasks.append((tt, xx, ss, part * df, cur.H))
                order.append((c, part))
        log(f"oracle CPU baseline: {sum(len(b) for b in sample.values())} bins on "
            f"{cur.n_curves} curves ({len(strat)} stratified) ...")
        res, el, cores = oracle_pool(tasks)
        dd = ref.float().cpu().numpy() if ref.dtype != torch.float64 else ref.cpu().numpy()
        errs, gates = [], []
        for (c, part), (d_ora, kappa, span) in zip(order, res):
            e = ora.rel_err(dd[c][:, part].astype(np.float64), d_ora)
            fr = part * df
            errs.append(e)
            gates.append((fr >= 1.0 / span) & (kappa <= 1e2) if span > 0 else kappa <= 1e2)
        nb = sum(len(p) for _, p in order)
        v_cpu = nb * cur.H / el
        # one core: every 32nd task of the same list, in this process
        sub = tasks[::32]
        t1 = time.perf_counter()
        for tk in sub:
            _oracle_task(tk)
        one = sum(len(tk[3]) for tk in sub) * cur.H / (time.perf_counter() - t1)
        out["cpu_baseline"] = {
            "value": round(v_cpu, 2), "unit": "freq*H/s", "cores": cores, "kind": "oracle",
            "sample": (f"{nb} bins (all H'=1..{cur.H}) of the batch workload: {len(strat)} "
                       f"curves stratified by length quartile and signal/noise with 96 "
                       f"seeded bins each, plus {BINS_EACH} seeded bins on every curve; "
                       f"{el:.1f} s wall"),
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "one_core_value": round(one, 2),
            "full_search_s_extrapolated": round(units / v_cpu, 1)}
        out["parity"] = parity_summary(errs, gates)
        out["parity"].update({"bins": nb, "gate": "k >= 1, f >= 1/span, kappa <= 100"})
        log(f"batch parity: max gated {out['parity']['max_rel_err_gated']:.3e}")
    plan.close()
    del dchi2, ref, ws
    torch.cuda.empty_cache()
    if not a.no_workloads:
        wl = {}
        wl["plain_fp64"] = workload_line("plain", a.steps, a.warmup, full_grid=True,
                                         tune_cache=a.tune_cache)
        # long: also +-8 bins around 1 and 2 cycles/day (the diurnal aliases)
        nf_l, fm_l = 2 ** 22, 50.0
        alias = np.concatenate([int(round(c * nf_l / fm_l)) + np.arange(-8, 9) for c in (1, 2)])
        wl["long_mixed"] = workload_line("long", a.steps, a.warmup, extra_bins=alias,
                                         tune_cache=a.tune_cache)
        wl["diff"] = gradient_timing(a.steps)
        wl["stress_mixed"] = workload_line("stress", max(3, a.steps // 2), 2, parity_bins=448,
                                           tune_cache=a.tune_cache)
        torch.cuda.empty_cache()
        wl["stress_fp64"] = workload_line("stress", max(3, a.steps // 2), 2, precision="fp64",
                                          parity_bins=448, tune_cache=a.tune_cache)
        out["workloads"] = wl
    if not a.no_extras:
        torch.cuda.empty_cache()
        out["multi"] = multi_vs_curves(max(3, a.steps // 2))
        out["variants"] = variants_timing(a.steps)
        out["fine"] = fine_timing(a.steps)
        out["band_share"] = band_share_timing(a.steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
