#!/usr/bin/env python3
"""Throughput of the F-chi2 hot path on one MI355X.

A step is one fchi2_search over the whole workload (moments, spreading, FFT
passes, per-bin assembly and Cholesky for every H'), with the inputs already
resident in device memory.  The value is trial frequencies x H per second.

Prints one JSON line.  Beside the throughput it reports, for the kernel that
takes the most time, its algorithmic bytes per launch divided by its average
launch time (HIP events recorded by the library on the search stream during
the timed steps), and the FP64 CPU oracle timed on a bounded sample of bins of
the same workload (whose values double as a parity spot check).
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
METRIC = ("trial freqs·H/sec for Δχ² (rel err ≤1e-5 vs FP64 oracle); "
          "batched vs plain")


def measured_traffic(workload):
    """HBM bytes per launch from the committed PMC summary, per stage, or None
    for a stage whose kernel source changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{workload}_mixed_hbm_traffic.md")
    if not os.path.exists(path):
        return {}
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return {}
    meta = json.loads(m.group(1))
    src = {"fft_first": ["fft.hip"], "fft_mid": ["fft.hip"], "fft_last": ["fft.hip"],
           "solve": ["solve.hip", "solve_bin.h"], "spread": ["spread.hip", "es_kernel.h"]}
    out = {}
    for st, nbytes in meta.get("bytes_per_launch", {}).items():
        h = hashlib.sha256()
        ok = st in src
        for f in src.get(st, []):
            path = os.path.join(ROOT, "paper_0901_1913_amd", "csrc", f)
            if not os.path.isfile(path):
                ok = False
                break
            h.update(open(path, "rb").read())
        ok = ok and h.hexdigest()[:16] == meta.get("source_sha256_16", {}).get(st)
        out[st] = int(nbytes) if ok else None
    return out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pair_extents(cur, w):
    """Nonzero cells of each packed grid (weight pairs, then data pairs)."""
    H, nf = cur.H, cur.n_freq
    L = 4 * nf
    df = cur.f_max / nf
    span = float(cur.t[-1] - cur.t[0])
    c_off = w // 2 + 2
    ms = [2 * p + 2 for p in range(H)] + [min(2 * j + 2, H) for j in range((H + 1) // 2)]
    return [min(L, int((m * (span * df)) * L + c_off) + w // 2 + 1) for m in ms]


def stage_bytes(cur, elem, out_elem, w):
    """Algorithmic HBM bytes per launch of each forward stage (one curve)."""
    H, nf = cur.H, cur.n_freq
    L = 4 * nf
    P = H + (H + 1) // 2
    E = pair_extents(cur, w)
    n = cur.t.shape[0]
    return {
        "moments": 24 * n,
        "spread": 24 * n + sum(E) * elem,
        "fft_first": sum(E) * elem + P * L * elem,
        "fft_mid": 2 * P * L * elem,
        "fft_last": P * L * elem + P * 2 * nf * elem,
        "solve": P * 2 * nf * elem + nf * elem + H * nf * out_elem + nf,
    }


def _oracle_chunk(args):
    t, x, s, freqs, H = args
    from threadpoolctl import threadpool_limits
    from oracle import fchi2_oracle as ora
    with threadpool_limits(1):
        r = ora.dchi2(t, x, s, freqs, H)
    return r["dchi2"], r["kappa"]


def cpu_baseline(cur, budget_s, seed=7):
    """Time the oracle on a seeded bin sample sized to ~budget_s of CPU work."""
    import multiprocessing as mp
    cores = max(1, min(16, os.cpu_count() or 1))
    t, x, s = cur.curve(0)
    rng = np.random.default_rng(seed)
    nf = cur.n_freq
    # Probe the cost of one bin on one core.
    probe = np.array([nf // 3], dtype=np.int64)
    t0 = time.perf_counter()
    _oracle_chunk((t, x, s, probe * (cur.f_max / nf), cur.H))
    per_bin = max(time.perf_counter() - t0, 1e-4)
    # One core on its own: a short run of consecutive bins in this process.
    one = np.arange(1, 33, dtype=np.int64) * (nf // 64)
    t0 = time.perf_counter()
    _oracle_chunk((t, x, s, one * (cur.f_max / nf), cur.H))
    one_core = len(one) * cur.H / (time.perf_counter() - t0)
    n_bins = int(max(cores, min(4096, budget_s * cores / per_bin)))
    n_bins = (n_bins // cores) * cores
    bins = np.sort(rng.choice(np.arange(1, nf), size=n_bins, replace=False))
    chunks = np.array_split(bins, cores)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        parts = pool.map(_oracle_chunk, [(t, x, s, c * (cur.f_max / nf), cur.H) for c in chunks])
    el = time.perf_counter() - t0
    return (bins, np.concatenate([p[0] for p in parts], axis=1),
            np.concatenate([p[1] for p in parts]), el, cores, one_core)


def batched_vs_plain(steps):
    """The batch workload as one graph-replayed search vs a loop of single-curve searches."""
    import torch
    from paper_0901_1913_amd import fchi2 as F
    from paper_0901_1913_amd import synth
    cur = synth.make("batch")
    log(f"batch: {cur.n_curves} curves, {cur.t.shape[0]} points, H={cur.H}, "
        f"n_freq={cur.n_freq}")
    t = torch.from_numpy(cur.t).cuda()
    x = torch.from_numpy(cur.x).cuda()
    s = torch.from_numpy(cur.sigma).cuda()
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=cur.precision,
                  graph=True)
    ws = plan.workspace()
    schedule = plan.autotune(t, x, s)
    log(f"batch autotuned: {schedule}")
    dchi2 = torch.empty((cur.n_curves, cur.H, cur.n_freq), dtype=plan.out_dtype, device="cuda")
    chi2_0 = torch.empty(cur.n_curves, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    units = cur.n_curves * cur.n_freq * cur.H
    with torch.cuda.stream(stream):
        plan.search(t, x, s, dchi2=dchi2, chi2_0=chi2_0, workspace=ws, want_flags=False)
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            plan.search(t, x, s, dchi2=dchi2, chi2_0=chi2_0, workspace=ws, want_flags=False)
        e1.record(stream)
        stream.synchronize()
        ms_b = e0.elapsed_time(e1) / steps
        ref = dchi2.clone()
        log(f"batched: {ms_b:.3f} ms/step")
        # Plain form: the same kernels, one curve per call, no graph.
        e0.record(stream)
        for c in range(cur.n_curves):
            plan.search_curves(c, 1, t, x, s, dchi2, chi2_0, workspace=ws, stream=stream)
        e1.record(stream)
        stream.synchronize()
        ms_p = e0.elapsed_time(e1)
        same = bool(torch.equal(ref, dchi2))
        log(f"plain loop: {ms_p:.3f} ms per pass (results identical: {same})")
        del ref, dchi2
        # Significance epilogue: K candidates per curve instead of the rows.
        K = 16
        plan.search_top(t, x, s, K=K, stream=stream)
        e0.record(stream)
        for _ in range(steps):
            top = plan.search_top(t, x, s, K=K, stream=stream)
        e1.record(stream)
        stream.synchronize()
        ms_top = e0.elapsed_time(e1) / steps
        log(f"fused top-{K}: {ms_top:.3f} ms/step")
    plan.close()
    torch.cuda.synchronize()
    return {"workload": "batch", "n_curves": cur.n_curves, "n_total": int(cur.t.shape[0]),
            "H": cur.H, "n_freq": cur.n_freq, "precision": cur.precision,
            "batched_value": round(units / (ms_b * 1e-3), 1), "batched_ms_per_step": round(ms_b, 4),
            "plain_value": round(units / (ms_p * 1e-3), 1), "plain_ms_per_pass": round(ms_p, 3),
            "speedup": round(ms_p / ms_b, 3), "identical_outputs": same,
            "schedule": schedule, "unit": "freq*H/s",
            "fused_top16_value": round(units / (ms_top * 1e-3), 1),
            "fused_top16_ms_per_step": round(ms_top, 4),
            "rows_bytes": int(cur.n_curves * cur.H * cur.n_freq * 4),
            "top16_bytes": int(sum(v.numel() * v.element_size() for v in top.values()))}


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
    of the sum of their Delta chi2 with respect to x and sigma."""
    import torch
    from paper_0901_1913_amd import fchi2 as F
    from paper_0901_1913_amd import synth
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
    idx = plan.top_peaks(d, cur.H - 1, int(np.ceil(1.0 / (span * df))), 16)
    g = torch.zeros_like(d)
    g[0, cur.H - 1, idx[0]] = 1.0
    plan.backward(t, x, s, g)
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
    plan.profile(True)
    e0.record(stream)
    for _ in range(steps):
        gx, gs = plan.backward(t, x, s, g)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1) / steps
    st = plan.profile_read()
    plan.profile(False)
    plan.close()
    units = cur.n_freq * cur.H
    log(f"gradient (diff): forward {ms_f:.4f} ms, backward {ms_b:.4f} ms")
    return {"workload": "diff", "n": int(cur.t.shape[0]), "H": cur.H, "n_freq": cur.n_freq,
            "precision": cur.precision, "forward_ms": round(ms_f, 5),
            "backward_ms": round(ms_b, 5),
            "backward_value": round(units / (ms_b * 1e-3), 1), "unit": "freq*H/s",
            "backward_stages_ms": {k: round(v[0] / steps, 5) for k, v in st.items()
                                   if v[1] and k.startswith("bwd")},
            "schedule": schedule}


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


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="long",
                    choices=["plain", "long", "diff", "stress"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-survey vs plain-loop comparison")
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--no-multi", action="store_true",
                    help="skip the shared-alpha multi-source comparison")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the floor-gridding and detrending timings")
    ap.add_argument("--no-gradient", action="store_true",
                    help="skip the adjoint timing on the diff workload")
    ap.add_argument("--no-band", action="store_true",
                    help="skip the frequency-band share of the stress curve")
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
    cur = synth.make(a.workload)
    log(f"workload {a.workload}: n={cur.t.shape[0]} H={cur.H} n_freq={cur.n_freq} "
        f"precision={cur.precision}")
    plan = F.Plan(cur.offsets, cur.f_max, cur.H, cur.n_freq, precision=cur.precision)
    t = torch.from_numpy(cur.t).cuda()
    x = torch.from_numpy(cur.x).cuda()
    s = torch.from_numpy(cur.sigma).cuda()
    ws = plan.workspace()
    t0 = time.perf_counter()
    schedule = plan.autotune(t, x, s)
    torch.cuda.synchronize()
    log(f"autotuned in {time.perf_counter() - t0:.2f} s (not timed): {schedule}")
    dchi2 = torch.empty((1, cur.H, cur.n_freq), dtype=plan.out_dtype, device="cuda")
    chi2_0 = torch.empty(1, dtype=torch.float64, device="cuda")
    flags = torch.empty((1, cur.n_freq), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    if a.calib_copy_mb > 0:
        nel = a.calib_copy_mb * (1 << 20) // 4
        c_src = torch.ones(nel, dtype=torch.float32, device="cuda")
        c_dst = torch.empty_like(c_src)
        torch.cuda.synchronize()
        c_dst.copy_(c_src)
        torch.cuda.synchronize()
        log(f"calibration copy: {a.calib_copy_mb} MiB read + {a.calib_copy_mb} MiB written")
        del c_src, c_dst
    for _ in range(a.warmup):
        plan.search(t, x, s, dchi2=dchi2, chi2_0=chi2_0, flags=flags, workspace=ws)
    torch.cuda.synchronize()
    log(f"warmup done ({a.warmup})")

    plan.profile(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(a.steps):
        plan.search(t, x, s, dchi2=dchi2, chi2_0=chi2_0, flags=flags, workspace=ws)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = ev0.elapsed_time(ev1) / a.steps
    stages = plan.profile_read()
    plan.profile(False)
    log(f"timed {a.steps} steps: {ms_step:.4f} ms/step (wall {1e3 * wall / a.steps:.4f})")

    units = cur.n_curves * cur.n_freq * cur.H
    value = units / (ms_step * 1e-3)
    w = plan.info()["kernel_width"]
    elem = 8 if cur.precision == "mixed" else 16
    out_elem = 4 if cur.precision == "mixed" else 8
    nbytes = stage_bytes(cur, elem, out_elem, w)
    st_avg = {k: (v[0] / v[1] if v[1] else 0.0, v[1] // a.steps) for k, v in stages.items()
              if v[1]}
    per_step = {k: round(v[0] * v[1], 5) for k, v in st_avg.items()}
    dom = max(per_step, key=per_step.get)
    dom_ms = st_avg[dom][0]
    achieved = nbytes[dom] / (dom_ms * 1e-3) / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (measured_traffic(a.workload).get(dom)
                        if cur.precision == "mixed" else None),
            "bytes_per_launch": int(nbytes[dom]),
            "avg_launch_ms": round(dom_ms, 5)}
    stage_gbs = {k: round(nbytes[k] / (v[0] * 1e-3) / 1e9, 1) for k, v in st_avg.items()
                 if k in nbytes and v[0] > 0}

    # Significance epilogue on the same plan: K candidates instead of the rows.
    K = 16
    top = plan.search_top(t, x, s, K=K)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(a.steps):
        top = plan.search_top(t, x, s, K=K)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_top = ev0.elapsed_time(ev1) / a.steps
    log(f"fused top-{K}: {ms_top:.4f} ms/step")
    signif = {"K": K, "ms_per_step": round(ms_top, 5), "value": round(units / (ms_top * 1e-3), 1),
              "best_bins": top["idx"][0, :4].tolist(),
              "best_log_p": [round(v, 3) for v in top["log_p"][0, :4].tolist()]}
    # Fine search on the ungridded points around those K candidates (R trials
    # over +-1 bin, three zoom levels), FP64 direct sums.
    R = 64
    fc = torch.where(top["idx"] >= 0, top["idx"].double() * (cur.f_max / cur.n_freq),
                     torch.full_like(top["log_p"], float("nan")))
    fine = plan.refine(t, x, s, fc, levels=3, R=R)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(a.steps):
        fine = plan.refine(t, x, s, fc, levels=3, R=R)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_fine = ev0.elapsed_time(ev1) / a.steps
    pairs = 3 * K * R * int(cur.t.shape[0])
    log(f"fine search, 3 levels x {K} x {R}: {ms_fine:.4f} ms")
    signif["fine"] = {"levels": 3, "R": R, "ms": round(ms_fine, 5),
                      "point_trials_per_s": round(pairs / (ms_fine * 1e-3), 1),
                      "f_best": [round(v, 9) for v in fine["f_best"][0, :4].tolist()]}

    d_gpu = dchi2.double().cpu().numpy()[0]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "freq*H/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if cur.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": a.workload, "n": int(cur.t.shape[0]), "H": cur.H,
                   "n_freq": cur.n_freq, "f_max": cur.f_max, "precision": cur.precision,
                   "schedule": plan.info()},
        "roofline": roof,
        "stages_ms_per_step": per_step,
        "stages_gbs": stage_gbs,
        "significance": signif,
    }
    if not a.no_cpu_baseline:
        from oracle import fchi2_oracle as ora
        log("oracle CPU baseline ...")
        bins, d_ora, kappa, el, cores, one_core = cpu_baseline(cur, a.cpu_seconds)
        v_cpu = len(bins) * cur.H / el
        out["cpu_baseline"] = {
            "value": round(v_cpu, 2), "unit": "freq*H/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{len(bins)} seeded random bins of the {a.workload} workload "
                      f"(all H'=1..{cur.H}), {el:.1f} s wall",
            "one_core_value": round(one_core, 2),
            "full_grid_s_extrapolated": round(units / v_cpu, 1)}
        span = float(cur.t[-1] - cur.t[0])
        freqs = bins * (cur.f_max / cur.n_freq)
        err = ora.rel_err(d_gpu[:, bins], d_ora)
        kmax = 1e2 if cur.precision == "mixed" else 1e6
        ok = (freqs >= 1.0 / span) & (kappa <= kmax)
        out["parity"] = {"bins": int(len(bins)), "gated_bins": int(ok.sum()),
                         "gate": f"f >= 1/span, kappa <= {kmax:g}",
                         "max_rel_err_gated": float(err[:, ok].max()) if ok.any() else None,
                         "median_rel_err_gated": float(np.median(err[:, ok])) if ok.any() else None,
                         "max_rel_err_all": float(err.max())}
    plan.close()
    del dchi2, ws
    if not a.no_batched:
        out["batched"] = batched_vs_plain(a.batched_steps)
    if not a.no_multi:
        out["multi"] = multi_vs_curves(a.batched_steps)
    if not a.no_gradient:
        out["gradient"] = gradient_timing(a.steps)
    if not a.no_variants:
        out["variants"] = variants_timing(a.steps)
    if not a.no_band:
        out["band_share"] = band_share_timing(a.steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
