"""Seeded synthetic light curves for the F-chi2 search.

This module only draws inputs (times, values, errors) and search settings.  It
holds none of the method's arithmetic and is shared by the tests, the
benchmark and the CPU oracle runs, so that every consumer sees bit-identical
FP64 inputs for a given (workload, seed, overrides).

The workloads stand in for the paper's Hipparcos Epoch Photometry test
(Section 4), which is not available: irregular sampling, per-point errors and
harmonic signal content of the kinds that section describes, at the sizes of
the five named workloads:

  plain    one curve, n=1000 over 100 d, two-harmonic signal, H=3,
           2^14 bins up to 10 /d, all-FP64
  long     one curve, n=100000 over 3000 d with diurnal gaps, five-term
           sawtooth of period 0.731 d, H=5, 2^22 bins up to 50 /d
  batch    10000 curves, n log-uniform in [50, 5000], spans 30..1000 d, half
           with a sinusoid, H=3, 2^16 bins up to 10 /d per curve
  diff     one curve, n=20000 over 500 d, four-harmonic signal of period
           3.3 d, H=4, 2^20 bins up to 100 /d (gradient workload)
  stress   one curve, n=1e6 over 1e4 d at t ~ 2.45e6, eight harmonics of
           period 0.1234 d, sigma log-uniform over [1e-3, 1], H=8,
           2^24 bins up to 40 /d (precision stress)

and one for the shared-alpha form (many sources at the same sampling times
with proportional errors, as an imager revisiting one field, Section 5):

  multi    2000 sources at 400 shared times over 1000 d, shared sigma
           uniform in [0.01, 0.05], per-source error scale log-uniform in
           [0.5, 4], a third of the sources with a sinusoid, H=3, 2^16 bins
           up to 10 /d
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

WORKLOADS = ("plain", "long", "batch", "diff", "stress", "multi")
SEEDS = {"plain": 1, "long": 2, "batch": 3, "diff": 4, "stress": 5, "multi": 6}


@dataclass
class Curves:
    """A batch of light curves in CSR form (offsets[c]..offsets[c+1])."""
    t: np.ndarray          # float64 [n_total], ascending within each curve
    x: np.ndarray          # float64 [n_total]
    sigma: np.ndarray      # float64 [n_total]
    offsets: np.ndarray    # int64 [n_curves + 1]
    H: int
    n_freq: int
    f_max: float
    precision: str         # "fp64" or "mixed"
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_curves(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def curve(self, c: int):
        a, b = int(self.offsets[c]), int(self.offsets[c + 1])
        return self.t[a:b], self.x[a:b], self.sigma[a:b]


def _single(t, x, s, H, n_freq, f_max, precision, name, meta=None):
    order = np.argsort(t, kind="stable")
    t, x, s = t[order], x[order], s[order]
    off = np.array([0, t.shape[0]], dtype=np.int64)
    return Curves(t=t.astype(np.float64), x=x.astype(np.float64),
                  sigma=s.astype(np.float64), offsets=off, H=H, n_freq=n_freq,
                  f_max=float(f_max), precision=precision, name=name,
                  meta=meta or {})


def plain(seed=1, n=1000, span=100.0, H=3, n_freq=2 ** 14, f_max=10.0,
          precision="fp64"):
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, span, n)
    s = rng.uniform(0.05, 0.2, n)
    P = 2.37
    x = 0.5 * np.sin(2 * np.pi * t / P) + 0.2 * np.cos(4 * np.pi * t / P)
    x = x + s * rng.standard_normal(n)
    return _single(t, x, s, H, n_freq, f_max, precision, "plain",
                   dict(period=P))


def long(seed=2, n=100_000, span=3000.0, H=5, n_freq=2 ** 22, f_max=50.0,
         precision="mixed"):
    """Diurnal-gapped long curve: keep samples whose fractional day is < 0.4."""
    rng = np.random.default_rng(seed)
    parts = []
    have = 0
    while have < n:
        cand = rng.uniform(0.0, span, 2 * (n - have) + 16)
        cand = cand[(cand - np.floor(cand)) < 0.4]
        parts.append(cand)
        have += cand.shape[0]
    t = np.concatenate(parts)[:n]
    s = 10.0 ** rng.uniform(-2.0, -1.0, n)
    P = 0.731
    x = np.zeros(n)
    for h in range(1, 6):
        x += ((-1) ** (h + 1)) * np.sin(2 * np.pi * h * t / P) / h
    x = 0.1 * (2.0 / np.pi) * x + s * rng.standard_normal(n)
    return _single(t, x, s, H, n_freq, f_max, precision, "long",
                   dict(period=P))


def diff(seed=4, n=20_000, span=500.0, H=4, n_freq=2 ** 20, f_max=100.0,
         precision="mixed"):
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, span, n)
    s = rng.uniform(0.05, 0.15, n)
    P = 3.3
    ph = rng.uniform(0.0, 2 * np.pi, 4)
    x = np.zeros(n)
    for h in range(1, 5):
        x += (0.4 / h) * np.sin(2 * np.pi * h * t / P + ph[h - 1])
    x = x + s * rng.standard_normal(n)
    return _single(t, x, s, H, n_freq, f_max, precision, "diff",
                   dict(period=P))


def stress(seed=5, n=1_000_000, span=1.0e4, H=8, n_freq=2 ** 24, f_max=40.0,
           precision="mixed", t_offset=2.45e6):
    rng = np.random.default_rng(seed)
    tr = rng.uniform(0.0, span, n)
    s = 10.0 ** rng.uniform(-3.0, 0.0, n)
    P = 0.1234
    ph = rng.uniform(0.0, 2 * np.pi, 8)
    x = np.zeros(n)
    for h in range(1, 9):
        x += (0.01 / h) * np.sin(2 * np.pi * h * tr / P + ph[h - 1])
    x = x + s * rng.standard_normal(n)
    return _single(tr + t_offset, x, s, H, n_freq, f_max, precision, "stress",
                   dict(period=P, t_offset=t_offset))


def batch(seed=3, n_curves=10_000, n_lo=50, n_hi=5000, span_lo=30.0,
          span_hi=1000.0, H=3, n_freq=2 ** 16, f_max=10.0, precision="mixed"):
    """Many curves of uneven length; exactly half carry a sinusoid."""
    ss = np.random.SeedSequence(seed)
    top = np.random.default_rng(ss.spawn(1)[0])
    with_signal = np.zeros(n_curves, dtype=bool)
    with_signal[top.permutation(n_curves)[: n_curves // 2]] = True
    children = ss.spawn(n_curves)
    ts, xs, sg, lens = [], [], [], []
    periods = np.full(n_curves, np.nan)
    for c in range(n_curves):
        rng = np.random.default_rng(children[c])
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        span = rng.uniform(span_lo, span_hi)
        t = np.sort(rng.uniform(0.0, span, n))
        s = rng.uniform(0.02, 0.3, n)
        x = s * rng.standard_normal(n)
        if with_signal[c]:
            P = 10.0 ** rng.uniform(-1.0, 2.0)
            A = rng.uniform(0.05, 0.5)
            phi = rng.uniform(0.0, 2 * np.pi)
            x = x + A * np.sin(2 * np.pi * t / P + phi)
            periods[c] = P
        ts.append(t)
        xs.append(x)
        sg.append(s)
        lens.append(n)
    off = np.zeros(n_curves + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    return Curves(t=np.concatenate(ts), x=np.concatenate(xs),
                  sigma=np.concatenate(sg), offsets=off, H=H, n_freq=n_freq,
                  f_max=float(f_max), precision=precision, name="batch",
                  meta=dict(periods=periods, with_signal=with_signal))


@dataclass
class Sources:
    """Many sources observed at one set of times with proportional errors."""
    t: np.ndarray          # float64 [n], ascending
    sigma: np.ndarray      # float64 [n], shared error shape
    x: np.ndarray          # float64 [n_sources, n]
    scale: np.ndarray      # float64 [n_sources]: source s has errors scale[s] * sigma
    H: int
    n_freq: int
    f_max: float
    precision: str
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_sources(self) -> int:
        return int(self.x.shape[0])

    @property
    def offsets(self) -> np.ndarray:
        return np.array([0, self.t.shape[0]], dtype=np.int64)

    def source(self, s: int):
        """(t, x, sigma) of source s as an ordinary curve."""
        return self.t, self.x[s], self.scale[s] * self.sigma


def multi(seed=6, n_sources=2000, n=400, span=1000.0, H=3, n_freq=2 ** 16, f_max=10.0,
          precision="mixed"):
    """Sources sharing sampling times; a third carry a sinusoid."""
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0.0, span, n))
    sigma = rng.uniform(0.01, 0.05, n)
    scale = 10.0 ** rng.uniform(np.log10(0.5), np.log10(4.0), n_sources)
    x = (scale[:, None] * sigma[None, :]) * rng.standard_normal((n_sources, n))
    x += rng.uniform(-1.0, 1.0, n_sources)[:, None]           # source mean levels
    periods = np.full(n_sources, np.nan)
    sig = rng.permutation(n_sources)[: n_sources // 3]
    for s_ in sig:
        P = 10.0 ** rng.uniform(-1.0, 1.5)
        A = rng.uniform(0.02, 0.2) * scale[s_]
        x[s_] += A * np.sin(2 * np.pi * t / P + rng.uniform(0.0, 2 * np.pi))
        periods[s_] = P
    return Sources(t=t, sigma=sigma, x=x, scale=scale, H=H, n_freq=n_freq,
                   f_max=float(f_max), precision=precision, name="multi",
                   meta=dict(periods=periods))


def make(name, **overrides):
    """Build the named workload; keyword overrides shrink it for tests."""
    fn = {"plain": plain, "long": long, "batch": batch, "diff": diff,
          "stress": stress, "multi": multi}[name]
    overrides.setdefault("seed", SEEDS[name])
    return fn(**overrides)
