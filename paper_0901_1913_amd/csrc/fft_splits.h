// FFT digit splits of the grid length L = 2^logL: the plan's default split
// and the autotuner's candidates.  Host code only (plain C++, no HIP), so a
// CPU test can pin its rules.
#pragma once

#include <vector>

#include "fchi2_internal.h"

namespace fchi2 {

// Choose the FFT digit split of L = 2^logL into np passes of radix <= 2^9.
// Constraints: each pass tile holds 2^LE elements as N_q rows x T columns and
// the T columns of one tile must share their other digits.
inline bool plan_fft(int logL, int LE, FftPlan& fp) {
  if (logL <= LE) {
    if (logL < 12) return false;
    fp.np = 1;
    fp.logn[1] = logL;
    fp.le[1] = logL;
    fp.logL = logL;
    return true;
  }
  for (int np = 2; np <= kMaxPasses; ++np) {
    int best_min = -1;
    int best[kMaxPasses + 1] = {0};
    int ln[kMaxPasses + 1];
    // Enumerate compositions of logL into np parts in [4, 9] (a tile then has
    // at least 8 columns, so global accesses are runs of >= 64 bytes).
    const int lo = 4, hi = 9;
    int total = 1;
    for (int q = 0; q < np; ++q) total *= (hi - lo + 1);
    for (int code = 0; code < total; ++code) {
      int c = code, sum = 0, mn = 99;
      for (int q = 1; q <= np; ++q) {
        ln[q] = lo + c % (hi - lo + 1);
        c /= (hi - lo + 1);
        sum += ln[q];
        mn = ln[q] < mn ? ln[q] : mn;
      }
      if (sum != logL) continue;
      bool ok = true;
      // PASS_FIRST (digit np): T = 2^(LE - ln[np]) columns within digit 1.
      if (LE - ln[np] > ln[1]) ok = false;
      // PASS_MID (digit q): T <= Tail_q = prod_{d > q} N_d.
      for (int q = 2; q < np && ok; ++q) {
        int tail = 0;
        for (int d = q + 1; d <= np; ++d) tail += ln[d];
        if (LE - ln[q] > tail) ok = false;
      }
      // PASS_LAST: T <= L / N_1.
      if (LE - ln[1] > logL - ln[1]) ok = false;
      for (int q = 1; q <= np; ++q)
        if (LE - ln[q] < 0) ok = false;
      if (!ok) continue;
      if (mn > best_min) {
        best_min = mn;
        for (int q = 1; q <= np; ++q) best[q] = ln[q];
      }
    }
    if (best_min >= 0) {
      fp.np = np;
      for (int q = 1; q <= np; ++q) {
        fp.logn[q] = best[q];
        fp.le[q] = LE;
      }
      fp.logL = logL;
      return true;
    }
  }
  return false;
}

// Valid digit splits of L = 2^logL for the autotuner: every split with the
// smallest pass count, plus (L <= 2^20) the most balanced splits with one
// pass more.  The
// extra pass costs a full read and write of the grids, but larger tiles in T
// (columns per tile) give longer contiguous runs: at L = 2^18 the two-pass
// split 2^9 x 2^9 moves runs of 8 elements (64 B), three passes of 2^6 move
// runs of 64.
inline std::vector<FftPlan> fft_splits_uniform(int logL, int LE) {
  std::vector<FftPlan> out;
  FftPlan best{};
  if (!plan_fft(logL, LE, best)) return out;
  if (best.np == 1) {
    out.push_back(best);
    return out;
  }
  const int lo = 4, hi = 9;
  auto valid = [&](const int* ln, int np) {
    bool ok = LE - ln[np] <= ln[1];
    for (int q = 2; q < np && ok; ++q) {
      int tail = 0;
      for (int d = q + 1; d <= np; ++d) tail += ln[d];
      if (LE - ln[q] > tail) ok = false;
    }
    return ok;
  };
  // The extra pass pays only on short grids (at L = 2^18 three passes of 2^6
  // beat two of 2^9); on grids above 2^20 cells it is slower and each pass
  // adds a rounding of the stored grid: measured on a curve of 1e6 points
  // with H = 8 and 2^24 bins (L = 2^26, mixed), every four-pass split gave
  // 6.3e-6 to 1.4e-5 against the oracle where the three-pass splits gave
  // 6.0e-6 to 9.9e-6.
  const int np_max = logL > 20 ? best.np : best.np + 1;
  for (int np = best.np; np <= np_max && np <= kMaxPasses; ++np) {
    std::vector<FftPlan> found;
    int total = 1;
    for (int q = 0; q < np; ++q) total *= (hi - lo + 1);
    int ln[kMaxPasses + 1];
    int best_min = 0;
    for (int code = 0; code < total; ++code) {
      int c = code, sum = 0, mn = 99;
      for (int q = 1; q <= np; ++q) {
        ln[q] = lo + c % (hi - lo + 1);
        c /= (hi - lo + 1);
        sum += ln[q];
        mn = ln[q] < mn ? ln[q] : mn;
      }
      if (sum != logL || !valid(ln, np)) continue;
      FftPlan f{};
      f.np = np;
      f.logL = logL;
      for (int q = 1; q <= np; ++q) {
        f.logn[q] = ln[q];
        f.le[q] = LE;
      }
      if (np == best.np) {
        out.push_back(f);
      } else if (mn >= best_min) {
        if (mn > best_min) found.clear();
        best_min = mn;
        found.push_back(f);
      }
    }
    out.insert(out.end(), found.begin(), found.end());
  }
  return out;
}

// Whether every pass q of the split fits its tile of 2^le[q] elements: the
// T = 2^(le[q] - logn[q]) columns of a tile must share their other digits.
inline bool split_valid(const FftPlan& f) {
  if (f.np == 1) return true;
  const int np = f.np;
  for (int q = 1; q <= np; ++q)
    if (f.le[q] - f.logn[q] < 0) return false;
  if (f.le[np] - f.logn[np] > f.logn[1]) return false;  // first pass
  for (int q = 2; q < np; ++q) {                          // middle passes
    int tail = 0;
    for (int d = q + 1; d <= np; ++d) tail += f.logn[d];
    if (f.le[q] - f.logn[q] > tail) return false;
  }
  return f.le[1] - f.logn[1] <= f.logL - f.logn[1];      // last pass
}

// Autotuner candidates: the splits of fft_splits_uniform for 2^12-element
// tiles and, for FP32 grids, for 2^13-element tiles (twice the columns, so
// runs twice as long), each also tried with its first pass on the smaller
// tile (that pass reads the sparse spread grid and writes whole columns).
inline std::vector<FftPlan> fft_splits(int logL, bool fp64) {
  std::vector<FftPlan> base = fft_splits_uniform(logL, 12);
  if (fp64 || logL <= 13) return base;
  for (const FftPlan& f : fft_splits_uniform(logL, 13)) base.push_back(f);
  std::vector<FftPlan> out;
  auto add = [&](const FftPlan& f) {
    if (!split_valid(f)) return;
    for (const FftPlan& g : out) {
      bool same = g.np == f.np;
      for (int q = 1; q <= f.np && same; ++q) same = g.logn[q] == f.logn[q] && g.le[q] == f.le[q];
      if (same) return;
    }
    out.push_back(f);
  };
  for (const FftPlan& f : base) {
    // All 2^12 tiles; all 2^13; first pass 2^12 and the rest 2^13; first pass
    // 2^13 and the rest 2^12.
    for (int v = 0; v < 4; ++v) {
      FftPlan g = f;
      for (int q = 1; q <= g.np; ++q) {
        const bool first = q == g.np;
        g.le[q] = (v == 1 || (v == 2 && !first) || (v == 3 && first)) ? 13 : 12;
      }
      add(g);
    }
  }
  return out;
}

}  // namespace fchi2
