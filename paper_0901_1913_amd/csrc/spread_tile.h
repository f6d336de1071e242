// Spreading tiles and their tile -> point-range table (shared by the
// spreading kernels and the persistent batched search); see spread.hip.
#pragma once

#include <cmath>

#include "fchi2_internal.h"
#include "es_kernel.h"

namespace fchi2 {

namespace {

constexpr int kNT = 256;

__device__ __forceinline__ double cell_pos(const double* __restrict__ t, int64_t i, double T0,
                                           double df, int m, double L, double c_off,
                                           bool flr) {
  return cell_at(t[i], T0, df, m, L, c_off, flr);
}

// Tile -> point-range table.  For harmonic m and tile t of B cells, the
// points a tile may need are those with position in
// [x_t, x_{t+2}), x_t = t B - w/2 - 2 (a superset of the kernel footprint).
// tb[t] = first point index i (relative to the curve) with pos_i >= x_t.  The
// intervals (pos_{i-1}, pos_i] partition the line, so thread i writes exactly
// the entries whose x_t falls in its interval: one scatter, no searches.
// Entries stop at tile_limit(): tiles past it hold no point of harmonic m.
// Last table entry written for harmonic m: the tile after the one holding the
// last point's footprint, plus the two-tile lookahead of the spreading.
__device__ __forceinline__ int64_t tile_limit_of(double t_last, const Moments& mo,
                                                 const Geom& g, int m, int log_tile) {
  const double last = cell_at(t_last, mo.T0, g.df, m, (double)g.L, (double)g.c_off, g.w == 1);
  return (int64_t)floor((last + (double)(g.w / 2 + 2)) / (double)((int64_t)1 << log_tile)) + 3;
}

__device__ __forceinline__ int64_t tile_limit(const double* __restrict__ t, const Moments& mo,
                                              const Geom& g, int m, int log_tile) {
  return tile_limit_of(t[mo.start + mo.n - 1], mo, g, m, log_tile);
}

// The table entries owned by point il (0..n; n: past the last point) of
// harmonic m for the curve mo in table slot cw.
__device__ __forceinline__ void tile_bounds_point(const double* __restrict__ t,
                                                  const Moments& mo, const Geom& g, int cw,
                                                  int m, int64_t il, int log_tile, int ntb,
                                                  int32_t* __restrict__ tb) {
  if (il > mo.n) return;
  const double Ld = (double)g.L, coff = (double)g.c_off;
  const double B = (double)((int64_t)1 << log_tile);
  const double shift = (double)(g.w / 2 + 2);
  int64_t t_min, t_max;
  if (il == 0) {
    t_min = 0;
  } else {
    const double lo = cell_pos(t, mo.start + il - 1, mo.T0, g.df, m, Ld, coff, g.w == 1);
    t_min = (int64_t)floor((lo + shift) / B) + 1;
  }
  if (il == mo.n) {
    t_max = tile_limit(t, mo, g, m, log_tile);
  } else {
    const double hi = cell_pos(t, mo.start + il, mo.T0, g.df, m, Ld, coff, g.w == 1);
    t_max = (int64_t)floor((hi + shift) / B);
  }
  if (t_min < 0) t_min = 0;
  if (t_max > ntb - 1) t_max = ntb - 1;
  int32_t* row = tb + ((int64_t)cw * (2 * g.H) + (m - 1)) * ntb;
  for (int64_t q = t_min; q <= t_max; ++q) row[q] = (int32_t)il;
}

constexpr int kSpreadCH = 1024;  // points staged through LDS at a time

// LDS of one spreading tile.
template <int LOGB>
struct SpreadSmem {
  double s_p[kSpreadCH];   // cell coordinate relative to the tile start (exact)
  double2 s_v[kSpreadCH];  // strengths of the real and imaginary parts
  int s_first[kNT];
  int s_first1[kNT];       // the second component's, when both are staged at once
};

// Point q of harmonic m (absolute index i) staged for a tile whose unwrapped
// first cell is base: its cell coordinate relative to base and its strengths
// (sre, sim) as the spreading adds them.
template <bool BAND>
__device__ __forceinline__ void stage_point(const double* __restrict__ t,
                                            const double* __restrict__ x,
                                            const double* __restrict__ sigma, const Moments& mo,
                                            const Geom& g, int comp, int m, int kind_a,
                                            int kind_b, bool both, int64_t i, int64_t base,
                                            double* s_p, double2* s_v, int q) {
  // floor gridding: pos is an integer and the kernel below is exp(0) = 1 at
  // d = 0 and 0 at |d| >= 1 (w = 1)
  const double pos = cell_pos(t, i, mo.T0, g.df, m, (double)g.L, (double)g.c_off, g.w == 1);
  const double si = sigma[i];
  const double w = 1.0 / (si * si);
  const double wy = w * (x[i + mo.xshift] - mo.xbar);
  const double sa = (kind_a == 0) ? w : wy;
  double sre, sim;
  if constexpr (BAND) {
    // Band plan: strength times exp(+2 pi i kc m u), kc = k0 + n_freq/2 the
    // band's middle bin, so that grid bin j (j - L for j >= L/2) is bin
    // kc + j of the search.  The phase kc m u in cycles is reduced modulo 1
    // from the FP64 product and its exact rounding residual.
    const double km = (double)((g.k0 + g.n_freq / 2) * (int64_t)m);
    const double u = (t[i] - mo.T0) * g.df;
    const double ph = km * u;
    const double r = fma(km, u, -ph);
    double fr = (ph - floor(ph)) + r;
    fr -= floor(fr);
    double sn, cs;
    sincospi(2.0 * fr, &sn, &cs);
    sre = sa * cs;
    sim = sa * sn;
  } else if (comp == 0) {
    sre = sa;
    sim = both ? ((kind_b == 0) ? w : wy) : 0.0;
  } else {
    sre = 0.0;
    sim = sa;
  }
  // pos - base is exact (a multiple of pos's ulp, smaller than pos), and so
  // is jl - s_p below: the same kernel argument as jl - cell - frac.
  s_p[q] = pos - (double)base;
  s_v[q] = make_double2(sre, sim);
}

// First staged point in [lo, hi) with coordinate >= key (binary search).
__device__ __forceinline__ int first_at_or_above(const double* s_p, int lo, int hi, double key) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (s_p[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Adds to cell jl (coordinate cl) the taps of the staged points [q, end)
// within the kernel's reach, in index order.
template <bool EXACT>
__device__ __forceinline__ void add_taps(const double* s_p, const double2* s_v, int q, int end,
                                         double cl, double hreach, double two_over_w,
                                         double beta, double& ar, double& ai) {
  while (q < end && cl - s_p[q] > hreach) ++q;
  for (int r = q; r < end; ++r) {
    const double d = cl - s_p[r];
    if (d <= -hreach) break;
    const double phi = es_kernel<EXACT>(d * two_over_w, beta);
    const double2 v = s_v[r];
    ar += phi * v.x;
    ai += phi * v.y;
  }
}

// One tile of B cells (tile `tile` of packed grid p) of the curve mo, whose
// table rows are in slot cw (or slot 0 with share_tb), written to out (the
// tile's first cell).  Every thread of the workgroup calls it.
template <typename S, int LOGB, bool BAND>
__device__ __forceinline__ void spread_tile(const double* __restrict__ t,
                                            const double* __restrict__ x,
                                            const double* __restrict__ sigma,
                                            const Moments& mo, const Geom& g, int cw,
                                            const int32_t* __restrict__ tb, int ntb,
                                            int share_tb, int p, int64_t tile,
                                            cplx<S>* __restrict__ out, SpreadSmem<LOGB>& sh,
                                            int tid) {
  constexpr bool EXACT = sizeof(S) == 8;
  constexpr int B = 1 << LOGB;
  constexpr int CPT = B / kNT;
  constexpr int CH = kSpreadCH;
  double* s_p = sh.s_p;
  double2* s_v = sh.s_v;
  int* s_first = sh.s_first;

  const double t_last = t[mo.start + mo.n - 1];
  const int64_t a0 = tile * B;

  const int hw = g.w / 2;
  const double two_over_w = 2.0 / (double)g.w;
  const double hreach = (double)(hw + 1);
  const double beta = g.beta;
  const double Ld = (double)g.L;
  const double coff = (double)g.c_off;
  const int64_t pa = mo.start;

  double acc_re[CPT], acc_im[CPT];
#pragma unroll
  for (int u = 0; u < CPT; ++u) {
    acc_re[u] = 0.0;
    acc_im[u] = 0.0;
  }

  // The grid is periodic in L cells: positions are kept unwrapped (the
  // phase m u of a long curve may span several periods) and the tile table
  // runs over g.laps periods, so the tile gathers its points lap after lap
  // (in index order: positions grow with t).
  const int64_t ntile = g.L >> LOGB;
  const int SPC = B / kNT;  // cells per binary search
  if constexpr (!BAND) {
    // A pair of two distinct harmonics on one lap whose points fit the LDS
    // chunk together: both components are staged in one round (one chain of
    // table and point loads, three barriers instead of six).  Each cell adds
    // component 0's taps, then component 1's, in index order, exactly as
    // the component-by-component loop below does.
    const int m0 = g.comp_m[p][0], m1 = g.comp_m[p][1];
    if (g.laps == 1 && m0 != 0 && m1 != 0 && m1 != m0) {
      const int32_t* row0 = tb + ((int64_t)(share_tb ? 0 : cw) * (2 * g.H) + (m0 - 1)) * ntb;
      const int32_t* row1 = tb + ((int64_t)(share_tb ? 0 : cw) * (2 * g.H) + (m1 - 1)) * ntb;
      const int64_t lim0 = tile_limit_of(t_last, mo, g, m0, LOGB);
      const int64_t lim1 = tile_limit_of(t_last, mo, g, m1, LOGB);
      int64_t lo0 = 0, lo1 = 0;
      int cnt0 = 0, cnt1 = 0;
      if (tile + 2 <= lim0) {
        lo0 = pa + row0[tile];
        const int64_t hi0 = pa + row0[tile + 2];
        cnt0 = hi0 > lo0 ? (int)(hi0 - lo0) : 0;
      }
      if (tile + 2 <= lim1) {
        lo1 = pa + row1[tile];
        const int64_t hi1 = pa + row1[tile + 2];
        cnt1 = hi1 > lo1 ? (int)(hi1 - lo1) : 0;
      }
      if ((int64_t)cnt0 + cnt1 <= CH) {
        const int n01 = cnt0 + cnt1;
        if (n01 > 0) {
          const int kind0 = g.comp_kind[p][0], kind1 = g.comp_kind[p][1];
          for (int q = tid; q < n01; q += kNT) {
            if (q < cnt0)
              stage_point<false>(t, x, sigma, mo, g, 0, m0, kind0, -1, false, lo0 + q, a0, s_p,
                                 s_v, q);
            else
              stage_point<false>(t, x, sigma, mo, g, 1, m1, kind1, -1, false, lo1 + (q - cnt0),
                                 a0, s_p, s_v, q);
          }
          __syncthreads();
          {
            const double key = (double)(tid * SPC - hw - 1);
            s_first[tid] = first_at_or_above(s_p, 0, cnt0, key);
            sh.s_first1[tid] = first_at_or_above(s_p, cnt0, n01, key);
          }
          __syncthreads();
#pragma unroll
          for (int u = 0; u < CPT; ++u) {
            const int jl = tid + u * kNT;
            const double cl = (double)jl;
            double ar = acc_re[u], ai = acc_im[u];
            add_taps<EXACT>(s_p, s_v, s_first[jl / SPC], cnt0, cl, hreach, two_over_w, beta, ar,
                            ai);
            add_taps<EXACT>(s_p, s_v, sh.s_first1[jl / SPC], n01, cl, hreach, two_over_w, beta,
                            ar, ai);
            acc_re[u] = ar;
            acc_im[u] = ai;
          }
          __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < CPT; ++u) out[tid + u * kNT] = cmk<S>((S)acc_re[u], (S)acc_im[u]);
        return;
      }
    }
  }
  for (int comp = 0; comp < 2; ++comp) {
    const int m = g.comp_m[p][comp];
    if (m == 0) continue;
    if (comp == 1 && m == g.comp_m[p][0]) continue;  // shared with component 0
    const bool both = (comp == 0) && (g.comp_m[p][1] == m);
    const int kind_a = g.comp_kind[p][comp];
    const int kind_b = both ? g.comp_kind[p][1] : -1;
    const int32_t* row = tb + ((int64_t)(share_tb ? 0 : cw) * (2 * g.H) + (m - 1)) * ntb;
    // No point of harmonic m reaches tiles past tile_limit - 2.
    const int64_t lim = tile_limit_of(t_last, mo, g, m, LOGB);
   for (int lap = 0; lap < g.laps; ++lap) {
    const int64_t ut = tile + (int64_t)lap * ntile;  // tile on the unwrapped axis
    if (ut + 2 > lim) break;
    const int64_t i_lo = pa + row[ut], i_hi = pa + row[ut + 2];
    if (i_hi <= i_lo) continue;  // no points in this lap
    const int64_t base = a0 + (int64_t)lap * g.L;

    for (int64_t ch = i_lo; ch < i_hi; ch += CH) {
      const int cnt = (int)((i_hi - ch) < CH ? (i_hi - ch) : CH);
      for (int q = tid; q < cnt; q += kNT)
        stage_point<BAND>(t, x, sigma, mo, g, comp, m, kind_a, kind_b, both, ch + q, base, s_p,
                          s_v, q);
      __syncthreads();
      // Cell jl takes the points with floor(p) in [jl - hw - 1, jl + hw], i.e.
      // jl - hw - 1 <= p < jl + hw + 1 (with d = jl - p the window is
      // -(hw + 1) < d <= hw + 1).  The first of them is found by binary
      // search for every (B / 256)-th cell (one search per thread); cells in
      // between advance from it.
      s_first[tid] = first_at_or_above(s_p, 0, cnt, (double)(tid * SPC - hw - 1));
      __syncthreads();
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int jl = tid + u * kNT;
        double ar = acc_re[u], ai = acc_im[u];
        add_taps<EXACT>(s_p, s_v, s_first[jl / SPC], cnt, (double)jl, hreach, two_over_w, beta,
                        ar, ai);
        acc_re[u] = ar;
        acc_im[u] = ai;
      }
      __syncthreads();
    }
   }
  }

#pragma unroll
  for (int u = 0; u < CPT; ++u) out[tid + u * kNT] = cmk<S>((S)acc_re[u], (S)acc_im[u]);
}


}  // namespace

}  // namespace fchi2
