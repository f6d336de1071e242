// FFT tiles of the multi-pass scheme (shared by the per-pass kernels and the
// persistent batched search); see fft.hip for the scheme.
#pragma once

#include "fchi2_internal.h"
#include "launch.h"
#include "es_kernel.h"

namespace fchi2 {

namespace {

constexpr double kC16[16] = {
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508978,
    0.0, -0.38268343236508978, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508978,
    0.0, 0.38268343236508978, 0.70710678118654752, 0.92387953251128674};
constexpr double kS16[16] = {
    0.0, 0.38268343236508978, 0.70710678118654752, 0.92387953251128674,
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508978,
    0.0, -0.38268343236508978, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508978};

// v * exp(+2 pi i E / N) for compile-time E, N <= 16.
template <typename R, int N, int E>
__device__ __forceinline__ cplx<R> mul_root(cplx<R> v) {
  constexpr int e = E % N;
  if constexpr (e == 0) {
    return v;
  } else if constexpr (4 * e == N) {
    return cmk<R>(-v.y, v.x);
  } else if constexpr (2 * e == N) {
    return cmk<R>(-v.x, -v.y);
  } else if constexpr (4 * e == 3 * N) {
    return cmk<R>(v.y, -v.x);
  } else {
    constexpr int k = e * (16 / N);
    const R c = (R)kC16[k];
    const R s = (R)kS16[k];
    return cmk<R>(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

template <int N, int I>
constexpr int bitrev() {
  int r = 0, x = I;
  for (int b = 1; b < N; b <<= 1) {
    r = (r << 1) | (x & 1);
    x >>= 1;
  }
  return r;
}

template <typename R, int N, int I>
__device__ __forceinline__ void bitrev_perm(cplx<R>* v) {
  if constexpr (I < N) {
    constexpr int J = bitrev<N, I>();
    if constexpr (I < J) {
      cplx<R> t = v[I];
      v[I] = v[J];
      v[J] = t;
    }
    bitrev_perm<R, N, I + 1>(v);
  }
}

template <typename R, int N, int S, int K, int J>
__device__ __forceinline__ void bfly_j(cplx<R>* v) {
  if constexpr (J < S) {
    constexpr int e = J * (N / (2 * S));
    cplx<R> t = mul_root<R, N, e>(v[K + J + S]);
    cplx<R> u = v[K + J];
    v[K + J] = cadd(u, t);
    v[K + J + S] = csub(u, t);
    bfly_j<R, N, S, K, J + 1>(v);
  }
}
template <typename R, int N, int S, int K>
__device__ __forceinline__ void bfly_k(cplx<R>* v) {
  if constexpr (K < N) {
    bfly_j<R, N, S, K, 0>(v);
    bfly_k<R, N, S, K + 2 * S>(v);
  }
}
template <typename R, int N, int S>
__device__ __forceinline__ void dit_stages(cplx<R>* v) {
  if constexpr (S < N) {
    bfly_k<R, N, S, 0>(v);
    dit_stages<R, N, 2 * S>(v);
  }
}

// In-register N-point DFT (N <= 16), natural order in and out, sign +i.
template <typename R, int N>
__device__ __forceinline__ void dft_reg(cplx<R>* v) {
  bitrev_perm<R, N, 0>(v);
  dit_stages<R, N, 1>(v);
}

// A tile holds 2^12 complex elements, or 2^13 with FP32 grids (the same LDS
// bytes as an FP64 tile of 2^12; twice the columns, so runs twice as long):
// the plan chooses per pass.  Every thread holds kEPT elements, so a
// workgroup has 256 or 512 threads.
constexpr int kEPT = 16;  // elements per thread
template <typename S>
constexpr int tile_log_max() {
  return sizeof(S) == 4 ? 13 : 12;
}
using C = cplx<double>;

// Grid data each pass touches once.  Runs of at least 128 bytes (NT) are
// loaded and stored non-temporally (streaming); shorter runs measured slower
// that way and use ordinary accesses.
template <bool NT, typename S>
__device__ __forceinline__ cplx<S> ntl(const cplx<S>* p) {
  if constexpr (NT) {
    cplx<S> r;
    r.x = __builtin_nontemporal_load(&p->x);
    r.y = __builtin_nontemporal_load(&p->y);
    return r;
  } else {
    return *p;
  }
}
template <bool NT, typename S>
__device__ __forceinline__ void nts(cplx<S>* p, cplx<S> v) {
  if constexpr (NT) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
  } else {
    *p = v;
  }
}
template <typename S>
__device__ __forceinline__ C widen(cplx<S> v) {
  return cmk<double>((double)v.x, (double)v.y);
}
template <typename S>
__device__ __forceinline__ cplx<S> narrow(C v) {
  return cmk<S>((S)v.x, (S)v.y);
}

// Stockham stage geometry over a tile of N rows x T columns, NT = N T / kEPT
// threads.  Butterfly bi of thread tid (slot it) is bi = tid + it * NT:
// column c = bi % T, butterfly
// b = bi / T; its element i is input row b + i N / RAD and output row
// (b / NS) NS RAD + b % NS + i NS.  Every thread holds kEPT elements.
template <int LOGN, int LOGT, int LOGNS>
struct Stage {
  static constexpr int N = 1 << LOGN;
  static constexpr int T = 1 << LOGT;
  static constexpr int NT = (N * T) / kEPT;
  static constexpr int LOGRAD = (LOGN - LOGNS) >= 4 ? 4 : (LOGN - LOGNS);
  static constexpr int RAD = 1 << LOGRAD;
  static constexpr int NS = 1 << LOGNS;
  static constexpr int PER = kEPT / RAD;
  static constexpr bool LAST = (LOGNS + LOGRAD) == LOGN;
  static_assert(PER * RAD == kEPT, "radix must divide the per-thread elements");
  __device__ static int col(int tid, int it) { return (tid + it * NT) & (T - 1); }
  __device__ static int bfly(int tid, int it) { return (tid + it * NT) >> LOGT; }
  __device__ static int in_row(int b, int i) { return b + i * (N / RAD); }
  __device__ static int out_row(int b, int i) {
    return ((b >> LOGNS) << (LOGNS + LOGRAD)) + (b & (NS - 1)) + i * NS;
  }
};

// Butterflies of one stage on the registers (FP64): stage twiddles from the
// omega_{2^13} table, then the in-register RAD-point DFT.
template <int LOGN, int LOGT, int LOGNS>
__device__ __forceinline__ void stage_compute(C* v, const C* __restrict__ tw, int tid) {
  using St = Stage<LOGN, LOGT, LOGNS>;
  constexpr int TWS = kStageLog - LOGNS - St::LOGRAD;
  static_assert(TWS >= 0, "stage twiddle table too small");
#pragma unroll
  for (int it = 0; it < St::PER; ++it) {
    C* u = v + it * St::RAD;
    if constexpr (St::NS > 1) {
      const int j = St::bfly(tid, it) & (St::NS - 1);
#pragma unroll
      for (int i = 1; i < St::RAD; ++i) u[i] = cmul(u[i], tw[(j * i) << TWS]);
    }
    dft_reg<double, St::RAD>(u);
  }
}

// Run the stages from LOGNS on; between stages the registers go through the
// LDS tile (type S) in Stockham order.  On return v holds the last stage's
// outputs: element i of slot it is row out_row(b, i) of column col(tid, it).
template <typename S, int LOGN, int LOGT, int LOGNS>
__device__ __forceinline__ void run_stages(C* v, cplx<S>* sm, const C* __restrict__ tw,
                                           int tid) {
  using St = Stage<LOGN, LOGT, LOGNS>;
  constexpr int PT = (St::T == 1) ? 1 : St::T + 1;
  stage_compute<LOGN, LOGT, LOGNS>(v, tw, tid);
  if constexpr (!St::LAST) {
    using Nx = Stage<LOGN, LOGT, LOGNS + St::LOGRAD>;
    __syncthreads();  // previous readers of sm are done
#pragma unroll
    for (int it = 0; it < St::PER; ++it) {
      const int c = St::col(tid, it), b = St::bfly(tid, it);
#pragma unroll
      for (int i = 0; i < St::RAD; ++i)
        sm[St::out_row(b, i) * PT + c] = narrow<S>(v[it * St::RAD + i]);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < Nx::PER; ++it) {
      const int c = Nx::col(tid, it), b = Nx::bfly(tid, it);
#pragma unroll
      for (int i = 0; i < Nx::RAD; ++i)
        v[it * Nx::RAD + i] = widen(sm[Nx::in_row(b, i) * PT + c]);
    }
    run_stages<S, LOGN, LOGT, LOGNS + St::LOGRAD>(v, sm, tw, tid);
  }
}

// LOGNS of the last stage: stages advance by radix 16 until the remainder.
constexpr int last_logns(int logn) {
  int ns = 0;
  while (ns + ((logn - ns) >= 4 ? 4 : (logn - ns)) < logn) ns += 4;
  return ns;
}

// exp(+2 pi i e / 2^logM) for 0 <= e < 2^logM (exact argument reduction).
__device__ __forceinline__ C root(int64_t e, int logM) {
  double s, c;
  sincospi(ldexp((double)e, 1 - logM), &s, &c);
  return cmk<double>(c, s);
}

// Cells of a first-pass tile (pair p, columns g0 + cc, rows r of stride
// Sd = L / N; rows r >= r_lim are beyond the pair's extent and stay zero)
// spread from the curve's points straight into the LDS tile sm, as S values in
// the tile layout (row r, column cc at r * PT + cc).  A thread owns kEPT
// cells, as one segment of a row (T >= kEPT) or whole rows.  The points that
// can reach a segment are a contiguous index range (positions grow with t):
// the fine tile table of the spreading (first point at or past each tile of
// 2^tb_log cells, minus the kernel's reach) gives it with two loads, and the
// thread reads those points, forms their cell coordinate on the component's
// harmonic grid and strength as the spreading kernel does, and adds
// phi(cell - pos) times the strength point by point in index order:
// component 0 of the pair into the real part (and the imaginary part when
// both components are the same harmonic), component 1 into the imaginary
// part.  FLR: floor gridding (kernel width 1).
template <typename S, int LOGN, int LOGT, bool FLR>
__device__ __forceinline__ void spread_into_tile(const FftPassArgs& a, const Moments& mo,
                                                 const Geom& g, int p, int cw, int64_t g0,
                                                 int64_t r_lim, cplx<S>* sm, int tid) {
  constexpr int N = 1 << LOGN;
  constexpr int T = 1 << LOGT;
  constexpr int PT = (T == 1) ? 1 : T + 1;
  constexpr int NTH = (N * T) / kEPT;
  constexpr int CPR = T >= kEPT ? kEPT : T;  // cells per owned row segment
  constexpr int RPT = kEPT / CPR;            // row segments per thread
  constexpr int TPR = T >= kEPT ? T / kEPT : 1;  // threads per row
  constexpr bool EXACT = sizeof(S) == 8;
  const int64_t Sd = g.L >> LOGN;
  double ar[RPT][CPR], ai[RPT][CPR];
#pragma unroll
  for (int j = 0; j < RPT; ++j)
#pragma unroll
    for (int u = 0; u < CPR; ++u) {
      ar[j][u] = 0.0;
      ai[j][u] = 0.0;
    }
  const int m0 = g.comp_m[p][0], m1 = g.comp_m[p][1];
  const bool both = m1 == m0;
  const int kd0 = g.comp_kind[p][0], kd1 = g.comp_kind[p][1];
  const double Ld = (double)g.L, coff = (double)g.c_off;
  const double two_over_w = 2.0 / (double)g.w;
  const double beta = g.beta;
  const double* __restrict__ t = a.t;
  const double* __restrict__ x = a.x;
  const double* __restrict__ sg = a.sigma;
  const int64_t pa = mo.start;
  const double t_last = t[pa + mo.n - 1];
  const int tbl = a.tb_log;
#pragma unroll
  for (int comp = 0; comp < 2; ++comp) {
    const int m = comp ? m1 : m0;
    if (m == 0 || (comp == 1 && both)) continue;
    const int kd = comp ? kd1 : kd0;
    const int32_t* row_tb = a.tb + ((int64_t)cw * (2 * g.H) + (m - 1)) * a.ntb;
    // Last table entry written for harmonic m (see the spreading kernel).
    const double last = cell_of((t_last - mo.T0) * g.df, m, Ld, coff, FLR);
    const int64_t lim = (int64_t)floor((last + (double)(g.w / 2 + 2)) / (double)((int64_t)1 << tbl)) + 3;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      int row, c0;
      if constexpr (TPR > 1) {
        row = tid / TPR;
        c0 = (tid % TPR) * kEPT;
      } else {
        row = tid + j * NTH;
        c0 = 0;
      }
      if (row >= r_lim) continue;
      const int64_t cell0 = g0 + c0 + Sd * (int64_t)row;
      // The grid is periodic: the segment gathers its points lap after lap
      // (positions on the unwrapped axis, table over g.laps periods).
     for (int lap = 0; lap < g.laps; ++lap) {
      const int64_t ucell = cell0 + (int64_t)lap * g.L;
      const int64_t ta = ucell >> tbl, tb2 = ((ucell + CPR - 1) >> tbl) + 2;
      if (ta > lim - 2) break;  // no point of harmonic m reaches this far
      const int64_t lo = pa + row_tb[ta];
      const int64_t hi = tb2 <= lim ? pa + row_tb[tb2] : pa + mo.n;
      const double c0d = (double)ucell;
      const double reach = (double)(g.w / 2 + 1);
      for (int64_t i = lo; i < hi; ++i) {
        const double pos = cell_at(t[i], mo.T0, g.df, m, Ld, coff, FLR);
        // Only points within the kernel's reach of the segment add a nonzero
        // tap (the others add exact zeros): skip those before it, stop after.
        if (pos < c0d - reach) continue;
        if (pos > c0d + (double)(CPR - 1) + reach) break;
        const double si = sg[i];
        const double w = 1.0 / (si * si);
        const double wy = w * (x[i + mo.xshift] - mo.xbar);
        const double va = kd == 0 ? w : wy;
        const double vb = both ? (kd1 == 0 ? w : wy) : 0.0;
#pragma unroll
        for (int u = 0; u < CPR; ++u) {
          const double phi = es_kernel<EXACT>(((c0d + (double)u) - pos) * two_over_w, beta);
          if (comp == 0) {
            ar[j][u] += phi * va;
            if (both) ai[j][u] += phi * vb;
          } else {
            ai[j][u] += phi * va;
          }
        }
      }
     }
    }
  }
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int row = (TPR > 1) ? tid / TPR : tid + j * NTH;
    const int c0 = (TPR > 1) ? (tid % TPR) * kEPT : 0;
#pragma unroll
    for (int u = 0; u < CPR; ++u)
      sm[row * PT + c0 + u] = cmk<S>((S)ar[j][u], (S)ai[j][u]);
  }
  __syncthreads();
}

// One pass.  Twiddles between passes, for output row k of tile column cc:
//   PASS_FIRST, np >= 3: w_M^{jd k}        (jd fixed for the tile)   = r[k]
//   PASS_FIRST, np == 2: w_L^{(g0+cc) k}   = r[k] * small[cc k]
//   PASS_MID:            w_M^{jd (K0+cc+Tail k)}                     = c[cc] r[k]
// with r, c built per workgroup in FP64 and small[e] = w_L^e, e < N T.
// LDS of one tile: the data tile, the row and column twiddles and, in the
// first pass, the output offset of each tile column.
// FP64 tiles keep the row twiddles in the padding column of the data tile
// (one 16-byte slot per row that no data access touches), which brings the
// 2^9 x 8 tile from 82 to 74 KB: two workgroups per CU instead of one.
template <typename S, int LOGN, int LOGT>
struct FftSmem {
  static constexpr int N = 1 << LOGN;
  static constexpr int T = 1 << LOGT;
  static constexpr int PT = (T == 1) ? 1 : T + 1;
  static constexpr bool kTrInPad = sizeof(cplx<S>) == sizeof(C) && T > 1;
  __align__(16) cplx<S> sm[N * PT];
  C tr[(T == 1 || kTrInPad) ? 1 : N];  // the single-pass tile has no twiddles
  C tc[T];
  int64_t s_rev[T];
  __device__ __forceinline__ C& row_tw(int k) {
    if constexpr (kTrInPad)
      return *reinterpret_cast<C*>(&sm[k * PT + T]);
    else
      return tr[k];
  }
};

// One tile of one pass: columns [bx T, bx T + T) of packed grid p of wave slot
// cw, whose grid is at in + grid_off (input) and out + grid_off (output) and
// whose pruned spectra (last forward pass) start at zpair.  Every thread of
// the workgroup calls it (it synchronises the workgroup).
template <typename S, int LOGN, int LOGT, bool FUSED>
__device__ __forceinline__ void fft_pass_tile(const FftPassArgs& a, const cplx<S>* in,
                                              cplx<S>* out, const Moments* __restrict__ mom,
                                              const Geom& g, const C* __restrict__ tw_stage,
                                              const C* __restrict__ tw_small, int bx, int p,
                                              int cw, int64_t grid_off, cplx<S>* zpair,
                                              FftSmem<S, LOGN, LOGT>& sh, int tid) {
  constexpr int N = 1 << LOGN;
  constexpr int T = 1 << LOGT;
  constexpr int PT = (T == 1) ? 1 : T + 1;
  constexpr int kNT = (N * T) / kEPT;  // threads of this tile
  static_assert(N * T == 4096 || (N * T == 8192 && sizeof(S) == 4), "tile size");
  constexpr bool NT = T * sizeof(cplx<S>) >= 128;
  using S0 = Stage<LOGN, LOGT, 0>;
  using SL = Stage<LOGN, LOGT, last_logns(LOGN)>;
  cplx<S>* sm = sh.sm;
  C* tc = sh.tc;
  int64_t* s_rev = sh.s_rev;

  const Moments mo = mom[a.curve0 + cw];
  if (mo.flags & kCurveFatal) return;

  const int64_t L = g.L;
  const int logL = a.logL;
  const cplx<S>* src = in + grid_off;
  const int64_t g0 = (int64_t)bx * T;  // first column of this tile

  int low_bits = 0;  // sum of log2 N over digits below q
  for (int d = 1; d < a.q; ++d) low_bits += a.logn[d];

  C v[kEPT];
  // Stage-0 inputs straight from HBM: element i of slot it is row
  // in_row(b, i) of column col(tid, it).
  if (a.kind == PASS_FIRST || a.kind == PASS_SINGLE) {
    const int64_t Sd = L >> LOGN;  // column c = g0 + cc, row r at c + Sd r
    int64_t r_skip_lo, r_skip_hi;  // rows in [r_skip_lo, r_skip_hi) are zero
    if (a.mode == MODE_FWD) {
      const int64_t E = pair_extent(mo, g, p);
      r_skip_lo = (E + Sd - 1) / Sd;
      r_skip_hi = N;
    } else {
      r_skip_lo = g.n_freq / Sd;
      r_skip_hi = (L - g.n_freq) / Sd;
    }
    if constexpr (FUSED) {
      // Forward first pass only (the launcher guarantees it).
      if (g.w == 1)
        spread_into_tile<S, LOGN, LOGT, true>(a, mo, g, p, cw, g0, r_skip_lo, sm, tid);
      else
        spread_into_tile<S, LOGN, LOGT, false>(a, mo, g, p, cw, g0, r_skip_lo, sm, tid);
#pragma unroll
      for (int it = 0; it < S0::PER; ++it) {
        const int cc = S0::col(tid, it), b = S0::bfly(tid, it);
#pragma unroll
        for (int i = 0; i < S0::RAD; ++i)
          v[it * S0::RAD + i] = widen(sm[S0::in_row(b, i) * PT + cc]);
      }
    } else {
#pragma unroll
      for (int it = 0; it < S0::PER; ++it) {
        const int cc = S0::col(tid, it), b = S0::bfly(tid, it);
#pragma unroll
        for (int i = 0; i < S0::RAD; ++i) {
          const int r = S0::in_row(b, i);
          C val = cmk<double>(0.0, 0.0);
          if (r < r_skip_lo || r >= r_skip_hi) val = widen(ntl<NT>(&src[g0 + cc + Sd * r]));
          v[it * S0::RAD + i] = val;
        }
      }
    }
    if (a.kind == PASS_FIRST) {
      const int np = a.np;
      const int logM = a.logn[np - 1] + LOGN;
      if (np >= 3) {
        int bits_below = 0;
        for (int d = 1; d < np - 1; ++d) bits_below += a.logn[d];
        const int64_t jd = g0 >> bits_below;
        const int64_t Mmask = ((int64_t)1 << logM) - 1;
        for (int k = tid; k < N; k += kNT) sh.row_tw(k) = root((jd * k) & Mmask, logM);
      } else {
        for (int k = tid; k < N; k += kNT) sh.row_tw(k) = root((g0 * k) & (L - 1), logL);
      }
    }
  } else {
    // PASS_MID: column (pre, K0 + cc), row r at pre N Tail + r Tail + K0 + cc.
    // PASS_LAST: pre = 0, Tail = L / N.
    const int64_t Tail = L >> (low_bits + LOGN);
    const int64_t pre = g0 / Tail;
    const int64_t K0 = g0 - pre * Tail;
    const cplx<S>* base = src + pre * ((int64_t)N * Tail) + K0;
#pragma unroll
    for (int it = 0; it < S0::PER; ++it) {
      const int cc = S0::col(tid, it), b = S0::bfly(tid, it);
#pragma unroll
      for (int i = 0; i < S0::RAD; ++i)
        v[it * S0::RAD + i] = widen(ntl<NT>(&base[(int64_t)S0::in_row(b, i) * Tail + cc]));
    }
    if (a.kind == PASS_MID) {
      const int64_t jd = pre & (((int64_t)1 << a.logn[a.q - 1]) - 1);
      const int logTail = logL - low_bits - LOGN;
      const int logM = a.logn[a.q - 1] + LOGN + logTail;
      const int64_t Mmask = ((int64_t)1 << logM) - 1;
      for (int k = tid; k < N; k += kNT) sh.row_tw(k) = root((jd * Tail * k) & Mmask, logM);
      for (int cc = tid; cc < T; cc += kNT) tc[cc] = root((jd * (K0 + cc)) & Mmask, logM);
    }
  }
  // tr/tc become visible at the first barrier inside run_stages, or below.
  run_stages<S, LOGN, LOGT, 0>(v, sm, tw_stage, tid);
  if constexpr (last_logns(LOGN) == 0) __syncthreads();  // single-stage tile

  cplx<S>* dst = out + grid_off;
  if (a.kind == PASS_FIRST) {
    // Twiddle in registers, then transpose through LDS so that each column's
    // N outputs leave as one contiguous run at row rev(c) of the output.
    const int np = a.np;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SL::PER; ++it) {
      const int cc = SL::col(tid, it), b = SL::bfly(tid, it);
#pragma unroll
      for (int i = 0; i < SL::RAD; ++i) {
        const int k = SL::out_row(b, i);
        C tw = sh.row_tw(k);
        if (np == 2) tw = cmul(tw, tw_small[cc * k]);
        sm[k * PT + cc] = narrow<S>(cmul(v[it * SL::RAD + i], tw));
      }
    }
    // Mixed-radix reversal of each of the tile's T columns, once per tile:
    // rev = ((j_1 N_2 + j_2) N_3 + j_3) ... + j_{np-1} for column c = g0 + cc.
    for (int cc = tid; cc < T; cc += kNT) {
      int64_t rev = 0, rest = g0 + cc;
      for (int d = 1; d < np; ++d) {
        const int64_t dig = rest & (((int64_t)1 << a.logn[d]) - 1);
        rest >>= a.logn[d];
        rev = (rev << a.logn[d]) | dig;
      }
      s_rev[cc] = rev * N;
    }
    __syncthreads();
#pragma unroll 4
    for (int it = 0; it < kEPT; ++it) {
      const int e = tid + it * kNT;
      const int k = e & (N - 1);
      const int cc = e >> LOGN;
      nts<NT>(&dst[s_rev[cc] + k], sm[k * PT + cc]);
    }
  } else if (a.kind == PASS_MID) {
    const int64_t Tail = L >> (low_bits + LOGN);
    const int64_t pre = g0 / Tail;
    const int64_t K0 = g0 - pre * Tail;
    cplx<S>* base = dst + pre * ((int64_t)N * Tail) + K0;
#pragma unroll
    for (int it = 0; it < SL::PER; ++it) {
      const int cc = SL::col(tid, it), b = SL::bfly(tid, it);
      const C fc = tc[cc];
#pragma unroll
      for (int i = 0; i < SL::RAD; ++i) {
        const int k = SL::out_row(b, i);
        nts<NT>(&base[(int64_t)k * Tail + cc], narrow<S>(cmul(v[it * SL::RAD + i], cmul(fc, sh.row_tw(k)))));
      }
    }
  } else {
    // PASS_LAST / PASS_SINGLE: X index = K + Tail * k, natural order.
    const int64_t Tail = L >> LOGN;
    const int64_t nf = g.n_freq;
    if (a.mode == MODE_FWD) {
      cplx<S>* z0 = zpair;
      cplx<S>* z1 = z0 + nf;
#pragma unroll
      for (int it = 0; it < SL::PER; ++it) {
        const int cc = SL::col(tid, it), b = SL::bfly(tid, it);
#pragma unroll
        for (int i = 0; i < SL::RAD; ++i) {
          const int64_t X = g0 + cc + Tail * SL::out_row(b, i);
          const cplx<S> val = narrow<S>(v[it * SL::RAD + i]);
          if (X < nf) z0[X] = val;
          const int64_t Xm = (L - X) & (L - 1);
          if (Xm < nf) z1[Xm] = val;
        }
      }
    } else {
      const int64_t E = pair_extent(mo, g, p);
      cplx<S>* go = (cplx<S>*)a.grid_out + grid_off;
#pragma unroll
      for (int it = 0; it < SL::PER; ++it) {
        const int cc = SL::col(tid, it), b = SL::bfly(tid, it);
#pragma unroll
        for (int i = 0; i < SL::RAD; ++i) {
          const int64_t X = g0 + cc + Tail * SL::out_row(b, i);
          if (X < E) go[X] = narrow<S>(v[it * SL::RAD + i]);
        }
      }
    }
  }
}

// Waves per SIMD a pass kernel is compiled for.  FP32 tiles of 8192
// elements are workgroups of eight waves with 72-78 KB of LDS, two per CU,
// which needs four waves per SIMD (at most 128 registers): left to itself the
// compiler gives the 2^9-row tiles 130 registers and the CU one workgroup
// (a curve of 1e6 points, H = 8, 2^24 bins: FFT 9.3 -> 8.1 ms).  The fused
// first pass (spreading inside the tile) keeps its own allocation: at 128
// registers it spills.
template <typename S, bool FUSED>
constexpr int fft_pass_waves() {
  return (sizeof(S) == 4 && !FUSED) ? 4 : 1;
}

// The pass over a wave of curves: grid (column tiles, pairs, curves).
template <typename S, int LOGN, int LOGT, bool FUSED>
__global__ __launch_bounds__(((1 << LOGN) << LOGT) / kEPT, (fft_pass_waves<S, FUSED>())) void k_fft_pass(
    FftPassArgs a, const cplx<S>* in, cplx<S>* out, const Moments* __restrict__ mom, Geom g,
    const C* __restrict__ tw_stage, const C* __restrict__ tw_small) {
  __shared__ FftSmem<S, LOGN, LOGT> sh;
  const int p = blockIdx.y;
  const int cw = blockIdx.z;
  const int64_t grid_off = ((int64_t)cw * g.P + p) * g.L;
  cplx<S>* zpair = a.zc ? (cplx<S>*)a.zc + ((int64_t)cw * g.P + p) * 2 * g.n_freq : nullptr;
  fft_pass_tile<S, LOGN, LOGT, FUSED>(a, in, out, mom, g, tw_stage, tw_small, blockIdx.x, p, cw,
                                      grid_off, zpair, sh, threadIdx.x);
}

}  // namespace

}  // namespace fchi2
