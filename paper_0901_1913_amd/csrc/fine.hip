// Fine search on the ungridded data (Section 3e): around each candidate
// frequency, Delta chi2 is evaluated directly from the points at R evenly
// spaced trial frequencies, with no gridding, and the locally best one is
// kept together with its coefficients.
//
// For a trial frequency f the sums of Section 2 are taken point by point in
// FP64:  Q(m f) = sum_i w_i e^{+i 2 pi m f tau_i}  (m = 1..2H) and
// P(m f) = sum_i w_i y_i e^{+i 2 pi m f tau_i}  (m = 1..H), tau = t - T0,
// y = x - xbar; Q(0) = W and P(0) = 0 (Section 3b).  The phase of the first
// harmonic is taken from the FP64 product f tau reduced to [0, 1) cycles; the
// higher harmonics follow by complex multiplication.  The normal equations,
// the prefix Cholesky solve and Delta chi2 for every H' are those of the grid
// search; the coefficients solve L^T A = z (eq. eqcoeffs) and xbar is added
// back to A_0.
//
// Phase 1 (k_fine_sums): a block holds 256 trial frequencies of one curve and
// one chunk of its points; the points are staged through LDS and every
// thread accumulates the 3H complex sums of its frequency.  Partial sums go
// to scratch, per chunk.  Phase 2 (k_fine_solve): one block per candidate
// adds the chunks in order (deterministic), solves every trial frequency and
// keeps the best one of row hrow (ties to the lower index).
#include <cmath>
#include <cstdint>

#include "fchi2_internal.h"
#include "launch.h"
#include "solve_bin.h"

namespace fchi2 {

namespace {

using namespace solve_detail;

constexpr int kNT = 256;
constexpr int kChunk = 1024;  // points per block of phase 1

// Trial frequency r of a candidate centred on fc with half-width hw.
__device__ __forceinline__ double fine_freq(double fc, double hw, int r, int R) {
  return R > 1 ? fc + hw * (2.0 * (double)r / (double)(R - 1) - 1.0) : fc;
}

template <int H>
__global__ __launch_bounds__(kNT) void k_fine_sums(const double* __restrict__ t,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ sigma,
                                                   const Moments* __restrict__ mom,
                                                   const double* __restrict__ fc, int K, int R,
                                                   double hw, int n_chunks,
                                                   double* __restrict__ part) {
  constexpr int NC = 6 * H;  // Re/Im of Q_1..Q_2H and P_1..P_H
  __shared__ double s_tau[kNT], s_w[kNT], s_wy[kNT];
  const int tid = threadIdx.x;
  const int c = blockIdx.z;
  const int chunk = blockIdx.y;
  const int KR = K * R;
  const int q = blockIdx.x * kNT + tid;
  const Moments mo = mom[c];
  const int64_t p0 = (int64_t)chunk * kChunk;
  if (p0 >= mo.n && chunk > 0) return;  // this curve has no such chunk
  const int64_t p1 = (p0 + kChunk < mo.n) ? p0 + kChunk : mo.n;

  double f = 0.0;
  bool active = q < KR && !(mo.flags & kCurveFatal);
  if (active) {
    f = fine_freq(fc[(int64_t)c * K + q / R], hw, q % R, R);
    active = f > 0.0 && isfinite(f);
  }
  double acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = 0.0;

  for (int64_t b = p0; b < p1; b += kNT) {
    const int64_t i = b + tid;
    if (i < p1) {
      const int64_t gi = mo.start + i;
      const double s = sigma[gi];
      const double w = 1.0 / (s * s);
      s_tau[tid] = t[gi] - mo.T0;
      s_w[tid] = w;
      s_wy[tid] = w * (x[gi] - mo.xbar);
    }
    __syncthreads();
    const int m = (p1 - b) < kNT ? (int)(p1 - b) : kNT;
    if (active) {
      for (int j = 0; j < m; ++j) {
        const double cyc = f * s_tau[j];
        const double fr = cyc - floor(cyc);
        double sn, cs;
        sincospi(2.0 * fr, &sn, &cs);
        const double w = s_w[j], wy = s_wy[j];
        double zr = cs, zi = sn;
        static_for<1, 2 * H + 1>([&](auto mc) {
          constexpr int mm = decltype(mc)::value;
          if constexpr (mm > 1) {
            const double nr = zr * cs - zi * sn;
            const double ni = zr * sn + zi * cs;
            zr = nr;
            zi = ni;
          }
          acc[2 * (mm - 1)] += w * zr;
          acc[2 * (mm - 1) + 1] += w * zi;
          if constexpr (mm <= H) {
            acc[4 * H + 2 * (mm - 1)] += wy * zr;
            acc[4 * H + 2 * (mm - 1) + 1] += wy * zi;
          }
        });
      }
    }
    __syncthreads();
  }
  if (q < KR) {
    double* o = part + ((int64_t)c * n_chunks + chunk) * NC * KR + q;
#pragma unroll
    for (int j = 0; j < NC; ++j) o[(int64_t)j * KR] = acc[j];
  }
}

// Spectra of trial frequency q of curve c: chunk partial sums added in order.
template <int H>
__device__ __forceinline__ void fine_spectra(const double* __restrict__ part, int64_t c,
                                             int n_chunks, int used, int KR, int q, double W,
                                             double* Qr, double* Qi, double* Pr, double* Pi) {
  constexpr int NC = 6 * H;
  double acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = 0.0;
  for (int ch = 0; ch < used; ++ch) {
    const double* p = part + (c * n_chunks + ch) * NC * KR + q;
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j] += p[(int64_t)j * KR];
  }
  Qr[0] = W;
  Qi[0] = 0.0;
  Pr[0] = 0.0;
  Pi[0] = 0.0;
#pragma unroll
  for (int m = 1; m <= 2 * H; ++m) {
    Qr[m] = acc[2 * (m - 1)];
    Qi[m] = acc[2 * (m - 1) + 1];
  }
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    Pr[m] = acc[4 * H + 2 * (m - 1)];
    Pi[m] = acc[4 * H + 2 * (m - 1) + 1];
  }
}

template <int H>
__global__ __launch_bounds__(kNT) void k_fine_solve(
    const Moments* __restrict__ mom, const double* __restrict__ fc, int K, int R, double hw,
    int n_chunks, const double* __restrict__ part, int hrow, double* __restrict__ out_rows,
    double* __restrict__ out_f, double* __restrict__ out_d, double* __restrict__ out_coef,
    uint8_t* __restrict__ out_flags) {
  constexpr int dd = 2 * H + 1;
  constexpr double kEps = 1e-13;
  __shared__ double r_v[kNT];
  __shared__ int r_i[kNT];
  const int tid = threadIdx.x;
  const int cand = blockIdx.x;
  const int c = blockIdx.y;
  const int KR = K * R;
  const Moments mo = mom[c];
  const bool fatal = (mo.flags & kCurveFatal) != 0;
  const int used = fatal ? 0 : (int)((mo.n + kChunk - 1) / kChunk);
  const double fcen = fc[(int64_t)c * K + cand];
  const bool cand_ok = !fatal && fcen > 0.0 && isfinite(fcen);
  const int64_t o = (int64_t)c * K + cand;

  double bv = -INFINITY;
  int bi = -1;
  for (int r = tid; r < R; r += kNT) {
    const double f = fine_freq(fcen, hw, r, R);
    double d[H];
    if (cand_ok && f > 0.0 && isfinite(f)) {
      double Qr[2 * H + 1], Qi[2 * H + 1], Pr[H + 1], Pi[H + 1];
      fine_spectra<H>(part, c, n_chunks, used, KR, cand * R + r, mo.W, Qr, Qi, Pr, Pi);
      uint8_t fl = 0;
      double Lm[dd][dd], inv[dd], z[dd];
      prefix_solve<H, double>(Qr, Qi, Pr, Pi, kEps, d, fl, Lm, inv, z);
    } else {
#pragma unroll
      for (int h = 0; h < H; ++h) d[h] = (double)NAN;
    }
    if (out_rows) {
      double* orow = out_rows + (((int64_t)c * K + cand) * R + r) * H;
#pragma unroll
      for (int h = 0; h < H; ++h) orow[h] = d[h];
    }
    double v = (double)NAN;
#pragma unroll
    for (int h = 0; h < H; ++h)
      if (h == hrow) v = d[h];
    if (v > bv) {  // r increases within a thread, so ties keep the lower r
      bv = v;
      bi = r;
    }
  }
  r_v[tid] = bv;
  r_i[tid] = bi;
  __syncthreads();
  for (int s = kNT / 2; s > 0; s >>= 1) {
    if (tid < s) {
      const double ov = r_v[tid + s];
      const int oi = r_i[tid + s];
      if (oi >= 0 && (r_i[tid] < 0 || ov > r_v[tid] || (ov == r_v[tid] && oi < r_i[tid]))) {
        r_v[tid] = ov;
        r_i[tid] = oi;
      }
    }
    __syncthreads();
  }
  if (tid != 0) return;
  const int win = r_i[0];
  if (win < 0) {
    out_f[o] = (double)NAN;
    for (int h = 0; h < H; ++h) out_d[o * H + h] = (double)NAN;
    if (out_coef)
      for (int j = 0; j < dd; ++j) out_coef[o * dd + j] = (double)NAN;
    if (out_flags) out_flags[o] = (uint8_t)(mo.flags & 0xF8u);
    return;
  }
  // The winner again, now with the coefficients: L^T A = z, a dropped pivot
  // leaving its A at 0; xbar added back to A_0.
  const double f = fine_freq(fcen, hw, win, R);
  double Qr[2 * H + 1], Qi[2 * H + 1], Pr[H + 1], Pi[H + 1];
  fine_spectra<H>(part, c, n_chunks, used, KR, cand * R + win, mo.W, Qr, Qi, Pr, Pi);
  uint8_t fl = 0;
  if (mo.span > 0.0 && f * mo.span < 1.0) fl |= BF_LOW_F;
  double d[H];
  double Lm[dd][dd], inv[dd], z[dd], A[dd];
  prefix_solve<H, double>(Qr, Qi, Pr, Pi, kEps, d, fl, Lm, inv, z);
  out_f[o] = f;
#pragma unroll
  for (int h = 0; h < H; ++h) out_d[o * H + h] = d[h];
  if (out_flags) out_flags[o] = fl;
  if (out_coef) {
    static_for<0, dd>([&](auto ic) {
      constexpr int i = dd - 1 - decltype(ic)::value;
      double s = z[i];
      static_for<i + 1, dd>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        s -= Lm[l][i] * A[l];
      });
      A[i] = s * inv[i];
    });
    A[0] += mo.xbar;
#pragma unroll
    for (int j = 0; j < dd; ++j) out_coef[o * dd + j] = A[j];
  }
}

template <int H>
hipError_t fine_h(const double* t, const double* x, const double* sigma, const Moments* mom,
                  int n_curves, const double* fc, int K, int R, double hw, int n_chunks,
                  double* part, int hrow, const FineOut& out, hipStream_t st) {
  dim3 g1((unsigned)((K * R + kNT - 1) / kNT), (unsigned)n_chunks, (unsigned)n_curves);
  hipLaunchKernelGGL((k_fine_sums<H>), g1, dim3(kNT), 0, st, t, x, sigma, mom, fc, K, R, hw,
                     n_chunks, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 g2((unsigned)K, (unsigned)n_curves);
  hipLaunchKernelGGL((k_fine_solve<H>), g2, dim3(kNT), 0, st, mom, fc, K, R, hw, n_chunks,
                     (const double*)part, hrow, out.rows, out.f_best, out.dchi2_best, out.coef,
                     out.flags);
  return hipGetLastError();
}

}  // namespace

int fine_chunks(int64_t max_n) {
  const int64_t n = (max_n + kChunk - 1) / kChunk;
  return n > 0 ? (int)n : 1;
}

size_t fine_part_bytes(int H, int n_curves, int64_t max_n, int K, int R) {
  return (size_t)6 * H * sizeof(double) * (size_t)K * (size_t)R * (size_t)fine_chunks(max_n) *
         (size_t)n_curves;
}

hipError_t launch_fine(const double* t, const double* x, const double* sigma, const Moments* mom,
                       int H, int n_curves, int64_t max_n, const double* fc, int K, int R,
                       double hw, double* part, int hrow, const FineOut& out, hipStream_t st) {
  const int nch = fine_chunks(max_n);
  switch (H) {
#define FCHI2_FINE_CASE(h) \
  case h: return fine_h<h>(t, x, sigma, mom, n_curves, fc, K, R, hw, nch, part, hrow, out, st);
    FCHI2_FINE_CASE(1)
    FCHI2_FINE_CASE(2)
    FCHI2_FINE_CASE(3)
    FCHI2_FINE_CASE(4)
    FCHI2_FINE_CASE(5)
    FCHI2_FINE_CASE(6)
    FCHI2_FINE_CASE(7)
    FCHI2_FINE_CASE(8)
#undef FCHI2_FINE_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fchi2
