// Internal definitions shared by the F-chi2 HIP kernels and the host layer.
// Not part of the public C ABI (that is include/fchi2.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace fchi2 {

constexpr int kHMax = 8;            // harmonics supported by the register solver
constexpr int kHWide = 16;          // harmonics supported by the wave-per-bin solver
constexpr int kMaxPairs = 24;       // 3 * kHMax (band plans: one grid per harmonic),
                                    // = kHWide + kHWide / 2 packed pairs
constexpr int kMaxPasses = 4;       // FFT passes (digits of the grid length)
constexpr int kStageLog = 13;       // stage twiddle table is omega_{2^13}

// Per-curve scalars produced by the moments kernel (FP64).
struct Moments {
  double W;       // sum of weights w = sigma^-2
  double xbar;    // weighted mean
  double chi2_0;  // chi2 of the constant model
  double T0;      // epoch: first (smallest) time
  double span;    // last minus first time
  int64_t start;  // CSR offset of the curve (of its t and sigma)
  int64_t n;      // number of points
  int64_t xshift; // x of point i is x[i + xshift] (nonzero for sources sharing t)
  uint32_t flags; // CF_* bits
  uint32_t pad;
};

// Partial moments of one chunk of a curve.
struct MomPart {
  double W;       // sum of weights
  double mean;    // weighted mean of the chunk
  double M2;      // sum w (x - mean)^2 over the chunk
  uint32_t bad;   // CF_* validity bits seen in the chunk
  uint32_t pad;
};

// Curve flags (also reported in the curve's first output flag byte).
enum : uint32_t {
  CF_NONFINITE = 1u << 3,  // a non-finite t, x or sigma, or sigma <= 0
  CF_UNSORTED = 1u << 4,   // t not ascending
  CF_WRAP = 1u << 5,       // 2H * df * span spans more grid periods than the plan covers
  CF_FEW = 1u << 6,        // fewer points than 2H+1 (pivots get dropped)
  CF_EMPTY = 1u << 7,      // no points
};
constexpr uint32_t kCurveFatal = CF_NONFINITE | CF_UNSORTED | CF_WRAP | CF_EMPTY;

// Bin flags.
enum : uint8_t { BF_PIVOT = 1, BF_LOW_F = 2, BF_DC = 4 };

// Compile-time loop: f(std::integral_constant<int, I>) for I = B..E-1, so
// every register-array index in the body is a constant (no scratch memory).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <typename R>
struct cplx {
  R x, y;
};

template <typename R>
__host__ __device__ inline cplx<R> cmk(R a, R b) {
  cplx<R> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename R>
__host__ __device__ inline cplx<R> cadd(cplx<R> a, cplx<R> b) {
  return cmk<R>(a.x + b.x, a.y + b.y);
}
template <typename R>
__host__ __device__ inline cplx<R> csub(cplx<R> a, cplx<R> b) {
  return cmk<R>(a.x - b.x, a.y - b.y);
}
template <typename R>
__host__ __device__ inline cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return cmk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Grid geometry and spreading kernel shared by spread, FFT, solve and gather.
struct Geom {
  int64_t L;        // complex grid length (cells): 4 n_freq (2 n_freq in a band plan)
  int64_t n_freq;   // trial bins per curve
  double df;        // bin spacing (cycles per unit time)
  double beta;      // exponential-of-semicircle kernel shape
  double half_w;    // w / 2
  int w;            // kernel width (taps)
  int c_off;        // grid origin shift (cells) so that no tap wraps
  int H;            // harmonics
  int P;            // packed complex grids per curve
  int chunk;        // extents are rounded up to a multiple of this
  int band;         // 1: band plan (first bin k0 > 0, one complex grid per harmonic,
                    //    centred on bin k0 + n_freq / 2)
  int64_t k0;       // first bin of the band (0 for the ordinary search)
  int laps;         // grid periods the tile tables cover: positions m u L + c_off
                    // up to laps * L (curves reaching further are flagged)
  // For pair p, component j (0 = real part, 1 = imaginary part):
  // harmonic multiple m (0 = unused) and strength kind (0: w, 1: w*(x-xbar)).
  int8_t comp_m[kMaxPairs][2];
  int8_t comp_kind[kMaxPairs][2];
};

// Cell extent [0, E) of the nonzero part of pair p of a curve (rounded up).
__host__ __device__ inline int64_t pair_extent(const Moments& mo, const Geom& g, int p) {
  int m = g.comp_m[p][0] > g.comp_m[p][1] ? g.comp_m[p][0] : g.comp_m[p][1];
  double v = mo.span * g.df;                 // same expression as the positions
  double pos = ((double)m * v) * (double)g.L + (double)g.c_off;
  int64_t e = (int64_t)pos + (int64_t)(g.w / 2) + 3;
  int64_t c = g.chunk;
  e = ((e + c - 1) / c) * c;
  if (e > g.L) e = g.L;
  return e;
}

// One FFT pass of the multi-pass decimation-in-time scheme (see fft kernel).
enum PassKind : int { PASS_FIRST = 0, PASS_MID = 1, PASS_LAST = 2, PASS_SINGLE = 3 };
enum PassMode : int { MODE_FWD = 0, MODE_BWD = 1 };

struct FftPlan {
  int np;                       // number of passes
  int logn[kMaxPasses + 1];     // logn[q] = log2 N_q, digit q = 1 (least significant)..np
  int le[kMaxPasses + 1];       // log2 of pass q's tile (N_q rows x 2^(le - logn) columns)
  int logL;
};

}  // namespace fchi2
