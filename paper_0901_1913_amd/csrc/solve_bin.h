// Per-bin normal equations and the prefix Cholesky solve, shared by the
// kernel that writes every Delta chi2 row and the one that keeps only the
// best candidates of each curve.
//
// For bin k the packed spectra give Q_m = Q(m f_k) (m = 1..2H) and
// P_m = P(m f_k) (m = 1..H).  The normal matrix alpha and right-hand side beta
// follow from the product-to-sum identities of Section 2 (equations
// eqalphafirst..eqalpha and the beta terms), with C'(g) = Re Q(g f),
// S'(g) = Im Q(g f), C'(-g) = C'(g), S'(-g) = -S'(g), Q(0) = W (the exact FP64
// sum of weights) and beta_0 = Re P(0) = 0 after centring (Section 3b).
// The basis order [1, sin f, cos f, ..., sin Hf, cos Hf] makes the H' model a
// prefix of the H model, so one Cholesky factor alpha = L L^T and
// z = L^-1 beta give Delta chi2(H') = sum_{j <= 2H'} z_j^2 for all H' at once
// (eq. eqchix with chi2_0 - chi2_min = beta^T alpha^-1 beta, Section 3d).
// A pivot below eps * alpha_jj is dropped (its direction adds nothing), which
// gives least-squares semantics for rank-deficient bins; the bin is flagged.
#pragma once

#include <cmath>

#include "fchi2_internal.h"

namespace fchi2 {
namespace solve_detail {

// Pair layout: pair p < H packs the weight grids (q_{2p+1}, q_{2p+2}); pair
// p >= H packs the weighted-data grids (p_{2j+1}, p_{2j+2}), j = p - H, the
// second part empty past H.
template <int H>
struct Layout {
  static constexpr int P = H + (H + 1) / 2;
};

// Unpack pair spectra at bin k into Qr/Qi (m = 0..2H) and Pr/Pi (m = 0..H),
// already multiplied by the deconvolution / origin-shift factor D[k].
template <int H, typename R>
__device__ __forceinline__ void load_spectra(const cplx<R>* __restrict__ zc, int64_t nf,
                                             int64_t base_pair, int64_t k, cplx<double> Dk_,
                                             double W, double* Qr, double* Qi, double* Pr,
                                             double* Pi) {
  constexpr int P = Layout<H>::P;
  const double Dr = (double)Dk_.x, Di = (double)Dk_.y;
  Qr[0] = W;
  Qi[0] = 0.0;
  Pr[0] = 0.0;
  Pi[0] = 0.0;
#pragma unroll
  for (int pp = 0; pp < P; ++pp) {
    const cplx<R> z0 = zc[((base_pair + pp) * 2 + 0) * nf + k];
    const cplx<R> z1 = zc[((base_pair + pp) * 2 + 1) * nf + k];
    const double ax = 0.5 * ((double)z0.x + (double)z1.x);
    const double ay = 0.5 * ((double)z0.y - (double)z1.y);
    const double bx = 0.5 * ((double)z0.y + (double)z1.y);
    const double by = -0.5 * ((double)z0.x - (double)z1.x);
    const double Ar = ax * Dr - ay * Di, Ai = ax * Di + ay * Dr;
    const double Br = bx * Dr - by * Di, Bi = bx * Di + by * Dr;
    if (pp < H) {
      Qr[2 * pp + 1] = Ar;
      Qi[2 * pp + 1] = Ai;
      Qr[2 * pp + 2] = Br;
      Qi[2 * pp + 2] = Bi;
    } else {
      const int j = pp - H;
      Pr[2 * j + 1] = Ar;
      Pi[2 * j + 1] = Ai;
      if (2 * j + 2 <= H) {
        Pr[2 * j + 2] = Br;
        Pi[2 * j + 2] = Bi;
      }
    }
  }
}

// Band plans: grid p holds one harmonic with complex (modulated) strengths,
// q_{p+1} for p < 2H and p_{p-2H+1} after, centred on the band's middle bin:
// band bin k is offset o = k - n_freq/2 from the centre, read from the direct
// half at o >= 0 (grid bin o) and from the mirror half at -o otherwise (grid
// bin L + o), times the deconvolution factor of o (D[-o] conjugated: the
// kernel transform is even and the origin-shift phase odd in o).
template <int H, typename R>
__device__ __forceinline__ void load_band(const cplx<R>* __restrict__ zc,
                                          const cplx<double>* __restrict__ D, int64_t nf,
                                          int64_t base_grid, int64_t k, double W, double* Qr,
                                          double* Qi, double* Pr, double* Pi) {
  const int64_t o = k - nf / 2;
  const bool neg = o < 0;
  const int64_t j = neg ? -o : o;
  const int64_t half = neg ? 1 : 0;
  const cplx<double> Dj = D[j];
  const double Dr = Dj.x, Di = neg ? -Dj.y : Dj.y;
  Qr[0] = W;
  Qi[0] = 0.0;
  Pr[0] = 0.0;
  Pi[0] = 0.0;
#pragma unroll
  for (int m = 1; m <= 2 * H; ++m) {
    const cplx<R> z = zc[((base_grid + m - 1) * 2 + half) * nf + j];
    Qr[m] = (double)z.x * Dr - (double)z.y * Di;
    Qi[m] = (double)z.x * Di + (double)z.y * Dr;
  }
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    const cplx<R> z = zc[((base_grid + 2 * H + m - 1) * 2 + half) * nf + j];
    Pr[m] = (double)z.x * Dr - (double)z.y * Di;
    Pi[m] = (double)z.x * Di + (double)z.y * Dr;
  }
}

__device__ __forceinline__ double Cp(const double* Qr, int gdiff) {
  return Qr[gdiff < 0 ? -gdiff : gdiff];
}
__device__ __forceinline__ double Sp(const double* Qi, int gdiff) {
  return gdiff < 0 ? -Qi[-gdiff] : Qi[gdiff];
}

// alpha_{ij} for basis indices i >= j (0 = constant, 2h-1 = sin h, 2h = cos h).
__device__ __forceinline__ double alpha_ij(int i, int j, const double* Qr, const double* Qi) {
  if (j == 0) {
    if (i == 0) return Qr[0];
    const int h = (i + 1) >> 1;
    return (i & 1) ? Qi[h] : Qr[h];
  }
  const int h = (i + 1) >> 1, hp = (j + 1) >> 1;
  const bool si = (i & 1), sj = (j & 1);
  if (si && sj) return 0.5 * (Cp(Qr, h - hp) - Cp(Qr, h + hp));
  if (si && !sj) return 0.5 * (Sp(Qi, h + hp) + Sp(Qi, h - hp));
  if (!si && sj) return 0.5 * (Sp(Qi, h + hp) - Sp(Qi, h - hp));
  return 0.5 * (Cp(Qr, h - hp) + Cp(Qr, h + hp));
}

__device__ __forceinline__ double beta_i(int i, const double* Pr, const double* Pi) {
  if (i == 0) return 0.0;
  const int h = (i + 1) >> 1;
  return (i & 1) ? Pi[h] : Pr[h];
}

template <typename O>
__device__ __forceinline__ O nan_of() {
  return (O)NAN;
}


// Prefix Cholesky solve of one bin from its assembled spectra: alpha = L L^T,
// z = L^-1 beta, d[H'-1] = sum_{j <= 2H'} z_j^2 (rounded to O).  Dropped
// pivots set inv[j] = 0 and the PIVOT flag.  L, inv and z are left for a
// caller that also wants the coefficients (L^T A = z).
template <int H, typename O>
__device__ __forceinline__ void prefix_solve(const double* Qr, const double* Qi,
                                             const double* Pr, const double* Pi, double eps,
                                             O* d, uint8_t& fl, double (&Lm)[2 * H + 1][2 * H + 1],
                                             double (&inv)[2 * H + 1], double (&z)[2 * H + 1]) {
  constexpr int dd = 2 * H + 1;
  double acc = 0.0;
  static_for<0, dd>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    static_for<0, i + 1>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      double s = alpha_ij(i, j, Qr, Qi);
      static_for<0, j>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        s -= Lm[i][l] * Lm[j][l];
      });
      if constexpr (i == j) {
        const double ajj = alpha_ij(i, i, Qr, Qi);
        if (s > eps * ajj && s > 0.0) {
          // only 1/L_ii enters the solve: one reciprocal square root
          inv[i] = rsqrt(s);
          Lm[i][i] = s * inv[i];
        } else {
          Lm[i][i] = 0.0;
          inv[i] = 0.0;
          fl |= BF_PIVOT;
        }
      } else {
        Lm[i][j] = s * inv[j];
      }
    });
    double s = beta_i(i, Pr, Pi);
    static_for<0, i>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      s -= Lm[i][l] * z[l];
    });
    z[i] = s * inv[i];
    acc += z[i] * z[i];
    if constexpr (i >= 2 && (i & 1) == 0) d[i / 2 - 1] = (O)acc;
  });
}

// Shared-alpha form (many sources observed at the same times with errors
// proportional to one sigma, Section 5): alpha depends on the times and the
// shared weights only, so it is factored once per bin and reused for every
// source's beta.  factor_alpha computes L (alpha = L L^T) with the pivot guard;
// solve_beta then gives Delta chi2(H') = sum_{j <= 2H'} z_j^2 * inv_scale2.
template <int H>
__device__ __forceinline__ void factor_alpha(const double* Qr, const double* Qi, double eps,
                                             uint8_t& fl, double (&Lm)[2 * H + 1][2 * H + 1],
                                             double (&inv)[2 * H + 1]) {
  constexpr int dd = 2 * H + 1;
  static_for<0, dd>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    static_for<0, i + 1>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      double s = alpha_ij(i, j, Qr, Qi);
      static_for<0, j>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        s -= Lm[i][l] * Lm[j][l];
      });
      if constexpr (i == j) {
        const double ajj = alpha_ij(i, i, Qr, Qi);
        if (s > eps * ajj && s > 0.0) {
          // only 1/L_ii enters the solve: one reciprocal square root
          inv[i] = rsqrt(s);
          Lm[i][i] = s * inv[i];
        } else {
          Lm[i][i] = 0.0;
          inv[i] = 0.0;
          fl |= BF_PIVOT;
        }
      } else {
        Lm[i][j] = s * inv[j];
      }
    });
  });
}

template <int H, typename O>
__device__ __forceinline__ void solve_beta(const double (&Lm)[2 * H + 1][2 * H + 1],
                                           const double (&inv)[2 * H + 1], const double* Pr,
                                           const double* Pi, double inv_scale2, O* d) {
  constexpr int dd = 2 * H + 1;
  double z[dd];
  double acc = 0.0;
  static_for<0, dd>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    double s = beta_i(i, Pr, Pi);
    static_for<0, i>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      s -= Lm[i][l] * z[l];
    });
    z[i] = s * inv[i];
    acc += z[i] * z[i];
    if constexpr (i >= 2 && (i & 1) == 0) d[i / 2 - 1] = (O)(acc * inv_scale2);
  });
}

// Unpack the weight pairs (q_{2p+1}, q_{2p+2}), p < H, of one grid slot.
template <int H, typename R>
__device__ __forceinline__ void load_q(const cplx<R>* __restrict__ zc, int64_t nf,
                                       int64_t base_pair, int64_t k, cplx<double> Dk_, double W,
                                       double* Qr, double* Qi) {
  const double Dr = (double)Dk_.x, Di = (double)Dk_.y;
  Qr[0] = W;
  Qi[0] = 0.0;
#pragma unroll
  for (int pp = 0; pp < H; ++pp) {
    const cplx<R> z0 = zc[((base_pair + pp) * 2 + 0) * nf + k];
    const cplx<R> z1 = zc[((base_pair + pp) * 2 + 1) * nf + k];
    const double ax = 0.5 * ((double)z0.x + (double)z1.x);
    const double ay = 0.5 * ((double)z0.y - (double)z1.y);
    const double bx = 0.5 * ((double)z0.y + (double)z1.y);
    const double by = -0.5 * ((double)z0.x - (double)z1.x);
    Qr[2 * pp + 1] = ax * Dr - ay * Di;
    Qi[2 * pp + 1] = ax * Di + ay * Dr;
    Qr[2 * pp + 2] = bx * Dr - by * Di;
    Qi[2 * pp + 2] = bx * Di + by * Dr;
  }
}

// Unpack the data pairs (p_{2j+1}, p_{2j+2}), j < ceil(H/2), of one grid slot.
template <int H, typename R>
__device__ __forceinline__ void load_p(const cplx<R>* __restrict__ zc, int64_t nf,
                                       int64_t base_pair, int64_t k, cplx<double> Dk_,
                                       double* Pr, double* Pi) {
  const double Dr = (double)Dk_.x, Di = (double)Dk_.y;
  Pr[0] = 0.0;
  Pi[0] = 0.0;
#pragma unroll
  for (int j = 0; j < (H + 1) / 2; ++j) {
    const cplx<R> z0 = zc[((base_pair + j) * 2 + 0) * nf + k];
    const cplx<R> z1 = zc[((base_pair + j) * 2 + 1) * nf + k];
    const double ax = 0.5 * ((double)z0.x + (double)z1.x);
    const double ay = 0.5 * ((double)z0.y - (double)z1.y);
    const double bx = 0.5 * ((double)z0.y + (double)z1.y);
    const double by = -0.5 * ((double)z0.x - (double)z1.x);
    Pr[2 * j + 1] = ax * Dr - ay * Di;
    Pi[2 * j + 1] = ax * Di + ay * Dr;
    if (2 * j + 2 <= H) {
      Pr[2 * j + 2] = bx * Dr - by * Di;
      Pi[2 * j + 2] = bx * Di + by * Dr;
    }
  }
}

// Delta chi2 of bin k of curve c (wave slot cw) for H' = 1..H, rounded to the
// output type, into d[0..H-1]; returns the bin's flags.  Curves with a fatal
// data flag give NaN rows; bin 0 gives zero rows and the DC flag.  BAND: a
// band plan's grids (bin k is bin k0 + k of the search).  COEF: also the
// coefficients of the H-harmonic model into A[0..2H] (eq. eqcoeffs,
// A = alpha^-1 beta by back substitution L^T A = z, basis [1, sin, cos, ...]
// in tau = t - T0), with the weighted mean added back to A_0 (Section 3b's
// centring); a dropped pivot's coefficient is 0; bin 0 gives A_0 = xbar and
// zeros; a rejected curve gives NaN.
template <int H, typename R, typename O, bool BAND = false, bool COEF = false>
__device__ __forceinline__ uint8_t solve_bin(const cplx<R>* __restrict__ zc,
                                             const cplx<double>* __restrict__ D,
                                             const Moments& mo, const Geom& g, int cw, int64_t k,
                                             double eps, O* d, double* A = nullptr) {
  constexpr int dd = 2 * H + 1;
  constexpr int P = Layout<H>::P;
  if (mo.flags & kCurveFatal) {
#pragma unroll
    for (int h = 0; h < H; ++h) d[h] = nan_of<O>();
    if constexpr (COEF) {
#pragma unroll
      for (int j = 0; j < dd; ++j) A[j] = (double)NAN;
    }
    return (uint8_t)(mo.flags & 0xF8u);
  }
  uint8_t fl = 0;
  const int64_t kg = BAND ? g.k0 + k : k;  // bin of the search
  const double f = (double)kg * g.df;
  if (mo.span > 0.0 && f * mo.span < 1.0) fl |= BF_LOW_F;
  if (kg == 0) {
#pragma unroll
    for (int h = 0; h < H; ++h) d[h] = (O)0;
    if constexpr (COEF) {
      A[0] = mo.xbar;
#pragma unroll
      for (int j = 1; j < dd; ++j) A[j] = 0.0;
    }
    return (uint8_t)(fl | BF_DC);
  }
  double Qr[2 * H + 1], Qi[2 * H + 1], Pr[H + 1], Pi[H + 1];
  if constexpr (BAND)
    load_band<H, R>(zc, D, g.n_freq, (int64_t)cw * g.P, k, mo.W, Qr, Qi, Pr, Pi);
  else
    load_spectra<H, R>(zc, g.n_freq, (int64_t)cw * P, k, D[k], mo.W, Qr, Qi, Pr, Pi);
  double Lm[dd][dd];
  double inv[dd];
  double z[dd];
  prefix_solve<H, O>(Qr, Qi, Pr, Pi, eps, d, fl, Lm, inv, z);
  if constexpr (COEF) {
    static_for<0, dd>([&](auto rc) {
      constexpr int ii = dd - 1 - decltype(rc)::value;
      double sacc = z[ii];
      static_for<ii + 1, dd>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        sacc -= Lm[l][ii] * A[l];
      });
      A[ii] = sacc * inv[ii];
    });
    A[0] += mo.xbar;
  }
  return fl;
}

}  // namespace solve_detail
}  // namespace fchi2
