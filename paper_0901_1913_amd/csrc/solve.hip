// Per-frequency Delta chi2 for every H' = 1..H: one thread per bin runs the
// shared per-bin solve and writes all H rows and the bin's flags.
#include <cmath>
#include <type_traits>

#include "fchi2_internal.h"
#include "launch.h"
#include "solve_bin.h"

namespace fchi2 {

namespace {

constexpr int kNT = 256;

using namespace solve_detail;

template <int H, typename R, typename O, bool BAND, bool COEF>
__global__ __launch_bounds__(kNT) void k_solve(const cplx<R>* __restrict__ zc,
                                               const cplx<double>* __restrict__ D,
                                               const Moments* __restrict__ mom, Geom g,
                                               int curve0, double eps, O* __restrict__ out,
                                               uint8_t* __restrict__ flags,
                                               O* __restrict__ coef) {
  const int64_t nf = g.n_freq;
  const int64_t k = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const int cw = blockIdx.y;
  const int c = curve0 + cw;
  if (k >= nf) return;
  const Moments mo = mom[c];
  O d[H];
  double A[COEF ? 2 * H + 1 : 1];
  const uint8_t fl = solve_bin<H, R, O, BAND, COEF>(zc, D, mo, g, cw, k, eps, d, A);
  O* o = out + (int64_t)c * H * nf + k;
#pragma unroll
  for (int h = 0; h < H; ++h) o[h * nf] = d[h];
  if (flags) flags[(int64_t)c * nf + k] = fl;
  if constexpr (COEF) {
    O* oc = coef + (int64_t)c * (2 * H + 1) * nf + k;
#pragma unroll
    for (int j = 0; j < 2 * H + 1; ++j) oc[j * nf] = (O)A[j];
  }
}

template <int H>
hipError_t solve_h(bool fp64, const void* zc, const void* D, const Moments* mom, const Geom& g,
                   int curve0, int n_curves, double eps, void* out, uint8_t* flags,
                   void* coef, hipStream_t st) {
  dim3 gr((unsigned)((g.n_freq + kNT - 1) / kNT), (unsigned)n_curves);
  auto launch = [&](auto band, auto cf) {
    constexpr bool B = decltype(band)::value;
    constexpr bool CF = decltype(cf)::value;
    if (fp64)
      hipLaunchKernelGGL((k_solve<H, double, double, B, CF>), gr, dim3(kNT), 0, st,
                         (const cplx<double>*)zc, (const cplx<double>*)D, mom, g, curve0, eps,
                         (double*)out, flags, (double*)coef);
    else
      hipLaunchKernelGGL((k_solve<H, float, float, B, CF>), gr, dim3(kNT), 0, st,
                         (const cplx<float>*)zc, (const cplx<double>*)D, mom, g, curve0, eps,
                         (float*)out, flags, (float*)coef);
  };
  auto by_coef = [&](auto band) {
    if (coef)
      launch(band, std::true_type{});
    else
      launch(band, std::false_type{});
  };
  if (g.band)
    by_coef(std::true_type{});
  else
    by_coef(std::false_type{});
  return hipGetLastError();
}

// Shared-alpha solve for sources observed at the same times (Section 5):
// thread k factors alpha of bin k once from the shared weight spectra, then
// solves beta of every source of the wave and scales by 1/scale^2 (the
// source's weights are the shared ones divided by scale^2).
template <int H, typename R, typename O>
__global__ __launch_bounds__(kNT) void k_solve_multi(
    const cplx<R>* __restrict__ zq, const cplx<R>* __restrict__ zp,
    const cplx<double>* __restrict__ D, const Moments* __restrict__ mom_t,
    const Moments* __restrict__ mom_s, const double* __restrict__ scale, Geom g, int src0,
    int n_src, double eps, O* __restrict__ out, uint8_t* __restrict__ flags) {
  constexpr int dd = 2 * H + 1;
  constexpr int PD = (H + 1) / 2;
  const int64_t nf = g.n_freq;
  const int64_t k = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (k >= nf) return;
  const Moments mt = mom_t[0];
  uint8_t fl = 0;
  const double f = (double)k * g.df;
  if (mt.span > 0.0 && f * mt.span < 1.0) fl |= BF_LOW_F;
  const bool base_bad = (mt.flags & kCurveFatal) != 0;
  double Lm[dd][dd], inv[dd];
  if (!base_bad && k > 0) {
    double Qr[2 * H + 1], Qi[2 * H + 1];
    load_q<H, R>(zq, nf, 0, k, D[k], mt.W, Qr, Qi);
    factor_alpha<H>(Qr, Qi, eps, fl, Lm, inv);
  }
  if (k == 0) fl |= BF_DC;
  if (base_bad) fl = (uint8_t)(mt.flags & 0xF8u);
  if (flags && src0 == 0) flags[k] = fl;
  const cplx<double> Dk = D[k];
  for (int sw = 0; sw < n_src; ++sw) {
    const int s = src0 + sw;
    const Moments ms = mom_s[s];
    O d[H];
    if (base_bad || (ms.flags & kCurveFatal)) {
#pragma unroll
      for (int h = 0; h < H; ++h) d[h] = nan_of<O>();
    } else if (k == 0) {
#pragma unroll
      for (int h = 0; h < H; ++h) d[h] = (O)0;
    } else {
      double Pr[H + 1], Pi[H + 1];
      load_p<H, R>(zp, nf, (int64_t)sw * PD, k, Dk, Pr, Pi);
      const double sc = scale[s];
      solve_beta<H, O>(Lm, inv, Pr, Pi, 1.0 / (sc * sc), d);
    }
    O* o = out + (int64_t)s * H * nf + k;
#pragma unroll
    for (int h = 0; h < H; ++h) o[h * nf] = d[h];
  }
}

// Wide solve for 9 <= H <= 16 (d = 2H + 1 <= 33 basis functions): the
// register solver's triangular factor would need d (d + 1) / 2 FP64 values per
// thread, so here one wave solves one bin with the matrix spread over its
// lanes, lane i holding row i of alpha.  Assembly (product-to-sum, Section 2),
// the pivot guard and the prefix sums are those of the register solver; the
// factorisation runs right-looking: at step j the pivot comes from lane j,
// every lane below scales its entry L_ij and updates its row with the L_kj
// of the lanes above it (shuffles), and the forward substitution z = L^-1 beta
// advances in the same step, so Delta chi2(H') = sum_{j <= 2H'} z_j^2 for
// every H' at once.  Coefficients (COEF) by back substitution L^T A = z, one
// wave reduction per unknown.  kNT / 64 bins per block.
constexpr int kDWide = 33;

template <typename R, typename O, bool COEF>
__global__ __launch_bounds__(kNT) void k_solve_wide(const cplx<R>* __restrict__ zc,
                                                    const cplx<double>* __restrict__ D,
                                                    const Moments* __restrict__ mom, Geom g,
                                                    int curve0, double eps, O* __restrict__ out,
                                                    uint8_t* __restrict__ flags,
                                                    O* __restrict__ coef) {
  const int H = g.H;
  const int dd = 2 * H + 1;
  const int P = g.P;
  const int64_t nf = g.n_freq;
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * (kNT / 64) + (threadIdx.x >> 6);
  const int cw = blockIdx.y;
  const int c = curve0 + cw;
  if (k >= nf) return;  // uniform per wave
  const Moments mo = mom[c];
  O* o = out + (int64_t)c * H * nf + k;
  O* oc = COEF ? coef + (int64_t)c * dd * nf + k : nullptr;
  if (mo.flags & kCurveFatal) {
    if (lane < H) o[lane * nf] = nan_of<O>();
    if (COEF && lane < dd) oc[lane * nf] = nan_of<O>();
    if (flags && lane == 0) flags[(int64_t)c * nf + k] = (uint8_t)(mo.flags & 0xF8u);
    return;
  }
  uint8_t fl = 0;
  const double f = (double)k * g.df;
  if (mo.span > 0.0 && f * mo.span < 1.0) fl |= BF_LOW_F;
  if (k == 0) {
    if (lane < H) o[lane * nf] = (O)0;
    if (COEF && lane < dd) oc[lane * nf] = (O)(lane == 0 ? mo.xbar : 0.0);
    if (flags && lane == 0) flags[(int64_t)c * nf + k] = (uint8_t)(fl | BF_DC);
    return;
  }
  // Lane m holds Q_m = Q(m f_k) for m <= 2H (Q_0 = W) and P_m for m <= H
  // (P_0 = 0), unpacked from the pair spectra and deconvolved as in the
  // register solver.
  const cplx<double> Dk = D[k];
  double qr = 0.0, qi = 0.0, pr = 0.0, pi = 0.0;
  auto unpack = [&](int pair, int comp, double& re, double& im) {
    const cplx<R> z0 = zc[(((int64_t)cw * P + pair) * 2 + 0) * nf + k];
    const cplx<R> z1 = zc[(((int64_t)cw * P + pair) * 2 + 1) * nf + k];
    double ax, ay;
    if (comp == 0) {
      ax = 0.5 * ((double)z0.x + (double)z1.x);
      ay = 0.5 * ((double)z0.y - (double)z1.y);
    } else {
      ax = 0.5 * ((double)z0.y + (double)z1.y);
      ay = -0.5 * ((double)z0.x - (double)z1.x);
    }
    re = ax * Dk.x - ay * Dk.y;
    im = ax * Dk.y + ay * Dk.x;
  };
  if (lane == 0) {
    qr = mo.W;
  } else if (lane <= 2 * H) {
    unpack((lane - 1) >> 1, (lane - 1) & 1, qr, qi);
  }
  if (lane >= 1 && lane <= H) unpack(H + ((lane - 1) >> 1), (lane - 1) & 1, pr, pi);
  auto Cp = [&](int gd) { return __shfl(qr, gd < 0 ? -gd : gd); };
  auto Sp = [&](int gd) {
    const double v = __shfl(qi, gd < 0 ? -gd : gd);
    return gd < 0 ? -v : v;
  };
  // Row `lane` of alpha (entries j <= lane), its original diagonal and beta.
  const int i = lane;
  const int hi_ = (i + 1) >> 1;
  const bool si = (i & 1);
  double a[kDWide];
  double diag = 0.0;
#pragma unroll
  for (int j = 0; j < kDWide; ++j) {
    double v = 0.0;
    if (j < dd) {
      const int hj = (j + 1) >> 1;
      const bool sj = (j & 1);
      // every lane takes part in the shuffles; only rows i >= j keep a value
      const double cm = Cp(hi_ - hj), cpl = Cp(hi_ + hj);
      const double sm_ = Sp(hi_ - hj), spl = Sp(hi_ + hj);
      const double q0r = __shfl(qr, hi_), q0i = __shfl(qi, hi_);
      if (j == 0) {
        v = (i == 0) ? mo.W : (si ? q0i : q0r);
      } else if (si && sj) {
        v = 0.5 * (cm - cpl);
      } else if (si && !sj) {
        v = 0.5 * (spl + sm_);
      } else if (!si && sj) {
        v = 0.5 * (spl - sm_);
      } else {
        v = 0.5 * (cm + cpl);
      }
      if (j > i || i >= dd) v = 0.0;
      if (j == i) diag = v;
    }
    a[j] = v;
  }
  const double bpi = __shfl(pi, hi_), bpr = __shfl(pr, hi_);
  double b = (i == 0 || i >= dd) ? 0.0 : (si ? bpi : bpr);
  // Right-looking factorisation with the forward substitution alongside.
  double inv_own = 0.0, acc = 0.0, dout = 0.0;
  double zall[kDWide];
#pragma unroll
  for (int j = 0; j < kDWide; ++j) {
    zall[j] = 0.0;
    if (j < dd) {
      const double piv = __shfl(a[j], j);
      const double ajj = __shfl(diag, j);
      double inv = 0.0;
      if (piv > eps * ajj && piv > 0.0) {
        inv = rsqrt(piv);
      } else {
        fl |= BF_PIVOT;
      }
      const double l = (i > j) ? a[j] * inv : (i == j ? piv * inv : 0.0);
      if (i >= j) a[j] = l;  // L_ij (L_jj on the diagonal)
      if (i == j) inv_own = inv;
      const double zj = __shfl(b, j) * inv;
      zall[j] = zj;
      if (i > j) b -= l * zj;
      acc += zj * zj;
      if (j >= 2 && (j & 1) == 0 && lane == j / 2 - 1) dout = acc;
#pragma unroll
      for (int kk = j + 1; kk < kDWide; ++kk) {
        if (kk < dd) {
          const double lkj = __shfl(l, kk);
          if (i >= kk) a[kk] -= l * lkj;
        }
      }
    }
  }
  if (lane < H) o[lane * nf] = (O)dout;
  if (flags && lane == 0) flags[(int64_t)c * nf + k] = fl;
  if constexpr (COEF) {
    // L^T A = z: A_j = (z_j - sum_{l > j} L_lj A_l) / L_jj, lane l holds L_lj.
    double Aown = 0.0;
#pragma unroll
    for (int jj = 0; jj < kDWide; ++jj) {
      const int j = kDWide - 1 - jj;
      if (j < dd) {
        double part = (i > j && i < dd) ? a[j] * Aown : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
        const double invj = __shfl(inv_own, j);
        const double Aj = (zall[j] - part) * invj;
        if (i == j) Aown = Aj;
      }
    }
    if (lane == 0) Aown += mo.xbar;
    if (lane < dd) oc[lane * nf] = (O)Aown;
  }
}

hipError_t solve_wide(bool fp64, const void* zc, const void* D, const Moments* mom,
                      const Geom& g, int curve0, int n_curves, double eps, void* out,
                      uint8_t* flags, void* coef, hipStream_t st) {
  if (2 * g.H + 1 > kDWide || g.band) return hipErrorInvalidValue;
  dim3 gr((unsigned)((g.n_freq + kNT / 64 - 1) / (kNT / 64)), (unsigned)n_curves);
  auto launch = [&](auto cf) {
    constexpr bool CF = decltype(cf)::value;
    if (fp64)
      hipLaunchKernelGGL((k_solve_wide<double, double, CF>), gr, dim3(kNT), 0, st,
                         (const cplx<double>*)zc, (const cplx<double>*)D, mom, g, curve0, eps,
                         (double*)out, flags, (double*)coef);
    else
      hipLaunchKernelGGL((k_solve_wide<float, float, CF>), gr, dim3(kNT), 0, st,
                         (const cplx<float>*)zc, (const cplx<double>*)D, mom, g, curve0, eps,
                         (float*)out, flags, (float*)coef);
  };
  if (coef)
    launch(std::true_type{});
  else
    launch(std::false_type{});
  return hipGetLastError();
}

template <int H>
hipError_t solve_multi_h(bool fp64, const void* zq, const void* zp, const void* D,
                         const Moments* mom_t, const Moments* mom_s, const double* scale,
                         const Geom& g, int src0, int n_src, double eps, void* out,
                         uint8_t* flags, hipStream_t st) {
  dim3 gr((unsigned)((g.n_freq + kNT - 1) / kNT));
  if (fp64)
    hipLaunchKernelGGL((k_solve_multi<H, double, double>), gr, dim3(kNT), 0, st,
                       (const cplx<double>*)zq, (const cplx<double>*)zp, (const cplx<double>*)D,
                       mom_t, mom_s, scale, g, src0, n_src, eps, (double*)out, flags);
  else
    hipLaunchKernelGGL((k_solve_multi<H, float, float>), gr, dim3(kNT), 0, st,
                       (const cplx<float>*)zq, (const cplx<float>*)zp, (const cplx<double>*)D,
                       mom_t, mom_s, scale, g, src0, n_src, eps, (float*)out, flags);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_solve(bool fp64, const void* zc, const void* D, const Moments* mom,
                        const Geom& g, int curve0, int n_curves, double eps_piv, void* dchi2,
                        uint8_t* flags, hipStream_t st, void* coef, bool wide) {
  if (wide)
    return solve_wide(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, coef, st);
  switch (g.H) {
    case 1: return solve_h<1>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, coef, st);
    case 2: return solve_h<2>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, coef, st);
    case 3: return solve_h<3>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, coef, st);
    case 4: return solve_h<4>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, coef, st);
    case 5: return solve_h<5>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, coef, st);
    case 6: return solve_h<6>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, coef, st);
    case 7: return solve_h<7>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, coef, st);
    case 8: return solve_h<8>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, coef, st);
    case 9: case 10: case 11: case 12: case 13: case 14: case 15: case 16:
      return solve_wide(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, coef, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_solve_multi(bool fp64, const void* zq, const void* zp, const void* D,
                              const Moments* mom_t, const Moments* mom_s, const double* scale,
                              const Geom& g, int src0, int n_src, double eps_piv, void* dchi2,
                              uint8_t* flags, hipStream_t st) {
  switch (g.H) {
    case 1: return solve_multi_h<1>(fp64, zq, zp, D, mom_t, mom_s, scale, g, src0, n_src, eps_piv, dchi2, flags, st);
    case 2: return solve_multi_h<2>(fp64, zq, zp, D, mom_t, mom_s, scale, g, src0, n_src, eps_piv, dchi2, flags, st);
    case 3: return solve_multi_h<3>(fp64, zq, zp, D, mom_t, mom_s, scale, g, src0, n_src, eps_piv, dchi2, flags, st);
    case 4: return solve_multi_h<4>(fp64, zq, zp, D, mom_t, mom_s, scale, g, src0, n_src, eps_piv, dchi2, flags, st);
    case 5: return solve_multi_h<5>(fp64, zq, zp, D, mom_t, mom_s, scale, g, src0, n_src, eps_piv, dchi2, flags, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fchi2
