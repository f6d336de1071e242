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

template <int H, typename R, typename O, bool BAND>
__global__ __launch_bounds__(kNT) void k_solve(const cplx<R>* __restrict__ zc,
                                               const cplx<double>* __restrict__ D,
                                               const Moments* __restrict__ mom, Geom g,
                                               int curve0, double eps, O* __restrict__ out,
                                               uint8_t* __restrict__ flags) {
  const int64_t nf = g.n_freq;
  const int64_t k = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const int cw = blockIdx.y;
  const int c = curve0 + cw;
  if (k >= nf) return;
  const Moments mo = mom[c];
  O d[H];
  const uint8_t fl = solve_bin<H, R, O, BAND>(zc, D, mo, g, cw, k, eps, d);
  O* o = out + (int64_t)c * H * nf + k;
#pragma unroll
  for (int h = 0; h < H; ++h) o[h * nf] = d[h];
  if (flags) flags[(int64_t)c * nf + k] = fl;
}

template <int H>
hipError_t solve_h(bool fp64, const void* zc, const void* D, const Moments* mom, const Geom& g,
                   int curve0, int n_curves, double eps, void* out, uint8_t* flags,
                   hipStream_t st) {
  dim3 gr((unsigned)((g.n_freq + kNT - 1) / kNT), (unsigned)n_curves);
  auto launch = [&](auto band) {
    constexpr bool B = decltype(band)::value;
    if (fp64)
      hipLaunchKernelGGL((k_solve<H, double, double, B>), gr, dim3(kNT), 0, st,
                         (const cplx<double>*)zc, (const cplx<double>*)D, mom, g, curve0, eps,
                         (double*)out, flags);
    else
      hipLaunchKernelGGL((k_solve<H, float, float, B>), gr, dim3(kNT), 0, st,
                         (const cplx<float>*)zc, (const cplx<double>*)D, mom, g, curve0, eps,
                         (float*)out, flags);
  };
  if (g.band)
    launch(std::true_type{});
  else
    launch(std::false_type{});
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
                        uint8_t* flags, hipStream_t st) {
  switch (g.H) {
    case 1: return solve_h<1>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, st);
    case 2: return solve_h<2>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, st);
    case 3: return solve_h<3>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, st);
    case 4: return solve_h<4>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, st);
    case 5: return solve_h<5>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, st);
    case 6: return solve_h<6>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, st);
    case 7: return solve_h<7>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, st);
    case 8: return solve_h<8>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, dchi2, flags, st);
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
