// Per-frequency Delta chi2 for every H' = 1..H: one thread per bin runs the
// shared per-bin solve and writes all H rows and the bin's flags.
#include <cmath>

#include "fchi2_internal.h"
#include "launch.h"
#include "solve_bin.h"

namespace fchi2 {

namespace {

constexpr int kNT = 256;

using namespace solve_detail;

template <int H, typename R, typename O>
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
  const uint8_t fl = solve_bin<H, R, O>(zc, D, mo, g, cw, k, eps, d);
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
  if (fp64)
    hipLaunchKernelGGL((k_solve<H, double, double>), gr, dim3(kNT), 0, st,
                       (const cplx<double>*)zc, (const cplx<double>*)D, mom, g, curve0, eps,
                       (double*)out, flags);
  else
    hipLaunchKernelGGL((k_solve<H, float, float>), gr, dim3(kNT), 0, st, (const cplx<float>*)zc,
                       (const cplx<double>*)D, mom, g, curve0, eps, (float*)out, flags);
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

}  // namespace fchi2
