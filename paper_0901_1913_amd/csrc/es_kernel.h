// Exponential-of-semicircle spreading kernel
//   phi(z) = exp(beta (sqrt(1 - z^2) - 1))  for |z| < 1,  0 elsewhere,
// evaluated with an FP64 argument by the spreading (standalone or fused into
// the first FFT pass) and by the adjoint's gather (the same values
// everywhere), and the cell coordinate of a point on a harmonic grid.
//
// EXACT (FP64 grids): correctly rounded FP64 sqrt and exp.
// Otherwise (FP32 grids), with no branch:
//   sqrt(q) = q * rsqrt(q), the hardware reciprocal-square-root estimate
//   refined by one Newton step (relative error ~1e-14);
//   exp(a) = 2^y, y = a log2(e) split in FP64 into an integer n and a
//   fraction |f| <= 1/2 (Cody-Waite range reduction), 2^f from the hardware
//   FP32 base-2 exponential of f rounded to FP32, scaled by 2^n.
// The FP32 path keeps phi within about two FP32 ulp over the whole support
// (the argument reaches -beta = -2.3 w), below what an FP32 grid stores.
#pragma once

#include <cmath>

namespace fchi2 {

template <bool EXACT>
__device__ __forceinline__ double es_kernel(double z, double beta) {
  const double q = 1.0 - z * z;
  if constexpr (EXACT) {
    if (!(q > 0.0)) return 0.0;
    return exp(beta * (sqrt(q) - 1.0));
  } else {
    const bool in = q > 0.0;
    const double qc = in ? q : 1.0;  // keeps the estimate finite off the support
    const double y0 = __builtin_amdgcn_rsq(qc);
    const double s0 = qc * y0;
    const double e0 = fma(-s0, 0.5 * y0, 0.5);
    const double s1 = fma(s0, e0, s0);                           // sqrt(qc)
    const double y = (beta * (s1 - 1.0)) * 1.4426950408889634;  // log2(e)
    const double n = rint(y);
    const float p2 = ldexpf(__builtin_amdgcn_exp2f((float)(y - n)), (int)n);
    return in ? (double)p2 : 0.0;
  }
}

// Cell coordinate of a point for harmonic multiple m (FP64 phase reduction),
// from v = (t - T0) df: m v L + c_off.  Floor gridding (kernel width 1,
// Section 3b): the point's time is replaced by the start of its cell,
// floor(v L), and harmonic m sits at m times that cell (an exact integer);
// the kernel weight is then 1 at that cell only.
__device__ __forceinline__ double cell_of(double v, int m, double L, double c_off, bool flr) {
  if (flr) return (double)m * floor(v * L);
  return ((double)m * v) * L + c_off;
}

__device__ __forceinline__ double cell_at(double ti, double T0, double df, int m, double L,
                                          double c_off, bool flr) {
  return cell_of((ti - T0) * df, m, L, c_off, flr);
}

}  // namespace fchi2
