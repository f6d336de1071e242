// Per-curve moments and the spreading (extirpolation) of the weighted data
// onto the packed harmonic grids.
//
// The transforms needed at trial frequency f_k = k * df are
//   Q(m f_k) = sum_i w_i exp(+2 pi i k u_i^(m)),
//   P(m f_k) = sum_i w_i (x_i - xbar) exp(+2 pi i k u_i^(m)),
// with w = sigma^-2 (Section 2, eq. eqPQ; centring as in Section 3b) and
// u_i^(m) = m * df * (t_i - T0) in cycles.  For every harmonic multiple m the
// points are spread with an exponential-of-semicircle kernel onto a periodic
// grid of L = 4 * n_freq cells at cell coordinate u * L + c_off, so that one
// FFT per grid gives all n_freq bins (the grid replaces the paper's Kronecker
// gridding of Section 3b; the kernel's Fourier transform is divided out
// afterwards).  The grid is periodic: when 2H * df * span exceeds 1 (the
// arrays of Section 3b cover fewer than 2H times the observed span) the
// phases m u wrap around it.  Positions are kept unwrapped, so they grow with
// t and every tile of cells owns a contiguous range of points in each period
// ("lap") of the grid; the tile table runs over the plan's laps.
//
// Two real grids are packed per complex grid (real part, imaginary part);
// each workgroup owns a tile of cells of one packed grid and sums the kernel
// contributions of its points cell by cell (deterministic, no atomics).  The
// arithmetic is FP64 (for float grids the kernel's exponential is taken to
// FP32 accuracy, see es_kernel.h); the grid is stored as S (float for mixed
// plans).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "fchi2_internal.h"
#include "launch.h"
#include "es_kernel.h"
#include "spread_tile.h"

namespace fchi2 {

namespace {

// Sum over the block in a fixed order (wave butterflies, then the four wave
// sums in order): deterministic, two barriers.  red holds kNT / 64 values.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  const int tid = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  T r = red[0];
#pragma unroll
  for (int w = 1; w < kNT / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}

// Phase 1: block b of curve c reduces a contiguous chunk of the curve to
// (W_b, mean_b, M2_b = sum w (x - mean_b)^2) and validity bits.  With
// shared_t every curve c uses the points [off[0], off[1]) of t and sigma and
// its own data x[c * n + i] (sources observed at the same times).
__global__ __launch_bounds__(kNT) void k_moments_part(const double* __restrict__ t,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ sigma,
                                                      const int64_t* __restrict__ off,
                                                      int bpc, int shared_t,
                                                      MomPart* __restrict__ part) {
  __shared__ double red[kNT / 64];
  __shared__ uint32_t bad_s;
  const int c = blockIdx.y;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t a = shared_t ? off[0] : off[c], e = shared_t ? off[1] : off[c + 1];
  const int64_t xs = shared_t ? (int64_t)c * (e - a) : 0;
  const int64_t n = e - a;
  const int64_t chunk = (n + bpc - 1) / bpc;
  const int64_t lo = a + (int64_t)b * chunk;
  const int64_t hi = (lo + chunk < e) ? lo + chunk : e;
  if (tid == 0) bad_s = 0;
  __syncthreads();
  double sw = 0.0, swx = 0.0;
  uint32_t bad = 0;
  for (int64_t i = lo + tid; i < hi; i += kNT) {
    const double ti = t[i], xi = x[i + xs], si = sigma[i];
    if (!isfinite(ti) || !isfinite(xi) || !isfinite(si) || !(si > 0.0)) bad |= CF_NONFINITE;
    if (i > a && !(ti >= t[i - 1])) bad |= CF_UNSORTED;
    const double w = 1.0 / (si * si);
    sw += w;
    swx += w * xi;
  }
  if (bad) atomicOr(&bad_s, bad);
  const double W = block_sum(sw, red);
  const double WX = block_sum(swx, red);
  const double mean = (W > 0.0) ? WX / W : 0.0;
  double sc = 0.0;
  for (int64_t i = lo + tid; i < hi; i += kNT) {
    const double si = sigma[i];
    const double y = x[i + xs] - mean;
    sc += y * y / (si * si);
  }
  const double M2 = block_sum(sc, red);
  if (tid == 0) {
    MomPart pp;
    pp.W = W;
    pp.mean = mean;
    pp.M2 = M2;
    pp.bad = bad_s;
    pp.pad = 0;
    part[(int64_t)c * bpc + b] = pp;
  }
}

// Pairwise combination of two chunk summaries (parallel variance update);
// an empty chunk (W = 0) leaves the other unchanged.
__device__ __forceinline__ void mom_combine(double& W, double& mean, double& M2, double W2,
                                            double mean2, double M22) {
  if (!(W2 > 0.0)) return;
  const double Wn = W + W2;
  const double dlt = mean2 - mean;
  mean += dlt * (W2 / Wn);
  M2 += M22 + dlt * dlt * (W * W2 / Wn);
  W = Wn;
}

// Phase 2: one wave per curve.  Lane j combines chunks j, j + 64, ... in
// order, then the 64 lane summaries are combined by a fixed pairwise tree
// (deterministic); lane 0 writes the curve's Moments and chi2_0.
__global__ __launch_bounds__(64) void k_moments_fin(const double* __restrict__ t,
                                                    const int64_t* __restrict__ off,
                                                    int n_curves, int bpc, int shared_t,
                                                    const double* __restrict__ scale,
                                                    const MomPart* __restrict__ part, Geom g,
                                                    Moments* __restrict__ mom,
                                                    double* __restrict__ chi2_out) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  double W = 0.0, mean = 0.0, M2 = 0.0;
  uint32_t fl = 0;
  for (int b = lane; b < bpc; b += 64) {
    const MomPart pp = part[(int64_t)c * bpc + b];
    fl |= pp.bad;
    mom_combine(W, mean, M2, pp.W, pp.mean, pp.M2);
  }
  for (int o = 1; o < 64; o <<= 1) {
    const double W2 = __shfl_down(W, o), mean2 = __shfl_down(mean, o), M22 = __shfl_down(M2, o);
    const uint32_t f2 = (uint32_t)__shfl_down((int)fl, o);
    if ((lane & (2 * o - 1)) == 0) {
      mom_combine(W, mean, M2, W2, mean2, M22);
      fl |= f2;
    }
  }
  if (lane != 0) return;
  const int64_t a = shared_t ? off[0] : off[c], e = shared_t ? off[1] : off[c + 1];
  const int64_t n = e - a;
  Moments m;
  m.W = W;
  m.xbar = mean;
  m.chi2_0 = M2;
  m.start = a;
  m.n = n;
  m.xshift = shared_t ? (int64_t)c * n : 0;
  if (n <= 0) {
    fl |= CF_EMPTY;
    m.T0 = 0.0;
    m.span = 0.0;
  } else {
    m.T0 = t[a];
    m.span = t[e - 1] - t[a];
  }
  if (n < 2 * g.H + 1) fl |= CF_FEW;
  if (!(fl & kCurveFatal)) {
    // The tile tables cover g.laps periods of the grid.
    const double v = m.span * g.df;
    const double pos = ((double)(2 * g.H) * v) * (double)g.L + (double)g.c_off;
    if (!(pos + (double)(g.w / 2) + 3.0 <= (double)g.laps * (double)g.L)) fl |= CF_WRAP;
  }
  // A source whose errors are scale[c] times the shared sigma: its chi2 is the
  // base-weight sum divided by scale^2 (the weights are sigma^-2 / scale^2).
  double sc2 = 1.0;
  if (scale) {
    const double sv = scale[c];
    if (!(sv > 0.0) || !isfinite(sv)) fl |= CF_NONFINITE;
    sc2 = sv * sv;
  }
  m.flags = fl;
  m.pad = 0;
  mom[c] = m;
  if (chi2_out) chi2_out[c] = (fl & kCurveFatal) ? NAN : M2 / sc2;
}

__global__ __launch_bounds__(kNT) void k_tile_bounds(const double* __restrict__ t,
                                                     const Moments* __restrict__ mom, Geom g,
                                                     int curve0, int log_tile, int ntb,
                                                     int32_t* __restrict__ tb) {
  const int cw = blockIdx.z;
  const int m = blockIdx.y + 1;
  const Moments mo = mom[curve0 + cw];
  if (mo.flags & kCurveFatal) return;
  const int64_t il = (int64_t)blockIdx.x * kNT + threadIdx.x;
  tile_bounds_point(t, mo, g, cw, m, il, log_tile, ntb, tb);
}

// Blocks of one curve (wave slot blockIdx.z) stride over the tiles below each
// pair's nonzero extent, pair after pair (cells beyond the extent are never
// read).
template <typename S, int LOGB, bool BAND>
__global__ __launch_bounds__(kNT) void k_spread(const double* __restrict__ t,
                                                const double* __restrict__ x,
                                                const double* __restrict__ sigma,
                                                const Moments* __restrict__ mom, Geom g,
                                                int curve0, const int32_t* __restrict__ tb,
                                                int ntb, int share_tb,
                                                cplx<S>* __restrict__ grid) {
  __shared__ SpreadSmem<LOGB> sh;
  const int cw = blockIdx.z;
  const Moments mo = mom[curve0 + cw];
  if (mo.flags & kCurveFatal) return;
  int64_t items = 0;
  for (int q = 0; q < g.P; ++q) items += pair_extent(mo, g, q) >> LOGB;
  for (int64_t wi = blockIdx.x; wi < items; wi += gridDim.x) {
    int p = 0;
    int64_t tile = wi;
    for (;;) {
      const int64_t nt = pair_extent(mo, g, p) >> LOGB;
      if (tile < nt) break;
      tile -= nt;
      ++p;
    }
    spread_tile<S, LOGB, BAND>(t, x, sigma, mo, g, cw, tb, ntb, share_tb, p, tile,
                               grid + ((int64_t)cw * g.P + p) * g.L + (tile << LOGB), sh, threadIdx.x);
  }
}

__global__ __launch_bounds__(kNT) void k_deconv(cplx<double>* __restrict__ D, Geom g,
                                                const double* __restrict__ gx,
                                                const double* __restrict__ gw, int ng) {
  const int64_t k = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (k >= g.n_freq) return;
  if (g.w == 1) {  // floor gridding: no kernel to divide out, no origin shift
    D[k] = cmk<double>(1.0, 0.0);
    return;
  }
  // phi_hat(k) = w * int_0^1 phi(z) cos(pi w k z / L) dz, phi(z) folded into gw.
  const double a = M_PI * (double)g.w * (double)k / (double)g.L;
  double s = 0.0;
  for (int q = 0; q < ng; ++q) s += gw[q] * cos(a * gx[q]);
  // exp(-2 pi i k c_off / L) with the exponent reduced exactly modulo L.
  const int64_t e = (k * (int64_t)g.c_off) & (g.L - 1);
  const double ang = -2.0 * (double)e / (double)g.L;
  double sn, cs;
  sincospi(ang, &sn, &cs);
  D[k] = cmk<double>(cs / s, sn / s);
}

}  // namespace

hipError_t launch_moments(const double* t, const double* x, const double* sigma,
                          const int64_t* offsets, int n_curves, int bpc, const Geom& g,
                          MomPart* part, Moments* mom, double* chi2_0, hipStream_t st,
                          bool shared_t, const double* scale) {
  hipLaunchKernelGGL(k_moments_part, dim3(bpc, n_curves), dim3(kNT), 0, st, t, x, sigma,
                     offsets, bpc, shared_t ? 1 : 0, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_moments_fin, dim3(n_curves), dim3(64), 0, st, t, offsets, n_curves, bpc,
                     shared_t ? 1 : 0, scale, part, g, mom, chi2_0);
  return hipGetLastError();
}

hipError_t launch_spread(bool fp64, const double* t, const double* x, const double* sigma,
                         const Moments* mom, const Geom& g, int curve0, int n_curves,
                         int64_t max_n, int32_t* tb, void* grid, int log_tile, hipStream_t st,
                         bool share_tb) {
  const int64_t tiles = g.L >> log_tile;
  const int ntb = (int)(tiles * g.laps) + 2;
  dim3 gb((unsigned)((max_n + 1 + kNT - 1) / kNT), (unsigned)(2 * g.H), (unsigned)n_curves);
  // Sources sharing one time base share the table of slot 0 (built already).
  if (!share_tb)
    hipLaunchKernelGGL(k_tile_bounds, gb, dim3(kNT), 0, st, t, mom, g, curve0, log_tile, ntb,
                       tb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Blocks stride over the non-empty tiles of each curve (counted on the device).
  const int64_t cap = std::max<int64_t>(8, 4096 / std::max(n_curves, 1));
  dim3 gr((unsigned)std::min<int64_t>(cap, tiles * g.P), 1u, (unsigned)n_curves);
  auto launch_b = [&](auto logb, auto band) -> void {
    constexpr int LB = decltype(logb)::value;
    constexpr bool BD = decltype(band)::value;
    if (fp64)
      hipLaunchKernelGGL((k_spread<double, LB, BD>), gr, dim3(kNT), 0, st, t, x, sigma, mom, g,
                         curve0, tb, ntb, share_tb ? 1 : 0, (cplx<double>*)grid);
    else
      hipLaunchKernelGGL((k_spread<float, LB, BD>), gr, dim3(kNT), 0, st, t, x, sigma, mom, g,
                         curve0, tb, ntb, share_tb ? 1 : 0, (cplx<float>*)grid);
  };
  auto launch = [&](auto logb) -> void {
    if (g.band)
      launch_b(logb, std::true_type{});
    else
      launch_b(logb, std::false_type{});
  };
  switch (log_tile) {
    case 10: launch(std::integral_constant<int, 10>{}); break;
    case 11: launch(std::integral_constant<int, 11>{}); break;
    case 12: launch(std::integral_constant<int, 12>{}); break;
    case 13: launch(std::integral_constant<int, 13>{}); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tile_bounds(const double* t, const Moments* mom, const Geom& g, int curve0,
                              int n_curves, int64_t max_n, int32_t* tb, int log_tile,
                              hipStream_t st) {
  const int ntb = (int)((g.L >> log_tile) * g.laps) + 2;
  dim3 gb((unsigned)((max_n + 1 + kNT - 1) / kNT), (unsigned)(2 * g.H), (unsigned)n_curves);
  hipLaunchKernelGGL(k_tile_bounds, gb, dim3(kNT), 0, st, t, mom, g, curve0, log_tile, ntb, tb);
  return hipGetLastError();
}

size_t tile_bounds_bytes(const Geom& g, int log_tile, int n_curves) {
  return sizeof(int32_t) * (size_t)n_curves * (size_t)(2 * g.H) *
         (size_t)((g.L >> log_tile) * g.laps + 2);
}

hipError_t launch_deconv_init(void* D, const Geom& g, const double* gl_x, const double* gl_w,
                              int n_gl, hipStream_t st) {
  const unsigned nb = (unsigned)((g.n_freq + kNT - 1) / kNT);
  hipLaunchKernelGGL(k_deconv, dim3(nb), dim3(kNT), 0, st, (cplx<double>*)D, g, gl_x, gl_w, n_gl);
  return hipGetLastError();
}

}  // namespace fchi2
