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
// afterwards).  Requiring 2H * df * span < 1 (the grid spans at least 2H times
// the observed period, Section 3b) means u never wraps, so positions are
// monotone in t and a tile of cells owns a contiguous range of points.
//
// Two real grids are packed per complex grid (real part, imaginary part);
// each workgroup owns a tile of cells of one packed grid and sums the kernel
// contributions of its points cell by cell (deterministic, no atomics).  The
// arithmetic is FP64; the grid is stored as S (float for mixed plans).
#include <cmath>

#include "fchi2_internal.h"
#include "launch.h"

namespace fchi2 {

namespace {

constexpr int kNT = 256;

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = kNT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  T r = red[0];
  __syncthreads();
  return r;
}

// Phase 1: block b of curve c reduces a contiguous chunk of the curve to
// (W_b, mean_b, M2_b = sum w (x - mean_b)^2) and validity bits.
__global__ __launch_bounds__(kNT) void k_moments_part(const double* __restrict__ t,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ sigma,
                                                      const int64_t* __restrict__ off,
                                                      int bpc, MomPart* __restrict__ part) {
  __shared__ double red[kNT];
  __shared__ uint32_t bad_s;
  const int c = blockIdx.y;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t a = off[c], e = off[c + 1];
  const int64_t n = e - a;
  const int64_t chunk = (n + bpc - 1) / bpc;
  const int64_t lo = a + (int64_t)b * chunk;
  const int64_t hi = (lo + chunk < e) ? lo + chunk : e;
  if (tid == 0) bad_s = 0;
  __syncthreads();
  double sw = 0.0, swx = 0.0;
  uint32_t bad = 0;
  for (int64_t i = lo + tid; i < hi; i += kNT) {
    const double ti = t[i], xi = x[i], si = sigma[i];
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
    const double y = x[i] - mean;
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

// Phase 2: one thread per curve combines the chunks in order (parallel
// variance update) and writes the curve's Moments and chi2_0.
__global__ __launch_bounds__(kNT) void k_moments_fin(const double* __restrict__ t,
                                                     const int64_t* __restrict__ off,
                                                     int n_curves, int bpc,
                                                     const MomPart* __restrict__ part, Geom g,
                                                     Moments* __restrict__ mom,
                                                     double* __restrict__ chi2_out) {
  const int c = blockIdx.x * kNT + threadIdx.x;
  if (c >= n_curves) return;
  const int64_t a = off[c], e = off[c + 1];
  const int64_t n = e - a;
  double W = 0.0, mean = 0.0, M2 = 0.0;
  uint32_t fl = 0;
  for (int b = 0; b < bpc; ++b) {
    const MomPart pp = part[(int64_t)c * bpc + b];
    fl |= pp.bad;
    if (!(pp.W > 0.0)) continue;
    const double Wn = W + pp.W;
    const double dlt = pp.mean - mean;
    mean += dlt * (pp.W / Wn);
    M2 += pp.M2 + dlt * dlt * (W * pp.W / Wn);
    W = Wn;
  }
  Moments m;
  m.W = W;
  m.xbar = mean;
  m.chi2_0 = M2;
  m.start = a;
  m.n = n;
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
    const double v = m.span * g.df;
    const double pos = ((double)(2 * g.H) * v) * (double)g.L + (double)g.c_off;
    if (!(pos + (double)(g.w / 2) + 3.0 <= (double)g.L)) fl |= CF_WRAP;
  }
  m.flags = fl;
  m.pad = 0;
  mom[c] = m;
  if (chi2_out) chi2_out[c] = (fl & kCurveFatal) ? NAN : M2;
}

// Cell coordinate of point i for harmonic multiple m (FP64 phase reduction).
__device__ __forceinline__ double cell_pos(const double* __restrict__ t, int64_t i, double T0,
                                           double df, int m, double L, double c_off) {
  const double v = (t[i] - T0) * df;
  return ((double)m * v) * L + c_off;
}

// First index in [lo, hi) whose cell position is >= target (positions are
// nondecreasing).  Executed by one full wavefront; 64-ary search.
__device__ int64_t wave_lower_bound(const double* __restrict__ t, int64_t lo, int64_t hi,
                                    double target, double T0, double df, int m, double L,
                                    double c_off) {
  const int lane = threadIdx.x & 63;
  while (hi - lo > 64) {
    const int64_t step = (hi - lo) / 64;
    const int64_t idx = lo + step * (lane + 1) - 1;
    const bool lt = cell_pos(t, idx, T0, df, m, L, c_off) < target;
    const int cnt = __popcll(__ballot(lt));
    const int64_t nlo = lo + step * cnt;
    const int64_t nhi = (cnt == 64) ? hi : lo + step * (cnt + 1);
    lo = nlo;
    hi = nhi;
  }
  const int64_t idx = lo + lane;
  const bool lt = (idx < hi) && (cell_pos(t, idx, T0, df, m, L, c_off) < target);
  return lo + __popcll(__ballot(lt));
}

// Exponential-of-semicircle kernel exp(beta (sqrt(1 - z^2) - 1)) on |z| < 1.
// The argument is formed in FP64.  With EXACT the exponential is FP64 too;
// otherwise the FP32 exponential of the rounded argument is corrected by the
// rounding residual, exp(a + r) = exp(a) (1 + r + O(r^2)), which keeps the
// kernel value within about one FP32 ulp although the argument reaches -2.3 w.
template <bool EXACT>
__device__ __forceinline__ double es_kernel(double z, double beta) {
  const double q = 1.0 - z * z;
  if (!(q > 0.0)) return 0.0;
  const double arg = beta * (sqrt(q) - 1.0);
  if constexpr (EXACT) {
    return exp(arg);
  } else {
    const float a = (float)arg;
    const double r = arg - (double)a;
    return (double)expf(a) * (1.0 + r);
  }
}

template <typename S, int LOGB>
__global__ __launch_bounds__(kNT) void k_spread(const double* __restrict__ t,
                                                const double* __restrict__ x,
                                                const double* __restrict__ sigma,
                                                const Moments* __restrict__ mom, Geom g,
                                                int curve0, cplx<S>* __restrict__ grid) {
  constexpr bool EXACT = sizeof(S) == 8;
  constexpr int B = 1 << LOGB;
  constexpr int CPT = B / kNT;
  constexpr int CH = 1024;
  __shared__ int s_j0[CH];
  __shared__ double s_fr[CH];
  __shared__ double s_re[CH];
  __shared__ double s_im[CH];
  __shared__ int64_t s_rng[2];

  const int tid = threadIdx.x;
  const int p = blockIdx.y;
  const int cw = blockIdx.z;
  const Moments mo = mom[curve0 + cw];
  if (mo.flags & kCurveFatal) return;
  const int64_t E = pair_extent(mo, g, p);
  const int64_t a0 = (int64_t)blockIdx.x * B;
  if (a0 >= E) return;

  const int hw = g.w / 2;
  const double two_over_w = 2.0 / (double)g.w;
  const double beta = g.beta;
  const double Ld = (double)g.L;
  const double coff = (double)g.c_off;
  const int64_t pa = mo.start, pb = mo.start + mo.n;

  double acc_re[CPT], acc_im[CPT];
#pragma unroll
  for (int u = 0; u < CPT; ++u) {
    acc_re[u] = 0.0;
    acc_im[u] = 0.0;
  }

  for (int comp = 0; comp < 2; ++comp) {
    const int m = g.comp_m[p][comp];
    if (m == 0) continue;
    if (comp == 1 && m == g.comp_m[p][0]) continue;  // shared with component 0
    const bool both = (comp == 0) && (g.comp_m[p][1] == m);
    const int kind_a = g.comp_kind[p][comp];
    const int kind_b = both ? g.comp_kind[p][1] : -1;

    const int wave = tid >> 6;
    if (wave < 2) {
      const double target = (wave == 0) ? (double)(a0 - hw - 2) : (double)(a0 + B + hw + 2);
      const int64_t r = wave_lower_bound(t, pa, pb, target, mo.T0, g.df, m, Ld, coff);
      if ((tid & 63) == 0) s_rng[wave] = r;
    }
    __syncthreads();
    const int64_t i_lo = s_rng[0], i_hi = s_rng[1];
    __syncthreads();

    for (int64_t ch = i_lo; ch < i_hi; ch += CH) {
      const int cnt = (int)((i_hi - ch) < CH ? (i_hi - ch) : CH);
      for (int q = tid; q < cnt; q += kNT) {
        const int64_t i = ch + q;
        const double pos = cell_pos(t, i, mo.T0, g.df, m, Ld, coff);
        const double fl = floor(pos);
        const double si = sigma[i];
        const double w = 1.0 / (si * si);
        const double wy = w * (x[i] - mo.xbar);
        const double sa = (kind_a == 0) ? w : wy;
        double sre, sim;
        if (comp == 0) {
          sre = sa;
          sim = both ? ((kind_b == 0) ? w : wy) : 0.0;
        } else {
          sre = 0.0;
          sim = sa;
        }
        s_j0[q] = (int)((int64_t)fl - a0);
        s_fr[q] = pos - fl;
        s_re[q] = sre;
        s_im[q] = sim;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int jl = tid + u * kNT;
        // First point with j0 >= jl - hw - 1.
        int lo = 0, hi = cnt;
        const int key = jl - hw - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (s_j0[mid] < key) lo = mid + 1;
          else hi = mid;
        }
        double ar = acc_re[u], ai = acc_im[u];
        for (int q = lo; q < cnt; ++q) {
          const int j0 = s_j0[q];
          if (j0 > jl + hw) break;
          const double d = (double)(jl - j0) - s_fr[q];
          const double phi = es_kernel<EXACT>(d * two_over_w, beta);
          ar += phi * s_re[q];
          ai += phi * s_im[q];
        }
        acc_re[u] = ar;
        acc_im[u] = ai;
      }
      __syncthreads();
    }
  }

  cplx<S>* out = grid + ((int64_t)cw * g.P + p) * g.L + a0;
#pragma unroll
  for (int u = 0; u < CPT; ++u) out[tid + u * kNT] = cmk<S>((S)acc_re[u], (S)acc_im[u]);
}

__global__ __launch_bounds__(kNT) void k_deconv(cplx<double>* __restrict__ D, Geom g,
                                                const double* __restrict__ gx,
                                                const double* __restrict__ gw, int ng) {
  const int64_t k = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (k >= g.n_freq) return;
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
                          MomPart* part, Moments* mom, double* chi2_0, hipStream_t st) {
  hipLaunchKernelGGL(k_moments_part, dim3(bpc, n_curves), dim3(kNT), 0, st, t, x, sigma,
                     offsets, bpc, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_moments_fin, dim3((n_curves + kNT - 1) / kNT), dim3(kNT), 0, st, t,
                     offsets, n_curves, bpc, part, g, mom, chi2_0);
  return hipGetLastError();
}

hipError_t launch_spread(bool fp64, const double* t, const double* x, const double* sigma,
                         const Moments* mom, const Geom& g, int curve0, int n_curves,
                         void* grid, int log_tile, hipStream_t st) {
  const int64_t tiles = g.L >> log_tile;
  dim3 gr((unsigned)tiles, (unsigned)g.P, (unsigned)n_curves);
  if (log_tile == 10) {
    if (fp64)
      hipLaunchKernelGGL((k_spread<double, 10>), gr, dim3(kNT), 0, st, t, x, sigma, mom, g,
                         curve0, (cplx<double>*)grid);
    else
      hipLaunchKernelGGL((k_spread<float, 10>), gr, dim3(kNT), 0, st, t, x, sigma, mom, g,
                         curve0, (cplx<float>*)grid);
  } else if (log_tile == 11) {
    if (fp64)
      hipLaunchKernelGGL((k_spread<double, 11>), gr, dim3(kNT), 0, st, t, x, sigma, mom, g,
                         curve0, (cplx<double>*)grid);
    else
      hipLaunchKernelGGL((k_spread<float, 11>), gr, dim3(kNT), 0, st, t, x, sigma, mom, g,
                         curve0, (cplx<float>*)grid);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_deconv_init(void* D, const Geom& g, const double* gl_x, const double* gl_w,
                              int n_gl, hipStream_t st) {
  const unsigned nb = (unsigned)((g.n_freq + kNT - 1) / kNT);
  hipLaunchKernelGGL(k_deconv, dim3(nb), dim3(kNT), 0, st, (cplx<double>*)D, g, gl_x, gl_w, n_gl);
  return hipGetLastError();
}

}  // namespace fchi2
