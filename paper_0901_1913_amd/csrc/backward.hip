// Adjoint of the search: gradient of a scalar loss L through Delta chi2 with
// respect to x_i and sigma_i.
//
// Per bin, Delta(H') = beta' alpha'^-1 beta' on the leading (2H'+1) block
// (eq. eqchix), so with A' = alpha'^-1 beta' (eq. eqcoeffs):
//   dDelta(H')/dbeta = 2 A',  dDelta(H')/dalpha = -A' A'^T.
// A' comes from the forward Cholesky factor by back substitution with its
// leading block.  The product-to-sum assembly (Section 2) is transposed onto
// the gradients of Re/Im Q(m f) and P(m f); the deconvolution factor and the
// unpacking of the packed grids are transposed; an FFT of the conjugated
// adjoint spectrum gives the conjugated grid gradient (the adjoint of the
// +i transform is the -i transform); and interpolation with the same kernel
// at the same positions (the transpose of the spreading) gives per-point
// gradients g_q (strength w) and g_p (strength w (x - xbar)).  Finally,
// with xbar = sum w x / W:
//   dL/dx_i     = w_i (g_p,i - gbar_p),  gbar_p = sum_j w_j g_p,j / W
//   dL/dw_i     = g_q,i + dL/dW + (x_i - xbar)(g_p,i - gbar_p)
//   dL/dsigma_i = -2 w_i / sigma_i * dL/dw_i
// where dL/dW collects the alpha entries that equal W = Q(0).
#include <cmath>

#include "fchi2_internal.h"
#include "launch.h"
#include "es_kernel.h"
#include "solve_bin.h"

namespace fchi2 {

namespace {

constexpr int kNT = 256;

// Spectra unpacking, assembly (product-to-sum) and the prefix Cholesky are
// the forward's own (solve_bin.h), so the adjoint differentiates exactly the
// factorisation the search used.
using namespace solve_detail;

// Add v * d alpha_ij / d(Q) for i >= j into dQr/dQi (index 0 of dQr is dW).
__device__ __forceinline__ void alpha_adj(int i, int j, double v, double* dQr, double* dQi) {
  if (j == 0) {
    if (i == 0) {
      dQr[0] += v;
      return;
    }
    const int h = (i + 1) >> 1;
    if (i & 1) dQi[h] += v;
    else dQr[h] += v;
    return;
  }
  const int h = (i + 1) >> 1, hp = (j + 1) >> 1;  // h >= hp for i >= j
  const int gm = h - hp, gpl = h + hp;
  const double hv = 0.5 * v;
  const bool si = (i & 1), sj = (j & 1);
  if (si && sj) {
    dQr[gm] += hv;
    dQr[gpl] -= hv;
  } else if (si && !sj) {
    dQi[gpl] += hv;
    if (gm > 0) dQi[gm] += hv;
  } else if (!si && sj) {
    dQi[gpl] += hv;
    if (gm > 0) dQi[gm] -= hv;
  } else {
    dQr[gm] += hv;
    dQr[gpl] += hv;
  }
}

template <int H, typename R, typename O>
__global__ __launch_bounds__(kNT) void k_adjoint(const cplx<R>* __restrict__ zc,
                                                 const cplx<double>* __restrict__ D,
                                                 const Moments* __restrict__ mom, Geom g,
                                                 int curve0, double eps,
                                                 const O* __restrict__ gin,
                                                 cplx<R>* __restrict__ spec,
                                                 double* __restrict__ dw_part, int bpc) {
  constexpr int d = 2 * H + 1;
  constexpr int P = Layout<H>::P;
  __shared__ double red[kNT];
  const int64_t nf = g.n_freq;
  const int64_t L = g.L;
  const int tid = threadIdx.x;
  const int64_t k = (int64_t)blockIdx.x * kNT + tid;
  const int cw = blockIdx.y;
  const int c = curve0 + cw;
  const Moments mo = mom[c];
  if (mo.flags & kCurveFatal) return;  // whole block: uniform per curve
  cplx<R>* sp = spec + (int64_t)cw * P * L;
  const cplx<R> zero = cmk<R>((R)0, (R)0);
  double dW = 0.0;

  if (k < nf) {
    if (k == 0) {
      for (int pp = 0; pp < P; ++pp) {
        sp[pp * L + 0] = zero;
        sp[pp * L + (L - nf)] = zero;
      }
    } else {
      // Forward spectra, assembly and Cholesky factor at bin k, as in the solve.
      double Qr[2 * H + 1], Qi[2 * H + 1], Pr[H + 1], Pi[H + 1];
      const cplx<double> Dk = D[k];
      const double Dr = (double)Dk.x, Di = (double)Dk.y;
      load_spectra<H, R>(zc, nf, (int64_t)cw * P, k, Dk, mo.W, Qr, Qi, Pr, Pi);
      double Lm[d][d];
      double inv[d];
      double z[d];
      double dfw[H];
      uint8_t fl = 0;
      prefix_solve<H, double>(Qr, Qi, Pr, Pi, eps, dfw, fl, Lm, inv, z);
      // Accumulate dQ (index 0 = dW) and dP over H' = 1..H.
      double dQr[2 * H + 1], dQi[2 * H + 1], dPr[H + 1], dPi[H + 1];
      static_for<0, 2 * H + 1>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        dQr[m] = 0.0;
        dQi[m] = 0.0;
      });
      static_for<0, H + 1>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        dPr[m] = 0.0;
        dPi[m] = 0.0;
      });
      const O* gk = gin + (int64_t)c * H * nf + k;
      static_for<1, H + 1>([&](auto hc) {
        constexpr int hp = decltype(hc)::value;
        constexpr int dp = 2 * hp + 1;
        const double gv = (double)gk[(hp - 1) * nf];
        // A' = L'^-T z' on the leading dp x dp block.
        double A[dp];
        static_for<0, dp>([&](auto rc) {
          constexpr int ii = dp - 1 - decltype(rc)::value;
          double s = z[ii];
          static_for<ii + 1, dp>([&](auto lc) {
            constexpr int l = decltype(lc)::value;
            s -= Lm[l][ii] * A[l];
          });
          A[ii] = s * inv[ii];
        });
        static_for<1, dp>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
          constexpr int h = (i + 1) >> 1;
          const double db = 2.0 * gv * A[i];
          if constexpr (i & 1) dPi[h] += db;
          else dPr[h] += db;
        });
        static_for<0, dp>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
          static_for<0, i + 1>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const double v = -gv * A[i] * A[j] * (i == j ? 1.0 : 2.0);
            alpha_adj(i, j, v, dQr, dQi);
          });
        });
      });
      dW = dQr[0];
      // Transpose of D and of the unpacking; write the conjugated adjoint
      // spectrum at k and L - k of every packed grid.
#pragma unroll
      for (int pp = 0; pp < P; ++pp) {
        double gar, gai, gbr, gbi;
        if (pp < H) {
          gar = dQr[2 * pp + 1];
          gai = dQi[2 * pp + 1];
          gbr = dQr[2 * pp + 2];
          gbi = dQi[2 * pp + 2];
        } else {
          const int j = pp - H;
          gar = dPr[2 * j + 1];
          gai = dPi[2 * j + 1];
          gbr = (2 * j + 2 <= H) ? dPr[2 * j + 2] : 0.0;
          gbi = (2 * j + 2 <= H) ? dPi[2 * j + 2] : 0.0;
        }
        // G_tilde = conj(D) * G
        const double tar = gar * Dr + gai * Di, tai = gai * Dr - gar * Di;
        const double tbr = gbr * Dr + gbi * Di, tbi = gbi * Dr - gbr * Di;
        // G_z0 = G_a/2 + (i/2) G_b ; G_z1 = conj(G_a)/2 + (i/2) conj(G_b)
        const double z0r = 0.5 * tar - 0.5 * tbi, z0i = 0.5 * tai + 0.5 * tbr;
        const double z1r = 0.5 * tar + 0.5 * tbi, z1i = -0.5 * tai + 0.5 * tbr;
        sp[pp * L + k] = cmk<R>((R)z0r, (R)(-z0i));
        sp[pp * L + (L - k)] = cmk<R>((R)z1r, (R)(-z1i));
      }
    }
  }
  // Block sum of dW (deterministic tree).
  red[tid] = dW;
  __syncthreads();
  for (int s = kNT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) dw_part[(int64_t)c * bpc + blockIdx.x] = red[0];
}

template <typename S>
__global__ __launch_bounds__(kNT) void k_gather(const double* __restrict__ t,
                                                const Moments* __restrict__ mom, Geom g,
                                                int curve0, const cplx<S>* __restrict__ grid,
                                                double* __restrict__ gq, double* __restrict__ gp) {
  constexpr bool EXACT = sizeof(S) == 8;
  const int cw = blockIdx.y;
  const Moments mo = mom[curve0 + cw];
  const int64_t il = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (il >= mo.n) return;
  if (mo.flags & kCurveFatal) return;
  const int64_t i = mo.start + il;
  const int hw = g.w / 2;
  const double two_over_w = 2.0 / (double)g.w;
  const double v = (t[i] - mo.T0) * g.df;
  double aq = 0.0, ap = 0.0;
  for (int p = 0; p < g.P; ++p) {
    const cplx<S>* gr = grid + ((int64_t)cw * g.P + p) * g.L;
    for (int comp = 0; comp < 2; ++comp) {
      const int m = g.comp_m[p][comp];
      if (m == 0) continue;
      const double pos = cell_of(v, m, (double)g.L, (double)g.c_off, false);
      const double fl = floor(pos);
      const int64_t j0 = (int64_t)fl;
      const double fr = pos - fl;
      double acc = 0.0;
      for (int dj = -hw - 1; dj <= hw + 1; ++dj) {
        const double phi = es_kernel<EXACT>(((double)dj - fr) * two_over_w, g.beta);
        if (phi != 0.0) {
          const cplx<S> val = gr[(j0 + dj) & (g.L - 1)];  // the grid is periodic
          acc += phi * (comp == 0 ? (double)val.x : -(double)val.y);
        }
      }
      if (g.comp_kind[p][comp] == 0) aq += acc;
      else ap += acc;
    }
  }
  gq[i] = aq;
  gp[i] = ap;
}

// Final step of the adjoint, in two chunked phases over each curve's points
// (the forward's moment partials buffer holds the per-chunk sums):
//   phase 1, block b of curve c: s1 = sum_chunk w g_p and s2 = its share of
//            the dW partials of the solve;
//   phase 2, block b of curve c: gbar = sum s1 / W, dW = sum s2, then
//            grad_x = w (g_p - gbar) and
//            grad_sigma = -2 w / sigma (g_q + dW + (x - xbar)(g_p - gbar)).
__global__ __launch_bounds__(kNT) void k_fin_reduce(const double* __restrict__ sigma,
                                                    const Moments* __restrict__ mom, int curve0,
                                                    const double* __restrict__ dw_part, int bpc,
                                                    const double* __restrict__ gp, int nch,
                                                    double* __restrict__ part) {
  __shared__ double red[2][kNT / 64];
  const int c = curve0 + blockIdx.y;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const Moments mo = mom[c];
  if (mo.flags & kCurveFatal) return;
  const int64_t chunk = (mo.n + nch - 1) / nch;
  const int64_t lo = mo.start + (int64_t)b * chunk;
  const int64_t hi = (lo + chunk < mo.start + mo.n) ? lo + chunk : mo.start + mo.n;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = lo + tid; i < hi; i += kNT) {
    const double si = sigma[i];
    s1 += gp[i] / (si * si);
  }
  const int per = (bpc + nch - 1) / nch;
  for (int q = b * per + tid; q < (b + 1) * per && q < bpc; q += kNT)
    s2 += dw_part[(int64_t)c * bpc + q];
  for (int o = 32; o > 0; o >>= 1) {
    s1 += __shfl_xor(s1, o);
    s2 += __shfl_xor(s2, o);
  }
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = s1;
    red[1][tid >> 6] = s2;
  }
  __syncthreads();
  if (tid == 0) {
    double a1 = 0.0, a2 = 0.0;
    for (int w = 0; w < kNT / 64; ++w) {
      a1 += red[0][w];
      a2 += red[1][w];
    }
    part[2 * ((int64_t)c * nch + b)] = a1;
    part[2 * ((int64_t)c * nch + b) + 1] = a2;
  }
}

__global__ __launch_bounds__(kNT) void k_finalize(const double* __restrict__ x,
                                                  const double* __restrict__ sigma,
                                                  const Moments* __restrict__ mom, int curve0,
                                                  const double* __restrict__ part, int nch,
                                                  const double* __restrict__ gq,
                                                  const double* __restrict__ gp,
                                                  double* __restrict__ grad_x,
                                                  double* __restrict__ grad_sigma) {
  __shared__ double red[2][kNT / 64];
  const int c = curve0 + blockIdx.y;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const Moments mo = mom[c];
  const int64_t chunk = (mo.n + nch - 1) / nch;
  const int64_t lo = mo.start + (int64_t)b * chunk;
  const int64_t hi = (lo + chunk < mo.start + mo.n) ? lo + chunk : mo.start + mo.n;
  if (mo.flags & kCurveFatal) {
    for (int64_t i = lo + tid; i < hi; i += kNT) {
      grad_x[i] = NAN;
      grad_sigma[i] = NAN;
    }
    return;
  }
  // Chunk sums in a fixed order (every block of the curve gets the same totals).
  double s1 = 0.0, s2 = 0.0;
  for (int q = tid; q < nch; q += kNT) {
    s1 += part[2 * ((int64_t)c * nch + q)];
    s2 += part[2 * ((int64_t)c * nch + q) + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    s1 += __shfl_xor(s1, o);
    s2 += __shfl_xor(s2, o);
  }
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = s1;
    red[1][tid >> 6] = s2;
  }
  __syncthreads();
  double a1 = 0.0, dW = 0.0;
  for (int w = 0; w < kNT / 64; ++w) {
    a1 += red[0][w];
    dW += red[1][w];
  }
  const double gbar = a1 / mo.W;
  for (int64_t i = lo + tid; i < hi; i += kNT) {
    const double si = sigma[i];
    const double w = 1.0 / (si * si);
    const double dp = gp[i] - gbar;
    grad_x[i] = w * dp;
    const double dLdw = gq[i] + dW + (x[i] - mo.xbar) * dp;
    grad_sigma[i] = -2.0 * w / si * dLdw;
  }
}

template <int H>
hipError_t adjoint_h(bool fp64, const void* zc, const void* D, const Moments* mom, const Geom& g,
                     int curve0, int n_curves, double eps, const void* gin, void* spec,
                     double* dw, int bpc, hipStream_t st) {
  dim3 gr((unsigned)bpc, (unsigned)n_curves);
  if (fp64)
    hipLaunchKernelGGL((k_adjoint<H, double, double>), gr, dim3(kNT), 0, st,
                       (const cplx<double>*)zc, (const cplx<double>*)D, mom, g, curve0, eps,
                       (const double*)gin, (cplx<double>*)spec, dw, bpc);
  else
    hipLaunchKernelGGL((k_adjoint<H, float, float>), gr, dim3(kNT), 0, st,
                       (const cplx<float>*)zc, (const cplx<double>*)D, mom, g, curve0, eps,
                       (const float*)gin, (cplx<float>*)spec, dw, bpc);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint_solve(bool fp64, const void* zc, const void* D, const Moments* mom,
                                const Geom& g, int curve0, int n_curves, double eps_piv,
                                const void* grad_dchi2, void* spec, double* dW_part,
                                int blocks_per_curve, hipStream_t st) {
  switch (g.H) {
#define FCHI2_ADJ(h) \
  case h:            \
    return adjoint_h<h>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, grad_dchi2, spec, dW_part, blocks_per_curve, st);
    FCHI2_ADJ(1)
    FCHI2_ADJ(2)
    FCHI2_ADJ(3)
    FCHI2_ADJ(4)
    FCHI2_ADJ(5)
    FCHI2_ADJ(6)
    FCHI2_ADJ(7)
    FCHI2_ADJ(8)
#undef FCHI2_ADJ
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_gather(bool fp64, const double* t, const Moments* mom, const Geom& g,
                         int curve0, int n_curves, const void* grid, double* gq, double* gp,
                         int64_t max_n, hipStream_t st) {
  dim3 gr((unsigned)((max_n + kNT - 1) / kNT), (unsigned)n_curves);
  if (gr.x == 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL((k_gather<double>), gr, dim3(kNT), 0, st, t, mom, g, curve0,
                       (const cplx<double>*)grid, gq, gp);
  else
    hipLaunchKernelGGL((k_gather<float>), gr, dim3(kNT), 0, st, t, mom, g, curve0,
                       (const cplx<float>*)grid, gq, gp);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* x, const double* sigma, const Moments* mom,
                           const Geom& g, int curve0, int n_curves, const double* dW_part,
                           int blocks_per_curve, const double* gq, const double* gp,
                           double* grad_x, double* grad_sigma, double* scratch, int nch,
                           hipStream_t st) {
  (void)g;
  dim3 gr((unsigned)nch, (unsigned)n_curves);
  hipLaunchKernelGGL(k_fin_reduce, gr, dim3(kNT), 0, st, sigma, mom, curve0, dW_part,
                     blocks_per_curve, gp, nch, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize, gr, dim3(kNT), 0, st, x, sigma, mom, curve0,
                     (const double*)scratch, nch, gq, gp, grad_x, grad_sigma);
  return hipGetLastError();
}

}  // namespace fchi2
