// Polynomial detrending before the search.  The paper's reference
// implementation can remove a slow polynomial variation (up to t^3 in the
// Section 4 example) so that the search looks for periodic variation on top
// of it.  For every curve the weighted least-squares polynomial of degree D,
// minimising sum w (x - p(t))^2 with w = sigma^-2, is subtracted from x.
//
// The fit uses Legendre polynomials of u = 2 (t - T0) / span - 1 in [-1, 1]
// (the same space as powers of t, well conditioned): one block per curve
// accumulates the Gram matrix G_jl = sum w P_j P_l and b_j = sum w x P_j in
// FP64, solves G c = b by Cholesky (a pivot below 1e-12 of its diagonal is
// dropped: too few points or a zero span), and writes x - sum c_j P_j(u).
// Blocks have 256 threads, or 512 when the longest curve has 8192 points or
// more (a single long curve is then spread over more lanes of its one CU;
// 1024 would cap the registers at 128 and spill the small solve).
#include <cmath>
#include <cstdint>

#include "fchi2_internal.h"
#include "launch.h"

namespace fchi2 {

namespace {

template <int NB>
__device__ __forceinline__ void legendre(double u, double* P) {
  P[0] = 1.0;
  if constexpr (NB > 1) P[1] = u;
#pragma unroll
  for (int j = 1; j + 1 < NB; ++j)
    P[j + 1] = ((double)(2 * j + 1) * u * P[j] - (double)j * P[j - 1]) / (double)(j + 1);
}

template <int D, int kNT>
__global__ __launch_bounds__(kNT) void k_detrend(const double* __restrict__ t,
                                                 const double* __restrict__ x,
                                                 const double* __restrict__ sigma,
                                                 const int64_t* __restrict__ off,
                                                 double* __restrict__ x_out,
                                                 double* __restrict__ coef) {
  constexpr int NB = D + 1;
  constexpr int NS = NB * (NB + 1) / 2 + NB;  // Gram upper triangle, then b
  __shared__ double red[NS][kNT / 64];
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t a = off[c], e = off[c + 1];
  if (e <= a) return;
  const double T0 = t[a];
  const double span = t[e - 1] - T0;
  const double sc = span > 0.0 ? 2.0 / span : 0.0;

  double acc[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) acc[q] = 0.0;
  for (int64_t i = a + tid; i < e; i += kNT) {
    const double u = (t[i] - T0) * sc - 1.0;
    const double s = sigma[i];
    const double w = 1.0 / (s * s);
    double P[NB];
    legendre<NB>(u, P);
    int q = 0;
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int l = j; l < NB; ++l) acc[q++] += w * P[j] * P[l];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[q++] += w * x[i] * P[j];
  }
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    double v = acc[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((tid & 63) == 0) red[q][tid >> 6] = v;
  }
  __syncthreads();
  double S[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    double v = red[q][0];
#pragma unroll
    for (int wv = 1; wv < kNT / 64; ++wv) v += red[q][wv];
    S[q] = v;
  }
  // Every thread solves the small system (identical inputs, identical result).
  double G[NB][NB], b[NB];
  {
    int q = 0;
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int l = j; l < NB; ++l) {
        G[j][l] = S[q];
        G[l][j] = S[q];
        ++q;
      }
#pragma unroll
    for (int j = 0; j < NB; ++j) b[j] = S[q++];
  }
  double Lm[NB][NB], inv[NB], z[NB], cf[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double s = G[i][j];
#pragma unroll
      for (int l = 0; l < j; ++l) s -= Lm[i][l] * Lm[j][l];
      if (i == j) {
        if (s > 1e-12 * G[i][i] && s > 0.0) {
          Lm[i][i] = sqrt(s);
          inv[i] = 1.0 / Lm[i][i];
        } else {
          Lm[i][i] = 0.0;
          inv[i] = 0.0;
        }
      } else {
        Lm[i][j] = s * inv[j];
      }
    }
    double s = b[i];
#pragma unroll
    for (int l = 0; l < i; ++l) s -= Lm[i][l] * z[l];
    z[i] = s * inv[i];
  }
#pragma unroll
  for (int i = NB - 1; i >= 0; --i) {
    double s = z[i];
#pragma unroll
    for (int l = i + 1; l < NB; ++l) s -= Lm[l][i] * cf[l];
    cf[i] = s * inv[i];
  }
  if (coef && tid < NB) {
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (j == tid) coef[(int64_t)c * NB + j] = cf[j];
  }
  for (int64_t i = a + tid; i < e; i += kNT) {
    const double u = (t[i] - T0) * sc - 1.0;
    double P[NB];
    legendre<NB>(u, P);
    double p = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) p += cf[j] * P[j];
    x_out[i] = x[i] - p;
  }
}

template <int NT>
hipError_t detrend_nt(const double* t, const double* x, const double* sigma,
                      const int64_t* offsets, int n_curves, int degree, double* x_out,
                      double* coef, hipStream_t st) {
  dim3 gr((unsigned)n_curves);
  switch (degree) {
    case 0: hipLaunchKernelGGL((k_detrend<0, NT>), gr, dim3(NT), 0, st, t, x, sigma, offsets, x_out, coef); break;
    case 1: hipLaunchKernelGGL((k_detrend<1, NT>), gr, dim3(NT), 0, st, t, x, sigma, offsets, x_out, coef); break;
    case 2: hipLaunchKernelGGL((k_detrend<2, NT>), gr, dim3(NT), 0, st, t, x, sigma, offsets, x_out, coef); break;
    case 3: hipLaunchKernelGGL((k_detrend<3, NT>), gr, dim3(NT), 0, st, t, x, sigma, offsets, x_out, coef); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_detrend(const double* t, const double* x, const double* sigma,
                          const int64_t* offsets, int n_curves, int degree, int64_t max_n,
                          double* x_out, double* coef, hipStream_t st) {
  if (max_n >= 8192)
    return detrend_nt<512>(t, x, sigma, offsets, n_curves, degree, x_out, coef, st);
  return detrend_nt<256>(t, x, sigma, offsets, n_curves, degree, x_out, coef, st);
}

}  // namespace fchi2
