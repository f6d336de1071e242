// Best frequencies (Section 3e: the bin with the largest Delta chi2 is the
// best fit; candidates near other large local maxima are kept for finer
// study).  Selects, per curve, the K largest strict local maxima
// D[k] > D[k-1], D[k] >= D[k+1] of one Delta chi2 row over k in
// [k_lo, n_freq - 2], ordered by value with ties to the lower k.
// Two deterministic phases: per block of bins, K rounds of block-wide
// arg-max; then the same selection over the per-block winners.
#include <cmath>

#include "fchi2_internal.h"
#include "launch.h"

namespace fchi2 {

namespace {

constexpr int kNT = 256;
constexpr int kPerThread = 64;
constexpr int64_t kBlockBins = (int64_t)kNT * kPerThread;

struct Cand {
  double v;
  int64_t k;
};

__device__ __forceinline__ bool better(double v, int64_t k, double bv, int64_t bk) {
  if (bk < 0) return k >= 0;
  if (k < 0) return false;
  return (v > bv) || (v == bv && k < bk);
}

__device__ Cand block_best(double v, int64_t k, double* rv, int64_t* rk) {
  const int tid = threadIdx.x;
  rv[tid] = v;
  rk[tid] = k;
  __syncthreads();
  for (int s = kNT / 2; s > 0; s >>= 1) {
    if (tid < s && better(rv[tid + s], rk[tid + s], rv[tid], rk[tid])) {
      rv[tid] = rv[tid + s];
      rk[tid] = rk[tid + s];
    }
    __syncthreads();
  }
  Cand c{rv[0], rk[0]};
  __syncthreads();
  return c;
}

template <typename O>
__global__ __launch_bounds__(kNT) void k_peaks_block(const O* __restrict__ dchi2, int64_t nf,
                                                     int H, int hrow, int64_t k_lo, int K,
                                                     Cand* __restrict__ part, int nblk) {
  __shared__ double rv[kNT];
  __shared__ int64_t rk[kNT];
  const int c = blockIdx.y;
  const int tid = threadIdx.x;
  const O* row = dchi2 + ((int64_t)c * H + hrow) * nf;
  const int64_t k0 = (int64_t)blockIdx.x * kBlockBins + (int64_t)tid * kPerThread;
  uint64_t is_max = 0;
  for (int u = 0; u < kPerThread; ++u) {
    const int64_t k = k0 + u;
    if (k < k_lo || k > nf - 2) continue;
    const double v = (double)row[k];
    if (v > (double)row[k - 1] && v >= (double)row[k + 1]) is_max |= (uint64_t)1 << u;
  }
  Cand* out = part + ((int64_t)c * nblk + blockIdx.x) * K;
  for (int r = 0; r < K; ++r) {
    double bv = 0.0;
    int64_t bk = -1;
    uint64_t m = is_max;
    while (m) {
      const int u = __ffsll((long long)m) - 1;
      m &= m - 1;
      const double v = (double)row[k0 + u];
      if (better(v, k0 + u, bv, bk)) {
        bv = v;
        bk = k0 + u;
      }
    }
    const Cand w = block_best(bv, bk, rv, rk);
    if (w.k >= 0 && w.k >= k0 && w.k < k0 + kPerThread) is_max &= ~((uint64_t)1 << (w.k - k0));
    if (tid == 0) out[r] = w;
  }
}

__global__ __launch_bounds__(kNT) void k_peaks_merge(const Cand* __restrict__ part, int nblk,
                                                     int K, int64_t* __restrict__ out_idx) {
  __shared__ double rv[kNT];
  __shared__ int64_t rk[kNT];
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const Cand* pc = part + (int64_t)c * nblk * K;
  const int n = nblk * K;
  int64_t last_k = -1;
  double last_v = INFINITY;
  for (int r = 0; r < K; ++r) {
    // Best candidate strictly after the previous winner in (value desc, k asc).
    double bv = 0.0;
    int64_t bk = -1;
    for (int q = tid; q < n; q += kNT) {
      const Cand cd = pc[q];
      if (cd.k < 0) continue;
      const bool after = (cd.v < last_v) || (cd.v == last_v && cd.k > last_k);
      if (after && better(cd.v, cd.k, bv, bk)) {
        bv = cd.v;
        bk = cd.k;
      }
    }
    const Cand w = block_best(bv, bk, rv, rk);
    if (tid == 0) out_idx[(int64_t)c * K + r] = w.k;
    if (w.k >= 0) {
      last_k = w.k;
      last_v = w.v;
    } else {
      last_k = INT64_MAX;
      last_v = -INFINITY;
    }
  }
}

}  // namespace

size_t peaks_scratch_bytes(int64_t n_freq, int n_curves, int K) {
  const int64_t nblk = (n_freq + kBlockBins - 1) / kBlockBins;
  return (size_t)nblk * (size_t)n_curves * (size_t)K * sizeof(Cand);
}

hipError_t launch_peaks(bool fp64, const void* dchi2, int64_t n_freq, int H, int hrow,
                        int n_curves, int64_t k_lo, int K, void* scratch, int64_t* out_idx,
                        hipStream_t st) {
  const int nblk = (int)((n_freq + kBlockBins - 1) / kBlockBins);
  dim3 g1((unsigned)nblk, (unsigned)n_curves);
  if (fp64)
    hipLaunchKernelGGL((k_peaks_block<double>), g1, dim3(kNT), 0, st, (const double*)dchi2,
                       n_freq, H, hrow, k_lo, K, (Cand*)scratch, nblk);
  else
    hipLaunchKernelGGL((k_peaks_block<float>), g1, dim3(kNT), 0, st, (const float*)dchi2, n_freq,
                       H, hrow, k_lo, K, (Cand*)scratch, nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_peaks_merge, dim3(n_curves), dim3(kNT), 0, st, (const Cand*)scratch, nblk,
                     K, out_idx);
  return hipGetLastError();
}

}  // namespace fchi2
