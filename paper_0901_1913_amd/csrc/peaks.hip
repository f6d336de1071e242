// Best frequencies (Section 3e: the bin with the largest Delta chi2 is the
// best fit; candidates near other large local maxima are kept for finer
// study).  Selects, per curve, the K largest strict local maxima
// D[k] > D[k-1], D[k] >= D[k+1] of one Delta chi2 row over k in
// [k_lo, n_freq - 2], ordered by value with ties to the lower k.
// Two deterministic phases: per block of bins, K rounds of a block-wide
// arg-max; then the same selection over the per-block winners.  In both,
// every thread keeps the best of its own remaining candidates; a round is a
// wave arg-max by lane shuffles, then the four wave winners compared through
// LDS (two barriers), and only the thread that owned the winner looks for
// its next best.
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

// (v, k) before (bv, bk) in the selection order: larger value first, ties to
// the lower bin; k < 0 marks no candidate and comes last.
__device__ __forceinline__ bool better(double v, int64_t k, double bv, int64_t bk) {
  if (bk < 0) return k >= 0;
  if (k < 0) return false;
  return (v > bv) || (v == bv && k < bk);
}

// The workgroup's best of the threads' (v, k), returned to every thread.
// s_v / s_k: LDS of one entry per wave.
__device__ __forceinline__ Cand block_best(double v, int64_t k, double* s_v, int64_t* s_k) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o);
    const int64_t ok = __shfl_xor(k, o);
    if (better(ov, ok, v, k)) {
      v = ov;
      k = ok;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    s_v[wv] = v;
    s_k[wv] = k;
  }
  __syncthreads();
  Cand c{s_v[0], s_k[0]};
#pragma unroll
  for (int w = 1; w < kNT / 64; ++w)
    if (better(s_v[w], s_k[w], c.v, c.k)) c = Cand{s_v[w], s_k[w]};
  __syncthreads();  // s_v / s_k are rewritten by the next round
  return c;
}

// Block b of a curve's row: bins B0 + u * 256 + tid (u < 64) of thread tid,
// so that every load of the local-maximum test is coalesced.
template <typename O>
__global__ __launch_bounds__(kNT) void k_peaks_block(const O* __restrict__ dchi2, int64_t nf,
                                                     int H, int hrow, int64_t k_lo, int K,
                                                     Cand* __restrict__ part, int nblk) {
  __shared__ double s_v[kNT / 64];
  __shared__ int64_t s_k[kNT / 64];
  const int c = blockIdx.y;
  const int tid = threadIdx.x;
  const O* row = dchi2 + ((int64_t)c * H + hrow) * nf;
  const int64_t B0 = (int64_t)blockIdx.x * kBlockBins + tid;  // this thread's first bin
  uint64_t is_max = 0;
  for (int u = 0; u < kPerThread; ++u) {
    const int64_t k = B0 + (int64_t)u * kNT;
    if (k < k_lo || k > nf - 2) continue;
    const double v = (double)row[k];
    if (v > (double)row[k - 1] && v >= (double)row[k + 1]) is_max |= (uint64_t)1 << u;
  }
  // The thread's best remaining candidate.
  auto own_best = [&](double& bv, int64_t& bk) {
    bv = 0.0;
    bk = -1;
    uint64_t m = is_max;
    while (m) {
      const int u = __ffsll((long long)m) - 1;
      m &= m - 1;
      const int64_t k = B0 + (int64_t)u * kNT;
      const double v = (double)row[k];
      if (better(v, k, bv, bk)) {
        bv = v;
        bk = k;
      }
    }
  };
  double bv;
  int64_t bk;
  own_best(bv, bk);
  Cand* out = part + ((int64_t)c * nblk + blockIdx.x) * K;
  for (int r = 0; r < K; ++r) {
    const Cand w = block_best(bv, bk, s_v, s_k);
    if (tid == 0) out[r] = w;
    if (w.k >= 0 && w.k == bk) {  // this thread held the winner
      is_max &= ~((uint64_t)1 << ((w.k - B0) / kNT));
      own_best(bv, bk);
    }
  }
}

// Merge of the per-block lists of a curve.  Each block's list is in
// selection order, so the merge is a tournament over list heads: thread tid
// owns lists tid + j * 256 (j < kListsPerThread: n_freq <= 2^24 gives at
// most 1024 blocks), offers the best of its heads, and the owner of a round's
// winner advances that list.
constexpr int kListsPerThread = 4;

__global__ __launch_bounds__(kNT) void k_peaks_merge(const Cand* __restrict__ part, int nblk,
                                                     int K, int64_t* __restrict__ out_idx) {
  __shared__ double s_v[kNT / 64];
  __shared__ int64_t s_k[kNT / 64];
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const Cand* pc = part + (int64_t)c * nblk * K;
  int head[kListsPerThread];
#pragma unroll
  for (int j = 0; j < kListsPerThread; ++j) head[j] = 0;
  auto own_best = [&](double& bv, int64_t& bk) {
    bv = 0.0;
    bk = -1;
#pragma unroll
    for (int j = 0; j < kListsPerThread; ++j) {
      const int l = tid + j * kNT;
      if (l >= nblk || head[j] >= K) continue;
      const Cand cd = pc[(int64_t)l * K + head[j]];
      if (better(cd.v, cd.k, bv, bk)) {
        bv = cd.v;
        bk = cd.k;
      }
    }
  };
  double bv;
  int64_t bk;
  own_best(bv, bk);
  for (int r = 0; r < K; ++r) {
    const Cand w = block_best(bv, bk, s_v, s_k);
    if (tid == 0) out_idx[(int64_t)c * K + r] = w.k;
    if (w.k >= 0 && w.k == bk) {  // advance the list whose head won
#pragma unroll
      for (int j = 0; j < kListsPerThread; ++j) {
        const int l = tid + j * kNT;
        if (l < nblk && head[j] < K && pc[(int64_t)l * K + head[j]].k == w.k) {
          ++head[j];
          break;
        }
      }
      own_best(bv, bk);
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
  if (nblk > kListsPerThread * kNT) return hipErrorInvalidValue;  // n_freq > 2^24
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
