// Significance epilogue of the search: per curve, the K candidate
// frequencies with the smallest false-alarm measure, without writing the
// Delta chi2 rows to memory.
//
// Section 3e: the best fit is the bin with the largest Delta chi2; its
// significance counts the trials searched so far (proportional to f, hence to
// the bin index k) times the upper tail of the chi2 distribution with 2H'
// degrees of freedom (the model's extra parameters), and the value to
// minimise is p(f) = k Q(Delta chi2 | 2H').  For an even number of degrees of
// freedom the tail has the closed form
//     Q(D | 2H') = exp(-D/2) sum_{j < H'} (D/2)^j / j!,
// evaluated here in logarithms so that no tail underflows.  Section 3e also
// defines the adjusted reduction Delta chi2 * N_dof / chi2_best, chi2_best
// being the minimum chi2 over the searched bins and N_dof = n - 2H' - 1
// (NaN when N_dof <= 0).
//
// Candidates are the strict local maxima D[k] > D[k-1], D[k] >= D[k+1] of
// row hrow over eligible bins (k >= k_lo, k >= 1, f_k >= 1/span, k <= n_freq-2),
// ranked by ln p ascending with ties to the lower k.  chi2_best uses the
// largest Delta chi2 of row hrow over all eligible bins (k <= n_freq - 1).
// The Delta chi2 values ranked are those the full search writes (rounded to
// the output type), so both paths select the same bins.
//
// Phase 1 (fused with the per-bin solve): one block of 256 threads solves
// 1024 consecutive bins, the first and last being halo bins whose values only
// serve the neighbour test, keeps all H rows in LDS, sorts its 1022 owned
// bins' keys (ln p, k) with a bitonic network and writes its K best in order.
// Phase 2: one block per curve merges the sorted per-block lists.
#include <cmath>
#include <cstdint>

#include "fchi2_internal.h"
#include "launch.h"
#include "solve_bin.h"

namespace fchi2 {

namespace {

using namespace solve_detail;

constexpr int kNT = 256;
constexpr int kBPT = 4;
constexpr int kSpan = kNT * kBPT;  // bins solved per block
constexpr int kOwn = kSpan - 2;    // bins owned per block (halo on both sides)
constexpr uint8_t kNoBin = 0xFF;   // LDS marker: bin outside 0..n_freq-1

// ln Q(D | 2 hp): log of the chi2 upper tail with an even number of degrees
// of freedom.  The partial exponential sum is evaluated by Horner's rule from
// the highest term down (all terms are positive, so nothing cancels) and
// log1p keeps the small-D end accurate.
__device__ __forceinline__ double log_q_even(double d, int hp) {
  const double u = 0.5 * (d > 0.0 ? d : 0.0);
  double r = 1.0;
  for (int j = hp - 1; j >= 2; --j) r = 1.0 + r * (u / (double)j);
  const double tail = hp > 1 ? u * r : 0.0;
  return -u + log1p(tail);
}

// (score, k) ordering: smaller score first, ties to the lower k.
__device__ __forceinline__ bool key_less(double sa, int ia, double sb, int ib) {
  return (sa < sb) || (sa == sb && ia < ib);
}

template <int H, typename R, typename O>
__global__ __launch_bounds__(kNT) void k_solve_top(
    const cplx<R>* __restrict__ zc, const cplx<double>* __restrict__ D,
    const Moments* __restrict__ mom, Geom g, int curve0, double eps, int hrow, int64_t k_lo,
    int K, int nblk, double* __restrict__ rs, int64_t* __restrict__ rk,
    uint8_t* __restrict__ rf, double* __restrict__ rd, double* __restrict__ bmax) {
  __shared__ O s_d[H][kSpan];
  __shared__ uint8_t s_fl[kSpan];
  __shared__ double s_ks[kSpan];
  __shared__ int s_ki[kSpan];
  __shared__ double s_red[kNT / 64];

  const int tid = threadIdx.x;
  const int cw = blockIdx.y;
  const Moments mo = mom[curve0 + cw];
  const int64_t nf = g.n_freq;
  const int64_t B0 = (int64_t)blockIdx.x * kOwn;  // first owned bin; s_* index i is bin B0-1+i

#pragma unroll 1
  for (int r = 0; r < kBPT; ++r) {
    const int i = r * kNT + tid;
    const int64_t k = B0 - 1 + i;
    if (k >= 0 && k < nf) {
      O d[H];
      const uint8_t fl = solve_bin<H, R, O>(zc, D, mo, g, cw, k, eps, d);
#pragma unroll
      for (int h = 0; h < H; ++h) s_d[h][i] = d[h];
      s_fl[i] = fl;
    } else {
      s_fl[i] = kNoBin;
    }
  }
  __syncthreads();

  const int hp = hrow + 1;
  const int64_t k_first = k_lo > 1 ? k_lo : 1;
  double vmax = -INFINITY;
#pragma unroll
  for (int r = 0; r < kBPT; ++r) {
    const int i = r * kNT + tid;
    const int64_t k = B0 - 1 + i;
    double score = INFINITY;
    const bool owned = i >= 1 && i <= kOwn && k < nf;
    if (owned) {
      const uint8_t fl = s_fl[i];
      const bool eligible = k >= k_first && !(fl & (BF_LOW_F | BF_DC | 0xF8u));
      if (eligible) {
        const double v = (double)s_d[hrow][i];
        if (v > vmax) vmax = v;  // NaN never raises the maximum
        if (k <= nf - 2 && v > (double)s_d[hrow][i - 1] && v >= (double)s_d[hrow][i + 1])
          score = log((double)k) + log_q_even(v, hp);
      }
    }
    s_ks[i] = score;
    s_ki[i] = i;
  }
  // Block maximum of the eligible Delta chi2 (for chi2_best).
  for (int o = 32; o > 0; o >>= 1) {
    const double other = __shfl_xor(vmax, o);
    vmax = other > vmax ? other : vmax;
  }
  if ((tid & 63) == 0) s_red[tid >> 6] = vmax;
  __syncthreads();

  // Bitonic sort of the kSpan keys, ascending.
  for (int size = 2; size <= kSpan; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int p = tid; p < kSpan / 2; p += kNT) {  // pair index
        const int a = ((p & ~(stride - 1)) << 1) | (p & (stride - 1));
        const int b = a + stride;
        const bool up = (a & size) == 0;
        const double sa = s_ks[a], sb = s_ks[b];
        const int ia = s_ki[a], ib = s_ki[b];
        if (key_less(sb, ib, sa, ia) == up) {
          s_ks[a] = sb;
          s_ki[a] = ib;
          s_ks[b] = sa;
          s_ki[b] = ia;
        }
      }
      __syncthreads();
    }
  }

  const int64_t base = ((int64_t)cw * nblk + blockIdx.x) * K;
  if (tid < K) {
    const double sc = s_ks[tid];
    const int i = s_ki[tid];
    const bool ok = sc < INFINITY;
    rs[base + tid] = ok ? sc : INFINITY;
    rk[base + tid] = ok ? B0 - 1 + i : -1;
    rf[base + tid] = ok ? s_fl[i] : 0;
#pragma unroll
    for (int h = 0; h < H; ++h) rd[(base + tid) * H + h] = ok ? (double)s_d[h][i] : (double)NAN;
  }
  if (tid == 0) {
    double m = s_red[0];
    for (int w = 1; w < kNT / 64; ++w) m = s_red[w] > m ? s_red[w] : m;
    bmax[(int64_t)cw * nblk + blockIdx.x] = m;
  }
}

// Merge of the per-block sorted lists of one curve: K rounds, each taking the
// smallest head key; the owner of the winning list advances its head.
__global__ __launch_bounds__(kNT) void k_top_merge(
    const double* __restrict__ rs, const int64_t* __restrict__ rk,
    const uint8_t* __restrict__ rf, const double* __restrict__ rd,
    const double* __restrict__ bmax, const Moments* __restrict__ mom, int curve0, int nblk,
    int K, int H, int hrow, int64_t* __restrict__ out_idx, double* __restrict__ out_logp,
    double* __restrict__ out_dchi2, double* __restrict__ out_adj,
    uint8_t* __restrict__ out_flags, double* __restrict__ out_best,
    uint8_t* __restrict__ out_cflags) {
  extern __shared__ uint8_t s_head[];  // [nblk] current head of each list
  __shared__ double r_s[kNT];
  __shared__ int64_t r_k[kNT];
  __shared__ int r_l[kNT];
  __shared__ int64_t s_win[64];  // winning record index per round (-1: none)
  __shared__ double s_mx[kNT];

  const int tid = threadIdx.x;
  const int cw = blockIdx.x;
  const int c = curve0 + cw;
  const Moments mo = mom[c];
  const int64_t lbase = (int64_t)cw * nblk;

  double mx = -INFINITY;
  for (int l = tid; l < nblk; l += kNT) {
    s_head[l] = 0;
    const double v = bmax[lbase + l];
    mx = v > mx ? v : mx;
  }
  s_mx[tid] = mx;
  __syncthreads();
  for (int s = kNT / 2; s > 0; s >>= 1) {
    if (tid < s && s_mx[tid + s] > s_mx[tid]) s_mx[tid] = s_mx[tid + s];
    __syncthreads();
  }
  const double vmax = s_mx[0];

  for (int r = 0; r < K; ++r) {
    double bs = INFINITY;
    int64_t bk = INT64_MAX;
    int bl = -1;
    for (int l = tid; l < nblk; l += kNT) {
      const int h = s_head[l];
      if (h >= K) continue;
      const int64_t q = (lbase + l) * K + h;
      const int64_t k = rk[q];
      if (k < 0) continue;
      const double s = rs[q];
      if (s < bs || (s == bs && k < bk)) {
        bs = s;
        bk = k;
        bl = l;
      }
    }
    r_s[tid] = bs;
    r_k[tid] = bk;
    r_l[tid] = bl;
    __syncthreads();
    for (int s = kNT / 2; s > 0; s >>= 1) {
      if (tid < s) {
        const double os = r_s[tid + s];
        const int64_t ok = r_k[tid + s];
        if (r_l[tid + s] >= 0 && (r_l[tid] < 0 || os < r_s[tid] || (os == r_s[tid] && ok < r_k[tid]))) {
          r_s[tid] = os;
          r_k[tid] = ok;
          r_l[tid] = r_l[tid + s];
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      const int wl = r_l[0];
      if (wl >= 0) {
        s_win[r] = (lbase + wl) * K + s_head[wl];
        s_head[wl] = (uint8_t)(s_head[wl] + 1);
      } else {
        s_win[r] = -1;
      }
    }
    __syncthreads();
  }

  const bool fatal = (mo.flags & kCurveFatal) != 0;
  const double best = (fatal || !(vmax > -INFINITY)) ? (double)NAN : mo.chi2_0 - vmax;
  const double ndof = (double)(mo.n - 2 * (hrow + 1) - 1);
  if (tid == 0 && out_best) out_best[c] = best;
  if (tid == 0 && out_cflags) out_cflags[c] = (uint8_t)(mo.flags & 0xF8u);
  if (tid < K) {
    const int64_t q = s_win[tid];
    const int64_t o = (int64_t)c * K + tid;
    if (q >= 0) {
      out_idx[o] = rk[q];
      out_logp[o] = rs[q];
      const double v = rd[q * H + hrow];
      if (out_adj) out_adj[o] = ndof > 0.0 ? v * ndof / best : (double)NAN;
      if (out_flags) out_flags[o] = rf[q];
      if (out_dchi2)
        for (int h = 0; h < H; ++h) out_dchi2[o * H + h] = rd[q * H + h];
    } else {
      out_idx[o] = -1;
      out_logp[o] = (double)NAN;
      if (out_adj) out_adj[o] = (double)NAN;
      if (out_flags) out_flags[o] = 0;
      if (out_dchi2)
        for (int h = 0; h < H; ++h) out_dchi2[o * H + h] = (double)NAN;
    }
  }
}

template <int H>
hipError_t solve_top_h(bool fp64, const void* zc, const void* D, const Moments* mom,
                       const Geom& g, int curve0, int n_curves, double eps, int hrow,
                       int64_t k_lo, int K, int nblk, const TopScratch& sc, hipStream_t st) {
  dim3 gr((unsigned)nblk, (unsigned)n_curves);
  if (fp64)
    hipLaunchKernelGGL((k_solve_top<H, double, double>), gr, dim3(kNT), 0, st,
                       (const cplx<double>*)zc, (const cplx<double>*)D, mom, g, curve0, eps, hrow,
                       k_lo, K, nblk, sc.score, sc.k, sc.flag, sc.d, sc.bmax);
  else
    hipLaunchKernelGGL((k_solve_top<H, float, float>), gr, dim3(kNT), 0, st,
                       (const cplx<float>*)zc, (const cplx<double>*)D, mom, g, curve0, eps, hrow,
                       k_lo, K, nblk, sc.score, sc.k, sc.flag, sc.d, sc.bmax);
  return hipGetLastError();
}

}  // namespace

int top_blocks(int64_t n_freq) { return (int)((n_freq + kOwn - 1) / kOwn); }

size_t top_scratch_bytes(int64_t n_freq, int H, int n_curves, int K) {
  const size_t rec = (size_t)top_blocks(n_freq) * (size_t)n_curves;
  auto a = [](size_t v) { return (v + 255) & ~(size_t)255; };
  return a(rec * K * sizeof(double)) + a(rec * K * sizeof(int64_t)) + a(rec * K) +
         a(rec * K * H * sizeof(double)) + a(rec * sizeof(double));
}

TopScratch top_scratch_carve(void* base, int64_t n_freq, int H, int n_curves, int K) {
  const size_t rec = (size_t)top_blocks(n_freq) * (size_t)n_curves;
  auto a = [](size_t v) { return (v + 255) & ~(size_t)255; };
  char* p = (char*)base;
  TopScratch s;
  s.score = (double*)p;
  p += a(rec * K * sizeof(double));
  s.k = (int64_t*)p;
  p += a(rec * K * sizeof(int64_t));
  s.flag = (uint8_t*)p;
  p += a(rec * K);
  s.d = (double*)p;
  p += a(rec * K * H * sizeof(double));
  s.bmax = (double*)p;
  return s;
}

hipError_t launch_solve_top(bool fp64, const void* zc, const void* D, const Moments* mom,
                            const Geom& g, int curve0, int n_curves, double eps_piv, int hrow,
                            int64_t k_lo, int K, const TopScratch& sc, hipStream_t st) {
  const int nblk = top_blocks(g.n_freq);
  switch (g.H) {
#define FCHI2_TOP_CASE(h) \
  case h: return solve_top_h<h>(fp64, zc, D, mom, g, curve0, n_curves, eps_piv, hrow, k_lo, K, nblk, sc, st);
    FCHI2_TOP_CASE(1)
    FCHI2_TOP_CASE(2)
    FCHI2_TOP_CASE(3)
    FCHI2_TOP_CASE(4)
    FCHI2_TOP_CASE(5)
    FCHI2_TOP_CASE(6)
    FCHI2_TOP_CASE(7)
    FCHI2_TOP_CASE(8)
#undef FCHI2_TOP_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_top_merge(const Moments* mom, const Geom& g, int curve0, int n_curves,
                            int hrow, int K, const TopScratch& sc, const TopOut& out,
                            hipStream_t st) {
  const int nblk = top_blocks(g.n_freq);
  hipLaunchKernelGGL(k_top_merge, dim3((unsigned)n_curves), dim3(kNT), (size_t)nblk, st,
                     (const double*)sc.score, (const int64_t*)sc.k, (const uint8_t*)sc.flag,
                     (const double*)sc.d, (const double*)sc.bmax, mom, curve0, nblk, K, g.H, hrow,
                     out.idx, out.log_p, out.dchi2, out.dchi2_adj, out.flags, out.chi2_best,
                     out.curve_flags);
  return hipGetLastError();
}

}  // namespace fchi2
