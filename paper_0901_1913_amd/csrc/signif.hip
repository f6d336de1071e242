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
// row hrow over eligible bins (k >= k_lo, k >= 1, f_k >= 1/span, k <= n_freq-2;
// band plans: every k >= k_lo, with one bin beyond each end solved as well),
// ranked by ln p ascending with ties to the lower k.  chi2_best uses the
// largest Delta chi2 of row hrow over all eligible bins (k <= n_freq - 1).
// The Delta chi2 values ranked are those the full search writes (rounded to
// the output type), so both paths select the same bins.
//
// Phase 1 (fused with the per-bin solve): one block of 256 threads solves
// 1024 consecutive bins, the first and last being halo bins whose values only
// serve the neighbour test, keeps all H rows in LDS and selects the K best of
// its 1022 owned bins: ln p is evaluated once per candidate on consecutive
// lanes, each thread keeps its four keys (ln p, k) sorted, each wave runs a
// tournament (K rounds of a wave arg-min over the threads' heads by DPP lane
// permutations, the owner of the winner advancing), and the four sorted wave
// lists are merged by rank.  The K winners are written in order.  Phase 2:
// the sorted per-block lists are merged in groups of up to 256 (one list per
// thread, the same wave tournaments and rank merge), and, where a curve has
// more than one group, the group lists once more, which gives the final K.
#include <cmath>
#include <type_traits>
#include <cstdint>

#include "fchi2_internal.h"
#include "launch.h"
#include "solve_bin.h"
#include "topk_keys.h"
#include "wave_min.h"

namespace fchi2 {

namespace {

using namespace solve_detail;

constexpr int kNT = 256;
constexpr int kBPT = 4;
constexpr int kSpan = kNT * kBPT;  // bins solved per block
constexpr int kOwn = kSpan - 2;    // bins owned per block (halo on both sides)
constexpr uint8_t kNoBin = 0xFF;   // LDS marker: bin outside 0..n_freq-1

template <int H, typename R, typename O, bool BAND>
__global__ __launch_bounds__(kNT) void k_solve_top(
    const cplx<R>* __restrict__ zc, const cplx<double>* __restrict__ D,
    const Moments* __restrict__ mom, Geom g, int curve0, double eps, int hrow, int64_t k_lo,
    int K, int nblk, double* __restrict__ rs, int64_t* __restrict__ rk,
    uint8_t* __restrict__ rf, double* __restrict__ rd, double* __restrict__ bmax) {
  __shared__ O s_d[H][kSpan];
  __shared__ uint8_t s_fl[kSpan];
  __shared__ double s_red[kNT / 64];
  __shared__ double w_s[kNT / 64][64];  // each wave's K best keys, in order
  __shared__ int w_i[kNT / 64][64];
  __shared__ int s_win[64];
  __shared__ int c_slot[kNT / 64][kNT];  // each wave's candidate slots
  __shared__ double s_sc[kSpan];         // ln p of the candidates

  const int tid = threadIdx.x;
  const int cw = blockIdx.y;
  const Moments mo = mom[curve0 + cw];
  const int64_t nf = g.n_freq;
  const int64_t B0 = (int64_t)blockIdx.x * kOwn;  // first owned bin; s_* index i is bin B0-1+i

#pragma unroll 1
  for (int r = 0; r < kBPT; ++r) {
    const int i = r * kNT + tid;
    const int64_t k = B0 - 1 + i;
    // A band plan also solves the bins just outside its band (offsets
    // -n_freq/2 - 1 and n_freq/2 from the centre, within the |o| < n_freq its
    // spectra hold), so that its first and last bins can be ranked too.
    if (BAND ? (k >= -1 && k <= nf) : (k >= 0 && k < nf)) {
      O d[H];
      const uint8_t fl = solve_bin<H, R, O, BAND>(zc, D, mo, g, cw, k, eps, d);
#pragma unroll
      for (int h = 0; h < H; ++h) s_d[h][i] = d[h];
      s_fl[i] = fl;
    } else {
      s_fl[i] = kNoBin;
    }
  }
  __syncthreads();

  const int hp = hrow + 1;
  // Band plans: bin 0 is bin k0 > 0 of the search.
  const int64_t k_first = k_lo > (BAND ? 0 : 1) ? k_lo : (BAND ? 0 : 1);
  const int64_t k_last = BAND ? nf - 1 : nf - 2;  // needs the bin after it
  const int lane = tid & 63, wv = tid >> 6;
  double vmax = -INFINITY;
  unsigned cand = 0;  // bit r: slot r * kNT + tid is a candidate
#pragma unroll
  for (int r = 0; r < kBPT; ++r) {
    const int i = r * kNT + tid;
    const int64_t k = B0 - 1 + i;
    const bool owned = i >= 1 && i <= kOwn && k < nf;
    if (owned) {
      const uint8_t fl = s_fl[i];
      const bool eligible = k >= k_first && !(fl & (BF_LOW_F | BF_DC | 0xF8u));
      if (eligible) {
        const double v = (double)s_d[hrow][i];
        if (v > vmax) vmax = v;  // NaN never raises the maximum
        if (k <= k_last && v > (double)s_d[hrow][i - 1] && v >= (double)s_d[hrow][i + 1])
          cand |= 1u << r;
      }
    }
  }
  // ln p of the wave's candidates (about a third of the bins), evaluated by
  // consecutive lanes: the wave's candidate slots are listed first, so the
  // logarithms run on full waves instead of on every lane for every slot.
  int ncand = 0;
#pragma unroll
  for (int r = 0; r < kBPT; ++r) {
    const bool c = (cand >> r) & 1u;
    const uint64_t m = __ballot(c);
    const int below = (int)__builtin_amdgcn_mbcnt_hi(
        (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (c) c_slot[wv][ncand + below] = r * kNT + tid;
    ncand += __popcll(m);
  }
  __syncthreads();
  for (int j = lane; j < ncand; j += 64) {
    const int i = c_slot[wv][j];
    // ln of the bin index of the search (a band plan's rows start at k0)
    const int64_t kg = (BAND ? g.k0 : 0) + B0 - 1 + i;
    s_sc[i] = rank_score(log((double)kg) + log_q_even((double)s_d[hrow][i], hp));
  }
  __syncthreads();
  double ks[kBPT];
  int ki[kBPT];
#pragma unroll
  for (int r = 0; r < kBPT; ++r) {
    const int i = r * kNT + tid;
    ks[r] = ((cand >> r) & 1u) ? s_sc[i] : INFINITY;
    ki[r] = i;
  }
  // Block maximum of the eligible Delta chi2 (for chi2_best).
  for (int o = 32; o > 0; o >>= 1) {
    const double other = __shfl_xor(vmax, o);
    vmax = other > vmax ? other : vmax;
  }
  if ((tid & 63) == 0) s_red[tid >> 6] = vmax;

  // Sort the thread's own keys (compile-time network).
#pragma unroll
  for (int a = 0; a < kBPT; ++a) {
#pragma unroll
    for (int b = kBPT - 1; b > a; --b) {
      if (key_less(ks[b], ki[b], ks[b - 1], ki[b - 1])) {
        const double ts = ks[b];
        const int ti = ki[b];
        ks[b] = ks[b - 1];
        ki[b] = ki[b - 1];
        ks[b - 1] = ts;
        ki[b - 1] = ti;
      }
    }
  }
  // Tournament inside each wave: K rounds of wave arg-min over the threads'
  // heads (DPP permutations, no barrier); lane r keeps the r-th winner and
  // the winner's owner advances.  Every key of a wave is held by that wave.
  int head = 0;
  double my_s = INFINITY;
  int my_i = INT_MAX;
  for (int r = 0; r < K; ++r) {
    double sv = INFINITY;
    int si = INT_MAX;
#pragma unroll
    for (int q = 0; q < kBPT; ++q) {
      if (q == head) {
        sv = ks[q];
        si = ki[q];
      }
    }
    wave_min_key(sv, si);
    if (!(sv < INFINITY)) break;  // the same decision in every lane of the wave
    if (lane == r) {
      my_s = sv;
      my_i = si;
    }
    if ((si & (kNT - 1)) == tid) ++head;
  }
  if (lane < K) {
    w_s[wv][lane] = my_s;
    w_i[wv][lane] = my_i;
  }
  if (tid < K) s_win[tid] = -1;  // a slot no rank fills stays marked empty
  __syncthreads();
  // Merge of the sorted wave lists: a finite key's rank is its position in its
  // list plus the number of smaller keys in the other lists (keys are
  // distinct, so ranks are); the K first ranks are the block's K best.
  bool wrote = false;
  if (tid < (kNT / 64) * K) {
    const int L = tid / K, pos = tid - L * K;
    const double sv = w_s[L][pos];
    const int si = w_i[L][pos];
    if (sv < INFINITY) {
      const int rank = merged_rank(&w_s[0][0], &w_i[0][0], 64, kNT / 64, K, L, pos);
      if (rank < K) {
        s_win[rank] = si;
        wrote = true;
      }
    }
  }
  const int rounds = __syncthreads_count(wrote);

  const int64_t base = ((int64_t)cw * nblk + blockIdx.x) * K;
  if (tid < K) {
    const bool ok = tid < rounds && s_win[tid] >= 0;
    const int i = ok ? s_win[tid] : 0;
    rs[base + tid] = ok ? s_sc[i] : INFINITY;
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

// One merge step: group g of curve slot cw takes up to 256 sorted lists (one
// per thread; list l = g * 256 + tid of the nl lists of the curve) and keeps
// their K smallest keys (ln p, k), in order: a tournament inside each wave as
// in the solve kernel (each thread holds its list's next four records in
// registers), then the rank merge of the four wave lists.  Records are
// referred to by their index q in the phase-1 arrays (in_q null: the input is
// phase 1 itself).  With `fin` set (one group per curve) it writes the user
// outputs instead of a list.
__global__ __launch_bounds__(kNT) void k_top_merge(
    const double* __restrict__ in_s, const int64_t* __restrict__ in_k,
    const int64_t* __restrict__ in_q, const double* __restrict__ in_max, int nl, int K,
    double* __restrict__ o_s, int64_t* __restrict__ o_k, int64_t* __restrict__ o_q,
    double* __restrict__ o_max, int fin, const Moments* __restrict__ mom, int curve0, int H,
    int hrow, const uint8_t* __restrict__ rf, const double* __restrict__ rd, TopOut out) {
  constexpr int PF = 4;  // records of a list held in registers at a time
  __shared__ double w_s[kNT / 64][64];  // each wave's K best, in order
  __shared__ int w_k[kNT / 64][64];
  __shared__ int64_t w_q[kNT / 64][64];
  __shared__ double s_ws[64];   // the group's K best: score,
  __shared__ int64_t s_wk[64];  // bin,
  __shared__ int64_t s_wq[64];  // phase-1 record
  __shared__ double s_mx[kNT / 64];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int g = blockIdx.x;
  const int cw = blockIdx.y;
  const int ng = gridDim.x;
  const int l = g * kNT + tid;
  const int64_t lbase = ((int64_t)cw * nl + l) * K;  // this thread's list

  double mx = -INFINITY;
  if (l < nl) mx = in_max[(int64_t)cw * nl + l];
  for (int o = 32; o > 0; o >>= 1) {
    const double other = __shfl_xor(mx, o);
    mx = other > mx ? other : mx;
  }
  if ((tid & 63) == 0) s_mx[tid >> 6] = mx;

  // Bins are below 2^24 (plan limit), so they serve as int keys.
  double cs[PF];
  int ck[PF];
  int64_t cq[PF];
  int head = 0;  // records of this list already taken
  auto fill = [&]() {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int idx = head + j;
      double sv = INFINITY;
      int kv = INT_MAX;
      int64_t qv = -1;
      if (l < nl && idx < K) {
        const int64_t kk = in_k[lbase + idx];
        if (kk >= 0) {
          sv = in_s[lbase + idx];
          kv = (int)kk;
          qv = in_q ? in_q[lbase + idx] : lbase + idx;
        }
      }
      cs[j] = sv;
      ck[j] = kv;
      cq[j] = qv;
    }
  };
  fill();
  int nwin = 0;
  for (int r = 0; r < K; ++r) {
    const int hq = head & (PF - 1);
    double sv = INFINITY;
    int sk = INT_MAX;
    int64_t sq = -1;
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      if (j == hq) {
        sv = cs[j];
        sk = ck[j];
        sq = cq[j];
      }
    }
    const int own_k = sk;
    wave_min_key(sv, sk);
    if (!(sv < INFINITY)) break;  // the same decision in every lane of the wave
    if (own_k == sk) {            // bins are distinct: this lane's list won
      w_s[wv][r] = sv;
      w_k[wv][r] = sk;
      w_q[wv][r] = sq;
      ++head;
      if ((head & (PF - 1)) == 0) fill();
    }
    nwin = r + 1;
  }
  if (lane >= nwin && lane < K) {
    w_s[wv][lane] = INFINITY;
    w_k[wv][lane] = INT_MAX;
    w_q[wv][lane] = -1;
  }
  if (tid < K) s_wq[tid] = -1;  // a slot no rank fills stays marked empty
  __syncthreads();
  bool wrote = false;
  if (tid < (kNT / 64) * K) {
    const int L = tid / K, pos = tid - L * K;
    const double sv = w_s[L][pos];
    const int sk = w_k[L][pos];
    if (sv < INFINITY) {
      const int rank = merged_rank(&w_s[0][0], &w_k[0][0], 64, kNT / 64, K, L, pos);
      if (rank < K) {
        s_ws[rank] = sv;
        s_wk[rank] = sk;
        s_wq[rank] = w_q[L][pos];
        wrote = true;
      }
    }
  }
  const int rounds = __syncthreads_count(wrote);
  double gmax = s_mx[0];
#pragma unroll
  for (int w = 1; w < kNT / 64; ++w) gmax = s_mx[w] > gmax ? s_mx[w] : gmax;

  if (!fin) {
    const int64_t ob = ((int64_t)cw * ng + g) * K;
    if (tid < K) {
      const bool ok = tid < rounds && s_wq[tid] >= 0;
      o_s[ob + tid] = ok ? s_ws[tid] : INFINITY;
      o_k[ob + tid] = ok ? s_wk[tid] : -1;
      o_q[ob + tid] = ok ? s_wq[tid] : -1;
    }
    if (tid == 0) o_max[(int64_t)cw * ng + g] = gmax;
    return;
  }

  const int c = curve0 + cw;
  const Moments mo = mom[c];
  const bool fatal = (mo.flags & kCurveFatal) != 0;
  const double best = (fatal || !(gmax > -INFINITY)) ? (double)NAN : mo.chi2_0 - gmax;
  const double ndof = (double)(mo.n - 2 * (hrow + 1) - 1);
  if (tid == 0) {
    if (out.chi2_best) out.chi2_best[c] = best;
    if (out.curve_flags) out.curve_flags[c] = (uint8_t)(mo.flags & 0xF8u);
  }
  if (tid < K) {
    const int64_t o = (int64_t)c * K + tid;
    if (tid < rounds && s_wq[tid] >= 0) {
      const int64_t q = s_wq[tid];
      out.idx[o] = s_wk[tid];
      out.log_p[o] = s_ws[tid];
      const double v = rd[q * H + hrow];
      if (out.dchi2_adj) out.dchi2_adj[o] = ndof > 0.0 ? v * ndof / best : (double)NAN;
      if (out.flags) out.flags[o] = rf[q];
      if (out.dchi2)
        for (int h = 0; h < H; ++h) out.dchi2[o * H + h] = rd[q * H + h];
    } else {
      out.idx[o] = -1;
      out.log_p[o] = (double)NAN;
      if (out.dchi2_adj) out.dchi2_adj[o] = (double)NAN;
      if (out.flags) out.flags[o] = 0;
      if (out.dchi2)
        for (int h = 0; h < H; ++h) out.dchi2[o * H + h] = (double)NAN;
    }
  }
}

template <int H>
hipError_t solve_top_h(bool fp64, const void* zc, const void* D, const Moments* mom,
                       const Geom& g, int curve0, int n_curves, double eps, int hrow,
                       int64_t k_lo, int K, int nblk, const TopScratch& sc, hipStream_t st) {
  dim3 gr((unsigned)nblk, (unsigned)n_curves);
  auto launch = [&](auto band) {
    constexpr bool B = decltype(band)::value;
    if (fp64)
      hipLaunchKernelGGL((k_solve_top<H, double, double, B>), gr, dim3(kNT), 0, st,
                         (const cplx<double>*)zc, (const cplx<double>*)D, mom, g, curve0, eps,
                         hrow, k_lo, K, nblk, sc.score, sc.k, sc.flag, sc.d, sc.bmax);
    else
      hipLaunchKernelGGL((k_solve_top<H, float, float, B>), gr, dim3(kNT), 0, st,
                         (const cplx<float>*)zc, (const cplx<double>*)D, mom, g, curve0, eps,
                         hrow, k_lo, K, nblk, sc.score, sc.k, sc.flag, sc.d, sc.bmax);
  };
  if (g.band)
    launch(std::true_type{});
  else
    launch(std::false_type{});
  return hipGetLastError();
}

}  // namespace

int top_blocks(int64_t n_freq) { return (int)((n_freq + kOwn - 1) / kOwn); }

namespace {
int top_groups(int64_t n_freq) { return (top_blocks(n_freq) + kNT - 1) / kNT; }
size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }
}  // namespace

size_t top_scratch_bytes(int64_t n_freq, int H, int n_curves, int K) {
  const size_t rec = (size_t)top_blocks(n_freq) * (size_t)n_curves;
  const size_t grp = (size_t)top_groups(n_freq) * (size_t)n_curves;
  return a256(rec * K * sizeof(double)) + a256(rec * K * sizeof(int64_t)) + a256(rec * K) +
         a256(rec * K * H * sizeof(double)) + a256(rec * sizeof(double)) +
         a256(grp * K * sizeof(double)) + 2 * a256(grp * K * sizeof(int64_t)) +
         a256(grp * sizeof(double));
}

TopScratch top_scratch_carve(void* base, int64_t n_freq, int H, int n_curves, int K) {
  const size_t rec = (size_t)top_blocks(n_freq) * (size_t)n_curves;
  const size_t grp = (size_t)top_groups(n_freq) * (size_t)n_curves;
  char* p = (char*)base;
  TopScratch s;
  s.score = (double*)p;
  p += a256(rec * K * sizeof(double));
  s.k = (int64_t*)p;
  p += a256(rec * K * sizeof(int64_t));
  s.flag = (uint8_t*)p;
  p += a256(rec * K);
  s.d = (double*)p;
  p += a256(rec * K * H * sizeof(double));
  s.bmax = (double*)p;
  p += a256(rec * sizeof(double));
  s.g_score = (double*)p;
  p += a256(grp * K * sizeof(double));
  s.g_k = (int64_t*)p;
  p += a256(grp * K * sizeof(int64_t));
  s.g_q = (int64_t*)p;
  p += a256(grp * K * sizeof(int64_t));
  s.g_max = (double*)p;
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
  const int ng = top_groups(g.n_freq);
  if (ng == 1) {
    // At most 256 per-block lists per curve: one step merges them and writes
    // the outputs (the same K smallest keys as two steps would keep).
    hipLaunchKernelGGL(k_top_merge, dim3(1u, (unsigned)n_curves), dim3(kNT), 0, st,
                       (const double*)sc.score, (const int64_t*)sc.k, (const int64_t*)nullptr,
                       (const double*)sc.bmax, nblk, K, (double*)nullptr, (int64_t*)nullptr,
                       (int64_t*)nullptr, (double*)nullptr, 1, mom, curve0, g.H, hrow,
                       (const uint8_t*)sc.flag, (const double*)sc.d, out);
    return hipGetLastError();
  }
  // Groups of up to 256 per-block lists, then the group lists of each curve.
  hipLaunchKernelGGL(k_top_merge, dim3((unsigned)ng, (unsigned)n_curves), dim3(kNT), 0, st,
                     (const double*)sc.score, (const int64_t*)sc.k, (const int64_t*)nullptr,
                     (const double*)sc.bmax, nblk, K, sc.g_score, sc.g_k, sc.g_q, sc.g_max, 0,
                     mom, curve0, g.H, hrow, (const uint8_t*)sc.flag, (const double*)sc.d, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_top_merge, dim3(1u, (unsigned)n_curves), dim3(kNT), 0, st,
                     (const double*)sc.g_score, (const int64_t*)sc.g_k, (const int64_t*)sc.g_q,
                     (const double*)sc.g_max, ng, K, (double*)nullptr, (int64_t*)nullptr,
                     (int64_t*)nullptr, (double*)nullptr, 1, mom, curve0, g.H, hrow,
                     (const uint8_t*)sc.flag, (const double*)sc.d, out);
  return hipGetLastError();
}

}  // namespace fchi2
