// Keys of the significance epilogue (Section 3e): the candidate score
// ln p = ln k + ln Q(Delta chi2 | 2H') paired with its bin, their order, and
// the rank merge of sorted key lists.  Host and device code share these
// functions, so the ordering and the merge are tested on the CPU as well.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

namespace fchi2 {

// ln Q(D | 2 hp): log of the chi2 upper tail with an even number of degrees
// of freedom, Q = exp(-D/2) sum_{j < hp} (D/2)^j / j!.  The partial sum is
// evaluated by Horner's rule from the highest term down (all terms are
// positive, so nothing cancels) and log1p keeps the small-D end accurate.
// D = +inf gives -inf (the tail vanishes); D <= 0 and NaN give 0 and NaN.
__host__ __device__ inline double log_q_even(double d, int hp) {
  const double u = 0.5 * (d > 0.0 ? d : 0.0);
  if (u == INFINITY) return -INFINITY;
  if (d != d) return d;
  double r = 1.0;
  for (int j = hp - 1; j >= 2; --j) r = 1.0 + r * (u / (double)j);
  const double tail = hp > 1 ? u * r : 0.0;
  return -u + log1p(tail);
}

// Score used for ranking: NaN ranks as +inf, i.e. never as a candidate, so
// every key entering a selection is ordered.
__host__ __device__ inline double rank_score(double s) { return s == s ? s : INFINITY; }

// (score, bin) order: smaller score first, ties to the lower bin.
__host__ __device__ inline bool key_less(double sa, int ia, double sb, int ib) {
  return (sa < sb) || (sa == sb && ia < ib);
}

// Rank of key `pos` of sorted list L among nl sorted lists of K keys each
// (list j at s[j * ld], k[j * ld]): its position plus, in every other list,
// the number of keys smaller than it (binary search).  With distinct keys the
// ranks of all keys are distinct; equal keys in two lists take one rank.
template <typename I>
__host__ __device__ inline int merged_rank(const double* s, const I* k, int ld, int nl, int K,
                                           int L, int pos) {
  const double sv = s[L * ld + pos];
  const int si = (int)k[L * ld + pos];
  int rank = pos;
  for (int L2 = 0; L2 < nl; ++L2) {
    if (L2 == L) continue;
    int a = 0, b = K;  // first index of list L2 whose key is not smaller
    while (a < b) {
      const int mid = (a + b) >> 1;
      if (key_less(s[L2 * ld + mid], (int)k[L2 * ld + mid], sv, si)) a = mid + 1;
      else b = mid;
    }
    rank += a;
  }
  return rank;
}

}  // namespace fchi2
