// Host-only checks of the top-K key order and rank merge shared by the
// significance kernels (no kernel is launched).  Prints "ALL OK" on success.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_0901_1913_amd/csrc/topk_keys.h"

using namespace fchi2;

static int g_fail = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);                \
      ++g_fail;                                                       \
    }                                                                 \
  } while (0)

struct Key {
  double s;
  int k;
};

// The block selection of the fused solve: 256 threads hold 4 keys each,
// every wave of 64 keeps its K best by repeated arg-min over the threads'
// heads (the owner of the winner advancing), then the four sorted wave lists
// are merged by rank into slots that start empty (-1).
static std::vector<int> block_select(const std::vector<Key>& keys, int K) {
  const int NT = 256, BPT = 4, NW = NT / 64;
  std::vector<double> ws(NW * 64, INFINITY);
  std::vector<int> wi(NW * 64, INT_MAX);
  for (int w = 0; w < NW; ++w) {
    std::vector<std::vector<Key>> own(64);
    for (int l = 0; l < 64; ++l) {
      for (int r = 0; r < BPT; ++r) own[l].push_back(keys[r * NT + w * 64 + l]);
      std::sort(own[l].begin(), own[l].end(),
                [](const Key& a, const Key& b) { return key_less(a.s, a.k, b.s, b.k); });
    }
    std::vector<int> head(64, 0);
    for (int r = 0; r < K; ++r) {
      double bs = INFINITY;
      int bi = INT_MAX, bl = -1;
      for (int l = 0; l < 64; ++l) {
        if (head[l] >= BPT) continue;
        const Key& c = own[l][head[l]];
        if (key_less(c.s, c.k, bs, bi)) {
          bs = c.s;
          bi = c.k;
          bl = l;
        }
      }
      if (!(bs < INFINITY)) break;
      ws[w * 64 + r] = bs;
      wi[w * 64 + r] = bi;
      ++head[bl];
    }
  }
  std::vector<int> win(K, -1);
  for (int L = 0; L < NW; ++L)
    for (int pos = 0; pos < K; ++pos) {
      if (!(ws[L * 64 + pos] < INFINITY)) continue;
      const int rank = merged_rank(ws.data(), wi.data(), 64, NW, K, L, pos);
      if (rank < K) win[rank] = wi[L * 64 + pos];
    }
  return win;
}

int main() {
  // ln Q for even dof: limits and closed forms.
  CHECK(log_q_even(INFINITY, 3) == -INFINITY);
  CHECK(std::isnan(log_q_even(NAN, 2)));
  CHECK(log_q_even(0.0, 4) == 0.0);
  CHECK(log_q_even(-5.0, 2) == 0.0);
  for (double d : {1e-6, 0.3, 7.0, 80.0, 3e4}) {
    CHECK(std::fabs(log_q_even(d, 1) - (-0.5 * d)) <= 1e-15 * std::max(1.0, d));
    const double u = 0.5 * d;
    CHECK(std::fabs(log_q_even(d, 2) - (-u + std::log1p(u))) <= 1e-14 * std::max(1.0, u));
  }
  CHECK(rank_score(NAN) == INFINITY);
  CHECK(rank_score(-INFINITY) == -INFINITY);
  CHECK(rank_score(2.5) == 2.5);
  CHECK(key_less(-INFINITY, 9, 0.0, 1));
  CHECK(key_less(1.0, 3, 1.0, 4));
  CHECK(!key_less(1.0, 4, 1.0, 4));

  std::mt19937_64 rng(7);
  for (int trial = 0; trial < 400; ++trial) {
    const int K = 1 + (int)(rng() % 64);
    std::vector<Key> keys(1024);
    const double levels[] = {-INFINITY, -3.0, -1.0, -1.0, 0.5, INFINITY, NAN};
    for (int i = 0; i < 1024; ++i) {
      double s;
      const int mode = (int)(rng() % 4);
      if (mode == 0) s = levels[rng() % 7];            // ties, infinities, NaN
      else s = -20.0 * (double)(rng() % 1000) / 1000.0;  // many equal scores too
      keys[i] = Key{rank_score(s), i};
    }
    const std::vector<int> got = block_select(keys, K);
    std::vector<Key> ref;
    for (const Key& k : keys)
      if (k.s < INFINITY) ref.push_back(k);
    std::sort(ref.begin(), ref.end(),
              [](const Key& a, const Key& b) { return key_less(a.s, a.k, b.s, b.k); });
    for (int r = 0; r < K; ++r) {
      const int want = r < (int)ref.size() ? ref[r].k : -1;
      if (got[r] != want) {
        std::printf("trial %d K %d slot %d: got %d want %d\n", trial, K, r, got[r], want);
        ++g_fail;
        break;
      }
    }
  }

  // A broken input with one key in two lists: both take one rank, so one slot
  // stays unfilled and must read as empty (-1), never as a stale index.
  {
    const int K = 4, NW = 4;
    std::vector<double> ws(NW * 64, INFINITY);
    std::vector<int> wi(NW * 64, INT_MAX);
    const double a[] = {1.0, 2.0, 3.0, 4.0};
    for (int p = 0; p < K; ++p) {
      ws[0 * 64 + p] = a[p];
      wi[0 * 64 + p] = 10 + p;
    }
    ws[1 * 64 + 0] = 1.0;  // duplicate of list 0's first key
    wi[1 * 64 + 0] = 10;
    std::vector<int> win(K, -1);
    for (int L = 0; L < NW; ++L)
      for (int pos = 0; pos < K; ++pos) {
        if (!(ws[L * 64 + pos] < INFINITY)) continue;
        const int rank = merged_rank(ws.data(), wi.data(), 64, NW, K, L, pos);
        if (rank < K) win[rank] = wi[L * 64 + pos];
      }
    int empty = 0;
    for (int r = 0; r < K; ++r) {
      CHECK(win[r] == -1 || (win[r] >= 10 && win[r] <= 13));
      empty += win[r] == -1;
    }
    CHECK(empty == 1);
  }

  if (g_fail == 0) std::printf("ALL OK\n");
  return g_fail == 0 ? 0 : 1;
}
