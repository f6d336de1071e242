// Host build of the FFT split planning (csrc/fft_splits.h): every candidate
// the autotuner may time is a valid split of the grid length, the plan's
// default split is one of them, and the extra-pass splits appear only for
// grids of at most 2^20 cells.
#include <cstdio>
#include <cstdlib>

#include "../../paper_0901_1913_amd/csrc/fft_splits.h"

using namespace fchi2;

static int fails = 0;
#define CHECK(c, ...)                              \
  do {                                             \
    if (!(c)) {                                    \
      ++fails;                                     \
      std::printf("FAIL %s: ", #c);                \
      std::printf(__VA_ARGS__);                    \
      std::printf("\n");                           \
    }                                              \
  } while (0)

static bool same(const FftPlan& a, const FftPlan& b) {
  if (a.np != b.np) return false;
  for (int q = 1; q <= a.np; ++q)
    if (a.logn[q] != b.logn[q] || a.le[q] != b.le[q]) return false;
  return true;
}

int main() {
  for (int fp64 = 0; fp64 <= 1; ++fp64) {
    for (int logL = 12; logL <= 26; ++logL) {
      FftPlan def{};
      CHECK(plan_fft(logL, 12, def), "logL %d has a default split", logL);
      const std::vector<FftPlan> c = fft_splits(logL, fp64 != 0);
      CHECK(!c.empty(), "logL %d has candidates", logL);
      int min_np = 99;
      for (const FftPlan& f : c) min_np = f.np < min_np ? f.np : min_np;
      CHECK(min_np == def.np, "logL %d: fewest passes %d = default %d", logL, min_np, def.np);
      bool has_default = false;
      for (size_t i = 0; i < c.size(); ++i) {
        const FftPlan& f = c[i];
        has_default = has_default || same(f, def);
        int sum = 0;
        for (int q = 1; q <= f.np; ++q) {
          sum += f.logn[q];
          CHECK(f.le[q] == 12 || (f.le[q] == 13 && !fp64) || (f.np == 1 && f.le[q] == logL),
                "logL %d tile 2^%d", logL, f.le[q]);
          if (f.np > 1) CHECK(f.logn[q] >= 4 && f.logn[q] <= 9, "digit 2^%d", f.logn[q]);
        }
        CHECK(sum == logL, "logL %d digits sum to %d", logL, sum);
        CHECK(f.logL == logL, "logL recorded");
        CHECK(split_valid(f), "logL %d candidate %zu valid", logL, i);
        CHECK(f.np <= min_np + 1, "logL %d: at most one pass more", logL);
        if (logL > 20) CHECK(f.np == min_np, "logL %d: no extra pass above 2^20", logL);
        for (size_t k = 0; k < i; ++k) CHECK(!same(f, c[k]), "logL %d duplicate candidate", logL);
      }
      CHECK(has_default, "logL %d: default split among the candidates", logL);
    }
  }
  // The batch grid (L = 2^18, FP32): three passes of 2^6 on 4096-element
  // tiles and the two-pass 2^9 x 2^9 split are both offered.
  {
    const std::vector<FftPlan> c = fft_splits(18, false);
    bool three = false, two = false;
    for (const FftPlan& f : c) {
      three = three || (f.np == 3 && f.logn[1] == 6 && f.logn[2] == 6 && f.logn[3] == 6 &&
                        f.le[1] == 12 && f.le[2] == 12 && f.le[3] == 12);
      two = two || (f.np == 2 && f.logn[1] == 9 && f.logn[2] == 9);
    }
    CHECK(three && two, "L = 2^18 offers 2^6 x 2^6 x 2^6 and 2^9 x 2^9");
  }
  // The stress grid (L = 2^26): three passes only.
  for (const FftPlan& f : fft_splits(26, false)) CHECK(f.np == 3, "L = 2^26 np %d", f.np);
  // Invalid splits are rejected: a first-pass tile wider than digit 1.
  {
    FftPlan f{};
    f.np = 3;
    f.logL = 18;
    f.logn[1] = 6; f.logn[2] = 6; f.logn[3] = 6;
    f.le[1] = 13; f.le[2] = 13; f.le[3] = 13;  // first pass: 2^7 columns > 2^6
    CHECK(!split_valid(f), "first-pass tile wider than digit 1 is rejected");
  }
  if (fails) {
    std::printf("%d FAILED\n", fails);
    return 1;
  }
  std::printf("ALL OK\n");
  return 0;
}
