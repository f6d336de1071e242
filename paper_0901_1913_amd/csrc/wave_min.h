// Wave-wide minimum of a (score, index) key, ordered by score and then by
// index (the candidate order of the significance epilogue), with DPP lane
// permutations instead of LDS-routed shuffles: a butterfly inside each row of
// 16 lanes (quad swaps, half-row and row mirrors), then the row broadcasts of
// lane 15 and lane 31 fold the four rows into lane 63, which is read back as
// a wave-uniform value.  Lanes that a permutation does not write see the
// identity key (+inf, INT_MAX).  Needs all 64 lanes active.
#pragma once

#include <climits>
#include <cmath>

#include "topk_keys.h"

namespace fchi2 {

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void wmin_step(double& s, int& i) {
  union {
    double d;
    int w[2];
  } a, b;
  a.d = s;
  const union {
    double d;
    int w[2];
  } id = {INFINITY};
  b.w[0] = __builtin_amdgcn_update_dpp(id.w[0], a.w[0], CTRL, ROW_MASK, 0xF, false);
  b.w[1] = __builtin_amdgcn_update_dpp(id.w[1], a.w[1], CTRL, ROW_MASK, 0xF, false);
  const int j = __builtin_amdgcn_update_dpp(INT_MAX, i, CTRL, ROW_MASK, 0xF, false);
  if (key_less(b.d, j, s, i)) {
    s = b.d;
    i = j;
  }
}

// On return every lane holds the wave's smallest key.
__device__ __forceinline__ void wave_min_key(double& s, int& i) {
  wmin_step<0xB1, 0xF>(s, i);   // quad_perm [1,0,3,2]
  wmin_step<0x4E, 0xF>(s, i);   // quad_perm [2,3,0,1]
  wmin_step<0x141, 0xF>(s, i);  // row_half_mirror
  wmin_step<0x140, 0xF>(s, i);  // row_mirror: every lane holds its row's minimum
  wmin_step<0x142, 0xA>(s, i);  // row_bcast:15 into rows 1 and 3
  wmin_step<0x143, 0xC>(s, i);  // row_bcast:31 into rows 2 and 3: lane 63 holds the minimum
  union {
    double d;
    int w[2];
  } r;
  r.d = s;
  r.w[0] = __builtin_amdgcn_readlane(r.w[0], 63);
  r.w[1] = __builtin_amdgcn_readlane(r.w[1], 63);
  s = r.d;
  i = __builtin_amdgcn_readlane(i, 63);
}

}  // namespace fchi2
