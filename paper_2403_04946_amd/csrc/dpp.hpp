// 16-lane reductions with DPP row permutations (CDNA: a row is 16 lanes of
// a 64-lane wavefront).  After the four steps every lane of the row holds
// the row sum: swap neighbours, swap pairs, mirror within 8, mirror within 16.
#pragma once

#include <hip/hip_runtime.h>

namespace ttf {

template <int CTRL>
__device__ inline double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double row16_sum(double x) {
  x += dpp_move<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_move<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_move<0x141>(x);  // row_half_mirror
  x += dpp_move<0x140>(x);  // row_mirror
  return x;
}

}  // namespace ttf
