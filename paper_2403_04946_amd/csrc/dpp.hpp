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

// x_a + x_b for the two 16-lane rows a, b of each 32-lane half: two copies
// of x go through V_PERMLANE16_SWAP (odd rows of one trade places with even
// rows of the other), which leaves row 2q of x in every lane of one result
// and row 2q+1 in the other; a VALU exchange, no trip through LDS.  Every
// lane adds the same two operands, so the sum is bitwise the same in both
// rows.
__device__ inline double row_pair_sum(double x) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = (unsigned)(b & 0xffffffffll), hi = (unsigned)(b >> 32);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const double even = __longlong_as_double(((long long)h[0] << 32) | l[0]);
  const double odd = __longlong_as_double(((long long)h[1] << 32) | l[1]);
  return even + odd;
}

// x_lo + x_hi for the two 32-lane halves of the wavefront (V_PERMLANE32_SWAP)
__device__ inline double half_pair_sum(double x) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = (unsigned)(b & 0xffffffffll), hi = (unsigned)(b >> 32);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double first = __longlong_as_double(((long long)h[0] << 32) | l[0]);
  const double second = __longlong_as_double(((long long)h[1] << 32) | l[1]);
  return first + second;
}

}  // namespace ttf
