// Reciprocal and reciprocal square root in FP64 from the hardware
// estimates (V_RCP_F64, V_RSQ_F64) refined by Newton's method: each step
// squares the relative error, and two steps bring the estimate to within a
// few units in the last place.  For normal, finite arguments only (callers
// keep subnormal and huge arguments on the exact library functions).
#pragma once

#include <hip/hip_runtime.h>

namespace ttf {

// 1 / sqrt(a), a > 0: y <- y + y (1/2 - a y^2 / 2), twice
__device__ inline double rsqrt_newton(double a) {
  double y = __builtin_amdgcn_rsq(a);
  const double h = 0.5 * a;
  double r = fma(-h * y, y, 0.5);
  y = fma(y, r, y);
  r = fma(-h * y, y, 0.5);
  return fma(y, r, y);
}

// 1 / a: y <- y + y (1 - a y), twice
__device__ inline double rcp_newton(double a) {
  double y = __builtin_amdgcn_rcp(a);
  double e = fma(-a, y, 1.0);
  y = fma(y, e, y);
  e = fma(-a, y, 1.0);
  return fma(y, e, y);
}

}  // namespace ttf
