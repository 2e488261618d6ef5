// Counter-based Gaussian random numbers on the device.
//
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64-bit multiplies and
// xors with a Weyl-sequence key schedule.  Box-Muller turns two uniforms into
// a pair of independent standard normals, used as the real and imaginary
// part of one complex sample.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ttf {

__device__ inline void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k0, k1);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// complex sample with independent N(0, 1) real and imaginary parts for
// counter (e, tag) under key (k0, k1)
__device__ inline double2 philox_gaussian(uint64_t e, uint32_t tag, uint32_t k0, uint32_t k1) {
  uint32_t c[4] = {(uint32_t)e, (uint32_t)(e >> 32), tag, 0x5EEDu};
  philox4x32_10(c, k0, k1);
  const double u1 = ((double)c[0] + 1.0) / 4294967297.0;  // (0, 1)
  const double u2 = (double)c[1] / 4294967296.0;          // [0, 1)
  const double r = sqrt(-2.0 * log(u1));
  double s, cs;
  sincospi(2.0 * u2, &s, &cs);
  return make_double2(r * cs, r * s);
}

}  // namespace ttf
