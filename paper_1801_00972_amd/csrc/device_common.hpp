// device_common.hpp -- small device helpers of the HIP path: the counter-based
// generator, uniform and normal conversions, index wrapping.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pic_types.hpp"

namespace pic {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): per round two 32x32->64
// products of counter words 0 and 2 with the published multipliers, xor-mixed
// with the other words and the round key; the key advances by the Weyl
// constants after each round.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// (w + 1/2) 2^-32: uniform on the open interval (0, 1)
__device__ __forceinline__ double u01_open(uint32_t w) {
  return ((double)w + 0.5) * 2.3283064365386962890625e-10;
}

// Box-Muller: two standard normals from two words, cosine branch first
__device__ __forceinline__ void normal_pair(uint32_t wa, uint32_t wb, double& n0, double& n1) {
  const double r = sqrt(-2.0 * log(u01_open(wa)));
  double s, c;
  sincos(2.0 * kPi * u01_open(wb), &s, &c);
  n0 = r * c;
  n1 = r * s;
}

__device__ __forceinline__ double rf_voltage(const RfDrive& d) {
  const double t = (double)(*d.step) * d.dt;
  return d.V_dc + d.V_rf * sin(2.0 * kPi * d.f_rf * t);
}

// wrap an index that is at most one period outside [0, n)
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

}  // namespace pic
