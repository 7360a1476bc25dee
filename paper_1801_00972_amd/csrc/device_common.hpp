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
// (also used on the host, for the seeded grain placement)
__host__ __device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                        uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 32x32 -> 64-bit product is one multiply-add instruction
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// word 0 of Philox4x32-10 for N counters (c0[q], c1, c2, c3) with one key:
// the rounds above, interleaved over the counters so each round key is
// formed once
template <int N>
__device__ __forceinline__ void philox_word0(const uint32_t* c0in, uint32_t c1, uint32_t c2,
                                             uint32_t c3, uint32_t k0, uint32_t k1,
                                             uint32_t* out) {
  uint32_t a[N], b[N], c[N], d[N];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    a[q] = c0in[q];
    b[q] = c1;
    c[q] = c2;
    d[q] = c3;
  }
#pragma unroll
  for (int r = 0; r < 10; ++r) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const uint64_t p0 = (uint64_t)0xD2511F53u * a[q];
      const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[q];
      const uint32_t na = (uint32_t)(p1 >> 32) ^ b[q] ^ k0;
      const uint32_t nc = (uint32_t)(p0 >> 32) ^ d[q] ^ k1;
      b[q] = (uint32_t)p1;
      d[q] = (uint32_t)p0;
      a[q] = na;
      c[q] = nc;
    }
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
#pragma unroll
  for (int q = 0; q < N; ++q) out[q] = a[q];
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

// rf-phase bin of step k for time averages: the phase f_rf k dt modulo one
// period, in nbins equal bins
__device__ __forceinline__ int phase_bin(uint32_t k, double f_rf, double dt, int nbins) {
  const double x = f_rf * ((double)k * dt);
  const int b = (int)((x - floor(x)) * (double)nbins);
  return b < 0 ? 0 : (b >= nbins ? nbins - 1 : b);
}

// phi at node (pn, k) (pn the node's index in its plane): stored (kLift
// false), or lifted from the interior potential psi of the refined solve:
// 0 and V on the electrodes, psi + V k / nz inside
template <bool kLift>
__device__ __forceinline__ double phi_node(const double* __restrict__ src, long plane, long pn,
                                           int k, int nz, double V) {
  if (!kLift) return src[(long)k * plane + pn];
  if (k == 0) return 0.0;
  if (k == nz) return V;
  return src[(long)(k - 1) * plane + pn] + V * (double)k / (double)nz;
}

// E = -grad phi at node (x, y, k): central differences, periodic in x, y;
// one-sided along z on the electrode planes
template <bool kLift>
__device__ __forceinline__ void node_field(const double* __restrict__ src, int nx, int ny, int nz,
                                           double dx, double V, int x, int y, int k, double& ex,
                                           double& ey, double& ez) {
  const long plane = (long)nx * ny, row = (long)y * nx, pn = row + x;
  const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
  const int yp = y + 1 == ny ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
  ex = -(phi_node<kLift>(src, plane, row + xp, k, nz, V) -
         phi_node<kLift>(src, plane, row + xm, k, nz, V)) /
       (2.0 * dx);
  ey = -(phi_node<kLift>(src, plane, (long)yp * nx + x, k, nz, V) -
         phi_node<kLift>(src, plane, (long)ym * nx + x, k, nz, V)) /
       (2.0 * dx);
  if (k == 0)
    ez = -(phi_node<kLift>(src, plane, pn, 1, nz, V) - phi_node<kLift>(src, plane, pn, 0, nz, V)) /
         dx;
  else if (k == nz)
    ez = -(phi_node<kLift>(src, plane, pn, nz, nz, V) -
           phi_node<kLift>(src, plane, pn, nz - 1, nz, V)) /
         dx;
  else
    ez = -(phi_node<kLift>(src, plane, pn, k + 1, nz, V) -
           phi_node<kLift>(src, plane, pn, k - 1, nz, V)) /
         (2.0 * dx);
}

// wrap an index that is at most one period outside [0, n)
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

}  // namespace pic
