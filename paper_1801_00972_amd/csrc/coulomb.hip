// coulomb.hip -- Coulomb collisions between the charged particles (Table I:
// e-e, e-Ar+, Ar+-Ar+), the binary Monte-Carlo model of Takizuka and Abe that
// the paper cites with its collision set.
//
// One pass, at the start of every interval-th step on (x_k, v_{k-1/2}):
//  1. count the alive particles of each species per cell and scan the counts
//     into per-cell ranges;
//  2. scatter (order key, slot) of every particle into its cell's range; the
//     key is the particle's Philox word (id, k, order purpose, species) above
//     its id, so the order inside a cell does not depend on the scatter's
//     atomics;
//  3. one 64-lane block per cell ranks each species' range by key, then runs
//     the like pairs (e-e and Ar+-Ar+, pairs in parallel, an odd count's
//     triplet on lane 0), a barrier, and the unlike pairs (one lane per
//     particle of the less numerous species, its partners in order).
// The collisions of one pass touch disjoint particles except where the
// pairing rule orders them, so this is the sequential pass of the rule.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "launch.hpp"

namespace pic {

namespace {

constexpr uint32_t kCOrder = 5;  // Philox counter word 2: pairing order
constexpr uint32_t kCPair = 6;   // Philox counter word 2: one collision's draws
constexpr int kScanChunk = 2048; // elements per block of the scan (256 threads x 8)

inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

__device__ __forceinline__ bool alive(const PartF64& P, long p) { return P.z[p] >= 0.0; }
__device__ __forceinline__ bool alive(const PartF32R& P, long p) { return P.cell[p] >= 0; }

// linear cell index (i + nx (j + ny k)) of an alive particle
__device__ __forceinline__ int cell_of(const PartF64& P, long p, int nx, int ny) {
  const int i = (int)floor(P.x[p]), j = (int)floor(P.y[p]), k = (int)floor(P.z[p]);
  return i + nx * (j + ny * k);
}
__device__ __forceinline__ int cell_of(const PartF32R& P, long p, int nx, int ny) {
  const int c = P.cell[p];
  return (c & 1023) + nx * (((c >> 10) & 1023) + ny * (c >> 20));
}

__device__ __forceinline__ void load_v(const PartF64& P, long p, double v[3]) {
  v[0] = P.vx[p];
  v[1] = P.vy[p];
  v[2] = P.vz[p];
}
__device__ __forceinline__ void load_v(const PartF32R& P, long p, double v[3]) {
  v[0] = P.vx[p];
  v[1] = P.vy[p];
  v[2] = P.vz[p];
}
__device__ __forceinline__ void store_v(const PartF64& P, long p, const double v[3]) {
  P.vx[p] = v[0];
  P.vy[p] = v[1];
  P.vz[p] = v[2];
}
__device__ __forceinline__ void store_v(const PartF32R& P, long p, const double v[3]) {
  P.vx[p] = (float)v[0];
  P.vy[p] = (float)v[1];
  P.vz[p] = (float)v[2];
}

template <typename PT>
__global__ __launch_bounds__(256) void coul_count_kernel(PT P, WorkLists L, int nx, int ny,
                                                         int* __restrict__ cnt) {
  const long total = L.tstart[L.ngrid];
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < total;
       p += (long)gridDim.x * blockDim.x)
    if (alive(P, p)) atomicAdd(&cnt[cell_of(P, p, nx, ny)], 1);
}

// exclusive scan of a[0..n) in place: blocks of kScanChunk, their totals in sums
__global__ __launch_bounds__(256) void coul_scan_local(int* __restrict__ a, long n,
                                                       int* __restrict__ sums) {
  __shared__ int s[256];
  const long base = (long)blockIdx.x * kScanChunk + (long)threadIdx.x * 8;
  int v[8], run = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    v[q] = base + q < n ? a[base + q] : 0;
    run += v[q];
  }
  s[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int acc = s[threadIdx.x] - run;  // exclusive prefix of this thread's eight
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (base + q < n) a[base + q] = acc;
    acc += v[q];
  }
  if (threadIdx.x == 255) sums[blockIdx.x] = s[255];
}

// exclusive scan of the block totals (one block, chunks of 256 with a carry)
__global__ __launch_bounds__(256) void coul_scan_sums(int* __restrict__ sums, int nb) {
  __shared__ int s[256];
  int carry = 0;
  for (int b0 = 0; b0 < nb; b0 += 256) {
    const int i = b0 + (int)threadIdx.x;
    const int v = i < nb ? sums[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) sums[i] = carry + s[threadIdx.x] - v;
    const int total = s[255];
    __syncthreads();
    carry += total;
  }
}

__global__ __launch_bounds__(256) void coul_scan_add(int* __restrict__ a, long n,
                                                     const int* __restrict__ sums) {
  const long i = (long)blockIdx.x * kScanChunk + threadIdx.x;
  const int add = sums[blockIdx.x];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const long e = i + q * 256;
    if (e < n) a[e] += add;
  }
}

template <typename PT>
__global__ __launch_bounds__(256) void coul_scatter_kernel(PT P, WorkLists L, CoulombConst C,
                                                           int sp, const int* __restrict__ start,
                                                           int* __restrict__ fill,
                                                           unsigned long long* __restrict__ key,
                                                           int* __restrict__ slot) {
  const long total = L.tstart[L.ngrid];
  const uint32_t k = *C.step;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < total;
       p += (long)gridDim.x * blockDim.x) {
    if (!alive(P, p)) continue;
    const int c = cell_of(P, p, C.nx, C.ny);
    const int at = start[c] + atomicAdd(&fill[c], 1);
    const uint32_t id = P.id[p];
    const uint4 r = philox4x32_10(id, k, kCOrder, (uint32_t)sp, C.key0, C.key1);
    key[at] = ((unsigned long long)r.x << 32) | id;
    slot[at] = (int)p;
  }
}

// One binary collision: draws from Philox(id, k, kCPair, word); delta normal
// (Box-Muller cosine branch of words 0, 1) with variance cv n_L / |u|^3, the
// azimuth 2 pi u(word 2); the relative velocity u = va - vb turns by
// theta = 2 atan(delta) about itself, va += fa du, vb -= fb du.
__device__ void coul_collide(const CoulombConst& C, uint32_t k, uint32_t word, double cv,
                             double fa, double fb, double* va, double* vb, uint32_t id) {
  const double u0 = va[0] - vb[0], u1 = va[1] - vb[1], u2 = va[2] - vb[2];
  const double um = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
  if (!(um > 0.0)) return;
  const uint4 r = philox4x32_10(id, k, kCPair, word, C.key0, C.key1);
  double n0, n1;
  normal_pair(r.x, r.y, n0, n1);
  const double delta = sqrt(cv / (um * um * um)) * n0;
  const double phi = 2.0 * kPi * u01_open(r.z);
  const double sn = 2.0 * delta / (1.0 + delta * delta);
  const double omc = 2.0 * delta * delta / (1.0 + delta * delta);
  const double cp = cos(phi), sp = sin(phi);
  const double up = sqrt(u0 * u0 + u1 * u1);
  double du[3];
  if (up > 0.0) {
    du[0] = (u0 / up) * u2 * sn * cp - (u1 / up) * um * sn * sp - u0 * omc;
    du[1] = (u1 / up) * u2 * sn * cp + (u0 / up) * um * sn * sp - u1 * omc;
    du[2] = -up * sn * cp - u2 * omc;
  } else {
    du[0] = um * sn * cp;
    du[1] = um * sn * sp;
    du[2] = -u2 * omc;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    va[a] += fa * du[a];
    vb[a] -= fb * du[a];
  }
}

template <typename PT>
__device__ __forceinline__ void like_pair(const PT& P, const CoulombConst& C, uint32_t k, int sp,
                                          const int* ord, int qa, int qb, double cv) {
  const long pa = ord[qa], pb = ord[qb];
  double va[3], vb[3];
  load_v(P, pa, va);
  load_v(P, pb, vb);
  coul_collide(C, k, (uint32_t)sp, cv, C.frac[sp][sp], C.frac[sp][sp], va, vb, P.id[pa]);
  store_v(P, pa, va);
  store_v(P, pb, vb);
}

template <typename PT>
__global__ __launch_bounds__(64) void coul_pair_kernel(PT Pe, PT Pi, CoulombBufs B,
                                                       CoulombConst C) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const PT P[2] = {Pe, Pi};
  int r0[2], n[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    r0[s] = B.start[s][c];
    n[s] = B.start[s][c + 1] - r0[s];
  }
  if (n[0] + n[1] < 2) return;
  const uint32_t k = *C.step;
  // rank by key (unique: the id is in the low word)
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const unsigned long long* key = B.key[s] + r0[s];
    for (int q = lane; q < n[s]; q += 64) {
      const unsigned long long kq = key[q];
      int rank = 0;
      for (int t = 0; t < n[s]; ++t) rank += key[t] < kq;
      B.ord[s][r0[s] + rank] = B.slot[s][r0[s] + q];
    }
  }
  __syncthreads();
  // like pairs, both species
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int N = n[s];
    if (N < 2) continue;
    const int* ord = B.ord[s] + r0[s];
    const double cv = C.c_var[s] * (double)N * C.w_vol;
    int first = 0;
    if (N & 1) {
      if (lane == 0) {
        like_pair(P[s], C, k, s, ord, 0, 1, 0.5 * cv);
        like_pair(P[s], C, k, s, ord, 1, 2, 0.5 * cv);
        like_pair(P[s], C, k, s, ord, 2, 0, 0.5 * cv);
      }
      first = 3;
    }
    for (int q = first + 2 * lane; q + 1 < N; q += 128) like_pair(P[s], C, k, s, ord, q, q + 1, cv);
  }
  __syncthreads();
  // unlike pairs: lane r takes particle r of the less numerous species b and
  // its partners j = r, r + N_b, ... of species a, in order
  if (n[0] > 0 && n[1] > 0) {
    const int sa = n[0] >= n[1] ? 0 : 1, sb = 1 - sa;
    const int Na = n[sa], Nb = n[sb];
    const int* oa = B.ord[sa] + r0[sa];
    const int* ob = B.ord[sb] + r0[sb];
    const double cv = C.c_var[2] * (double)Nb * C.w_vol;
    for (int r = lane; r < Nb; r += 64) {
      const long pb = ob[r];
      double vb[3];
      load_v(P[sb], pb, vb);
      for (int j = r; j < Na; j += Nb) {
        const long pa = oa[j];
        double va[3];
        load_v(P[sa], pa, va);
        coul_collide(C, k, 2u + (uint32_t)sa, cv, C.frac[2][sa], C.frac[2][sb], va, vb,
                     P[sa].id[pa]);
        store_v(P[sa], pa, va);
        // the b particle's velocity is kept in registers between its
        // collisions but rounded to the record's precision after each, as the
        // records hold it
        store_v(P[sb], pb, vb);
        load_v(P[sb], pb, vb);
      }
    }
  }
  if (lane == 0) {
    unsigned long long m = 0;
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (n[s] >= 2) m += (n[s] & 1) ? 3 + (n[s] - 3) / 2 : n[s] / 2;
    if (n[0] > 0 && n[1] > 0) m += n[0] > n[1] ? n[0] : n[1];
    if (m) atomicAdd(B.count, m);
  }
}

template <typename PT>
void coulomb_impl(const PT P[2], const WorkLists L[2], const CoulombBufs& B, const CoulombConst& C,
                  const long cap[2], hipStream_t st) {
  const long ncell = C.ncell;
  for (int s = 0; s < 2; ++s) {
    launch_zero_i32(B.start[s], ncell + 1, st);
    launch_zero_i32(B.fill[s], ncell, st);
    const int g = std::min(nblk(cap[s], 256), 65536);
    if (g > 0)
      hipLaunchKernelGGL(coul_count_kernel<PT>, dim3(g), dim3(256), 0, st, P[s], L[s], C.nx, C.ny,
                         B.start[s]);
    const long n = ncell + 1;
    const int nb = nblk(n, kScanChunk);
    hipLaunchKernelGGL(coul_scan_local, dim3(nb), dim3(256), 0, st, B.start[s], n, B.sums);
    hipLaunchKernelGGL(coul_scan_sums, dim3(1), dim3(256), 0, st, B.sums, nb);
    hipLaunchKernelGGL(coul_scan_add, dim3(nb), dim3(256), 0, st, B.start[s], n, B.sums);
    if (g > 0)
      hipLaunchKernelGGL(coul_scatter_kernel<PT>, dim3(g), dim3(256), 0, st, P[s], L[s], C, s,
                         B.start[s], B.fill[s], B.key[s], B.slot[s]);
  }
  hipLaunchKernelGGL(coul_pair_kernel<PT>, dim3((unsigned)ncell), dim3(64), 0, st, P[0], P[1], B, C);
}

}  // namespace

long coulomb_scan_sums(long ncell) { return nblk(ncell + 1, kScanChunk); }

void launch_coulomb(const PartF64* P64, const PartF32R* P32, const WorkLists L[2],
                    const CoulombBufs& B, const CoulombConst& C, const long cap[2],
                    hipStream_t st) {
  if (C.ncell <= 0) return;
  if (P64)
    coulomb_impl<PartF64>(P64, L, B, C, cap, st);
  else
    coulomb_impl<PartF32R>(P32, L, B, C, cap, st);
}

}  // namespace pic
