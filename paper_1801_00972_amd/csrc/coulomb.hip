// coulomb.hip -- Coulomb collisions between the charged particles (Table I:
// e-e, e-Ar+, Ar+-Ar+), the binary Monte-Carlo model of Takizuka and Abe that
// the paper cites with its collision set.
//
// One pass, at the start of every interval-th step on (x_k, v_{k-1/2}):
//  1. count the alive particles of each species per cell (cells numbered in
//     the tile order of the particle bins) and scan the counts into per-cell
//     ranges;
//  2. scatter (order key, slot) of every particle into its cell's range; the
//     key is the particle's Philox word (id, k, order purpose, species) above
//     its id, so the order inside a cell does not depend on the scatter's
//     atomics;
//  3. a block of 256 threads takes 16 groups of 8 consecutive cells in turn
//     (each a contiguous range of the key / slot arrays): it stages a group's
//     keys in LDS (the next group's keys and slots already load meanwhile),
//     ranks each particle inside its cell by key and puts the id (the key's
//     low word) and the velocity in that order, then 32 lanes per
//     cell run the like items (e-e and Ar+-Ar+ pairs, an odd count's triplet
//     as one item), a barrier, and the unlike pairs (one lane per particle of
//     the less numerous species, its partners in order), and the velocities
//     go back once; the arithmetic is in the velocities' precision (FP64 or
//     FP32); a group with a cell above 64 particles of a species runs its
//     cells in turn through global memory with the whole block.
// Counting and scattering go a block per tile of the particle bins: an LDS
// histogram and one global atomic per cell, one more per particle that has
// left its tile since the last binning.
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


// Cells are numbered in tile order: tile (i/4 + ntx (j/4 + nty k/4)), the
// tile order of the particle bins, times 64 plus the cell inside its tile
// (x fastest); cells of a tile past the box edge stay empty.  -1: not alive.
__device__ __forceinline__ int tiled_cell(int i, int j, int k, int ntx, int nty) {
  return (((k >> 2) * nty + (j >> 2)) * ntx + (i >> 2)) * 64 + ((k & 3) * 4 + (j & 3)) * 4 + (i & 3);
}
__device__ __forceinline__ int coul_cell(const PartF64& P, long p, int ntx, int nty) {
  if (!(P.z[p] >= 0.0)) return -1;
  return tiled_cell((int)floor(P.x[p]), (int)floor(P.y[p]), (int)floor(P.z[p]), ntx, nty);
}
__device__ __forceinline__ int coul_cell(const PartF32R& P, long p, int ntx, int nty) {
  const int c = P.cell[p];
  if (c < 0) return -1;
  return tiled_cell(c & 1023, (c >> 10) & 1023, c >> 20, ntx, nty);
}

// The collision arithmetic runs in the precision the velocities are stored
// in: FP64 for the FP64 records, FP32 for the FP32R records (whose velocities
// are FP32 already; the pass's rounding is then of the order of the FP32
// velocities' own).
template <typename PT> struct CoulReal { using T = double; };
template <> struct CoulReal<PartF32R> { using T = float; };

__device__ __forceinline__ void load_v(const PartF64& P, long p, double v[3]) {
  v[0] = P.vx[p];
  v[1] = P.vy[p];
  v[2] = P.vz[p];
}
__device__ __forceinline__ void load_v(const PartF32R& P, long p, float v[3]) {
  v[0] = P.vx[p];
  v[1] = P.vy[p];
  v[2] = P.vz[p];
}
__device__ __forceinline__ void store_v(const PartF64& P, long p, const double v[3]) {
  P.vx[p] = v[0];
  P.vy[p] = v[1];
  P.vz[p] = v[2];
}
__device__ __forceinline__ void store_v(const PartF32R& P, long p, const float v[3]) {
  P.vx[p] = v[0];
  P.vy[p] = v[1];
  P.vz[p] = v[2];
}

// Runs of equal cells in consecutive lanes of a wave (the slots of a tile are
// grouped by cell after a re-binning): each lane learns its run's first lane,
// the first lane also the run's length.  All 64 lanes must call it.
__device__ __forceinline__ void wave_run(int cell, int& head, int& len) {
  const int lane = (int)(threadIdx.x & 63);
  const int prev = __shfl_up(cell, 1);
  const bool first = lane == 0 || prev != cell;
  const unsigned long long heads = __ballot(first);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
  head = 63 - __clzll(heads & upto);
  const unsigned long long after = heads & ~upto;
  len = (after ? __ffsll((long long)after) - 1 : 64) - lane;
}

// A block per tile of the particle bins: an LDS histogram of the tile's cells
// (one atomic per run of equal cells in a wave), kept in thist for the
// scatter, then one global atomic per cell; a run of particles that have left
// the tile since the last binning adds itself.
template <typename PT>
__global__ __launch_bounds__(256) void coul_count_kernel(PT P, WorkLists L,
                                                         int* __restrict__ cnt,
                                                         int* __restrict__ thist) {
  __shared__ int h[64];
  for (int t = blockIdx.x; t < L.ngrid; t += gridDim.x) {
    if (threadIdx.x < 64) h[threadIdx.x] = 0;
    __syncthreads();
    const long p0 = L.tstart[t], p1 = L.tstart[t + 1];
    const int lane = (int)(threadIdx.x & 63);
    for (long base = p0 + (threadIdx.x & ~63); base < p1; base += 256) {
      const long p = base + lane;
      const int c = p < p1 ? coul_cell(P, p, L.ntx, L.nty) : -1;
      int head, len;
      wave_run(c, head, len);
      if (head != lane || c < 0) continue;
      if ((c >> 6) == t)
        atomicAdd(&h[c & 63], len);
      else
        atomicAdd(&cnt[c], len);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      thist[64 * t + threadIdx.x] = h[threadIdx.x];
      if (h[threadIdx.x] > 0) atomicAdd(&cnt[64 * t + threadIdx.x], h[threadIdx.x]);
    }
    __syncthreads();
  }
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

// (order key, slot) of every particle into its cell's range, a block per
// tile: the tile's histogram (from the counting kernel), one atomic per cell
// reserves the tile's run of each cell, LDS atomics (one per run of equal
// cells in a wave) place the particles in it; particles that have left the
// tile reserve their own places.
template <typename PT>
__global__ __launch_bounds__(256) void coul_scatter_kernel(PT P, WorkLists L, CoulombConst C,
                                                           int sp, const int* __restrict__ start,
                                                           int* __restrict__ fill,
                                                           const int* __restrict__ thist,
                                                           unsigned long long* __restrict__ key,
                                                           int* __restrict__ slot) {
  __shared__ int h[64], at[64];
  const uint32_t k = *C.step;
  for (int t = blockIdx.x; t < L.ngrid; t += gridDim.x) {
    const long p0 = L.tstart[t], p1 = L.tstart[t + 1];
    const int lane = (int)(threadIdx.x & 63);
    if (threadIdx.x < 64) {
      const int c = 64 * t + threadIdx.x, n = thist[c];
      at[threadIdx.x] = n > 0 ? start[c] + atomicAdd(&fill[c], n) : 0;
      h[threadIdx.x] = 0;
    }
    __syncthreads();
    for (long base = p0 + (threadIdx.x & ~63); base < p1; base += 256) {
      const long p = base + lane;
      const int c = p < p1 ? coul_cell(P, p, L.ntx, L.nty) : -1;
      int head, len;
      wave_run(c, head, len);
      int off = 0;
      if (head == lane && c >= 0)
        off = (c >> 6) == t ? at[c & 63] + atomicAdd(&h[c & 63], len)
                            : start[c] + atomicAdd(&fill[c], len);
      const int pos = __shfl(off, head) + (lane - head);
      if (c < 0) continue;
      const uint32_t id = P.id[p];
      const uint4 r = philox4x32_10(id, k, kCOrder, (uint32_t)sp, C.key0, C.key1);
      key[pos] = ((unsigned long long)r.x << 32) | id;
      slot[pos] = (int)p;
    }
    __syncthreads();
  }
}

// One binary collision: draws from Philox(id, k, kCPair, word); delta normal
// (Box-Muller cosine branch of words 0, 1) with variance cv n_L / |u|^3, the
// azimuth 2 pi u(word 2); the relative velocity u = va - vb turns by
// theta = 2 atan(delta) about itself, va += fa du, vb -= fb du.
// The draws' three functions of the uniforms, per precision: the normal
// deviate sqrt(-2 ln u1) cos(2 pi u2) and cos, sin of 2 pi u3.
struct CoulDraw64 {
  __device__ static double normal(uint32_t a, uint32_t b) {
    // cospi / sincospi take the angle in half turns: no range reduction by pi
    return sqrt(-2.0 * log(u01_open(a))) * cospi(2.0 * u01_open(b));
  }
  __device__ static void azimuth(uint32_t c, double* s, double* co) {
    sincospi(2.0 * u01_open(c), s, co);
  }
};
struct CoulDraw32 {
  // (w + 1/2) 2^-32 in FP32: w rounded to 24 bits, relative error <= 2^-24
  __device__ static float u01(uint32_t w) {
    return __builtin_fmaf((float)w, 2.3283064365386963e-10f, 1.1641532182693481e-10f);
  }
  // the hardware log2, and cos / sin of 2 pi x taken in turns (x in (0, 1))
  __device__ static float normal(uint32_t a, uint32_t b) {
    const float ln_u = __builtin_amdgcn_logf(u01(a)) * 0.69314718055994531f;
    return __builtin_amdgcn_sqrtf(-2.0f * ln_u) * __builtin_amdgcn_cosf(u01(b));
  }
  __device__ static void azimuth(uint32_t c, float* s, float* co) {
    const float x = u01(c);
    *s = __builtin_amdgcn_sinf(x);
    *co = __builtin_amdgcn_cosf(x);
  }
};
template <typename R> struct CoulDraw;
template <> struct CoulDraw<double> : CoulDraw64 {};
template <> struct CoulDraw<float> : CoulDraw32 {};
__device__ __forceinline__ double coul_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float coul_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double coul_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float coul_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename R>
__device__ void coul_collide(const CoulombConst& C, uint32_t k, uint32_t word, R cv, R fa, R fb,
                             R* va, R* vb, uint32_t id) {
  const R u0 = va[0] - vb[0], u1 = va[1] - vb[1], u2 = va[2] - vb[2];
  const R um2 = u0 * u0 + u1 * u1 + u2 * u2;
  if (!(um2 > (R)0)) return;
  const R um = coul_sqrt(um2);
  const uint4 r = philox4x32_10(id, k, kCPair, word, C.key0, C.key1);
  const R delta = coul_sqrt(cv * coul_rcp(um2 * um)) * CoulDraw<R>::normal(r.x, r.y);
  R sp, cp;
  CoulDraw<R>::azimuth(r.z, &sp, &cp);
  const R inv = coul_rcp((R)1 + delta * delta);
  const R sn = (R)2 * delta * inv;
  const R omc = (R)2 * delta * delta * inv;
  const R up = coul_sqrt(u0 * u0 + u1 * u1);
  R du[3];
  if (up > (R)0) {
    const R iu = coul_rcp(up);
    du[0] = (u0 * iu) * u2 * sn * cp - (u1 * iu) * um * sn * sp - u0 * omc;
    du[1] = (u1 * iu) * u2 * sn * cp + (u0 * iu) * um * sn * sp - u1 * omc;
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

// The pairing rule on velocities held in a cell's arrays (LDS), in key order:
// like items of both species (pairs, an odd count's triplet as one item) over
// the cell's W lanes, a barrier, then the unlike pairs (lane r takes particle r
// of the less numerous species b and its partners j = r, r + N_b, ... of a).
// V(s, q) is the velocity of the q-th particle of species s in key order,
// ID(s, q) its id; LANE is the lane's index among the cell's W lanes.
#define COUL_PAIRS(V, ID, LANE, W)                                                            \
  {                                                                                         \
    /* like items of both species in one list: species 0's, then 1's; an */                \
    /* odd count's triplet is its species' first item */                                   \
    int items[2];                                                                           \
    _Pragma("unroll") for (int s = 0; s < 2; ++s)                                            \
      items[s] = n[s] < 2 ? 0 : ((n[s] & 1) ? 1 + (n[s] - 3) / 2 : n[s] / 2);                 \
    for (int it = (LANE); it < items[0] + items[1]; it += (W)) {                            \
      const int s = it < items[0] ? 0 : 1;                                                  \
      const int i = it - (s ? items[0] : 0);                                                \
      const int N = n[s];                                                                   \
      const R cv = (R)(C.c_var[s] * (double)N * C.w_vol);                                   \
      const R f = (R)C.frac[s][s];                                                          \
      if ((N & 1) && i == 0) {                                                              \
        coul_collide<R>(C, k, (uint32_t)s, (R)0.5 * cv, f, f, V(s, 0), V(s, 1), ID(s, 0));  \
        coul_collide<R>(C, k, (uint32_t)s, (R)0.5 * cv, f, f, V(s, 1), V(s, 2), ID(s, 1));  \
        coul_collide<R>(C, k, (uint32_t)s, (R)0.5 * cv, f, f, V(s, 2), V(s, 0), ID(s, 2));  \
      } else {                                                                              \
        const int q = (N & 1) ? 3 + 2 * (i - 1) : 2 * i;                                     \
        coul_collide<R>(C, k, (uint32_t)s, cv, f, f, V(s, q), V(s, q + 1), ID(s, q));       \
      }                                                                                     \
    }                                                                                       \
    __syncthreads();                                                                        \
    if (n[0] > 0 && n[1] > 0) {                                                             \
      const int sa = n[0] >= n[1] ? 0 : 1, sb = 1 - sa;                                     \
      const int Na = n[sa], Nb = n[sb];                                                     \
      const R cv = (R)(C.c_var[2] * (double)Nb * C.w_vol);                                  \
      for (int r = (LANE); r < Nb; r += (W))                                                \
        for (int j = r; j < Na; j += Nb)                                                    \
          coul_collide<R>(C, k, 2u + (uint32_t)sa, cv, (R)C.frac[2][sa], (R)C.frac[2][sb],  \
                          V(sa, j), V(sb, r), ID(sa, j));                                   \
    }                                                                                       \
    __syncthreads();                                                                        \
  }

// cells whose species each hold at most kCellCap particles go through LDS
constexpr int kCellCap = 64;
constexpr int kPairThreads = 256;  // threads of a pair block: 32 lanes per cell of a group
constexpr int kGroup = kPairThreads / 32;  // consecutive cells staged together
constexpr int kGroupCap = 512;     // staged particles of a species per group
constexpr int kStagePer = kGroupCap / kPairThreads;  // staged particles per thread and species
constexpr int kRunGroups = 16;     // groups of one block: two tiles of 64 cells
template <typename R>
struct GroupStage {
  unsigned long long key[2][kGroupCap];
  int slot[2][kGroupCap];  // in key order inside each cell
  uint32_t id[2][kGroupCap];
  R v[2][kGroupCap][3];
  int start[2][kRunGroups * kGroup + 1];  // the block's cells' starts in the key / slot arrays
};

// cells above the LDS capacity: the rule through global memory, the slots
// ranked into the order array, one cell at a time with the whole block
template <typename PT>
__device__ void global_collide(const PT P[2], const int* const ord[2], const CoulombConst& C,
                               uint32_t k, uint32_t word, typename CoulReal<PT>::T cv,
                               typename CoulReal<PT>::T fa, typename CoulReal<PT>::T fb, int sa,
                               int qa, int sb, int qb, uint32_t id) {
  using R = typename CoulReal<PT>::T;
  const long pa = ord[sa][qa], pb = ord[sb][qb];
  R va[3], vb[3];
  load_v(P[sa], pa, va);
  load_v(P[sb], pb, vb);
  coul_collide<R>(C, k, word, cv, fa, fb, va, vb, id);
  store_v(P[sa], pa, va);
  store_v(P[sb], pb, vb);
}

template <typename PT>
__device__ void cell_global(const PT P[2], const CoulombBufs& B, const CoulombConst& C, uint32_t k,
                            int c, int lane) {
  using R = typename CoulReal<PT>::T;
  int r0[2], n[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    r0[s] = B.start[s][c];
    n[s] = B.start[s][c + 1] - r0[s];
  }
  if (n[0] + n[1] < 2) return;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const unsigned long long* key = B.key[s] + r0[s];
    for (int q = lane; q < n[s]; q += kPairThreads) {
      const unsigned long long kq = key[q];
      int rank = 0;
      for (int t = 0; t < n[s]; ++t) rank += key[t] < kq;
      B.ord[s][r0[s] + rank] = B.slot[s][r0[s] + q];
    }
  }
  __syncthreads();
  const int* const ord[2] = {B.ord[0] + r0[0], B.ord[1] + r0[1]};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int N = n[s];
    if (N < 2) continue;
    const R cv = (R)(C.c_var[s] * (double)N * C.w_vol);
    const R f = (R)C.frac[s][s];
    int first = 0;
    if (N & 1) {
      if (lane == 0) {
        global_collide(P, ord, C, k, (uint32_t)s, (R)0.5 * cv, f, f, s, 0, s, 1, P[s].id[ord[s][0]]);
        global_collide(P, ord, C, k, (uint32_t)s, (R)0.5 * cv, f, f, s, 1, s, 2, P[s].id[ord[s][1]]);
        global_collide(P, ord, C, k, (uint32_t)s, (R)0.5 * cv, f, f, s, 2, s, 0, P[s].id[ord[s][2]]);
      }
      first = 3;
    }
    for (int q = first + 2 * lane; q + 1 < N; q += 2 * kPairThreads)
      global_collide(P, ord, C, k, (uint32_t)s, cv, f, f, s, q, s, q + 1, P[s].id[ord[s][q]]);
  }
  __syncthreads();
  if (n[0] > 0 && n[1] > 0) {
    const int sa = n[0] >= n[1] ? 0 : 1, sb = 1 - sa;
    const int Na = n[sa], Nb = n[sb];
    const R cv = (R)(C.c_var[2] * (double)Nb * C.w_vol);
    const R fa = (R)C.frac[2][sa], fb = (R)C.frac[2][sb];
    for (int r = lane; r < Nb; r += kPairThreads) {
      const long pb = ord[sb][r];
      R vb[3];
      load_v(P[sb], pb, vb);
      for (int j = r; j < Na; j += Nb) {
        const long pa = ord[sa][j];
        R va[3];
        load_v(P[sa], pa, va);
        coul_collide<R>(C, k, 2u + (uint32_t)sa, cv, fa, fb, va, vb, P[sa].id[pa]);
        store_v(P[sa], pa, va);
      }
      store_v(P[sb], pb, vb);
    }
  }
  __syncthreads();
}

// A block takes a run of kRunGroups groups of kGroup consecutive cells (two
// tiles: their key / slot ranges are contiguous, and a tile's particle records
// are gathered and written by one block, through one XCD's L2).  The run's
// cell starts are staged once.  For each group the block stages the keys in
// LDS (a key's low word is the particle's id), ranks each particle inside its
// cell by key, puts slot, id and velocity at the ranked place, runs the pairing
// rule with 32 lanes per cell and writes the velocities back.  The next
// group's keys and slots are loaded into registers while the current group is
// worked on, and the FP32 velocities are gathered before the ranking, so the
// loads overlap the arithmetic instead of waiting in turn.  A group with a
// cell above kCellCap particles of a species, or with more than kGroupCap of a
// species, runs its cells one by one through global memory with the whole
// block.
template <typename PT>
__global__ __launch_bounds__(kPairThreads) void coul_pair_kernel(PT Pe, PT Pi, CoulombBufs B,
                                                                 CoulombConst C) {
  using R = typename CoulReal<PT>::T;
  // FP32 velocities are gathered in registers before the ranking; the FP64
  // ones after it, straight into LDS (their registers would cost occupancy)
  constexpr bool kEarlyV = std::is_same<R, float>::value;
  __shared__ GroupStage<R> sm;
  const int tid = threadIdx.x, cl = tid >> 5, hl = tid & 31;
  const PT P[2] = {Pe, Pi};
  const uint32_t k = *C.step;
  unsigned long long pairings = 0;  // this half-wave's cells, added to the counter once
  const int ngroup = (C.ncell + kGroup - 1) / kGroup;
  const int g_beg = (int)blockIdx.x * kRunGroups;
  const int g_end = min(ngroup, g_beg + kRunGroups);
  if (g_beg >= g_end) return;
  const int c_beg = g_beg * kGroup;
  const int nst = min(C.ncell, g_end * kGroup) - c_beg + 1;  // starts staged per species
  for (int i = tid; i < 2 * nst; i += kPairThreads) {
    const int s = i >= nst ? 1 : 0, j = i - s * nst;
    sm.start[s][j] = B.start[s][c_beg + j];
  }
  __syncthreads();
  // start of cell j of the run (cells past the box are empty)
  auto st_at = [&](int s, int j) { return sm.start[s][min(j, nst - 1)]; };
  unsigned long long pk[2][kStagePer];
  int ps[2][kStagePer];
  auto prefetch = [&](int g) {
    const int j0 = (g - g_beg) * kGroup;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int b = st_at(s, j0), N = min(st_at(s, j0 + kGroup) - b, kGroupCap);
#pragma unroll
      for (int u = 0; u < kStagePer; ++u) {
        const int i = tid + u * kPairThreads;
        if (i < N) {
          pk[s][u] = B.key[s][b + i];
          ps[s][u] = B.slot[s][b + i];
        }
      }
    }
  };
  prefetch(g_beg);
  for (int g = g_beg; g < g_end; ++g) {
    const int c0 = g * kGroup, j0 = (g - g_beg) * kGroup;
    int b[2], N[2], n[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      b[s] = st_at(s, j0);
      N[s] = st_at(s, j0 + kGroup) - b[s];
      n[s] = st_at(s, j0 + cl + 1) - st_at(s, j0 + cl);
    }
    bool fits = N[0] <= kGroupCap && N[1] <= kGroupCap;
#pragma unroll
    for (int j = 0; j < kGroup; ++j)
      fits = fits && st_at(0, j0 + j + 1) - st_at(0, j0 + j) <= kCellCap &&
             st_at(1, j0 + j + 1) - st_at(1, j0 + j) <= kCellCap;
    if (hl == 0) {
#pragma unroll
      for (int s = 0; s < 2; ++s)
        if (n[s] >= 2) pairings += (n[s] & 1) ? 3 + (n[s] - 3) / 2 : n[s] / 2;
      if (n[0] > 0 && n[1] > 0) pairings += n[0] > n[1] ? n[0] : n[1];
    }
    // this group's keys and slots; the next group's start loading
    unsigned long long kk[2][kStagePer];
    int sl[2][kStagePer];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int u = 0; u < kStagePer; ++u) {
        kk[s][u] = pk[s][u];
        sl[s][u] = ps[s][u];
      }
    if (g + 1 < g_end) prefetch(g + 1);
    if (!fits) {  // (block-uniform)
      for (int j = 0; j < kGroup && c0 + j < C.ncell; ++j) cell_global(P, B, C, k, c0 + j, tid);
      __syncthreads();
      continue;
    }
    R vv[2][kStagePer][3];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int u = 0; u < kStagePer; ++u) {
        const int i = tid + u * kPairThreads;
        if (i < N[s]) {
          sm.key[s][i] = kk[s][u];
          if (kEarlyV) load_v(P[s], sl[s][u], vv[s][u]);
        }
      }
    __syncthreads();
    // rank inside the cell; slot, id and velocity to the ranked place
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int u = 0; u < kStagePer; ++u) {
        const int i = tid + u * kPairThreads;
        if (i >= N[s]) continue;
        int j = 0;
        while (j + 1 < kGroup && st_at(s, j0 + j + 1) - b[s] <= i) ++j;
        const int lo = st_at(s, j0 + j) - b[s], hi = st_at(s, j0 + j + 1) - b[s];
        const unsigned long long kq = kk[s][u];
        int rank = lo;
        for (int t = lo; t < hi; ++t) rank += sm.key[s][t] < kq;
        sm.slot[s][rank] = sl[s][u];
        sm.id[s][rank] = (uint32_t)kq;
        if (kEarlyV) {
#pragma unroll
          for (int a = 0; a < 3; ++a) sm.v[s][rank][a] = vv[s][u][a];
        } else {
          load_v(P[s], sl[s][u], sm.v[s][rank]);
        }
      }
    __syncthreads();
    const int o0 = st_at(0, j0 + cl) - b[0], o1 = st_at(1, j0 + cl) - b[1];
#define GRP_V(s, q) (sm.v[s][((s) ? o1 : o0) + (q)])
#define GRP_ID(s, q) (sm.id[s][((s) ? o1 : o0) + (q)])
    COUL_PAIRS(GRP_V, GRP_ID, hl, 32)
#undef GRP_V
#undef GRP_ID
#pragma unroll
    for (int s = 0; s < 2; ++s)
      for (int i = tid; i < N[s]; i += kPairThreads) store_v(P[s], sm.slot[s][i], sm.v[s][i]);
    __syncthreads();
  }
  if (hl == 0 && pairings) atomicAdd(B.count, pairings);
}

template <typename PT>
void coulomb_impl(const PT P[2], const WorkLists L[2], const CoulombBufs& B, const CoulombConst& C,
                  const long cap[2], hipStream_t st) {
  const long ncell = C.ncell;
  for (int s = 0; s < 2; ++s) {
    launch_zero_i32(B.start[s], ncell + 1, st);
    launch_zero_i32(B.fill[s], ncell, st);
    const int g = std::min(L[s].ngrid, 65536);
    if (cap[s] > 0 && g > 0)
      hipLaunchKernelGGL(coul_count_kernel<PT>, dim3(g), dim3(256), 0, st, P[s], L[s], B.start[s],
                         B.thist[s]);
    const long n = ncell + 1;
    const int nb = nblk(n, kScanChunk);
    hipLaunchKernelGGL(coul_scan_local, dim3(nb), dim3(256), 0, st, B.start[s], n, B.sums);
    hipLaunchKernelGGL(coul_scan_sums, dim3(1), dim3(256), 0, st, B.sums, nb);
    hipLaunchKernelGGL(coul_scan_add, dim3(nb), dim3(256), 0, st, B.start[s], n, B.sums);
    if (cap[s] > 0 && g > 0)
      hipLaunchKernelGGL(coul_scatter_kernel<PT>, dim3(g), dim3(256), 0, st, P[s], L[s], C, s,
                         B.start[s], B.fill[s], B.thist[s], B.key[s], B.slot[s]);
  }
  const long ngroup = (ncell + kGroup - 1) / kGroup;
  const int grid = (int)((ngroup + kRunGroups - 1) / kRunGroups);
  hipLaunchKernelGGL(coul_pair_kernel<PT>, dim3(grid), dim3(kPairThreads), 0, st, P[0], P[1], B,
                     C);
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
