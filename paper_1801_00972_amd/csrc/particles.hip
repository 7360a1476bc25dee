// particles.hip -- particle kernels of the hot path (gfx950, wave64):
//   loading, the fused gather / leapfrog / wall / grain / collision / deposit
//   kernel in its FP64 and FP32R forms, the standalone deposit, and the
//   counting sort that keeps the particle arrays ordered by cell.
//
// Method (arXiv:1801.00972, Sec. III): CIC charge assignment and field gather
// on the cell corners, leapfrog Eq. (1)-(2), PPPM near-grain field Eq. (5)-(6)
// with dt_MD = dt/40, perfect absorption at electrodes and grains, binary
// collisions with the neutral reservoir (Table I) in null-collision form.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "launch.hpp"

namespace pic {

enum { ST_ALIVE = 0, ST_WALL0 = 1, ST_WALL1 = 2, ST_GRAIN = 3, ST_NONE = 4, ST_BAD = 5 };

// electrode test of a position already wrapped in x,y; a non-finite or
// out-of-range coordinate (which no valid input produces) removes the particle
__device__ __forceinline__ int z_status(const double x[3], const SpeciesStep& S) {
  if (x[2] >= 0.0 && x[2] < (double)S.nz) {
    return (x[0] >= 0.0 && x[0] < (double)S.nx && x[1] >= 0.0 && x[1] < (double)S.ny) ? ST_ALIVE
                                                                                     : ST_BAD;
  }
  if (x[2] < 0.0) return ST_WALL0;
  if (x[2] >= (double)S.nz) return ST_WALL1;
  return ST_BAD;
}

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// ---------------------------------------------------------------- field loads
__device__ __forceinline__ void load_node(const double2* __restrict__ E, long n, double& ex,
                                          double& ey, double& ez) {
  const double2 a = E[2 * n], b = E[2 * n + 1];
  ex = a.x;
  ey = a.y;
  ez = b.x;
}
__device__ __forceinline__ void load_node(const float4* __restrict__ E, long n, double& ex,
                                          double& ey, double& ez) {
  const float4 a = E[n];
  ex = a.x;
  ey = a.y;
  ez = a.z;
}

// CIC gather in double precision at cell (i0,j0,k0), offsets (fx,fy,fz)
template <typename ET>
__device__ __forceinline__ void gather_d(const ET* __restrict__ E, const SpeciesStep& S, int i0,
                                         int j0, int k0, double fx, double fy, double fz,
                                         double out[3]) {
  const int i1 = i0 + 1 == S.nx ? 0 : i0 + 1;
  const int j1 = j0 + 1 == S.ny ? 0 : j0 + 1;
  const long r00 = (long)S.nx * j0 + (long)S.nxy * k0;
  const long r10 = (long)S.nx * j1 + (long)S.nxy * k0;
  const long r01 = r00 + S.nxy, r11 = r10 + S.nxy;
  const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
  const long base[4] = {r00, r10, r01, r11};
  out[0] = out[1] = out[2] = 0.0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const double wyz = wy[t & 1] * wz[t >> 1];
    double ex, ey, ez;
    load_node(E, base[t] + i0, ex, ey, ez);
    out[0] += wx[0] * wyz * ex;
    out[1] += wx[0] * wyz * ey;
    out[2] += wx[0] * wyz * ez;
    load_node(E, base[t] + i1, ex, ey, ez);
    out[0] += wx[1] * wyz * ex;
    out[1] += wx[1] * wyz * ey;
    out[2] += wx[1] * wyz * ez;
  }
}

// ---------------------------------------------------------------- MD region
__device__ __forceinline__ uint32_t md_lookup(const MdTables& md, int nx, int ny, int i, int j,
                                              int k) {
  if (md.n_grains == 0) return 0u;
  int a = i - md.bx0;
  if (a < 0) a += nx;
  if (a >= md.bsx) return 0u;
  int b = j - md.by0;
  if (b < 0) b += ny;
  if (b >= md.bsy) return 0u;
  const int c = k - md.bz0;
  if (c < 0 || c >= md.bsz) return 0u;
  return md.cell_list[((long)c * md.bsy + b) * md.bsx + a];
}

// separation x - x_g (cell units), minimum image across the periodic x,y
__device__ __forceinline__ void grain_sep(const MdTables& md, const SpeciesStep& S, int g,
                                          const double x[3], double r[3]) {
  r[0] = x[0] - md.gpos[3 * g + 0];
  r[1] = x[1] - md.gpos[3 * g + 1];
  r[2] = x[2] - md.gpos[3 * g + 2];
  if (r[0] > 0.5 * S.nx) r[0] -= S.nx;
  else if (r[0] < -0.5 * S.nx) r[0] += S.nx;
  if (r[1] > 0.5 * S.ny) r[1] -= S.ny;
  else if (r[1] < -0.5 * S.ny) r[1] += S.ny;
}

// CIC gather of grain g's unit-charge field from its cube of nodes
__device__ __forceinline__ void gather_unit(const MdTables& md, const SpeciesStep& S, int g,
                                            int i0, int j0, int k0, double fx, double fy,
                                            double fz, double out[3]) {
  const int c = md.cutoff, side = md.side;
  const long cube = (long)side * side * side;
  int lx = i0 - (md.gcell[3 * g + 0] - c);
  lx = ((lx % S.nx) + S.nx) % S.nx;
  int ly = j0 - (md.gcell[3 * g + 1] - c);
  ly = ((ly % S.ny) + S.ny) % S.ny;
  const int lz = k0 - (md.gcell[3 * g + 2] - c);
  const double* U = md.U + (long)g * 3 * cube;
  out[0] = out[1] = out[2] = 0.0;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int a = t & 1, b = (t >> 1) & 1, cc = t >> 2;
    const double w = (a ? fx : 1.0 - fx) * (b ? fy : 1.0 - fy) * (cc ? fz : 1.0 - fz);
    const long l = ((long)(lz + cc) * side + (ly + b)) * side + (lx + a);
    out[0] += w * U[l];
    out[1] += w * U[cube + l];
    out[2] += w * U[2 * cube + l];
  }
}

__device__ __forceinline__ double wrap_coord(double X, int n) {
  if (X < 0.0) X += (double)n;
  else if (X >= (double)n) X -= (double)n;
  if (X >= (double)n) X -= (double)n;  // -tiny + n rounds to n
  if (X < 0.0 || X >= (double)n) X = X - (double)n * floor(X / (double)n);
  return X;
}

// Sub-cycled PPPM motion near grains, Eq. (5)-(6): md_sub sub-steps of
// h = dt/md_sub with E = E_mesh - sum_g Q_g U_g + sum_g Q_g r / (4 pi eps0 r^3)
// over the grains whose cube holds the current cell; hit when |r| <= a.
template <typename ET>
__device__ int md_move(const ET* __restrict__ E, const MdTables& md, const SpeciesStep& S,
                       double x[3], double v[3], int& hit) {
  for (int sub = 0; sub < S.md_sub; ++sub) {
    int i0 = (int)floor(x[0]), j0 = (int)floor(x[1]), k0 = (int)floor(x[2]);
    double fx = x[0] - i0, fy = x[1] - j0, fz = x[2] - k0;
    double Ep[3];
    gather_d(E, S, i0, j0, k0, fx, fy, fz, Ep);
    uint32_t cl = md_lookup(md, S.nx, S.ny, i0, j0, k0);
    for (uint32_t t = 0; t < (cl & 255u); ++t) {
      const int g = md.grain_idx[(cl >> 8) + t];
      const double Q = md.Q[g];
      if (Q == 0.0) continue;
      double r[3];
      grain_sep(md, S, g, x, r);
      r[0] *= S.dx;
      r[1] *= S.dx;
      r[2] *= S.dx;
      const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      const double inv = 1.0 / (4.0 * kPi * kEps0 * r2 * sqrt(r2));
      double Um[3];
      gather_unit(md, S, g, i0, j0, k0, fx, fy, fz, Um);
      Ep[0] += Q * (r[0] * inv - Um[0]);
      Ep[1] += Q * (r[1] * inv - Um[1]);
      Ep[2] += Q * (r[2] * inv - Um[2]);
    }
    v[0] += S.qm_h * Ep[0];
    v[1] += S.qm_h * Ep[1];
    v[2] += S.qm_h * Ep[2];
    x[0] = wrap_coord(x[0] + v[0] * S.h_dx, S.nx);
    x[1] = wrap_coord(x[1] + v[1] * S.h_dx, S.ny);
    x[2] += v[2] * S.h_dx;
    const int zs = z_status(x, S);
    if (zs != ST_ALIVE) return zs;
    i0 = (int)floor(x[0]);
    j0 = (int)floor(x[1]);
    k0 = (int)floor(x[2]);
    cl = md_lookup(md, S.nx, S.ny, i0, j0, k0);
    for (uint32_t t = 0; t < (cl & 255u); ++t) {
      const int g = md.grain_idx[(cl >> 8) + t];
      double r[3];
      grain_sep(md, S, g, x, r);
      r[0] *= S.dx;
      r[1] *= S.dx;
      r[2] *= S.dx;
      if (r[0] * r[0] + r[1] * r[1] + r[2] * r[2] <= md.a2) {
        hit = g;
        return ST_GRAIN;
      }
    }
  }
  return ST_ALIVE;
}

// ---------------------------------------------------------------- collisions
// Null-collision MCC against the neutral reservoir: candidate iff Philox word 0
// is below the integer threshold of P' = 1 - exp(-n_g sigma g_cap dt); accept
// with probability g / g_cap.  e-Ar: elastic, isotropic in the CM frame with
// the neutral at rest.  Ar+-Ar: charge exchange, the ion takes the velocity of
// the neutral drawn from the 300 K reservoir.
__device__ __forceinline__ void collide(const SpeciesStep& S, uint32_t id, double v[3], bool& coll,
                                        bool& capv) {
  const uint4 r = philox4x32_10(id, S.step, kColl, (uint32_t)S.sp, S.key0, S.key1);
  if ((uint64_t)r.x >= S.T_null) return;
  double vn[3] = {0.0, 0.0, 0.0};
  if (S.sp == 1) {
    const uint4 q = philox4x32_10(id, S.step, kNeutral, 1u, S.key0, S.key1);
    double n0, n1, n2, n3;
    normal_pair(q.x, q.y, n0, n1);
    normal_pair(q.z, q.w, n2, n3);
    vn[0] = S.vth_gas * n0;
    vn[1] = S.vth_gas * n1;
    vn[2] = S.vth_gas * n2;
  }
  const double gx = v[0] - vn[0], gy = v[1] - vn[1], gz = v[2] - vn[2];
  const double g = sqrt(gx * gx + gy * gy + gz * gz);
  const double ratio = g * S.inv_g_cap;
  bool accept;
  if (ratio > 1.0) {
    capv = true;
    accept = true;
  } else {
    accept = u01_open(r.y) < ratio;
  }
  if (!accept) return;
  coll = true;
  if (S.sp == 0) {
    const double cost = 1.0 - 2.0 * u01_open(r.z);
    const double sint = sqrt(fmax(0.0, 1.0 - cost * cost));
    double sp, cp;
    sincos(2.0 * kPi * u01_open(r.w), &sp, &cp);
    const double nh[3] = {sint * cp, sint * sp, cost};
    for (int a = 0; a < 3; ++a) v[a] = S.mass_ratio_e * v[a] + S.mass_ratio_n * g * nh[a];
  } else {
    v[0] = vn[0];
    v[1] = vn[1];
    v[2] = vn[2];
  }
}

// ---------------------------------------------------------------- deposit
// FP64 form: rho accumulates sign * W in units of the macro charge w e.
__device__ __forceinline__ void deposit_f64(double* __restrict__ rho, const SpeciesStep& S,
                                            double X, double Y, double Z) {
  const int i0 = (int)floor(X), j0 = (int)floor(Y), k0 = (int)floor(Z);
  const double fx = X - i0, fy = Y - j0, fz = Z - k0;
  const int i1 = i0 + 1 == S.nx ? 0 : i0 + 1;
  const int j1 = j0 + 1 == S.ny ? 0 : j0 + 1;
  const double s = S.sign;
  const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
  const int ii[2] = {i0, i1}, jj[2] = {j0, j1};
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int a = t & 1, b = (t >> 1) & 1, c = t >> 2;
    const long n = ii[a] + (long)S.nx * jj[b] + (long)S.nxy * (k0 + c);
    unsafeAtomicAdd(&rho[n], s * wx[a] * wy[b] * wz[c]);
  }
}

// FP32R form: the macro charge Qp (2^-32 e) split exactly into 8 non-negative
// parts, along x by q1 = (Q f24) >> 24 with f24 = floor(offset 2^24), then each
// half along y, each quarter along z; integer atomics, so the sum is exact and
// independent of order.
__device__ __forceinline__ void split8(long long Q, float ox, float oy, float oz,
                                       long long part[8]) {
  const long long qx = (long long)(ox * 16777216.0f);
  const long long qy = (long long)(oy * 16777216.0f);
  const long long qz = (long long)(oz * 16777216.0f);
  long long ax[2];
  ax[1] = (Q * qx) >> 24;
  ax[0] = Q - ax[1];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const long long y1 = (ax[a] * qy) >> 24;
    const long long yy[2] = {ax[a] - y1, y1};
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const long long z1 = (yy[b] * qz) >> 24;
      part[a + 2 * b] = yy[b] - z1;
      part[a + 2 * b + 4] = z1;
    }
  }
}

__device__ __forceinline__ void deposit_fixed(long long* __restrict__ rho, const SpeciesStep& S,
                                              int i0, int j0, int k0, float ox, float oy,
                                              float oz) {
  long long part[8];
  split8(S.Qp, ox, oy, oz, part);
  const int i1 = i0 + 1 == S.nx ? 0 : i0 + 1;
  const int j1 = j0 + 1 == S.ny ? 0 : j0 + 1;
  const int ii[2] = {i0, i1}, jj[2] = {j0, j1};
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int a = t & 1, b = (t >> 1) & 1, c = t >> 2;
    const long n = ii[a] + (long)S.nx * jj[b] + (long)S.nxy * (k0 + c);
    atomicAdd((unsigned long long*)&rho[n], (unsigned long long)(S.isign * part[t]));
  }
}

// ---------------------------------------------------------------- helpers
// Block-wide stream compaction: each kept thread gets a slot in the output;
// the block reserves its range with one atomic.
__device__ __forceinline__ int compact_slot(bool keep, int* n_out, int* s_wave, int* s_base) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long m = __ballot(keep);
  const int before = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) s_wave[wave] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < kWaves; ++w) {
      const int cnt = s_wave[w];
      s_wave[w] = tot;
      tot += cnt;
    }
    *s_base = tot ? atomicAdd(n_out, tot) : 0;
  }
  __syncthreads();
  return *s_base + s_wave[wave] + before;
}

__device__ __forceinline__ void wave_count(bool flag, unsigned long long* dst) {
  const unsigned long long m = __ballot(flag);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(dst, (unsigned long long)__popcll(m));
}

// ---------------------------------------------------------------- push, FP64
__global__ __launch_bounds__(kBlock) void push_f64_kernel(
    PartF64 in, PartF64 out, const int* __restrict__ n_in, int* __restrict__ n_out,
    const double2* __restrict__ E, double* __restrict__ rho_next, MdTables md, SpeciesStep S,
    Tallies* __restrict__ T, unsigned long long* __restrict__ grain_count, int do_mcc) {
  __shared__ int s_wave[kWaves];
  __shared__ int s_base;
  const int n = *n_in;
  if ((long)blockIdx.x * kBlock >= n) return;
  const int p = blockIdx.x * kBlock + threadIdx.x;
  int st = ST_NONE;
  double x[3], v[3];
  uint32_t id = 0;
  bool coll = false, capv = false, is_md = false;
  if (p < n) {
    x[0] = in.x[p];
    x[1] = in.y[p];
    x[2] = in.z[p];
    v[0] = in.vx[p];
    v[1] = in.vy[p];
    v[2] = in.vz[p];
    id = in.id[p];
    const int i0 = (int)floor(x[0]), j0 = (int)floor(x[1]), k0 = (int)floor(x[2]);
    if (md_lookup(md, S.nx, S.ny, i0, j0, k0) == 0u) {
      // plain PIC particle: gather, kick Eq. (2), drift Eq. (1)
      double Ep[3];
      gather_d(E, S, i0, j0, k0, x[0] - i0, x[1] - j0, x[2] - k0, Ep);
      v[0] += S.qm_dt * Ep[0];
      v[1] += S.qm_dt * Ep[1];
      v[2] += S.qm_dt * Ep[2];
      x[0] = wrap_coord(x[0] + v[0] * S.dt_dx, S.nx);
      x[1] = wrap_coord(x[1] + v[1] * S.dt_dx, S.ny);
      x[2] += v[2] * S.dt_dx;
      st = z_status(x, S);
    } else {
      is_md = true;
      int hit = -1;
      st = md_move(E, md, S, x, v, hit);
      if (st == ST_GRAIN) atomicAdd(&grain_count[2 * hit + S.sp], 1ull);
    }
    if (st == ST_ALIVE && do_mcc) collide(S, id, v, coll, capv);
  }
  const bool keep = st == ST_ALIVE;
  const int dst = compact_slot(keep, n_out, s_wave, &s_base);
  if (keep) {
    out.x[dst] = x[0];
    out.y[dst] = x[1];
    out.z[dst] = x[2];
    out.vx[dst] = v[0];
    out.vy[dst] = v[1];
    out.vz[dst] = v[2];
    out.id[dst] = id;
    deposit_f64(rho_next, S, x[0], x[1], x[2]);
  }
  wave_count(st == ST_WALL0, &T->wall[0][S.sp]);
  wave_count(st == ST_WALL1, &T->wall[1][S.sp]);
  wave_count(coll, &T->n_coll[S.sp]);
  wave_count(capv, &T->cap_viol[S.sp]);
  wave_count(is_md, &T->md[S.sp]);
  wave_count(st == ST_BAD, &T->numeric_bad);
}

// ---------------------------------------------------------------- push, FP32R
__device__ __forceinline__ float gather1(const float4 e, int comp) {
  return comp == 0 ? e.x : (comp == 1 ? e.y : e.z);
}

__global__ __launch_bounds__(kBlock) void push_f32r_kernel(
    PartF32R in, PartF32R out, const int* __restrict__ n_in, int* __restrict__ n_out,
    const float4* __restrict__ E, long long* __restrict__ rho_next, MdTables md, SpeciesStep S,
    Tallies* __restrict__ T, unsigned long long* __restrict__ grain_count, int do_mcc) {
  __shared__ int s_wave[kWaves];
  __shared__ int s_base;
  const int n = *n_in;
  if ((long)blockIdx.x * kBlock >= n) return;
  const int p = blockIdx.x * kBlock + threadIdx.x;
  int st = ST_NONE;
  int ci = 0, cj = 0, ck = 0;
  float o[3] = {0.f, 0.f, 0.f}, vf[3] = {0.f, 0.f, 0.f};
  uint32_t id = 0;
  bool coll = false, capv = false, is_md = false;
  if (p < n) {
    const int cell = in.cell[p];
    o[0] = in.ox[p];
    o[1] = in.oy[p];
    o[2] = in.oz[p];
    vf[0] = in.vx[p];
    vf[1] = in.vy[p];
    vf[2] = in.vz[p];
    id = in.id[p];
    ck = cell / S.nxy;
    const int rem = cell - ck * S.nxy;
    cj = rem / S.nx;
    ci = rem - cj * S.nx;
    if (md_lookup(md, S.nx, S.ny, ci, cj, ck) == 0u) {
      // gather in FP32 from the FP32 field
      const int i1 = ci + 1 == S.nx ? 0 : ci + 1;
      const int j1 = cj + 1 == S.ny ? 0 : cj + 1;
      const long r00 = (long)S.nx * cj + (long)S.nxy * ck;
      const long r10 = (long)S.nx * j1 + (long)S.nxy * ck;
      const long base[4] = {r00, r10, r00 + S.nxy, r10 + S.nxy};
      const float wx0 = 1.0f - o[0], wx1 = o[0];
      const float wy[2] = {1.0f - o[1], o[1]}, wz[2] = {1.0f - o[2], o[2]};
      float e0 = 0.f, e1 = 0.f, e2 = 0.f;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float wyz = wy[t & 1] * wz[t >> 1];
        const float4 a = E[base[t] + ci];
        const float4 b = E[base[t] + i1];
        e0 += wyz * (wx0 * a.x + wx1 * b.x);
        e1 += wyz * (wx0 * a.y + wx1 * b.y);
        e2 += wyz * (wx0 * a.z + wx1 * b.z);
      }
      vf[0] += S.qm_dt_f * e0;
      vf[1] += S.qm_dt_f * e1;
      vf[2] += S.qm_dt_f * e2;
      int d[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        float f = o[a] + vf[a] * S.dt_dx_f;
        const float fl = floorf(f);
        f -= fl;
        d[a] = (int)fl;
        if (f >= 1.0f) {  // -tiny + 1 rounds to 1
          f = 0.0f;
          d[a] += 1;
        }
        o[a] = f;
      }
      ci += d[0];
      cj += d[1];
      ck += d[2];
      if (ci < 0 || ci >= S.nx) ci = ((ci % S.nx) + S.nx) % S.nx;
      if (cj < 0 || cj >= S.ny) cj = ((cj % S.ny) + S.ny) % S.ny;
      st = ck < 0 ? ST_WALL0 : (ck >= S.nz ? ST_WALL1 : ST_ALIVE);
      if (!(o[0] >= 0.0f && o[0] < 1.0f && o[1] >= 0.0f && o[1] < 1.0f && o[2] >= 0.0f &&
            o[2] < 1.0f && vf[0] == vf[0] && vf[1] == vf[1] && vf[2] == vf[2]))
        st = ST_BAD;
    } else {
      // near a grain: the sub-cycled path runs in FP64 on the exact position
      is_md = true;
      double x[3] = {(double)ci + (double)o[0], (double)cj + (double)o[1],
                     (double)ck + (double)o[2]};
      double v[3] = {vf[0], vf[1], vf[2]};
      int hit = -1;
      st = md_move(E, md, S, x, v, hit);
      if (st == ST_GRAIN) atomicAdd(&grain_count[2 * hit + S.sp], 1ull);
      if (st == ST_ALIVE) {
        ci = (int)floor(x[0]);
        cj = (int)floor(x[1]);
        ck = (int)floor(x[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int c = a == 0 ? ci : (a == 1 ? cj : ck);
          float f = (float)(x[a] - (double)c);
          if (f >= 1.0f) {
            f = 0.0f;
            if (a == 0) ci = ci + 1 == S.nx ? 0 : ci + 1;
            if (a == 1) cj = cj + 1 == S.ny ? 0 : cj + 1;
            if (a == 2) ck += 1;
          }
          o[a] = f;
        }
        if (ck >= S.nz) st = ST_WALL1;
      }
      vf[0] = (float)v[0];
      vf[1] = (float)v[1];
      vf[2] = (float)v[2];
    }
    if (st == ST_ALIVE && do_mcc) {
      // the candidate test is integer; the kinematics of the few candidates run in FP64
      const uint4 r = philox4x32_10(id, S.step, kColl, (uint32_t)S.sp, S.key0, S.key1);
      if ((uint64_t)r.x < S.T_null) {
        double v[3] = {vf[0], vf[1], vf[2]};
        collide(S, id, v, coll, capv);
        vf[0] = (float)v[0];
        vf[1] = (float)v[1];
        vf[2] = (float)v[2];
      }
    }
  }
  const bool keep = st == ST_ALIVE;
  const int dst = compact_slot(keep, n_out, s_wave, &s_base);
  if (keep) {
    out.cell[dst] = ci + S.nx * (cj + S.ny * ck);
    out.ox[dst] = o[0];
    out.oy[dst] = o[1];
    out.oz[dst] = o[2];
    out.vx[dst] = vf[0];
    out.vy[dst] = vf[1];
    out.vz[dst] = vf[2];
    out.id[dst] = id;
    deposit_fixed(rho_next, S, ci, cj, ck, o[0], o[1], o[2]);
  }
  wave_count(st == ST_WALL0, &T->wall[0][S.sp]);
  wave_count(st == ST_WALL1, &T->wall[1][S.sp]);
  wave_count(coll, &T->n_coll[S.sp]);
  wave_count(capv, &T->cap_viol[S.sp]);
  wave_count(is_md, &T->md[S.sp]);
  wave_count(st == ST_BAD, &T->numeric_bad);
}

// ---------------------------------------------------------------- loading
// Particle p of a species sits in cell p / ppc (x fastest); offsets are the top
// 24 bits of three Philox words (exact in FP32); velocities are Maxwellian by
// Box-Muller, per-component sigma = sqrt(kT/m), taken as v_{-1/2}.
__device__ __forceinline__ void load_draws(uint32_t p, int sp, uint32_t k0, uint32_t k1,
                                           double vth, double off[3], double vel[3]) {
  const uint4 a = philox4x32_10(p, 0u, kInitPos, (uint32_t)sp, k0, k1);
  off[0] = (double)(a.x >> 8) * 5.9604644775390625e-08;
  off[1] = (double)(a.y >> 8) * 5.9604644775390625e-08;
  off[2] = (double)(a.z >> 8) * 5.9604644775390625e-08;
  const uint4 b = philox4x32_10(p, 0u, kInitVel, (uint32_t)sp, k0, k1);
  double n0, n1, n2, n3;
  normal_pair(b.x, b.y, n0, n1);
  normal_pair(b.z, b.w, n2, n3);
  vel[0] = vth * n0;
  vel[1] = vth * n1;
  vel[2] = vth * n2;
}

__global__ void init_f64_kernel(PartF64 P, int n, int ppc, int nx, int ny, int sp, uint32_t k0,
                                uint32_t k1, double vth) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int cell = p / ppc;
  const int i = cell % nx, j = (cell / nx) % ny, k = cell / (nx * ny);
  double off[3], vel[3];
  load_draws((uint32_t)p, sp, k0, k1, vth, off, vel);
  P.x[p] = i + off[0];
  P.y[p] = j + off[1];
  P.z[p] = k + off[2];
  P.vx[p] = vel[0];
  P.vy[p] = vel[1];
  P.vz[p] = vel[2];
  P.id[p] = (uint32_t)p;
}

__global__ void init_f32r_kernel(PartF32R P, int n, int ppc, int sp, uint32_t k0, uint32_t k1,
                                 double vth) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double off[3], vel[3];
  load_draws((uint32_t)p, sp, k0, k1, vth, off, vel);
  P.cell[p] = p / ppc;
  P.ox[p] = (float)off[0];
  P.oy[p] = (float)off[1];
  P.oz[p] = (float)off[2];
  P.vx[p] = (float)vel[0];
  P.vy[p] = (float)vel[1];
  P.vz[p] = (float)vel[2];
  P.id[p] = (uint32_t)p;
}

// ---------------------------------------------------------------- deposit only
__global__ void deposit_f64_kernel(PartF64 P, const int* __restrict__ n_in,
                                   double* __restrict__ rho, SpeciesStep S) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= *n_in) return;
  deposit_f64(rho, S, P.x[p], P.y[p], P.z[p]);
}

__global__ void deposit_f32r_kernel(PartF32R P, const int* __restrict__ n_in,
                                    long long* __restrict__ rho, SpeciesStep S) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= *n_in) return;
  const int cell = P.cell[p];
  const int k = cell / S.nxy, rem = cell - k * S.nxy, j = rem / S.nx, i = rem - j * S.nx;
  deposit_fixed(rho, S, i, j, k, P.ox[p], P.oy[p], P.oz[p]);
}

// ---------------------------------------------------------------- cell sort
__device__ __forceinline__ int cell_of(const PartF64& P, int p, int nx, int ny) {
  return (int)floor(P.x[p]) + nx * ((int)floor(P.y[p]) + ny * (int)floor(P.z[p]));
}
__device__ __forceinline__ int cell_of(const PartF32R& P, int p, int, int) { return P.cell[p]; }

template <typename PT>
__global__ void sort_hist_kernel(PT P, const int* __restrict__ n_in, int* __restrict__ hist,
                                 int nx, int ny) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= *n_in) return;
  atomicAdd(&hist[cell_of(P, p, nx, ny)], 1);
}

__device__ __forceinline__ void copy_particle(const PartF64& a, int i, const PartF64& b, int j) {
  b.x[j] = a.x[i];
  b.y[j] = a.y[i];
  b.z[j] = a.z[i];
  b.vx[j] = a.vx[i];
  b.vy[j] = a.vy[i];
  b.vz[j] = a.vz[i];
  b.id[j] = a.id[i];
}
__device__ __forceinline__ void copy_particle(const PartF32R& a, int i, const PartF32R& b, int j) {
  b.cell[j] = a.cell[i];
  b.ox[j] = a.ox[i];
  b.oy[j] = a.oy[i];
  b.oz[j] = a.oz[i];
  b.vx[j] = a.vx[i];
  b.vy[j] = a.vy[i];
  b.vz[j] = a.vz[i];
  b.id[j] = a.id[i];
}

template <typename PT>
__global__ void sort_scatter_kernel(PT src, PT dst, const int* __restrict__ n_in,
                                    int* __restrict__ cursor, int nx, int ny) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= *n_in) return;
  const int d = atomicAdd(&cursor[cell_of(src, p, nx, ny)], 1);
  copy_particle(src, p, dst, d);
}

// exclusive scan of an int array: per-block sums, scan of the sums, per-block scan
constexpr int kScanBlock = 1024;
__global__ void scan_block_sums(const int* __restrict__ a, int n, int* __restrict__ sums) {
  __shared__ int s[kScanBlock];
  const int i = blockIdx.x * kScanBlock + threadIdx.x;
  s[threadIdx.x] = i < n ? a[i] : 0;
  __syncthreads();
  for (int off = kScanBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = s[0];
}

__global__ void scan_sums_serial(int* __restrict__ sums, int nb) {
  // one block: exclusive scan of the block sums, chunk by chunk
  __shared__ int s[kScanBlock];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += kScanBlock) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? sums[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
      const int t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) sums[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == kScanBlock - 1) carry += s[threadIdx.x];
    __syncthreads();
  }
}

__global__ void scan_apply(const int* __restrict__ a, int n, const int* __restrict__ sums,
                           int* __restrict__ out) {
  __shared__ int s[kScanBlock];
  const int i = blockIdx.x * kScanBlock + threadIdx.x;
  const int v = i < n ? a[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const int t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) out[i] = sums[blockIdx.x] + s[threadIdx.x] - v;
}

__global__ void fill_int_kernel(int* a, long n, int v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// ---------------------------------------------------------------- launchers
static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

void launch_push_f64(const PartF64& in, const PartF64& out, const int* n_in, int* n_out,
                     const double* E, double* rho_next, const MdTables& md,
                     const SpeciesStep& S, Tallies* T, unsigned long long* gc, int do_mcc,
                     long capacity, hipStream_t st) {
  if (capacity <= 0) return;
  hipLaunchKernelGGL(push_f64_kernel, dim3(nblk(capacity, kBlock)), dim3(kBlock), 0, st, in, out,
                     n_in, n_out, (const double2*)E, rho_next, md, S, T, gc, do_mcc);
}

void launch_push_f32r(const PartF32R& in, const PartF32R& out, const int* n_in, int* n_out,
                      const float* E, long long* rho_next, const MdTables& md,
                      const SpeciesStep& S, Tallies* T, unsigned long long* gc, int do_mcc,
                      long capacity, hipStream_t st) {
  if (capacity <= 0) return;
  hipLaunchKernelGGL(push_f32r_kernel, dim3(nblk(capacity, kBlock)), dim3(kBlock), 0, st, in,
                     out, n_in, n_out, (const float4*)E, rho_next, md, S, T, gc, do_mcc);
}

void launch_init_f64(const PartF64& P, int n, int ppc, int nx, int ny, int sp, uint32_t k0,
                     uint32_t k1, double vth, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(init_f64_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, P, n, ppc, nx, ny, sp,
                     k0, k1, vth);
}

void launch_init_f32r(const PartF32R& P, int n, int ppc, int sp, uint32_t k0, uint32_t k1,
                      double vth, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(init_f32r_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, P, n, ppc, sp, k0,
                     k1, vth);
}

void launch_deposit_f64(const PartF64& P, const int* n_in, double* rho, const SpeciesStep& S,
                        long capacity, hipStream_t st) {
  if (capacity <= 0) return;
  hipLaunchKernelGGL(deposit_f64_kernel, dim3(nblk(capacity, 256)), dim3(256), 0, st, P, n_in,
                     rho, S);
}

void launch_deposit_f32r(const PartF32R& P, const int* n_in, long long* rho,
                         const SpeciesStep& S, long capacity, hipStream_t st) {
  if (capacity <= 0) return;
  hipLaunchKernelGGL(deposit_f32r_kernel, dim3(nblk(capacity, 256)), dim3(256), 0, st, P, n_in,
                     rho, S);
}

void launch_fill_int(int* a, long n, int v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_int_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, a, n, v);
}

template <typename PT>
static void sort_impl(const PT& src, const PT& dst, const int* n_in, int* hist, int* sums,
                      long ncell, int nx, int ny, long capacity, hipStream_t st) {
  launch_fill_int(hist, ncell, 0, st);
  hipLaunchKernelGGL(sort_hist_kernel<PT>, dim3(nblk(capacity, 256)), dim3(256), 0, st, src, n_in,
                     hist, nx, ny);
  const int nb = nblk(ncell, kScanBlock);
  hipLaunchKernelGGL(scan_block_sums, dim3(nb), dim3(kScanBlock), 0, st, hist, (int)ncell, sums);
  hipLaunchKernelGGL(scan_sums_serial, dim3(1), dim3(kScanBlock), 0, st, sums, nb);
  hipLaunchKernelGGL(scan_apply, dim3(nb), dim3(kScanBlock), 0, st, hist, (int)ncell, sums, hist);
  hipLaunchKernelGGL(sort_scatter_kernel<PT>, dim3(nblk(capacity, 256)), dim3(256), 0, st, src,
                     dst, n_in, hist, nx, ny);
}

void launch_sort_f64(const PartF64& src, const PartF64& dst, const int* n_in, int* hist,
                     int* sums, long ncell, int nx, int ny, long capacity, hipStream_t st) {
  if (capacity <= 0) return;
  sort_impl(src, dst, n_in, hist, sums, ncell, nx, ny, capacity, st);
}

void launch_sort_f32r(const PartF32R& src, const PartF32R& dst, const int* n_in, int* hist,
                      int* sums, long ncell, int nx, int ny, long capacity, hipStream_t st) {
  if (capacity <= 0) return;
  sort_impl(src, dst, n_in, hist, sums, ncell, nx, ny, capacity, st);
}

}  // namespace pic
