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

#include <climits>
#include <type_traits>

#include "device_common.hpp"
#include "launch.hpp"

namespace pic {

enum { ST_ALIVE = 0, ST_WALL0 = 1, ST_WALL1 = 2, ST_GRAIN = 3, ST_NONE = 4, ST_BAD = 5, ST_MD = 6, ST_OUT = 7 };

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
constexpr int kPPT = 4;                   // consecutive particles per thread
constexpr int kChunk = kBlock * kPPT;     // slots one pass of a push block streams

// int32 cell index of the FP32R form: i | j << 10 | k << 20 (nx, ny <= 1024, nz < 2048);
// -1 marks an empty slot
__device__ __forceinline__ int cell_i(int c) { return c & 1023; }
__device__ __forceinline__ int cell_j(int c) { return (c >> 10) & 1023; }
__device__ __forceinline__ int cell_k(int c) { return c >> 20; }
__device__ __forceinline__ int pack_cell(int i, int j, int k) { return i | (j << 10) | (k << 20); }

// Blocks are dealt round-robin to the 8 XCDs; give each XCD one contiguous
// run of tiles (a slab in z) so neighbouring tiles share that XCD's L2.  nb is
// a multiple of 8, so this is a permutation of [0, nb).
__device__ __forceinline__ long xcd_chunk(long b, long nb) { return (b % 8) * (nb / 8) + b / 8; }

// The same dealing with the XCDs' runs cut into chunks of `chunk` items and
// interleaved (XCD x takes chunks x, x + 8, ...): with a chunk of one z-layer
// of tiles every XCD works on layers spread over the whole height, so the
// particle density's variation along z (the sheaths) does not load some XCDs
// more than others, while neighbouring tiles of a layer still share an L2.
// nb / 8 must be a multiple of chunk (then it is a permutation of [0, nb)).
__device__ __forceinline__ long xcd_interleave(long b, long chunk) {
  const long x = b % 8, i = b / 8;
  return ((i / chunk) * 8 + x) * chunk + i % chunk;
}

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
// index of cell (i, j, k) in the bounding box of the MD cubes, or -1
__device__ __forceinline__ long md_box_index(const MdTables& md, int nx, int ny, int i, int j,
                                             int k) {
  if (md.n_grains == 0) return -1;
  int a = i - md.bx0;
  if (a < 0) a += nx;
  if (a >= md.bsx) return -1;
  int b = j - md.by0;
  if (b < 0) b += ny;
  if (b >= md.bsy) return -1;
  const int c = k - md.bz0;
  if (c < 0 || c >= md.bsz) return -1;
  return ((long)c * md.bsy + b) * md.bsx + a;
}

__device__ __forceinline__ uint32_t md_lookup(const MdTables& md, int nx, int ny, int i, int j,
                                              int k) {
  const long bi = md_box_index(md, nx, ny, i, j, k);
  if (bi < 0) return 0u;
  const uint32_t cl = md.cell_list[bi];
  return (cl & 255u) ? cl : 0u;  // a cell of the box outside every cube has no grains
}

// per-grain data the sub-stepping reads every sub-step (staged in LDS)
struct GrainView {
  const double* gpos;   // [g][3] cell units
  const double* Q;      // [g] grain charge frozen for the step, times qscale:
  double qscale;        // Q qscale = Q / (4 pi eps0 dx^2)
};

// 1 / sqrt(a), a > 0: the hardware estimate refined by two Newton steps
// y <- y (3 - a y^2) / 2 (each squares the relative error)
__device__ __forceinline__ double rsqrt_refined(double a) {
  double y = __builtin_amdgcn_rsq(a);
  y = y * (1.5 - 0.5 * a * y * y);
  y = y * (1.5 - 0.5 * a * y * y);
  return y;
}

// separation x - x_g (cell units), minimum image across the periodic x,y
__device__ __forceinline__ void grain_sep(const GrainView& G, const SpeciesStep& S, int g,
                                          const double x[3], double r[3]) {
  r[0] = x[0] - G.gpos[3 * g + 0];
  r[1] = x[1] - G.gpos[3 * g + 1];
  r[2] = x[2] - G.gpos[3 * g + 2];
  if (r[0] > 0.5 * S.nx) r[0] -= S.nx;
  else if (r[0] < -0.5 * S.nx) r[0] += S.nx;
  if (r[1] > 0.5 * S.ny) r[1] -= S.ny;
  else if (r[1] < -0.5 * S.ny) r[1] += S.ny;
}

__device__ __forceinline__ double wrap_coord(double X, int n) {
  if (X < 0.0) X += (double)n;
  else if (X >= (double)n) X -= (double)n;
  if (X >= (double)n) X -= (double)n;  // -tiny + n rounds to n
  if (X < 0.0 || X >= (double)n) X = X - (double)n * floor(X / (double)n);
  return X;
}

constexpr int kMdCache = 8;  // grains of the current cell kept in registers

// Sub-cycled PPPM motion near grains, Eq. (5)-(6): md_sub sub-steps of
// h = dt/md_sub with E = E_mesh - sum_g Q_g U_g + sum_g Q_g r / (4 pi eps0 r^3)
// over the grains whose cube holds the current cell; hit when |r| <= a (the
// lowest grain index of the cell's list wins).  The first two terms are
// gathered from the cell's corrected node fields (built once per step by
// md_field_kernel).  A particle crosses a cell boundary in only a few of its
// sub-steps, so the cell's node fields and grain list are kept until the cell
// changes.
template <typename ET>
__device__ int md_move(const ET* __restrict__ E, const MdTables& md, const GrainView& G,
                       const SpeciesStep& S, double x[3], double v[3], int& hit) {
  int e_cell = -1;
  double ec[8][3];
  uint32_t cl = 0u;
  int cnt = 0;
  int gl[kMdCache];
  auto load_cell = [&](int cell, int i0, int j0, int k0) {
    if (cell == e_cell) return;
    e_cell = cell;
    const long bi = md_box_index(md, S.nx, S.ny, i0, j0, k0);
    cl = bi >= 0 ? md.cell_list[bi] : 0u;
    cnt = (int)(cl & 255u);
    if (cnt > 0) {
      const double* src = md.ecorr + bi * 24;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        ec[c][0] = src[3 * c];
        ec[c][1] = src[3 * c + 1];
        ec[c][2] = src[3 * c + 2];
      }
    } else {
      const int i1 = i0 + 1 == S.nx ? 0 : i0 + 1;
      const int j1 = j0 + 1 == S.ny ? 0 : j0 + 1;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        load_node(E, ((c & 1) ? i1 : i0) + (long)S.nx * (((c >> 1) & 1) ? j1 : j0) +
                         (long)S.nxy * (k0 + (c >> 2)),
                  ec[c][0], ec[c][1], ec[c][2]);
    }
#pragma unroll
    for (int u = 0; u < kMdCache; ++u) gl[u] = u < cnt ? md.grain_idx[(cl >> 8) + u] : 0;
  };
  auto grain_at = [&](int t) -> int {
    int g = 0;
#pragma unroll
    for (int u = 0; u < kMdCache; ++u)
      if (u == t) g = gl[u];
    return t < kMdCache ? g : md.grain_idx[(cl >> 8) + t];
  };
  // the field at x: the mesh part from the cell's corrected node fields,
  // then the grains' Coulomb fields (their mesh parts are in the corrected
  // nodes): Q r / (4 pi eps0 |r|^3) with r in cells and Q qscale = Q / (4 pi eps0 dx^2)
  auto mesh_field = [&](double Ep[3]) {
    const int i0 = (int)floor(x[0]), j0 = (int)floor(x[1]), k0 = (int)floor(x[2]);
    const double fx = x[0] - i0, fy = x[1] - j0, fz = x[2] - k0;
    load_cell(pack_cell(i0, j0, k0), i0, j0, k0);
    const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
    Ep[0] = Ep[1] = Ep[2] = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double wt = wx[c & 1] * wy[(c >> 1) & 1] * wz[c >> 2];
      Ep[0] += wt * ec[c][0];
      Ep[1] += wt * ec[c][1];
      Ep[2] += wt * ec[c][2];
    }
  };
  auto grain_field = [&](int g, const double r[3], double Ep[3]) {
    const double Qc = G.Q[g] * G.qscale;
    if (Qc == 0.0) return;
    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double rs = rsqrt_refined(r2);
    const double inv = Qc * rs * rs * rs;
    Ep[0] += r[0] * inv;
    Ep[1] += r[1] * inv;
    Ep[2] += r[2] * inv;
  };
  // position x_s, s = 0 .. md_sub: after a drift (s > 0) the hit test, in list
  // order (the first grain that holds the particle wins), and, before the
  // next kick, the field, from one walk over the cell's grains
  double Ep[3];
  for (int sub = 0;; ++sub) {
    mesh_field(Ep);
    for (int t = 0; t < cnt; ++t) {
      const int g = grain_at(t);
      double r[3];
      grain_sep(G, S, g, x, r);
      const double d0 = r[0] * S.dx, d1 = r[1] * S.dx, d2 = r[2] * S.dx;
      if (sub > 0 && d0 * d0 + d1 * d1 + d2 * d2 <= md.a2) {
        hit = g;
        return ST_GRAIN;
      }
      grain_field(g, r, Ep);
    }
    if (sub == S.md_sub) break;
    v[0] += S.qm_h * Ep[0];
    v[1] += S.qm_h * Ep[1];
    v[2] += S.qm_h * Ep[2];
    x[0] = wrap_coord(x[0] + v[0] * S.h_dx, S.nx);
    x[1] = wrap_coord(x[1] + v[1] * S.h_dx, S.ny);
    x[2] += v[2] * S.h_dx;
    const int zs = z_status(x, S);
    if (zs != ST_ALIVE) return zs;
  }
  return ST_ALIVE;
}

// The corrected node field of Eq. (5) at corner (ta, tb, tc) of MD box cell
// bi, whose lowest node is (i0, j0, k0): E_k(node) - sum_g Q_g U_g(node) over
// the cell's grains (cl: its list entry), in list order; E holds E_k(node).
__device__ __forceinline__ void md_corner(const MdTables& md, int nx, int ny, uint32_t cl, int i0,
                                          int j0, int k0, int ta, int tb, int tc, double E[3]) {
  const int cnt = (int)(cl & 255u);
  const int side = md.side;
  const long cube = (long)side * side * side;
  for (int u = 0; u < cnt; ++u) {
    const int g = md.grain_idx[(cl >> 8) + u];
    const double Q = md.Q[g];
    if (Q == 0.0) continue;
    int lx = i0 - (md.gcell[3 * g + 0] - md.cutoff);
    lx = ((lx % nx) + nx) % nx;
    int ly = j0 - (md.gcell[3 * g + 1] - md.cutoff);
    ly = ((ly % ny) + ny) % ny;
    const int lz = k0 - (md.gcell[3 * g + 2] - md.cutoff);
    const long l = ((long)(lz + tc) * side + (ly + tb)) * side + (lx + ta);
    const double* U = md.U + (long)g * 3 * cube;
    E[0] -= Q * U[l];
    E[1] -= Q * U[cube + l];
    E[2] -= Q * U[2 * cube + l];
  }
}

// The fields of a step in one launch.  Blocks [0, nbm): one thread per (MD box
// cell in a cube, corner) forms the corrected node field; E at the node is
// formed from phi and rounded to the storage type first, so it is what a read
// of E returns (these blocks come first: their dependent table loads then
// overlap the node blocks' streaming).  Blocks from nbm on: one thread per
// node writes phi (kLift: from the refined solve's interior potential psi and
// the electrode voltages; otherwise phi is the stored src), E = -grad phi in
// the storage type, and clears the next step's charge accumulator.
template <typename ET, bool kLift>
__global__ __launch_bounds__(256) void field_out_kernel(const double* __restrict__ src,
                                                        double* __restrict__ phi,
                                                        ET* __restrict__ E,
                                                        unsigned long long* __restrict__ zero_next,
                                                        MdTables md, int nx, int ny, int nz,
                                                        double dx, RfDrive rf, int nbm) {
  const double V = kLift ? rf_voltage(rf) : 0.0;
  if ((int)blockIdx.x >= nbm) {
    const int plane = nx * ny;
    const int n = ((int)blockIdx.x - nbm) * (int)blockDim.x + (int)threadIdx.x;
    if (n >= plane * (nz + 1)) return;
    const int k = n / plane, pn = n - k * plane;
    const int y = pn / nx, x = pn - y * nx;
    if (kLift) phi[n] = phi_node<true>(src, plane, pn, k, nz, V);
    double ex, ey, ez;
    node_field<kLift>(src, nx, ny, nz, dx, V, x, y, k, ex, ey, ez);
    if constexpr (std::is_same<ET, double2>::value) {
      E[2 * (long)n] = make_double2(ex, ey);
      E[2 * (long)n + 1] = make_double2(ez, 0.0);
    } else {
      E[n] = make_float4((float)ex, (float)ey, (float)ez, 0.0f);
    }
    if (zero_next) zero_next[n] = 0ull;
    return;
  }
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nbox = (long)md.bsx * md.bsy * md.bsz;
  if (gid >= 8 * nbox) return;
  const long bi = gid >> 3;
  const int t = (int)(gid & 7);
  const uint32_t cl = md.cell_list[bi];
  if ((cl & 255u) == 0u) return;
  const int a = (int)(bi % md.bsx), b = (int)((bi / md.bsx) % md.bsy);
  const int c = (int)(bi / ((long)md.bsx * md.bsy));
  const int i0 = (md.bx0 + a) % nx, j0 = (md.by0 + b) % ny, k0 = md.bz0 + c;
  const int ta = t & 1, tb = (t >> 1) & 1, tc = t >> 2;
  const int in = i0 + ta == nx ? 0 : i0 + ta, jn = j0 + tb == ny ? 0 : j0 + tb;
  double En[3];
  node_field<kLift>(src, nx, ny, nz, dx, V, in, jn, k0 + tc, En[0], En[1], En[2]);
  if constexpr (!std::is_same<ET, double2>::value) {
#pragma unroll
    for (int q = 0; q < 3; ++q) En[q] = (double)(float)En[q];
  }
  md_corner(md, nx, ny, cl, i0, j0, k0, ta, tb, tc, En);
  double* dst = md.ecorr + bi * 24 + 3 * t;
  dst[0] = En[0];
  dst[1] = En[1];
  dst[2] = En[2];
}

// ---------------------------------------------------------------- collisions
// Null-collision MCC against the neutral reservoir: candidate iff Philox word 0
// is below the integer threshold of P' = 1 - exp(-n_g sigma g_cap dt); accept
// with probability g / g_cap.  e-Ar: elastic, isotropic in the CM frame with
// the neutral at rest.  Ar+-Ar: charge exchange, the ion takes the velocity of
// the neutral drawn from the 300 K reservoir.  T is the arithmetic of the
// form: double for FP64; float for FP32R, whose velocities are FP32 (its
// uniforms are the top 24 bits of the word plus one half, times 2^-24).
template <typename PT>
struct VelOf {
  using type = double;
};
template <>
struct VelOf<PartF32R> {
  using type = float;
};

template <typename T>
__device__ __forceinline__ T u01(uint32_t w) {
  if constexpr (sizeof(T) == 8) return u01_open(w);
  else return ((float)(w >> 8) + 0.5f) * 5.9604644775390625e-08f;
}

template <typename T>
__device__ __forceinline__ void normal_pair_t(uint32_t wa, uint32_t wb, T& n0, T& n1) {
  if constexpr (sizeof(T) == 8) {
    normal_pair(wa, wb, n0, n1);
  } else {
    const float r = sqrtf(-2.0f * logf(u01<float>(wa)));
    float sn, cs;
    sincosf(2.0f * (float)kPi * u01<float>(wb), &sn, &cs);
    n0 = r * cs;
    n1 = r * sn;
  }
}

// sigma of table column `col` at energy E (eV): linear between the grid
// points, the end values past them
__device__ inline double xs_at(const SpeciesStep& S, int col, double E) {
  const double* x = S.xs;
  const double* t = S.xs + (long)col * S.xs_n;
  const int n = S.xs_n;
  if (E <= x[0]) return t[0];
  if (E >= x[n - 1]) return t[n - 1];
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (x[mid] <= E) lo = mid;
    else hi = mid;
  }
  const double f = (E - x[lo]) / (x[hi] - x[lo]);
  return t[lo] + f * (t[hi] - t[lo]);
}

// A candidate's collision with energy-dependent cross sections (FP64 in
// both forms): the process is picked by u1 against the cumulative
// g sigma_k(E) / (g sigma)_max, E the projectile's energy with the target at
// rest.  Electrons: elastic, then excitation (CM energy above E_ex; the CM
// energy drops by E_ex, isotropic scattering), then ionisation (CM energy
// above E_iz; what is left is shared, a uniform fraction s from
// Philox(id, k, IONIZE, 0) word 0 to the ejected electron, 1 - s to this one,
// which scatters isotropically; the event is recorded for ionize_kernel);
// ions: charge exchange, then isotropic elastic scattering in the CM frame of
// ion and neutral (equal masses).  Above the bound the collision happens
// (counted) and u1 splits the cross section.
template <typename T>
__device__ void collide_xs(const SpeciesStep& S, const uint4& r, const T vn[3], T v[3], bool& coll,
                           bool& capv, uint32_t id, long slot) {
  const double gx = (double)v[0] - (double)vn[0], gy = (double)v[1] - (double)vn[1],
               gz = (double)v[2] - (double)vn[2];
  const double g2 = gx * gx + gy * gy + gz * gz;
  const double g = sqrt(g2);
  const double E = 0.5 * g2 / fabs(S.qm);  // m g^2 / 2 in eV (|q| = e)
  double s1, s2, s3 = 0.0;
  if (S.sp == 0) {
    s1 = xs_at(S, 1, E);
    s2 = g2 > S.ex_g2 ? xs_at(S, 2, E) : 0.0;
    if (S.iz_ev && g2 > S.iz_g2) s3 = xs_at(S, 5, E);
  } else {
    s1 = xs_at(S, 3, E);
    s2 = xs_at(S, 4, E);
  }
  const double a1 = g * s1 / S.sg_max, a2 = g * (s1 + s2) / S.sg_max;
  const double a3 = g * (s1 + s2 + s3) / S.sg_max;
  const double u1 = u01_open(r.y);
  int proc;
  if (a3 > 1.0) {
    capv = true;
    const double x = u1 * (s1 + s2 + s3);
    proc = x < s1 ? 1 : (x < s1 + s2 ? 2 : 3);
  } else {
    proc = u1 < a1 ? 1 : (u1 < a2 ? 2 : (u1 < a3 ? 3 : 0));
  }
  if (proc == 0) return;
  coll = true;
  if (S.sp == 1 && proc == 1) {
    v[0] = vn[0];
    v[1] = vn[1];
    v[2] = vn[2];
    return;
  }
  const double cost = 1.0 - 2.0 * u01_open(r.z);
  const double sint = sqrt(fmax(0.0, 1.0 - cost * cost));
  double sp, cp;
  sincos(2.0 * kPi * u01_open(r.w), &sp, &cp);
  const double nh[3] = {sint * cp, sint * sp, cost};
  if (S.sp == 0) {
    double gp = proc == 2 ? sqrt(g2 - S.ex_g2) : g;
    if (proc == 3) {
      const double gsq = g2 - S.iz_g2;
      const uint4 w = philox4x32_10(id, *S.step, kIonize, 0u, S.key0, S.key1);
      gp = sqrt((1.0 - u01_open(w.x)) * gsq);
      const int e = atomicAdd(S.iz_cnt, 1);
      if (e < S.iz_cap) {
        IzEvent& ev = S.iz_ev[e];
        ev.id = id;
        ev.slot = (int32_t)slot;
        for (int a = 0; a < 3; ++a) ev.v[a] = (double)v[a];
        ev.gsq = gsq;
      }
    }
    for (int a = 0; a < 3; ++a) v[a] = (T)(S.mass_ratio_e * (double)v[a] + S.mass_ratio_n * gp * nh[a]);
  } else {
    for (int a = 0; a < 3; ++a) v[a] = (T)(0.5 * ((double)v[a] + (double)vn[a]) + 0.5 * g * nh[a]);
  }
}

template <typename T>
__device__ __forceinline__ void collide(const SpeciesStep& S, uint32_t id, T v[3], bool& coll,
                                        bool& capv, long slot) {
  if constexpr (sizeof(T) == 4) {
    // FP32R records: the collision in FP64 (2 % of the particles per step),
    // rounded once; a 24-bit uniform in the Box-Muller radius or the
    // scattering angle could put a tail draw 1e-4 off
    double vd[3] = {v[0], v[1], v[2]};
    collide<double>(S, id, vd, coll, capv, slot);
    if (coll) {
      v[0] = (T)vd[0];
      v[1] = (T)vd[1];
      v[2] = (T)vd[2];
    }
    return;
  }
  const uint4 r = philox4x32_10(id, *S.step, kColl, (uint32_t)S.sp, S.key0, S.key1);
  if ((uint64_t)r.x >= S.T_null) return;
  T vn[3] = {(T)0, (T)0, (T)0};
  if (S.sp == 1) {
    const uint4 q = philox4x32_10(id, *S.step, kNeutral, 1u, S.key0, S.key1);
    T n0, n1, n2, n3;
    normal_pair_t<T>(q.x, q.y, n0, n1);
    normal_pair_t<T>(q.z, q.w, n2, n3);
    const T vg = (T)S.vth_gas;
    vn[0] = vg * n0;
    vn[1] = vg * n1;
    vn[2] = vg * n2;
  }
  if (S.xs_n > 0) {
    collide_xs<T>(S, r, vn, v, coll, capv, id, slot);
    return;
  }
  const T gx = v[0] - vn[0], gy = v[1] - vn[1], gz = v[2] - vn[2];
  const T g = sqrt(gx * gx + gy * gy + gz * gz);
  const T ratio = g / (T)S.g_cap;
  bool accept;
  if (ratio > (T)1) {
    capv = true;
    accept = true;
  } else {
    accept = u01<T>(r.y) < ratio;
  }
  if (!accept) return;
  coll = true;
  if (S.sp == 0) {
    const T cost = (T)1 - (T)2 * u01<T>(r.z);
    const T sint = sqrt(fmax((T)0, (T)1 - cost * cost));
    T sp, cp;
    if constexpr (sizeof(T) == 8) sincos(2.0 * kPi * u01<T>(r.w), &sp, &cp);
    else sincosf(2.0f * (float)kPi * u01<T>(r.w), &sp, &cp);
    const T nh[3] = {sint * cp, sint * sp, cost};
    const T ae = (T)S.mass_ratio_e, an = (T)S.mass_ratio_n;
    for (int a = 0; a < 3; ++a) v[a] = ae * v[a] + an * g * nh[a];
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
// a * b for 0 <= a < 2^63, 0 <= b < 2^32 with a * b < 2^63: two 32x32 -> 64-bit
// multiply-adds instead of a general 64-bit product
__device__ __forceinline__ long long mul_q(long long a, uint32_t b) {
  const unsigned long long ua = (unsigned long long)a;
  const unsigned long long lo = (unsigned long long)(uint32_t)ua * b;
  const unsigned long long hi = (unsigned long long)(uint32_t)(ua >> 32) * b;
  return (long long)(lo + (hi << 32));
}

__device__ __forceinline__ void split8(long long Q, float ox, float oy, float oz,
                                       long long part[8]) {
  // offsets in [0, 1): f24 in [0, 2^24), the parts stay in [0, Q]
  const uint32_t qx = (uint32_t)(ox * 16777216.0f);
  const uint32_t qy = (uint32_t)(oy * 16777216.0f);
  const uint32_t qz = (uint32_t)(oz * 16777216.0f);
  long long ax[2];
  ax[1] = mul_q(Q, qx) >> 24;
  ax[0] = Q - ax[1];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const long long y1 = mul_q(ax[a], qy) >> 24;
    const long long yy[2] = {ax[a] - y1, y1};
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const long long z1 = mul_q(yy[b], qz) >> 24;
      part[a + 2 * b] = yy[b] - z1;
      part[a + 2 * b + 4] = z1;
    }
  }
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ void wave_add_count(int v, unsigned long long* dst) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, (unsigned long long)v);
}

// ---------------------------------------------------------------- one particle
// FP32R: gather from the 8 node fields ec, kick Eq. (2), drift Eq. (1) in cell +
// offset form, periodic wrap; returns the electrode status
__device__ __forceinline__ int push_one_f32(const SpeciesStep& S, const float ec[8][3], float o[3],
                                            float v[3], int& ci, int& cj, int& ck) {
  const float wx[2] = {1.0f - o[0], o[0]};
  const float wy[2] = {1.0f - o[1], o[1]};
  const float wz[2] = {1.0f - o[2], o[2]};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float e = 0.0f;
#pragma unroll
    for (int t = 0; t < 8; ++t) e += wx[t & 1] * wy[(t >> 1) & 1] * wz[t >> 2] * ec[t][a];
    v[a] += S.qm_dt_f * e;
  }
  int d[3];
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float f = o[a] + v[a] * S.dt_dx_f;
    const float fl = floorf(f);
    f -= fl;
    d[a] = (int)fl;
    if (f >= 1.0f) {  // -tiny + 1 rounds to 1
      f = 0.0f;
      d[a] += 1;
    }
    ok = ok && (f >= 0.0f && f < 1.0f);
    o[a] = f;
  }
  ci += d[0];
  cj += d[1];
  ck += d[2];
  // periodic wrap: one box length covers any move below it (the general
  // remainder only past that)
  if (ci < 0) ci += S.nx;
  else if (ci >= S.nx) ci -= S.nx;
  if (cj < 0) cj += S.ny;
  else if (cj >= S.ny) cj -= S.ny;
  if (ci < 0 || ci >= S.nx) ci = ((ci % S.nx) + S.nx) % S.nx;
  if (cj < 0 || cj >= S.ny) cj = ((cj % S.ny) + S.ny) % S.ny;
  return !ok ? ST_BAD : (ck < 0 ? ST_WALL0 : (ck >= S.nz ? ST_WALL1 : ST_ALIVE));
}

// FP64: kick with the gathered field, drift, wrap; returns the electrode status
__device__ __forceinline__ int push_one_f64(const SpeciesStep& S, const double Ep[3], double x[3],
                                            double v[3]) {
  v[0] += S.qm_dt * Ep[0];
  v[1] += S.qm_dt * Ep[1];
  v[2] += S.qm_dt * Ep[2];
  x[0] = wrap_coord(x[0] + v[0] * S.dt_dx, S.nx);
  x[1] = wrap_coord(x[1] + v[1] * S.dt_dx, S.ny);
  x[2] += v[2] * S.dt_dx;
  return z_status(x, S);
}

// ---------------------------------------------------------------- tile windows
// The arrays are binned by tiles of 4x4x4 cells.  One push block takes one
// tile: it stages the field on the tile's cells plus a margin of cells (the
// window) in LDS and accumulates its deposit there.  Particles that have
// drifted beyond the window since the last sort (fast electrons) are left to
// the outlier kernel, which gathers and deposits through global memory.
struct Tile {
  int x0, y0, k0;  // first node (x0, y0 may be negative: periodic)
  int tx, ty, tz;  // nodes per edge
  bool on;
  bool wraps;      // the window crosses the periodic seam in x or y
};

// the window of tiles t .. t + span - 1 (consecutive along x): their cells
// plus m cells on each side, in nodes; the margin shrinks until the window
// fits `cap` nodes
__device__ __forceinline__ Tile make_tile(int t, const WorkLists& L, int nx, int ny, int nz,
                                          int margin, int cap, int span = 1) {
  Tile w;
  w.on = false;
  w.wraps = false;
  w.x0 = w.y0 = w.k0 = 0;
  w.tx = w.ty = w.tz = 0;
  // a padding tile of the grid (its slots, if any, hold particles made by
  // ionisation since the last re-binning): no window, every particle takes
  // the global-memory paths
  if (t >= L.ntx * L.nty * L.ntz) return w;
  const int ti = t % L.ntx, tj = (t / L.ntx) % L.nty, tk = t / (L.ntx * L.nty);
  const int i0 = 4 * ti, ni = min(4 * span, nx - i0), j0 = 4 * tj, nj = min(4, ny - j0);
  const int k0 = 4 * tk, nk = min(4, nz - k0);
  for (int m = margin; m >= 0; --m) {
    int x0 = i0 - m, tx = ni + 2 * m + 1;
    if (ni + 2 * m >= nx) {
      x0 = 0;
      tx = nx + 1;
    }
    int y0 = j0 - m, ty = nj + 2 * m + 1;
    if (nj + 2 * m >= ny) {
      y0 = 0;
      ty = ny + 1;
    }
    const int klo = max(0, k0 - m), khi = min(nz - 1, k0 + nk - 1 + m);
    const int tz = khi - klo + 2;
    if (tx * ty * tz <= cap) {
      w.x0 = x0;
      w.y0 = y0;
      w.k0 = klo;
      w.tx = tx;
      w.ty = ty;
      w.tz = tz;
      w.on = true;
      w.wraps = x0 < 0 || x0 + tx - 1 >= nx || y0 < 0 || y0 + ty - 1 >= ny;
      return w;
    }
  }
  return w;
}

// tile-local index of the cell's lower corner node, or -1 if the cell's 8
// nodes are not all in the tile
__device__ __forceinline__ int tile_cell(const Tile& t, int i, int j, int k, int nx, int ny) {
  if (!t.on) return -1;
  int lx = i - t.x0;
  int ly = j - t.y0;
  if (t.wraps) {  // (block-uniform)
    if (lx >= nx) lx -= nx;
    else if (lx < 0) lx += nx;
    if (ly >= ny) ly -= ny;
    else if (ly < 0) ly += ny;
  }
  const int lz = k - t.k0;
  // (unsigned: a negative index, possible without the wrap, is out too)
  if ((unsigned)lx > (unsigned)(t.tx - 2) || (unsigned)ly > (unsigned)(t.ty - 2) ||
      (unsigned)lz > (unsigned)(t.tz - 2))
    return -1;
  return (lz * t.ty + ly) * t.tx + lx;
}

// a / b for 0 <= a < 2^24 without an integer divide (rb = 1/b)
__device__ __forceinline__ int qdiv(int a, int b, float rb) {
  int q = (int)((float)a * rb);
  if (q * b > a) --q;
  else if ((q + 1) * b <= a) ++q;
  return q;
}

// global node of tile entry t
__device__ __forceinline__ long tile_node(const Tile& T, int t, float rtx, float rtxy, int nx,
                                          int ny, long nxy) {
  const int lz = qdiv(t, T.tx * T.ty, rtxy);
  const int r = t - lz * T.tx * T.ty;
  const int ly = qdiv(r, T.tx, rtx);
  const int lx = r - ly * T.tx;
  int gi = T.x0 + lx;
  if (gi < 0) gi += nx;
  else if (gi >= nx) gi -= nx;
  if (gi < 0 || gi >= nx) gi = ((gi % nx) + nx) % nx;
  int gj = T.y0 + ly;
  if (gj < 0) gj += ny;
  else if (gj >= ny) gj -= ny;
  if (gj < 0 || gj >= ny) gj = ((gj % ny) + ny) % ny;
  return gi + (long)nx * gj + nxy * (T.k0 + lz);
}

template <typename A>
__device__ __forceinline__ void atomic_add_acc(A* p, A v) {
  if constexpr (std::is_same<A, long long>::value)
    atomicAdd((unsigned long long*)p, (unsigned long long)v);
  else
    unsafeAtomicAdd(p, v);
}

// the 8 corner contributions of one cell into the tile (lbase >= 0) or to global
template <typename A>
__device__ __forceinline__ void corner_add(const Tile& T, int lbase, A* s_rho, A* __restrict__ rho,
                                           const SpeciesStep& S, int i, int j, int k,
                                           const A acc[8]) {
  if (lbase >= 0) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int off = (t & 1) + T.tx * (((t >> 1) & 1) + T.ty * (t >> 2));
      if constexpr (std::is_same<A, long long>::value)
        atomicAdd((unsigned long long*)&s_rho[lbase + off], (unsigned long long)acc[t]);
      else
        atomicAdd(&s_rho[lbase + off], acc[t]);
    }
  } else {
    const int i1 = i + 1 == S.nx ? 0 : i + 1;
    const int j1 = j + 1 == S.ny ? 0 : j + 1;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const long node = ((t & 1) ? i1 : i) + (long)S.nx * (((t >> 1) & 1) ? j1 : j) +
                        (long)S.nxy * (k + (t >> 2));
      atomic_add_acc(&rho[node], acc[t]);
    }
  }
}

// one particle's CIC charge straight to the global mesh (particles outside their tile's window)
__device__ __forceinline__ void deposit_global_fixed(long long* __restrict__ rho,
                                                     const SpeciesStep& S, int i, int j, int k,
                                                     float ox, float oy, float oz) {
  long long part[8];
  split8(S.Qp, ox, oy, oz, part);
#pragma unroll
  for (int t = 0; t < 8; ++t) part[t] *= S.isign;
  Tile none{};
  corner_add<long long>(none, -1, nullptr, rho, S, i, j, k, part);
}

__device__ __forceinline__ void cic_weights_d(double fx, double fy, double fz, double s,
                                              double w[8]) {
  const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
#pragma unroll
  for (int t = 0; t < 8; ++t) w[t] = s * wx[t & 1] * wy[(t >> 1) & 1] * wz[t >> 2];
}

// append to a list segment: one LDS atomic per wave
__device__ __forceinline__ void chunk_append(bool flag, int32_t* seg, int* s_n, int value) {
  const unsigned long long m = __ballot(flag);
  if (!m) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(s_n, __popcll(m));
  base = __shfl(base, leader, 64);
  if (flag) seg[base + __popcll(m & ((1ull << lane) - 1ull))] = value;
}

// the same for the slots p0 .. p0 + kPPT - 1 of every lane at once: one LDS
// reservation for the whole wave (entries lane-ordered per q); every lane of
// the wave must take part.  (Used by the FP64 push; in the FP32R push the
// flags' registers cost more than the atomics saved.)
__device__ __forceinline__ void chunk_append4(const bool (&flag)[kPPT], int32_t* seg, int* s_n,
                                              int p0) {
  unsigned long long m[kPPT];
  int total = 0;
#pragma unroll
  for (int q = 0; q < kPPT; ++q) {
    m[q] = __ballot(flag[q]);
    total += __popcll(m[q]);
  }
  if (!total) return;
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == 0) base = atomicAdd(s_n, total);
  base = __shfl(base, 0, 64);
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int q = 0; q < kPPT; ++q) {
    if (flag[q]) seg[base + __popcll(m[q] & below)] = p0 + q;
    base += __popcll(m[q]);
  }
}

// the slots p0 + q of every lane whose status st[q] is `want`, appended in
// slot order (lane by lane, q ascending within a lane) with one reservation
// for the wave: the dense MD list then runs through the cells in order, so the
// MD kernel's waves meet few distinct cells when they deposit; every lane of
// the wave must take part
__device__ __forceinline__ void append_slot_order(const int (&st)[kPPT], int want, int32_t* seg,
                                                  int* s_n, int p0) {
  unsigned long long m[kPPT];
  int total = 0;
#pragma unroll
  for (int q = 0; q < kPPT; ++q) {
    m[q] = __ballot(st[q] == want);
    total += __popcll(m[q]);
  }
  if (!total) return;
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == 0) base = atomicAdd(s_n, total);
  base = __shfl(base, 0, 64);
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int q = 0; q < kPPT; ++q) base += __popcll(m[q] & below);
#pragma unroll
  for (int q = 0; q < kPPT; ++q)
    if (st[q] == want) seg[base++] = p0 + q;
}

// block-level tallies: wave sums into LDS; thread 0 then adds them to the
// tile's own accumulators (each tile has one writer per kernel: no atomics)
__device__ __forceinline__ void tally_add(unsigned* s_t, int which, int v) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(&s_t[which], (unsigned)v);
}
__device__ __forceinline__ void tally_store(const unsigned* s_t, unsigned long long* tally) {
  if (threadIdx.x != 0) return;
  for (int w = 0; w < TL_N; ++w)
    if (s_t[w]) tally[w] += s_t[w];
}

// The MD particles of one pass of a push block are staged in LDS and appended
// to the dense MD list with one reservation.  Every thread calls this after a
// barrier that follows the pass's last append.
constexpr int kMdStage = kBlock * kPPT;
__device__ __forceinline__ void md_flush(int32_t* s_md, int* s_nmd, int* s_mdbase,
                                         const WorkLists& L) {
  const int nmd = *s_nmd;
  __syncthreads();  // every thread has read the count before it changes
  if (nmd == 0) return;
  if (threadIdx.x == 0) {
    *s_mdbase = atomicAdd(&L.cnt[2], nmd);
    *s_nmd = 0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nmd; t += kBlock) L.md[*s_mdbase + t] = s_md[t];
  __syncthreads();  // the stage is free again
}

// one run of same-cell charge parts (magnitudes) into the window, or, outside
// it, with the species' sign straight to the global mesh (and the block's
// stray flag set)
__device__ __forceinline__ void deposit_run(const Tile& tile, long long* s_rho,
                                            long long* __restrict__ rho, const SpeciesStep& S,
                                            int c, long long acc[8], int* s_stray) {
  const int ai = cell_i(c), aj = cell_j(c), ak = cell_k(c);
  const int lb = tile_cell(tile, ai, aj, ak, S.nx, S.ny);
  if (lb < 0) *s_stray = 1;  // the run ends the push outside the window
  if (lb < 0 && S.isign < 0) {
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = -acc[t];
  }
  corner_add<long long>(tile, lb, s_rho, rho, S, ai, aj, ak, acc);
}

// whether any cell of the window lies in the bounding box of the MD cubes
// (periodic in x, y)
__device__ __forceinline__ bool window_meets_md(const Tile& w, const MdTables& md, int nx, int ny) {
  if (md.n_grains == 0) return false;
  if (!w.on) return true;
  const int wx = w.tx - 1, wy = w.ty - 1;  // cells of the window per axis
  int dx = (w.x0 - md.bx0) % nx;
  if (dx < 0) dx += nx;
  int dy = (w.y0 - md.by0) % ny;
  if (dy < 0) dy += ny;
  const bool mx = wx >= nx || dx < md.bsx || dx + wx > nx;
  const bool my = wy >= ny || dy < md.bsy || dy + wy > ny;
  const bool mz = w.k0 < md.bz0 + md.bsz && md.bz0 < w.k0 + w.tz - 1;
  return mx && my && mz;
}

// ---------------------------------------------------------------- push, FP32R
// One block streams the slots of its tile, 1024 per pass, four consecutive
// slots per thread with 16-byte loads and stores, and updates them in place:
// gather from the LDS field window (the 8 node fields are reused while
// consecutive particles share a cell), kick Eq. (2), drift Eq. (1) in cell +
// offset form, periodic wrap, electrode absorption, collision candidate test;
// the new positions are deposited into the LDS window (per-thread sums over a
// run of particles in one cell first), whose occupied nodes are then added to
// rho.  Particles starting inside an MD cube are left untouched (their list
// is formed before the push, md_scan_kernel, and the sub-cycled kernel moves
// them meanwhile into the other record buffer); candidates are listed for the
// collision kernel, which runs right after the push while the records it
// wrote are still in cache.
constexpr int kWinF32 = 1331;  // window capacity (nodes): a tile with a 3-cell margin

// The FP32R push streams the particle records once per step in each direction
// and they are not reread before they would have left the caches: their
// 16-byte loads and stores carry the non-temporal hint, which keeps the field
// and deposit windows and the lists cached instead.  (Measured: faster here;
// slower for the FP64 records' 16-byte pairs and the re-binning's 4-byte
// scatter, which keep the default.)
typedef int vi4 __attribute__((ext_vector_type(4)));
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef unsigned vu4 __attribute__((ext_vector_type(4)));
template <typename Out, typename V, typename T>
__device__ __forceinline__ Out nt_load4(const T* p, long g4) {
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p) + g4);
  Out o;
  o.x = v.x;
  o.y = v.y;
  o.z = v.z;
  o.w = v.w;
  return o;
}
template <typename V, typename T>
__device__ __forceinline__ void nt_store4(T* p, long g4, V v) {
  __builtin_nontemporal_store(v, reinterpret_cast<V*>(p) + g4);
}
// the kPPT consecutive values of one field at group g (FP32R push records)
typedef int viP __attribute__((ext_vector_type(kPPT)));
typedef float vfP __attribute__((ext_vector_type(kPPT)));
typedef unsigned vuP __attribute__((ext_vector_type(kPPT)));
template <typename V, typename T>
__device__ __forceinline__ V nt_loadP(const T* p, long g) {
  return __builtin_nontemporal_load(reinterpret_cast<const V*>(p) + g);
}

// LDS of one push block (FP32R)
struct PushSmemF32 {
  float4 E[kWinF32];
  long long rho[kWinF32];
  unsigned tally[TL_N];
  int ncoll, nout, stray;
};

// A block takes `span` tiles that are consecutive along x (1 or 2): their
// slots are one contiguous range and they share one window; the lists of the
// span go to the first tile's segments, the others' counts are zero.
template <bool kMove>
__device__ __forceinline__ void push_tile_f32r(const PartF32R& P, const float4* __restrict__ E,
                                               long long* __restrict__ rho, const MdTables& md,
                                               const SpeciesStep& S, const WorkLists& L, int tidx,
                                               int span, PushSmemF32& sm) {
  const int beg = L.tstart[tidx], end = L.tstart[tidx + span];
  if (kMove && threadIdx.x < span) {
    L.coll_cnt[tidx + threadIdx.x] = 0;
    L.out_cnt[tidx + threadIdx.x] = 0;
  }
  if (beg >= end) return;
  const Tile tile = make_tile(tidx, L, S.nx, S.ny, S.nz, S.margin, kWinF32, span);
  const int vol = tile.on ? tile.tx * tile.ty * tile.tz : 0;
  const float rtx = 1.0f / (float)max(tile.tx, 1), rtxy = 1.0f / (float)max(tile.tx * tile.ty, 1);
  for (int t = threadIdx.x; t < vol; t += kBlock) {
    if (kMove) sm.E[t] = E[tile_node(tile, t, rtx, rtxy, S.nx, S.ny, S.nxy)];
    sm.rho[t] = 0;
  }
  if (threadIdx.x < TL_N) sm.tally[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    sm.ncoll = 0;
    sm.nout = 0;
    sm.stray = 0;
  }
  // MD cubes near the window: only then does every particle need the lookup
  const bool md_near = window_meets_md(tile, md, S.nx, S.ny);
  __syncthreads();
  // event counts per thread, one byte per status, added up every 32 passes
  unsigned long long packed = 0ull;
  int n_w0 = 0, n_w1 = 0, n_bad = 0, n_md = 0, n_out = 0, n_fast = 0;
  for (int base = beg, pass = 0; base < end; base += kChunk, ++pass) {
    // tile ranges are multiples of 4 slots: a thread's kPPT slots are all in
    // the tile or all beyond it
    const int p0 = base + kPPT * (int)threadIdx.x;
    const bool have = p0 < end;
    const long g4 = p0 / kPPT;
    int cell[kPPT];
    float o[kPPT][3], v[kPPT][3];
    uint32_t id[kPPT];
    {
      viP c4 = -1;
      vfP X4 = 0.0f, Y4 = 0.0f, Z4 = 0.0f, U4 = 0.0f, V4 = 0.0f, W4 = 0.0f;
      vuP I4 = 0u;
      if (have) {
        c4 = nt_loadP<viP>(P.cell, g4);
        X4 = nt_loadP<vfP>(P.ox, g4);
        Y4 = nt_loadP<vfP>(P.oy, g4);
        Z4 = nt_loadP<vfP>(P.oz, g4);
        U4 = nt_loadP<vfP>(P.vx, g4);
        V4 = nt_loadP<vfP>(P.vy, g4);
        W4 = nt_loadP<vfP>(P.vz, g4);
        I4 = nt_loadP<vuP>(P.id, g4);
      }
#pragma unroll
      for (int q = 0; q < kPPT; ++q) {
        cell[q] = c4[q];
        o[q][0] = X4[q];
        o[q][1] = Y4[q];
        o[q][2] = Z4[q];
        v[q][0] = U4[q];
        v[q][1] = V4[q];
        v[q][2] = W4[q];
        id[q] = I4[q];
      }
    }
    int st[kPPT];
    bool cand[kPPT];
    int cached = -1;
    float ec[8][3];
#pragma unroll
    for (int q = 0; q < kPPT; ++q) {
      st[q] = ST_NONE;
      cand[q] = false;
      if (cell[q] < 0) continue;
      if (!kMove) {
        st[q] = ST_ALIVE;
        continue;
      }
      int ci = cell_i(cell[q]), cj = cell_j(cell[q]), ck = cell_k(cell[q]);
      // (a cached cell has passed both tests already)
      const int lb = cell[q] == cached ? 0 : tile_cell(tile, ci, cj, ck, S.nx, S.ny);
      if ((md_near && cell[q] != cached) || lb < 0) {
        if (md_lookup(md, S.nx, S.ny, ci, cj, ck) != 0u) {
          st[q] = ST_MD;
          continue;
        }
      }
      if (lb < 0) {
        // outside the window: left for the outlier kernel (no global gather
        // here, so no wave waits on a dependent memory round trip)
        st[q] = ST_OUT;
        continue;
      }
      if (cell[q] != cached) {
        cached = cell[q];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float4 e = sm.E[lb + (t & 1) + tile.tx * (((t >> 1) & 1) + tile.ty * (t >> 2))];
          ec[t][0] = e.x;
          ec[t][1] = e.y;
          ec[t][2] = e.z;
        }
      }
      st[q] = push_one_f32(S, ec, o[q], v[q], ci, cj, ck);
      cell[q] = st[q] == ST_ALIVE ? pack_cell(ci, cj, ck) : -1;
      n_fast += v[q][0] * v[q][0] + v[q][1] * v[q][1] + v[q][2] * v[q][2] >= S.vfast2_f;
    }
    if (kMove) {
      // collision candidates of the survivors: word 0 of Philox(id, k, COLL, s)
      uint32_t w0[kPPT];
      philox_word0<kPPT>(id, *S.step, kColl, (uint32_t)S.sp, S.key0, S.key1, w0);
#pragma unroll
      for (int q = 0; q < kPPT; ++q) {
        cand[q] = st[q] == ST_ALIVE && (uint64_t)w0[q] < S.T_null;
        chunk_append(cand[q], L.coll + beg, &sm.ncoll, p0 + q);
        chunk_append(st[q] == ST_OUT, L.out + beg, &sm.nout, p0 + q);
        packed += 1ull << (8 * st[q]);
      }
      if ((pass & 31) == 31) {
        n_w0 += (int)((packed >> (8 * ST_WALL0)) & 255u);
        n_w1 += (int)((packed >> (8 * ST_WALL1)) & 255u);
        n_bad += (int)((packed >> (8 * ST_BAD)) & 255u);
        n_md += (int)((packed >> (8 * ST_MD)) & 255u);
        n_out += (int)((packed >> (8 * ST_OUT)) & 255u);
        packed = 0ull;
      }
      if (have) {
        viP c;
        vfP a0, a1, a2, b0, b1, b2;
#pragma unroll
        for (int q = 0; q < kPPT; ++q) {
          c[q] = cell[q];
          a0[q] = o[q][0];
          a1[q] = o[q][1];
          a2[q] = o[q][2];
          b0[q] = v[q][0];
          b1[q] = v[q][1];
          b2[q] = v[q][2];
        }
        nt_store4<viP>(P.cell, g4, c);
        nt_store4<vfP>(P.ox, g4, a0);
        nt_store4<vfP>(P.oy, g4, a1);
        nt_store4<vfP>(P.oz, g4, a2);
        nt_store4<vfP>(P.vx, g4, b0);
        nt_store4<vfP>(P.vy, g4, b1);
        nt_store4<vfP>(P.vz, g4, b2);
      }
    }

    // deposit of rho_{k+1}
    long long acc[8];
    int acc_cell = -1;
#pragma unroll
    for (int q = 0; q < kPPT; ++q) {
      if (st[q] != ST_ALIVE) continue;
      long long part[8];
      split8(S.Qp, o[q][0], o[q][1], o[q][2], part);
      if (cell[q] == acc_cell) {
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] += part[t];
      } else {
        if (acc_cell >= 0) deposit_run(tile, sm.rho, rho, S, acc_cell, acc, &sm.stray);
        acc_cell = cell[q];
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] = part[t];
      }
    }
    if (acc_cell >= 0) deposit_run(tile, sm.rho, rho, S, acc_cell, acc, &sm.stray);
  }
  if (kMove) {
    n_w0 += (int)((packed >> (8 * ST_WALL0)) & 255u);
    n_w1 += (int)((packed >> (8 * ST_WALL1)) & 255u);
    n_bad += (int)((packed >> (8 * ST_BAD)) & 255u);
    n_md += (int)((packed >> (8 * ST_MD)) & 255u);
    n_out += (int)((packed >> (8 * ST_OUT)) & 255u);
    tally_add(sm.tally, TL_W0, n_w0);
    tally_add(sm.tally, TL_W1, n_w1);
    tally_add(sm.tally, TL_BAD, n_bad);
    tally_add(sm.tally, TL_MD, n_md);
    tally_add(sm.tally, TL_DEAD, n_w0 + n_w1 + n_bad);
    tally_add(sm.tally, TL_FALL, n_out);
    tally_add(sm.tally, TL_FAST, n_fast);
  }
  __syncthreads();
  // the window holds the magnitudes; the species' sign is applied here
  for (int t = threadIdx.x; t < vol; t += kBlock) {
    const long long val = sm.rho[t];
    if (val != 0)
      atomicAdd((unsigned long long*)&rho[tile_node(tile, t, rtx, rtxy, S.nx, S.ny, S.nxy)],
                (unsigned long long)(S.isign < 0 ? -val : val));
  }
  if (kMove) {
    if (threadIdx.x == 0) {
      L.coll_cnt[tidx] = sm.ncoll;
      L.out_cnt[tidx] = sm.nout;
      if (sm.stray) L.stray[tidx] = 1;
    }
    tally_store(sm.tally, L.tally + (long)TL_N * tidx);
  }
}

// (at most 128 VGPRs: four waves per SIMD, which the streaming needs)
template <bool kMove>
__global__ __launch_bounds__(kBlock, 4) void push_f32r_kernel(PartF32R P,
                                                           const float4* __restrict__ E,
                                                           long long* __restrict__ rho, MdTables md,
                                                           SpeciesStep S, WorkLists L, int span,
                                                           int chunk) {
  __shared__ PushSmemF32 sm;
  push_tile_f32r<kMove>(P, E, rho, md, S, L, span * (int)xcd_interleave(blockIdx.x, chunk), span,
                        sm);
}

// ---------------------------------------------------------------- push, ensemble
// One persistent launch over the tile spans of every (replica, species) of an
// ensemble: work item i belongs to descriptor d with start[d] <= i < start[d+1]
// (each descriptor has a multiple of 8 items).  Items are dealt dynamically
// from eight queues, one per residue of the item index modulo 8: block b takes
// the next item of queue b % 8 (one atomic per item), so item i still runs on
// XCD i % 8 as the tile interleave expects, and blocks that drew light tiles
// take more of them.  A queue's items come in increasing order, so a block
// finds its descriptor by walking forward.  queue[0..7] are zero at launch.
__global__ __launch_bounds__(kBlock, 4) void push_batch_f32r_kernel(const PushDescF32* __restrict__ descs,
                                                                 const int32_t* __restrict__ start,
                                                                 int ndesc, int* __restrict__ queue) {
  __shared__ PushSmemF32 sm;
  __shared__ int s_item;
  const int total = start[ndesc];
  const int x = (int)(blockIdx.x & 7u);
  int lo = 0;
  for (;;) {
    if (threadIdx.x == 0) s_item = x + 8 * atomicAdd(&queue[x], 1);
    __syncthreads();
    const int item = s_item;
    if (item >= total) break;
    while (lo + 1 < ndesc && start[lo + 1] <= item) ++lo;
    const int local = item - start[lo];
    const PushDescF32& d = descs[lo];
    push_tile_f32r<true>(d.P, d.E, d.rho, d.md, d.S, d.L,
                         d.span * (int)xcd_interleave(local, d.chunk), d.span, sm);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- push, FP64
// The same kernel on FP64 records: positions in cell units, velocities in m/s;
// an empty slot has z = -1.  The field window holds (Ex,Ey),(Ez,0) pairs.
constexpr int kWinF64 = 729;  // window capacity (nodes): a tile with a 2-cell margin

// (at most 168 VGPRs: three waves per SIMD)
template <bool kMove>
__global__ __launch_bounds__(kBlock, 3) void push_f64_kernel(PartF64 P, const double2* __restrict__ E,
                                                          double* __restrict__ rho, MdTables md,
                                                          SpeciesStep S, WorkLists L, int chunk) {
  __shared__ double2 s_E[2 * kWinF64];
  __shared__ double s_rho[kWinF64];
  __shared__ unsigned s_tally[TL_N];
  __shared__ int s_nmd, s_ncoll, s_nout, s_mdbase;
  __shared__ int32_t s_md[kMdStage];
  const int tidx = (int)xcd_interleave(blockIdx.x, chunk);
  const int beg = L.tstart[tidx], end = L.tstart[tidx + 1];
  if (beg >= end) {
    if (kMove && threadIdx.x == 0) {
      L.coll_cnt[tidx] = 0;
      L.out_cnt[tidx] = 0;
    }
    return;
  }
  const Tile tile = make_tile(tidx, L, S.nx, S.ny, S.nz, S.margin, kWinF64);
  const int vol = tile.on ? tile.tx * tile.ty * tile.tz : 0;
  const float rtx = 1.0f / (float)max(tile.tx, 1), rtxy = 1.0f / (float)max(tile.tx * tile.ty, 1);
  for (int t = threadIdx.x; t < vol; t += kBlock) {
    if (kMove) {
      const long node = tile_node(tile, t, rtx, rtxy, S.nx, S.ny, S.nxy);
      s_E[2 * t] = E[2 * node];
      s_E[2 * t + 1] = E[2 * node + 1];
    }
    s_rho[t] = 0.0;
  }
  if (threadIdx.x < TL_N) s_tally[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    s_nmd = 0;
    s_ncoll = 0;
    s_nout = 0;
  }
  __syncthreads();
  int n_w0 = 0, n_w1 = 0, n_bad = 0, n_md = 0, n_out = 0, n_fast = 0;
  for (int base = beg; base < end; base += kChunk) {
    const int p0 = base + kPPT * (int)threadIdx.x;
    const bool have = p0 < end;  // four slots in the tile, or none
    const long g4 = p0 / kPPT;
    double x[kPPT][3], v[kPPT][3];
    uint32_t id[kPPT] = {};
#pragma unroll
    for (int q = 0; q < kPPT; ++q) {
      x[q][0] = x[q][1] = v[q][0] = v[q][1] = v[q][2] = 0.0;
      x[q][2] = -1.0;
    }
    if (have) {
#define PIC_LOAD4(arr, dst, a)                                            \
  {                                                                       \
    const double2 lo = reinterpret_cast<const double2*>(arr)[2 * g4];     \
    const double2 hi = reinterpret_cast<const double2*>(arr)[2 * g4 + 1]; \
    dst[0][a] = lo.x;                                                     \
    dst[1][a] = lo.y;                                                     \
    dst[2][a] = hi.x;                                                     \
    dst[3][a] = hi.y;                                                     \
  }
      PIC_LOAD4(P.x, x, 0)
      PIC_LOAD4(P.y, x, 1)
      PIC_LOAD4(P.z, x, 2)
      PIC_LOAD4(P.vx, v, 0)
      PIC_LOAD4(P.vy, v, 1)
      PIC_LOAD4(P.vz, v, 2)
#undef PIC_LOAD4
      const uint4 I4 = reinterpret_cast<const uint4*>(P.id)[g4];
      id[0] = I4.x;
      id[1] = I4.y;
      id[2] = I4.z;
      id[3] = I4.w;
    }
    int st[kPPT], cell[kPPT];
    bool cand[kPPT];
#pragma unroll
    for (int q = 0; q < kPPT; ++q) {
      st[q] = ST_NONE;
      cand[q] = false;
      cell[q] = -1;
      if (!(x[q][2] >= 0.0)) continue;
      const int i0 = (int)floor(x[q][0]), j0 = (int)floor(x[q][1]), k0 = (int)floor(x[q][2]);
      if (!kMove) {
        st[q] = ST_ALIVE;
        cell[q] = pack_cell(i0, j0, k0);
        continue;
      }
      if (md_lookup(md, S.nx, S.ny, i0, j0, k0) != 0u) {
        st[q] = ST_MD;
        continue;
      }
      const int lb = tile_cell(tile, i0, j0, k0, S.nx, S.ny);
      if (lb < 0) {
        st[q] = ST_OUT;  // left for the outlier kernel
        continue;
      }
      double Ep[3];
      {
        const double fx = x[q][0] - i0, fy = x[q][1] - j0, fz = x[q][2] - k0;
        const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
        Ep[0] = Ep[1] = Ep[2] = 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int l = lb + (t & 1) + tile.tx * (((t >> 1) & 1) + tile.ty * (t >> 2));
          const double w = wx[t & 1] * wy[(t >> 1) & 1] * wz[t >> 2];
          const double2 a = s_E[2 * l], b2 = s_E[2 * l + 1];
          Ep[0] += w * a.x;
          Ep[1] += w * a.y;
          Ep[2] += w * b2.x;
        }
      }
      st[q] = push_one_f64(S, Ep, x[q], v[q]);
      n_fast += v[q][0] * v[q][0] + v[q][1] * v[q][1] + v[q][2] * v[q][2] >= S.vfast2;
      if (st[q] == ST_ALIVE) {
        cell[q] = pack_cell((int)floor(x[q][0]), (int)floor(x[q][1]), (int)floor(x[q][2]));
        const uint4 r = philox4x32_10(id[q], *S.step, kColl, (uint32_t)S.sp, S.key0, S.key1);
        cand[q] = (uint64_t)r.x < S.T_null;
      } else {
        x[q][2] = -1.0;
      }
    }
    if (kMove) {
      bool is_out[kPPT];
#pragma unroll
      for (int q = 0; q < kPPT; ++q) is_out[q] = st[q] == ST_OUT;
      append_slot_order(st, ST_MD, s_md, &s_nmd, p0);
      chunk_append4(cand, L.coll + beg, &s_ncoll, p0);
      chunk_append4(is_out, L.out + beg, &s_nout, p0);
#pragma unroll
      for (int q = 0; q < kPPT; ++q) {
        n_out += st[q] == ST_OUT;
        n_w0 += st[q] == ST_WALL0;
        n_w1 += st[q] == ST_WALL1;
        n_bad += st[q] == ST_BAD;
        n_md += st[q] == ST_MD;
      }
      if (have) {
#define PIC_STORE4(arr, srcv, a)                                                          \
  {                                                                                       \
    reinterpret_cast<double2*>(arr)[2 * g4] = make_double2(srcv[0][a], srcv[1][a]);     \
    reinterpret_cast<double2*>(arr)[2 * g4 + 1] = make_double2(srcv[2][a], srcv[3][a]); \
  }
        PIC_STORE4(P.x, x, 0)
        PIC_STORE4(P.y, x, 1)
        PIC_STORE4(P.z, x, 2)
        PIC_STORE4(P.vx, v, 0)
        PIC_STORE4(P.vy, v, 1)
        PIC_STORE4(P.vz, v, 2)
#undef PIC_STORE4
      }
    }

    double acc[8];
    int acc_cell = -1;
#pragma unroll
    for (int q = 0; q < kPPT; ++q) {
      if (st[q] != ST_ALIVE) continue;
      double w[8];
      const int i = cell_i(cell[q]), j = cell_j(cell[q]), k = cell_k(cell[q]);
      cic_weights_d(x[q][0] - i, x[q][1] - j, x[q][2] - k, S.sign, w);
      if (cell[q] == acc_cell) {
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] += w[t];
      } else {
        if (acc_cell >= 0) {
          const int ai = cell_i(acc_cell), aj = cell_j(acc_cell), ak = cell_k(acc_cell);
          corner_add<double>(tile, tile_cell(tile, ai, aj, ak, S.nx, S.ny), s_rho, rho, S, ai, aj,
                             ak, acc);
        }
        acc_cell = cell[q];
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] = w[t];
      }
    }
    if (acc_cell >= 0) {
      const int ai = cell_i(acc_cell), aj = cell_j(acc_cell), ak = cell_k(acc_cell);
      corner_add<double>(tile, tile_cell(tile, ai, aj, ak, S.nx, S.ny), s_rho, rho, S, ai, aj, ak,
                         acc);
    }
    if (kMove) {
      __syncthreads();
      md_flush(s_md, &s_nmd, &s_mdbase, L);
    }
  }
  if (kMove) {
    tally_add(s_tally, TL_W0, n_w0);
    tally_add(s_tally, TL_W1, n_w1);
    tally_add(s_tally, TL_BAD, n_bad);
    tally_add(s_tally, TL_MD, n_md);
    tally_add(s_tally, TL_DEAD, n_w0 + n_w1 + n_bad);
    tally_add(s_tally, TL_FALL, n_out);
    tally_add(s_tally, TL_FAST, n_fast);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < vol; t += kBlock) {
    const double val = s_rho[t];
    if (val != 0.0) unsafeAtomicAdd(&rho[tile_node(tile, t, rtx, rtxy, S.nx, S.ny, S.nxy)], val);
  }
  if (kMove) {
    if (threadIdx.x == 0) {
      L.coll_cnt[tidx] = s_ncoll;
      L.out_cnt[tidx] = s_nout;
    }
    tally_store(s_tally, L.tally + (long)TL_N * tidx);
  }
}

// ---------------------------------------------------------------- MD particles
// The particles that started the step inside an MD cube: the sub-cycled PPPM
// motion in FP64, grain and electrode absorption, the collision, the deposit.
// One thread per entry of the dense list.
__device__ __forceinline__ void load_d(const PartF64& P, long p, double x[3], double v[3]) {
  x[0] = P.x[p];
  x[1] = P.y[p];
  x[2] = P.z[p];
  v[0] = P.vx[p];
  v[1] = P.vy[p];
  v[2] = P.vz[p];
}
__device__ __forceinline__ void load_d(const PartF32R& P, long p, double x[3], double v[3]) {
  const int c = P.cell[p];
  x[0] = (double)cell_i(c) + (double)P.ox[p];
  x[1] = (double)cell_j(c) + (double)P.oy[p];
  x[2] = (double)cell_k(c) + (double)P.oz[p];
  v[0] = P.vx[p];
  v[1] = P.vy[p];
  v[2] = P.vz[p];
}

// store the survivor; returns its cell (-1 if rounding put it on the rf
// electrode) and the eight corner shares of its charge
__device__ __forceinline__ int store_d(const PartF64& P, long p, const double x[3],
                                       const double v[3], const SpeciesStep& S, double part[8]) {
  P.x[p] = x[0];
  P.y[p] = x[1];
  P.z[p] = x[2];
  P.vx[p] = v[0];
  P.vy[p] = v[1];
  P.vz[p] = v[2];
  const int i = (int)floor(x[0]), j = (int)floor(x[1]), k = (int)floor(x[2]);
  cic_weights_d(x[0] - i, x[1] - j, x[2] - k, S.sign, part);
  return pack_cell(i, j, k);
}
__device__ __forceinline__ int store_d(const PartF32R& P, long p, const double x[3],
                                       const double v[3], const SpeciesStep& S,
                                       long long part[8]) {
  int c[3];
  float f[3];
  const int n3[3] = {S.nx, S.ny, S.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c[a] = (int)floor(x[a]);
    f[a] = (float)(x[a] - (double)c[a]);
    if (f[a] >= 1.0f) {
      f[a] = 0.0f;
      c[a] += 1;
      if (a < 2 && c[a] == n3[a]) c[a] = 0;
    }
  }
  P.vx[p] = (float)v[0];
  P.vy[p] = (float)v[1];
  P.vz[p] = (float)v[2];
  if (c[2] >= S.nz) {
    P.cell[p] = -1;
    return -1;
  }
  P.cell[p] = pack_cell(c[0], c[1], c[2]);
  P.ox[p] = f[0];
  P.oy[p] = f[1];
  P.oz[p] = f[2];
  split8(S.Qp, f[0], f[1], f[2], part);
#pragma unroll
  for (int t = 0; t < 8; ++t) part[t] *= S.isign;
  return P.cell[p];
}

template <typename T>
__device__ __forceinline__ T wave_sum_t(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The charges of a wave's MD particles to the global mesh.  The particles of
// a cell of the dense list tend to sit in neighbouring lanes and hit the same
// eight nodes, which all MD blocks share, so per distinct cell the wave first
// sums the corner shares and one lane adds them (for the fixed-point charge
// the sums are exact and the mesh does not depend on the grouping).  After
// kDepGroups distinct cells the remaining lanes add their own shares.
constexpr int kDepGroups = 16;
template <typename A>
__device__ __forceinline__ void deposit_wave(A* __restrict__ rho, const SpeciesStep& S, int cell,
                                             const A part[8]) {
  const int lane = threadIdx.x & 63;
  unsigned long long pending = __ballot(cell >= 0);
  Tile none{};
  for (int it = 0; it < kDepGroups && pending; ++it) {
    const int leader = __ffsll((long long)pending) - 1;
    const int key = __shfl(cell, leader, 64);
    const bool mine = cell == key;
    const unsigned long long m = __ballot(mine);
    pending &= ~m;
    A sum[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) sum[t] = wave_sum_t<A>(mine ? part[t] : (A)0);
    if (lane == leader)
      corner_add<A>(none, -1, nullptr, rho, S, cell_i(key), cell_j(key), cell_k(key), sum);
  }
  if ((pending >> lane) & 1ull)
    corner_add<A>(none, -1, nullptr, rho, S, cell_i(cell), cell_j(cell), cell_k(cell), part);
}

__device__ __forceinline__ void kill(const PartF64& P, long p) { P.z[p] = -1.0; }
__device__ __forceinline__ void kill(const PartF32R& P, long p) { P.cell[p] = -1; }
// slot p of src into slot p of dst (an empty src slot empties dst's)
__device__ __forceinline__ void copy_rec(const PartF64& src, const PartF64& dst, long p) {
  dst.x[p] = src.x[p];
  dst.y[p] = src.y[p];
  dst.z[p] = src.z[p];
  dst.vx[p] = src.vx[p];
  dst.vy[p] = src.vy[p];
  dst.vz[p] = src.vz[p];
}
__device__ __forceinline__ void copy_rec(const PartF32R& src, const PartF32R& dst, long p) {
  const int c = src.cell[p];
  dst.cell[p] = c;
  if (c < 0) return;
  dst.ox[p] = src.ox[p];
  dst.oy[p] = src.oy[p];
  dst.oz[p] = src.oz[p];
  dst.vx[p] = src.vx[p];
  dst.vy[p] = src.vy[p];
  dst.vz[p] = src.vz[p];
}

// one thread per MD particle of the dense list of this step, both species in
// one launch (blocks [0, nb) electrons, [nb, 2 nb) ions); events go to the
// block's own tally row, grain hits to LDS counters first.  The particles are
// read from P and their new states written to the same slots of D: D = P for
// the FP64 records (in place, after the push); the FP32R step runs this kernel
// beside the push with D the species' other record buffer, and
// md_collide_kernel copies the states back afterwards.  The survivors'
// collisions follow in md_collide_kernel (kept out of this kernel so that its
// registers allow three waves per SIMD).
constexpr int kMdThreads = 64;
template <typename PT, typename ET, typename RT>
__global__ __launch_bounds__(kMdThreads) void md_kernel(SpeciesPair<PT> pr, PT D0, PT D1,
                                                        const ET* __restrict__ E,
                                                        RT* __restrict__ rho, MdTables md,
                                                        unsigned long long* __restrict__ grain_count) {
  const int sp = (int)blockIdx.x >= pr.nb;
  const PT P = pr.P[sp];
  const PT D = sp ? D1 : D0;
  const SpeciesStep S = pr.S[sp];
  const WorkLists L = pr.L[sp];
  const int bid = (int)blockIdx.x - sp * pr.nb;
  const int total = L.cnt[2];
  if ((long)bid * kMdThreads >= total) return;
  constexpr int kStage = 256;
  __shared__ double s_gpos[3 * kStage], s_Qc[kStage];
  __shared__ unsigned s_hits[kStage];
  for (int t = threadIdx.x; t < min(md.n_grains, kStage); t += blockDim.x) {
    s_Qc[t] = md.Q[t] * S.coul_c;
    s_hits[t] = 0u;
    for (int a = 0; a < 3; ++a) s_gpos[3 * t + a] = md.gpos[3 * t + a];
  }
  __syncthreads();
  const GrainView G = md.n_grains <= kStage ? GrainView{s_gpos, s_Qc, 1.0}
                                            : GrainView{md.gpos, md.Q, S.coul_c};
  int n_w0 = 0, n_w1 = 0, n_bad = 0, n_dead = 0;
  for (long base = (long)bid * kMdThreads; base < total; base += (long)pr.nb * kMdThreads) {
    const long idx = base + threadIdx.x;
    int st = ST_NONE, cell = -1;
    RT part[8];
    if (idx < total) {
      const long p = L.md[idx];
      double x[3], v[3];
      load_d(P, p, x, v);
      int hit = -1;
      st = md_move(E, md, G, S, x, v, hit);
      if (st == ST_GRAIN) {
        if (hit < kStage) atomicAdd(&s_hits[hit], 1u);
        else atomicAdd(&grain_count[2 * hit + S.sp], 1ull);
      }
      if (st == ST_ALIVE) {
        cell = store_d(D, p, x, v, S, part);
        if (cell < 0) st = ST_WALL1;
      } else {
        kill(D, p);
      }
    }
    deposit_wave<RT>(rho, S, cell, part);
    n_w0 += st == ST_WALL0;
    n_w1 += st == ST_WALL1;
    n_bad += st == ST_BAD;
    n_dead += st == ST_WALL0 || st == ST_WALL1 || st == ST_BAD || st == ST_GRAIN;
  }
  int c4[4] = {n_w0, n_w1, n_bad, n_dead};
#pragma unroll
  for (int k = 0; k < 4; ++k) c4[k] = wave_sum(c4[k]);
  if (threadIdx.x == 0) {  // this block's own tally row (no atomics)
    unsigned long long* tally = L.tally + (long)TL_N * (L.ngrid + bid);
    const int kinds[4] = {TL_W0, TL_W1, TL_BAD, TL_DEAD};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (c4[k]) tally[kinds[k]] += (unsigned long long)c4[k];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < min(md.n_grains, kStage); t += blockDim.x)
    if (s_hits[t]) atomicAdd(&grain_count[2 * t + S.sp], (unsigned long long)s_hits[t]);
}

// ---------------------------------------------------------------- moments
// Density and flux moments of one species on the mesh nodes (the densities
// and fluxes of Sec. IV): per node the sums over the particles of W and of
// v W, where W is the particle's CIC weight for the node, the same
// assignment as the charge deposit of Sec. III.  The host scales them by
// w / dx^3.  v is the stored half-step velocity v_{k-1/2}.  One block per
// tile: the tile's (4+1)^3 nodes accumulate in LDS and are then added to the
// mesh; particles that left the tile since the last re-binning add to the
// mesh directly.  mom is [4][nn]: W, v_x W, v_y W, v_z W.  For the time
// averages (avg.step non-null) the sums go to the rf-phase bin of the
// current step, avg.stride doubles further per bin.
// the moment window: the tile's nodes plus the species' drift margin (as the
// push stages them; at most 2 cells here), so particles that drifted out of
// their tile since the last re-binning still add in LDS
constexpr int kMomWin = 729;
// copies of the window: thread t adds into copy t % kMomCopies (summed at the flush)
constexpr int kMomCopies = 1;
__device__ __forceinline__ bool slot_alive(const PartF64& P, long p) { return P.z[p] >= 0.0; }
__device__ __forceinline__ bool slot_alive(const PartF32R& P, long p) { return P.cell[p] >= 0; }

template <typename PT>
__global__ __launch_bounds__(256) void moments_kernel(PT P, SpeciesStep S, WorkLists L,
                                                      double* __restrict__ mom, long nn,
                                                      AvgBins avg) {
  const int t = blockIdx.x;
  if (avg.step) mom += avg.stride * phase_bin(*avg.step, avg.f_rf, avg.dt, avg.nbins);
  const long a = L.tstart[t], b = L.tstart[t + 1];
  if (a == b) return;
  __shared__ double s_m[kMomCopies][4][kMomWin];
  const Tile T = make_tile(t, L, S.nx, S.ny, S.nz, S.margin, kMomWin);
  for (int u = threadIdx.x; u < kMomCopies * 4 * kMomWin; u += blockDim.x) (&s_m[0][0][0])[u] = 0.0;
  __syncthreads();
  const int cp = (int)threadIdx.x % kMomCopies;
  // each thread walks a contiguous run of slots: the slots of a tile are grouped
  // by cell, so consecutive particles of one cell are summed in registers and
  // reach the LDS window once per run
  const long per = (b - a + blockDim.x - 1) / blockDim.x;
  const long p0 = a + (long)threadIdx.x * per, p1 = p0 + per < b ? p0 + per : b;
  int run_lb = -1;
  double acc[4][8];
  for (long p = p0; p < p1; ++p) {
    if (!slot_alive(P, p)) continue;
    double x[3], v[3], w[8];
    load_d(P, p, x, v);
    const int i = (int)floor(x[0]), j = (int)floor(x[1]), k = (int)floor(x[2]);
    cic_weights_d(x[0] - i, x[1] - j, x[2] - k, 1.0, w);
    const int lb = tile_cell(T, i, j, k, S.nx, S.ny);
    if (lb < 0) {
      // outside the window: straight to the mesh
      double val[8];
      corner_add<double>(T, -1, s_m[cp][0], mom, S, i, j, k, w);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
#pragma unroll
        for (int c = 0; c < 8; ++c) val[c] = v[q] * w[c];
        corner_add<double>(T, -1, s_m[cp][q + 1], mom + (q + 1) * nn, S, i, j, k, val);
      }
      continue;
    }
    if (lb != run_lb) {
      if (run_lb >= 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) corner_add<double>(T, run_lb, s_m[cp][q], mom, S, 0, 0, 0, acc[q]);
      }
      run_lb = lb;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        acc[0][c] = w[c];
        acc[1][c] = v[0] * w[c];
        acc[2][c] = v[1] * w[c];
        acc[3][c] = v[2] * w[c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        acc[0][c] += w[c];
        acc[1][c] += v[0] * w[c];
        acc[2][c] += v[1] * w[c];
        acc[3][c] += v[2] * w[c];
      }
    }
  }
  if (run_lb >= 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) corner_add<double>(T, run_lb, s_m[cp][q], mom, S, 0, 0, 0, acc[q]);
  }
  __syncthreads();
  if (!T.on) return;
  const int nt = T.tx * T.ty * T.tz;
  const float rtx = 1.0f / (float)T.tx, rtxy = 1.0f / (float)(T.tx * T.ty);
  for (int u = threadIdx.x; u < nt; u += blockDim.x) {
    const long node = tile_node(T, u, rtx, rtxy, S.nx, S.ny, S.nxy);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double sum = 0.0;
#pragma unroll
      for (int c = 0; c < kMomCopies; ++c) sum += s_m[c][q][u];
      if (sum != 0.0) unsafeAtomicAdd(&mom[q * nn + node], sum);
    }
  }
}

// Fine diagnostic grid (the grid finer than the PIC cells over the grains'
// region, Sec. IV): a particle whose u = (x - o) / h lies in [0, m) on every
// axis adds its cloud-in-cell weights W and v W to the 8 nodes of its fine
// cell.  Grid-stride over the slots in use; the PIC cell is tested first, so
// the records of particles far from the box are not read whole.  Global FP64
// atomics: the box holds few particles per fine cell.
__device__ __forceinline__ bool fine_cell_near(const FineBox& fb, int i, int j, int k) {
  return i >= fb.lo[0] && i < fb.hi[0] && j >= fb.lo[1] && j < fb.hi[1] && k >= fb.lo[2] &&
         k < fb.hi[2];
}
__device__ __forceinline__ bool fine_near(const PartF64& P, long p, const FineBox& fb) {
  const double z = P.z[p];
  if (!(z >= 0.0)) return false;
  return fine_cell_near(fb, (int)floor(P.x[p]), (int)floor(P.y[p]), (int)floor(z));
}
__device__ __forceinline__ bool fine_near(const PartF32R& P, long p, const FineBox& fb) {
  const int c = P.cell[p];
  return c >= 0 && fine_cell_near(fb, cell_i(c), cell_j(c), cell_k(c));
}

template <typename PT>
__global__ __launch_bounds__(256) void fine_moments_kernel(PT P, WorkLists L, FineBox fb,
                                                           double* __restrict__ mom,
                                                           AvgBins avg) {
  if (avg.step) mom += avg.stride * phase_bin(*avg.step, avg.f_rf, avg.dt, avg.nbins);
  const long total = L.tstart[L.ngrid];
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < total;
       p += (long)gridDim.x * blockDim.x) {
    if (!fine_near(P, p, fb)) continue;
    double x[3], v[3], u[3];
    load_d(P, p, x, v);
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      u[a] = (x[a] - fb.o[a]) / fb.h;
      in = in && u[a] >= 0.0 && u[a] < (double)fb.m[a];
    }
    if (!in) continue;
    const long i = (long)floor(u[0]), j = (long)floor(u[1]), k = (long)floor(u[2]);
    const double fx = u[0] - (double)i, fy = u[1] - (double)j, fz = u[2] - (double)k;
    const long base = (k * fb.my + j) * fb.mx + i;
#pragma unroll
    for (int cc = 0; cc < 2; ++cc)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const double wt = (a ? fx : 1.0 - fx) * (b ? fy : 1.0 - fy) * (cc ? fz : 1.0 - fz);
          const long node = base + ((long)cc * fb.my + b) * fb.mx + a;
          unsafeAtomicAdd(&mom[node], wt);
#pragma unroll
          for (int q = 0; q < 3; ++q) unsafeAtomicAdd(&mom[(q + 1) * fb.fn + node], v[q] * wt);
        }
  }
}

// The collisions of the MD particles that survived their sub-cycled motion,
// from their stored velocities (same list, blocks and tally rows as md_kernel).
template <typename PT>
__device__ __forceinline__ void md_collide_block(const SpeciesPair<PT>& pr, const PT& D, int sp,
                                                 int bid, int commit, int mcc) {
  const PT P = pr.P[sp];
  const SpeciesStep S = pr.S[sp];
  const WorkLists L = pr.L[sp];
  const int total = L.cnt[2];
  if ((long)bid * kMdThreads >= total) return;
  int n_coll = 0, n_cap = 0;
  for (long idx = (long)bid * kMdThreads + threadIdx.x; idx < total;
       idx += (long)pr.nb * kMdThreads) {
    const long p = L.md[idx];
    if (commit) copy_rec(D, P, p);  // the sub-cycled kernel's result
    if (!mcc || !slot_alive(P, p)) continue;
    bool coll = false, capv = false;
    typename VelOf<PT>::type v[3] = {P.vx[p], P.vy[p], P.vz[p]};
    collide(S, P.id[p], v, coll, capv, p);
    if (coll) {
      P.vx[p] = v[0];
      P.vy[p] = v[1];
      P.vz[p] = v[2];
    }
    n_coll += coll;
    n_cap += capv;
  }
  n_coll = wave_sum(n_coll);
  n_cap = wave_sum(n_cap);
  if (threadIdx.x == 0) {
    unsigned long long* tally = L.tally + (long)TL_N * (L.ngrid + bid);
    if (n_coll) tally[TL_COLL] += (unsigned long long)n_coll;
    if (n_cap) tally[TL_CAP] += (unsigned long long)n_cap;
  }
}
template <typename PT>
__global__ __launch_bounds__(kMdThreads) void md_collide_kernel(SpeciesPair<PT> pr, PT D0, PT D1,
                                                                int commit, int mcc,
                                                                int sp_only) {
  // both species (blocks [0, nb) electrons) or species sp_only alone
  const int sp = sp_only >= 0 ? sp_only : ((int)blockIdx.x >= pr.nb ? 1 : 0);
  const int bid = (int)blockIdx.x - (sp_only >= 0 ? 0 : sp * pr.nb);
  md_collide_block(pr, sp ? D1 : D0, sp, bid, commit, mcc);
}

// ---------------------------------------------------------------- MD list
// The dense MD list of an FP32R step, formed before the push: every slot
// whose particle starts the step in a cell of an MD cube (the push leaves
// those to the sub-cycled kernel; the same test as the push's).  A particle
// in an MD cube either lies inside its push block's window, which then meets
// the MD cubes' bounding box, or has left that window since the last sort,
// which set the block's stray flag; the grid's padding tiles (new particles of
// ionisation) have no window.  So one block per push block (blocks [0, npb)
// electrons, the rest ions) scans the block's slots only in those cases, in
// chunks of kMdScanSlots, compacting a chunk's hits in slot order and
// reserving their place in the list with one atomic; L.cnt[2] is zero at the
// start of a step.
constexpr int kMdScanPer = 8;  // slots per thread and chunk (two 16-byte loads)
constexpr int kMdScanSlots = 256 * kMdScanPer;
__global__ __launch_bounds__(256) void md_scan_kernel(PartF32R P0, PartF32R P1, WorkLists L0,
                                                      WorkLists L1, MdTables md, int nx, int ny,
                                                      int nz, int m0, int m1, int span, int npb) {
  __shared__ int s_wave[4];
  __shared__ int s_base;
  const int sp = (int)blockIdx.x >= npb ? 1 : 0;
  const PartF32R P = sp ? P1 : P0;
  const WorkLists L = sp ? L1 : L0;
  const int t0 = ((int)blockIdx.x - sp * npb) * span;
  const int beg = L.tstart[t0], end = L.tstart[t0 + span];  // multiples of 4
  if (beg >= end) return;
  if (!L.stray[t0] &&
      !window_meets_md(make_tile(t0, L, nx, ny, nz, sp ? m1 : m0, kWinF32, span), md, nx, ny))
    return;
  const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
  for (int s0 = beg; s0 < end; s0 += kMdScanSlots) {
    const int p0 = s0 + kMdScanPer * (int)threadIdx.x;
    int c[kMdScanPer];
#pragma unroll
    for (int h = 0; h < kMdScanPer / 4; ++h) {
      int4 v = make_int4(-1, -1, -1, -1);
      if (p0 + 4 * h < end) v = reinterpret_cast<const int4*>(P.cell)[(p0 >> 2) + h];
      c[4 * h] = v.x;
      c[4 * h + 1] = v.y;
      c[4 * h + 2] = v.z;
      c[4 * h + 3] = v.w;
    }
    bool hit[kMdScanPer];
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < kMdScanPer; ++q) {
      hit[q] = c[q] >= 0 && md_lookup(md, nx, ny, cell_i(c[q]), cell_j(c[q]), cell_k(c[q])) != 0u;
      cnt += hit[q];
    }
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      const int total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
      s_base = total ? atomicAdd(&L.cnt[2], total) : 0;
    }
    __syncthreads();
    int at = s_base + incl - cnt;
    for (int w = 0; w < wave; ++w) at += s_wave[w];
#pragma unroll
    for (int q = 0; q < kMdScanPer; ++q)
      if (hit[q]) L.md[at++] = p0 + q;
    __syncthreads();  // s_wave and s_base are reused by the next chunk
  }
}

// ---------------------------------------------------------------- outliers
// Particles that started outside their tile's window (they drifted since the
// last sort): the same push with the field gathered from global memory and the
// charge deposited with global atomics, the collision done in place.  One wave
// per tile segment.
// the outliers of push block bid of species sp
__device__ __forceinline__ void outlier_block(const SpeciesPair<PartF32R>& pr,
                                              const float4* __restrict__ E,
                                              long long* __restrict__ rho, int do_mcc, int sp,
                                              int bid) {
  const PartF32R P = pr.P[sp];
  const SpeciesStep S = pr.S[sp];
  const WorkLists L = pr.L[sp];
  const int tidx = bid * pr.span;
  const int count = L.out_cnt[tidx];
  if (count == 0) return;
  if (threadIdx.x == 0) L.stray[tidx] = 1;  // (already set when these left the window)
  const int32_t* seg = L.out + L.tstart[tidx];
  int t_w0 = 0, t_w1 = 0, t_bad = 0, t_coll = 0, t_cap = 0, t_fast = 0;
  for (int idx = threadIdx.x; idx < count; idx += 64) {
    const long p = seg[idx];
    const int c = P.cell[p];
    int ci = cell_i(c), cj = cell_j(c), ck = cell_k(c);
    float o[3] = {P.ox[p], P.oy[p], P.oz[p]};
    float v[3] = {P.vx[p], P.vy[p], P.vz[p]};
    float ec[8][3];
    const int i1 = ci + 1 == S.nx ? 0 : ci + 1;
    const int j1 = cj + 1 == S.ny ? 0 : cj + 1;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const float4 e = E[((t & 1) ? i1 : ci) + (long)S.nx * (((t >> 1) & 1) ? j1 : cj) +
                         (long)S.nxy * (ck + (t >> 2))];
      ec[t][0] = e.x;
      ec[t][1] = e.y;
      ec[t][2] = e.z;
    }
    const int st = push_one_f32(S, ec, o, v, ci, cj, ck);
    t_fast += v[0] * v[0] + v[1] * v[1] + v[2] * v[2] >= S.vfast2_f;
    if (st == ST_ALIVE) {
      bool coll = false, capv = false;
      if (do_mcc) {
        const uint32_t id = P.id[p];
        const uint4 r = philox4x32_10(id, *S.step, kColl, (uint32_t)S.sp, S.key0, S.key1);
        if ((uint64_t)r.x < S.T_null) collide(S, id, v, coll, capv, p);
      }
      t_coll += coll;
      t_cap += capv;
      P.cell[p] = pack_cell(ci, cj, ck);
      P.ox[p] = o[0];
      P.oy[p] = o[1];
      P.oz[p] = o[2];
      deposit_global_fixed(rho, S, ci, cj, ck, o[0], o[1], o[2]);
    } else {
      P.cell[p] = -1;
    }
    P.vx[p] = v[0];
    P.vy[p] = v[1];
    P.vz[p] = v[2];
    t_w0 += st == ST_WALL0;
    t_w1 += st == ST_WALL1;
    t_bad += st == ST_BAD;
  }
  t_w0 = wave_sum(t_w0);
  t_w1 = wave_sum(t_w1);
  t_bad = wave_sum(t_bad);
  t_coll = wave_sum(t_coll);
  t_cap = wave_sum(t_cap);
  t_fast = wave_sum(t_fast);
  if (threadIdx.x == 0) {
    unsigned long long* tl = L.tally + (long)TL_N * tidx;
    tl[TL_W0] += t_w0;
    tl[TL_W1] += t_w1;
    tl[TL_BAD] += t_bad;
    tl[TL_COLL] += t_coll;
    tl[TL_CAP] += t_cap;
    tl[TL_DEAD] += t_w0 + t_w1 + t_bad;
    tl[TL_FAST] += t_fast;
  }
}
__global__ __launch_bounds__(64) void outlier_f32r_kernel(SpeciesPair<PartF32R> pr,
                                                          const float4* __restrict__ E,
                                                          long long* __restrict__ rho, int do_mcc,
                                                          int sp_only) {
  // both species (blocks [0, nb) electrons) or species sp_only alone
  const int sp = sp_only >= 0 ? sp_only : ((int)blockIdx.x >= pr.nb ? 1 : 0);
  outlier_block(pr, E, rho, do_mcc, sp, (int)blockIdx.x - (sp_only >= 0 ? 0 : sp * pr.nb));
}

__global__ __launch_bounds__(64) void outlier_f64_kernel(SpeciesPair<PartF64> pr,
                                                         const double2* __restrict__ E,
                                                         double* __restrict__ rho, int do_mcc) {
  const int sp = (int)blockIdx.x >= pr.nb;
  const PartF64 P = pr.P[sp];
  const SpeciesStep S = pr.S[sp];
  const WorkLists L = pr.L[sp];
  const int tidx = (int)blockIdx.x - sp * pr.nb;
  const int count = L.out_cnt[tidx];
  if (count == 0) return;
  const int32_t* seg = L.out + L.tstart[tidx];
  int t_w0 = 0, t_w1 = 0, t_bad = 0, t_coll = 0, t_cap = 0, t_fast = 0;
  for (int idx = threadIdx.x; idx < count; idx += 64) {
    const long p = seg[idx];
    double x[3], v[3];
    load_d(P, p, x, v);
    const int i0 = (int)floor(x[0]), j0 = (int)floor(x[1]), k0 = (int)floor(x[2]);
    double Ep[3];
    gather_d(E, S, i0, j0, k0, x[0] - i0, x[1] - j0, x[2] - k0, Ep);
    const int st = push_one_f64(S, Ep, x, v);
    t_fast += v[0] * v[0] + v[1] * v[1] + v[2] * v[2] >= S.vfast2;
    if (st == ST_ALIVE) {
      bool coll = false, capv = false;
      if (do_mcc) {
        const uint32_t id = P.id[p];
        const uint4 r = philox4x32_10(id, *S.step, kColl, (uint32_t)S.sp, S.key0, S.key1);
        if ((uint64_t)r.x < S.T_null) collide(S, id, v, coll, capv, p);
      }
      t_coll += coll;
      t_cap += capv;
      double part[8];
      const int c = store_d(P, p, x, v, S, part);
      Tile none{};
      corner_add<double>(none, -1, nullptr, rho, S, cell_i(c), cell_j(c), cell_k(c), part);
    } else {
      kill(P, p);
      P.vx[p] = v[0];
      P.vy[p] = v[1];
      P.vz[p] = v[2];
    }
    t_w0 += st == ST_WALL0;
    t_w1 += st == ST_WALL1;
    t_bad += st == ST_BAD;
  }
  t_w0 = wave_sum(t_w0);
  t_w1 = wave_sum(t_w1);
  t_bad = wave_sum(t_bad);
  t_coll = wave_sum(t_coll);
  t_cap = wave_sum(t_cap);
  t_fast = wave_sum(t_fast);
  if (threadIdx.x == 0) {
    unsigned long long* tl = L.tally + (long)TL_N * tidx;
    tl[TL_W0] += t_w0;
    tl[TL_W1] += t_w1;
    tl[TL_BAD] += t_bad;
    tl[TL_COLL] += t_coll;
    tl[TL_CAP] += t_cap;
    tl[TL_DEAD] += t_w0 + t_w1 + t_bad;
    tl[TL_FAST] += t_fast;
  }
}

// ---------------------------------------------------------------- collisions
// One wave per push block's segment of collision candidates (the push block
// of `span` tiles lists them at its first tile).
template <typename PT>
__device__ __forceinline__ void collide_block(const PT& P, const SpeciesStep& S, const WorkLists& L,
                                              int tidx) {
  const int count = L.coll_cnt[tidx];
  if (count == 0) return;
  const int32_t* seg = L.coll + L.tstart[tidx];
  int n_coll = 0, n_cap = 0;
  for (int idx = threadIdx.x; idx < count; idx += 64) {
    const long p = seg[idx];
    bool coll = false, capv = false;
    typename VelOf<PT>::type v[3] = {P.vx[p], P.vy[p], P.vz[p]};
    collide(S, P.id[p], v, coll, capv, p);
    if (coll) {
      P.vx[p] = v[0];
      P.vy[p] = v[1];
      P.vz[p] = v[2];
    }
    n_coll += coll;
    n_cap += capv;
  }
  n_coll = wave_sum(n_coll);
  n_cap = wave_sum(n_cap);
  if (threadIdx.x == 0) {
    unsigned long long* tl = L.tally + (long)TL_N * tidx;
    tl[TL_COLL] += (unsigned long long)n_coll;
    tl[TL_CAP] += (unsigned long long)n_cap;
  }
}
template <typename PT>
__global__ __launch_bounds__(64) void collide_kernel(PT P, SpeciesStep S, WorkLists L, int span) {
  collide_block(P, S, L, (int)blockIdx.x * span);
}

// Everything after one FP32R species' push in one launch: block b < npb takes
// push block b's collision candidates and then its outliers (disjoint sets of
// particles, one tally row), and the kMdListBlocks blocks after those copy the
// MD particles' states back and collide them.
constexpr int kMdListBlocks = 512;
__global__ __launch_bounds__(64) void species_lists_f32r_kernel(SpeciesPair<PartF32R> pr,
                                                                PartF32R D, const float4* E,
                                                                long long* rho, int do_mcc, int sp,
                                                                int npb, int md) {
  const int b = (int)blockIdx.x;
  if (b < npb) {
    collide_block(pr.P[sp], pr.S[sp], pr.L[sp], b * pr.span);
    outlier_block(pr, E, rho, do_mcc, sp, b);
  } else if (md) {
    SpeciesPair<PartF32R> pm = pr;
    pm.nb = kMdListBlocks;  // the blocks' stride over the MD list (tally rows 0 .. 511)
    md_collide_block(pm, D, sp, b - npb, 1, do_mcc);
  }
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

__global__ void init_f32r_kernel(PartF32R P, int n, int ppc, int nx, int ny, int sp, uint32_t k0,
                                 uint32_t k1, double vth) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int cell = p / ppc;
  double off[3], vel[3];
  load_draws((uint32_t)p, sp, k0, k1, vth, off, vel);
  P.cell[p] = pack_cell(cell % nx, (cell / nx) % ny, cell / (nx * ny));
  P.ox[p] = (float)off[0];
  P.oy[p] = (float)off[1];
  P.oz[p] = (float)off[2];
  P.vx[p] = (float)vel[0];
  P.vy[p] = (float)vel[1];
  P.vz[p] = (float)vel[2];
  P.id[p] = (uint32_t)p;
}

// ---------------------------------------------------------------- re-binning
// Counting sort of one species into the other buffer by tile, and by cell
// inside each tile, dropping the empty slots.  Each block takes kSortSlots
// consecutive slots of the (nearly binned) source:
//  1. count: the block's particles per destination tile, aggregated in an LDS
//     table, then one global atomic per (block, tile);
//  2. the tile sizes rounded up to a multiple of 4 and their exclusive scan
//     (the tile starts); each tile's cursor starts at its start; the padding
//     slots are marked empty;
//  3. scatter: per block again, one returning atomic per (block, tile)
//     reserves a contiguous run of the tile, and an LDS counting sort of the
//     block's particles by (tile, cell) places them in their runs in cell
//     order.
// A destination tile is thus a concatenation of cell-sorted runs, one per
// source block that sends particles into it (mostly one or two).  No atomic
// is taken per cell, so the cost does not grow with how far the particles
// have drifted since the last sort.
struct TileOrder {
  int ntx, nty;  // tiles along x, y
};
// key of a cell: tile index (tiles x fastest) * 64 + cell inside the tile (x fastest)
__device__ __forceinline__ int tiled_key(int i, int j, int k, TileOrder o) {
  return (((k >> 2) * o.nty + (j >> 2)) * o.ntx + (i >> 2)) * 64 + ((k & 3) * 4 + (j & 3)) * 4 +
         (i & 3);
}
__device__ __forceinline__ int sort_key(const PartF64& P, int p, TileOrder o) {
  if (!(P.z[p] >= 0.0)) return -1;
  return tiled_key((int)floor(P.x[p]), (int)floor(P.y[p]), (int)floor(P.z[p]), o);
}
__device__ __forceinline__ int sort_key(const PartF32R& P, int p, TileOrder o) {
  const int c = P.cell[p];
  if (c < 0) return -1;
  return tiled_key(cell_i(c), cell_j(c), cell_k(c), o);
}

// Runs of equal keys in neighbouring lanes (the input is nearly sorted): each
// lane learns the lane that heads its run, its rank in the run and, for the
// head, the run length, so one operation serves the whole run.
struct Run {
  int head, rank, len;
};
__device__ __forceinline__ Run lane_run(int key) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1, 64);
  const bool is_head = lane == 0 || key != prev;
  const unsigned long long heads = __ballot(is_head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  Run r;
  r.head = 63 - __clzll((long long)(heads & upto));
  r.rank = lane - r.head;
  const unsigned long long above = lane == 63 ? 0ull : (heads & ~upto);
  r.len = (above ? __ffsll((long long)above) - 1 : 64) - lane;
  return r;
}

// Each wave takes kSortRounds rounds of 64 consecutive slots (a block covers
// kSortSlots slots); every load of a thread is issued before its first atomic.
constexpr int kSortRounds = 4;
constexpr int kSortSlots = 4 * 64 * kSortRounds;
constexpr int kTable = 64;  // destination tiles per block held in LDS (open addressing)

template <int Rounds = kSortRounds>
__device__ __forceinline__ int sort_first_slot() {
  return blockIdx.x * (256 * Rounds) + (threadIdx.x >> 6) * 64 * Rounds + (threadIdx.x & 63);
}
// rounds per wave of the scatter: half for FP64 records, so that a block's
// staged records fit in LDS
template <typename PT>
constexpr int scatter_rounds() {
  return std::is_same<PT, PartF64>::value ? kSortRounds / 2 : kSortRounds;
}

// the LDS table slot of tile t, inserted if new; -1 when the table is full
__device__ __forceinline__ int table_slot(int* s_tile, int t) {
  const unsigned h = ((unsigned)t * 2654435761u) >> 26;
  for (int probe = 0; probe < kTable; ++probe) {
    const int i = (int)((h + probe) & (kTable - 1));
    const int old = atomicCAS(&s_tile[i], -1, t);
    if (old == -1 || old == t) return i;
  }
  return -1;
}

template <typename PT>
__global__ __launch_bounds__(256) void bin_count_kernel(PT P, const int* __restrict__ cnt,
                                                        int* __restrict__ tcount, TileOrder o) {
  __shared__ int s_tile[kTable], s_n[kTable];
  if (threadIdx.x < kTable) {
    s_tile[threadIdx.x] = -1;
    s_n[threadIdx.x] = 0;
  }
  __syncthreads();
  const int n = cnt[0];
  const int first = sort_first_slot();
  int key[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int p = first + 64 * r;
    key[r] = p < n ? sort_key(P, p, o) : -1;
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int t = key[r] >= 0 ? key[r] >> 6 : -1;
    const Run run = lane_run(t);
    if (t >= 0 && run.rank == 0) {
      const int sl = table_slot(s_tile, t);
      if (sl >= 0) atomicAdd(&s_n[sl], run.len);
      else atomicAdd(&tcount[t], run.len);
    }
  }
  __syncthreads();
  if (threadIdx.x < kTable && s_tile[threadIdx.x] >= 0)
    atomicAdd(&tcount[s_tile[threadIdx.x]], s_n[threadIdx.x]);
}

// one particle record in registers
struct RecF64 {
  double x, y, z, vx, vy, vz;
  uint32_t id;
};
struct RecF32R {
  int cell;
  float ox, oy, oz, vx, vy, vz;
  uint32_t id;
};
__device__ __forceinline__ void load_rec(const PartF64& a, int i, RecF64& r) {
  r.x = a.x[i];
  r.y = a.y[i];
  r.z = a.z[i];
  r.vx = a.vx[i];
  r.vy = a.vy[i];
  r.vz = a.vz[i];
  r.id = a.id[i];
}
__device__ __forceinline__ void store_rec(const PartF64& b, int j, const RecF64& r) {
  b.x[j] = r.x;
  b.y[j] = r.y;
  b.z[j] = r.z;
  b.vx[j] = r.vx;
  b.vy[j] = r.vy;
  b.vz[j] = r.vz;
  b.id[j] = r.id;
}
__device__ __forceinline__ int rec_key(const RecF64& r, TileOrder o) {
  if (!(r.z >= 0.0)) return -1;
  return tiled_key((int)floor(r.x), (int)floor(r.y), (int)floor(r.z), o);
}
__device__ __forceinline__ void load_rec(const PartF32R& a, int i, RecF32R& r) {
  r.cell = a.cell[i];
  r.ox = a.ox[i];
  r.oy = a.oy[i];
  r.oz = a.oz[i];
  r.vx = a.vx[i];
  r.vy = a.vy[i];
  r.vz = a.vz[i];
  r.id = a.id[i];
}
__device__ __forceinline__ void store_rec(const PartF32R& b, int j, const RecF32R& r) {
  b.cell[j] = r.cell;
  b.ox[j] = r.ox;
  b.oy[j] = r.oy;
  b.oz[j] = r.oz;
  b.vx[j] = r.vx;
  b.vy[j] = r.vy;
  b.vz[j] = r.vz;
  b.id[j] = r.id;
}
__device__ __forceinline__ int rec_key(const RecF32R& r, TileOrder o) {
  if (r.cell < 0) return -1;
  return tiled_key(cell_i(r.cell), cell_j(r.cell), cell_k(r.cell), o);
}
template <typename PT>
struct RecOf;
template <>
struct RecOf<PartF64> {
  using type = RecF64;
};
template <>
struct RecOf<PartF32R> {
  using type = RecF32R;
};

// LDS staging of a block's records (one array per field, so neighbouring
// lanes touch neighbouring words) and their destinations
template <typename Rec, int N>
struct SortStage;
template <int N>
struct SortStage<RecF32R, N> {
  int cell[N];
  float ox[N], oy[N], oz[N], vx[N], vy[N], vz[N];
  uint32_t id[N];
  int dest[N];
  __device__ void put(int u, const RecF32R& r) {
    cell[u] = r.cell;
    ox[u] = r.ox;
    oy[u] = r.oy;
    oz[u] = r.oz;
    vx[u] = r.vx;
    vy[u] = r.vy;
    vz[u] = r.vz;
    id[u] = r.id;
  }
  __device__ RecF32R get(int u) const {
    return RecF32R{cell[u], ox[u], oy[u], oz[u], vx[u], vy[u], vz[u], id[u]};
  }
};
template <int N>
struct SortStage<RecF64, N> {
  double x[N], y[N], z[N], vx[N], vy[N], vz[N];
  uint32_t id[N];
  int dest[N];
  __device__ void put(int u, const RecF64& r) {
    x[u] = r.x;
    y[u] = r.y;
    z[u] = r.z;
    vx[u] = r.vx;
    vy[u] = r.vy;
    vz[u] = r.vz;
    id[u] = r.id;
  }
  __device__ RecF64 get(int u) const {
    return RecF64{x[u], y[u], z[u], vx[u], vy[u], vz[u], id[u]};
  }
};

template <typename PT>
__global__ __launch_bounds__(256) void bin_scatter_kernel(PT src, PT dst, const int* __restrict__ cnt,
                                                          int* __restrict__ cursor, TileOrder o) {
  using Rec = typename RecOf<PT>::type;
  constexpr int kBins = kTable * 64;         // (table slot, cell in tile)
  constexpr int kPerThread = kBins / 256;    // bins scanned per thread
  __shared__ int s_tile[kTable], s_base[kTable];
  __shared__ int s_bin[kBins];
  __shared__ int s_wsum[4];
  for (int i = threadIdx.x; i < kBins; i += 256) s_bin[i] = 0;
  if (threadIdx.x < kTable) s_tile[threadIdx.x] = -1;
  const int n = cnt[0];
  constexpr int R = scatter_rounds<PT>();
  const int first = sort_first_slot<R>();
  Rec rec[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = first + 64 * r;
    if (p < n) load_rec(src, p, rec[r]);
  }
  __syncthreads();
  int key[R], slot[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    key[r] = first + 64 * r < n ? rec_key(rec[r], o) : -1;
    const int t = key[r] >= 0 ? key[r] >> 6 : -1;
    const Run run = lane_run(t);
    int sl = -1;
    if (t >= 0 && run.rank == 0) sl = table_slot(s_tile, t);
    sl = __shfl(sl, run.head, 64);
    slot[r] = t >= 0 ? sl : -1;
    // one LDS atomic per run of equal bins (the input is nearly sorted)
    const int bk = slot[r] >= 0 ? slot[r] * 64 + (key[r] & 63) : -1;
    const Run brun = lane_run(bk);
    if (bk >= 0 && brun.rank == 0) atomicAdd(&s_bin[bk], brun.len);
  }
  __syncthreads();
  // exclusive scan of the bins in (slot, cell) order: block-local positions
  int local[kPerThread], sum = 0;
#pragma unroll
  for (int b = 0; b < kPerThread; ++b) {
    local[b] = s_bin[kPerThread * threadIdx.x + b];
    sum += local[b];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(incl, off, 64);
    if (lane >= off) incl += u;
  }
  if (lane == 63) s_wsum[w] = incl;
  __syncthreads();
  int run = incl - sum, total = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k < w) run += s_wsum[k];
    total += s_wsum[k];
  }
#pragma unroll
  for (int b = 0; b < kPerThread; ++b) {
    s_bin[kPerThread * threadIdx.x + b] = run;
    run += local[b];
  }
  __syncthreads();
  // one reservation per (block, tile): the run of the tile this block fills
  if (threadIdx.x < kTable && s_tile[threadIdx.x] >= 0) {
    const int g0 = s_bin[64 * threadIdx.x];
    const int g1 = threadIdx.x + 1 < kTable ? s_bin[64 * (threadIdx.x + 1)] : total;
    s_base[threadIdx.x] = atomicAdd(&cursor[s_tile[threadIdx.x]], g1 - g0) - g0;
  }
  __syncthreads();
  // the records are staged in LDS at their block-local places and then
  // written out in destination order (whole lines)
  __shared__ SortStage<Rec, 256 * R> s_stage;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    // places in the bin: one LDS atomic per run, lanes of a run in lane order
    const int bk = slot[r] >= 0 ? slot[r] * 64 + (key[r] & 63) : -1;
    const Run brun = lane_run(bk);
    int d0 = 0;
    if (bk >= 0 && brun.rank == 0) d0 = atomicAdd(&s_bin[bk], brun.len);
    d0 = __shfl(d0, brun.head, 64);
    if (key[r] < 0) continue;
    if (slot[r] >= 0) {
      const int u = d0 + brun.rank;
      s_stage.put(u, rec[r]);
      s_stage.dest[u] = s_base[slot[r]] + u;
    } else {
      store_rec(dst, atomicAdd(&cursor[key[r] >> 6], 1), rec[r]);  // the table was full
    }
  }
  __syncthreads();
  for (int u = threadIdx.x; u < total; u += 256) store_rec(dst, s_stage.dest[u], s_stage.get(u));
}

// t <= ngrid: the tile's size rounded up to a multiple of 4 (0 for the grid's
// padding tiles and the end entry), scanned afterwards into the tile starts
__global__ void tile_size_kernel(const int* __restrict__ tcount, int* __restrict__ tsize,
                                 int ngrid) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > ngrid) return;
  tsize[t] = t < ngrid ? (tcount[t] + 3) & ~3 : 0;
}

// every tile's cursor at its start; its padding slots marked empty
template <typename PT>
__global__ void tile_pad_kernel(const int* __restrict__ tcount, const int* __restrict__ tstart,
                                int* __restrict__ cursor, PT dst, int ngrid) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ngrid) return;
  const int s = tstart[t];
  cursor[t] = s;
  for (int p = s + tcount[t]; p < tstart[t + 1]; ++p) kill(dst, p);
}

// after the scatter the tiles fill [0, tstart[ngrid]) of the other buffer
__global__ void sort_finish_kernel(int* cnt, const int* tstart, int ngrid) {
  if (threadIdx.x == 0 && blockIdx.x == 0) cnt[0] = tstart[ngrid];
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

__global__ void scan_sums_serial(int* __restrict__ sums, int nb, int* __restrict__ total) {
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
  if (threadIdx.x == 0 && total) *total = carry;
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

// k -> k + 1 at the end of a step
// the end of a step: the step counter advances and the dense MD lists start
// empty for the next step
__global__ void advance_step_kernel(uint32_t* step, int32_t* cnt0, int32_t* cnt1) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *step += 1u;
    cnt0[2] = 0;
    cnt1[2] = 0;
  }
}

// ---------------------------------------------------------------- ionisation
// The ionisations of the step, after every particle has moved and collided
// and before any re-binning: in the order of the parent electrons' ids (an
// event's rank is the number of events with a smaller id), each makes an
// electron and an ion at the parent's new position, in the slots after the
// last tile's -- the range of the grid's last padding tile, whose push block
// takes them through the global-memory paths until the next re-binning puts
// them in their tiles -- with ids next_id[s] + rank.  The ejected electron
// takes the fraction s (Philox(id, k, IONIZE, 0) word 0) of the shared
// centre-of-mass energy, an isotropic direction (words 1 and 2), the neutral
// at rest; the ion a Maxwellian velocity of the gas temperature
// (Philox(id, k, IONIZE, 1), Box-Muller, cosine branch first).  Their charges
// cancel on the mesh (same position), so rho_{k+1} is left as it is.  If the
// new particles do not fit (room_* slots in use at most, so that the next
// re-binning fits too) or events exceeded the list, they are counted in
// *dropped.  One block.
constexpr int kIzThreads = 1024;
constexpr int kIzChunk = 4096;
__device__ __forceinline__ void copy_pos(const PartF64& s, long p, const PartF64& d, long q) {
  d.x[q] = s.x[p];
  d.y[q] = s.y[p];
  d.z[q] = s.z[p];
}
__device__ __forceinline__ void copy_pos(const PartF32R& s, long p, const PartF32R& d, long q) {
  d.cell[q] = s.cell[p];
  d.ox[q] = s.ox[p];
  d.oy[q] = s.oy[p];
  d.oz[q] = s.oz[p];
}

template <typename PT>
__global__ __launch_bounds__(kIzThreads) void ionize_kernel(PT Pe, PT Pi, WorkLists Le,
                                                            WorkLists Li, SpeciesStep Se,
                                                            uint32_t* __restrict__ next_id,
                                                            long room_e, long room_i,
                                                            unsigned long long* dropped) {
  using V = typename VelOf<PT>::type;
  __shared__ uint32_t s_id[kIzChunk];
  const int total = *Se.iz_cnt;
  const int n = min(total, Se.iz_cap);
  const int ng = Le.ngrid;
  const long be = Le.tstart[ng], bi = Li.tstart[ng];
  // the tail stays a multiple of 4 slots long (a push thread streams four
  // slots at once): the slots after the new particles up to that are emptied
  const int n4 = (n + 3) & ~3;
  const bool fit = be + n4 <= room_e && bi + n4 <= room_i;
  const uint32_t k = *Se.step;
  for (int j0 = 0; fit && j0 < n; j0 += kIzThreads) {
    const int q = j0 + (int)threadIdx.x;
    const bool mine = q < n;
    const uint32_t myid = mine ? Se.iz_ev[q].id : 0u;
    int rank = 0;
    for (int c0 = 0; c0 < n; c0 += kIzChunk) {
      __syncthreads();
      for (int t = threadIdx.x; t < kIzChunk && c0 + t < n; t += kIzThreads) s_id[t] = Se.iz_ev[c0 + t].id;
      __syncthreads();
      const int m = min(kIzChunk, n - c0);
      if (mine)
        for (int t = 0; t < m; ++t) rank += s_id[t] < myid;
    }
    if (!mine) continue;
    const IzEvent ev = Se.iz_ev[q];
    const uint4 w0 = philox4x32_10(ev.id, k, kIonize, 0u, Se.key0, Se.key1);
    const uint4 w1 = philox4x32_10(ev.id, k, kIonize, 1u, Se.key0, Se.key1);
    const double ge = sqrt(u01_open(w0.x) * ev.gsq);
    const double cost = 1.0 - 2.0 * u01_open(w0.y);
    const double sint = sqrt(fmax(0.0, 1.0 - cost * cost));
    double sp, cp;
    sincos(2.0 * kPi * u01_open(w0.z), &sp, &cp);
    const double nh[3] = {sint * cp, sint * sp, cost};
    const long pe = be + rank, pi = bi + rank;
    copy_pos(Pe, ev.slot, Pe, pe);
    copy_pos(Pe, ev.slot, Pi, pi);
    Pe.vx[pe] = (V)(Se.mass_ratio_e * ev.v[0] + Se.mass_ratio_n * ge * nh[0]);
    Pe.vy[pe] = (V)(Se.mass_ratio_e * ev.v[1] + Se.mass_ratio_n * ge * nh[1]);
    Pe.vz[pe] = (V)(Se.mass_ratio_e * ev.v[2] + Se.mass_ratio_n * ge * nh[2]);
    double n0, n1, n2, n3;
    normal_pair(w1.x, w1.y, n0, n1);
    normal_pair(w1.z, w1.w, n2, n3);
    Pi.vx[pi] = (V)(Se.vth_gas * n0);
    Pi.vy[pi] = (V)(Se.vth_gas * n1);
    Pi.vz[pi] = (V)(Se.vth_gas * n2);
    Pe.id[pe] = next_id[0] + (uint32_t)rank;
    Pi.id[pi] = next_id[1] + (uint32_t)rank;
  }
  if (fit && (int)threadIdx.x < n4 - n) {
    kill(Pe, be + n + threadIdx.x);
    kill(Pi, bi + n + threadIdx.x);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (fit && n > 0) {
    Le.tstart[ng] = (int32_t)(be + n4);
    Li.tstart[ng] = (int32_t)(bi + n4);
    Le.cnt[0] = (int32_t)(be + n4);
    Li.cnt[0] = (int32_t)(bi + n4);
    next_id[0] += (uint32_t)n;
    next_id[1] += (uint32_t)n;
    Le.tally[TL_BORN] += (unsigned long long)n;
    Li.tally[TL_BORN] += (unsigned long long)n;
  }
  const int lost = fit ? total - n : total;
  if (lost > 0) *dropped += (unsigned long long)lost;
  *Se.iz_cnt = 0;
}

// ---------------------------------------------------------------- energy
// FP64 energy diagnostic.  Per block: the sum of |v|^2 over the live slots it
// strides (kinetic), or of |E|^2 times the node's share of a cell volume (half
// on the two electrode planes) over the nodes it strides (field); block b
// writes out[b].  A fixed grid and order make the sums repeatable.
constexpr int kEnergyBlocks = 1024;
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double s_w[kBlock / 64];
  v = wave_sum_t<double>(v);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) t += s_w[w];
  return t;
}

template <typename PT>
__global__ __launch_bounds__(kBlock) void kinetic_kernel(PT P, const int32_t* __restrict__ cnt,
                                                         double* __restrict__ out) {
  const long slots = cnt[0];
  double s = 0.0;
  for (long p = (long)blockIdx.x * kBlock + threadIdx.x; p < slots; p += (long)gridDim.x * kBlock) {
    if (!slot_alive(P, p)) continue;
    const double vx = P.vx[p], vy = P.vy[p], vz = P.vz[p];
    s += vx * vx + vy * vy + vz * vz;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

template <typename ET>
__global__ __launch_bounds__(kBlock) void field_energy_kernel(const ET* __restrict__ E, long nxy,
                                                              int nz, double* __restrict__ out) {
  const long nn = nxy * (nz + 1);
  double s = 0.0;
  for (long n = (long)blockIdx.x * kBlock + threadIdx.x; n < nn; n += (long)gridDim.x * kBlock) {
    double ex, ey, ez;
    load_node(E, n, ex, ey, ez);
    const long k = n / nxy;
    s += (k == 0 || k == nz ? 0.5 : 1.0) * (ex * ex + ey * ey + ez * ez);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// ---------------------------------------------------------------- launchers
static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

int tile_grid(int nx, int ny, int nz, int extra) {
  return (((nx + 3) / 4) * ((ny + 3) / 4) * ((nz + 3) / 4) + extra + 15) / 16 * 16;
}


void launch_advance_step(uint32_t* step, int32_t* cnt0, int32_t* cnt1, hipStream_t st) {
  hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, st, step, cnt0, cnt1);
}

void launch_push_f64(const PartF64& P, const double* E, double* rho, const MdTables& md,
                     const SpeciesStep& S, const WorkLists& L, hipStream_t st) {
  if (L.ngrid <= 0) return;
  hipLaunchKernelGGL(push_f64_kernel<true>, dim3(L.ngrid), dim3(kBlock), 0, st, P,
                     (const double2*)E, rho, md, S, L, push_chunk(L, 1));
}

void launch_push_f32r(const PartF32R& P, const float* E, long long* rho, const MdTables& md,
                      const SpeciesStep& S, const WorkLists& L, hipStream_t st) {
  if (L.ngrid <= 0) return;
  const int span = push_span(L);
  hipLaunchKernelGGL(push_f32r_kernel<true>, dim3(L.ngrid / span), dim3(kBlock), 0, st, P,
                     (const float4*)E, rho, md, S, L, span, push_chunk(L, span));
}

void launch_push_batch_f32r(const PushDescF32* descs, const int32_t* start, int ndesc, int grid,
                            int* queue, hipStream_t st) {
  if (ndesc <= 0 || grid <= 0) return;
  launch_zero_i32(queue, 8, st);
  hipLaunchKernelGGL(push_batch_f32r_kernel, dim3(grid), dim3(kBlock), 0, st, descs, start, ndesc,
                     queue);
}

constexpr int kMdBlocks = kMdTallyRows;

void launch_field_out(const double* psi, double* phi, void* E, int e_f64,
                      unsigned long long* zero_next, const MdTables& md, int nx, int ny, int nz,
                      double dx, RfDrive rf, hipStream_t st) {
  const long nn = (long)nx * ny * (nz + 1);
  const int nbe = nblk(nn, 256);
  const int nbm = md.n_grains > 0 ? nblk(8L * md.bsx * md.bsy * md.bsz, 256) : 0;
  const double* src = psi ? psi : phi;
  if (e_f64) {
    if (psi)
      hipLaunchKernelGGL((field_out_kernel<double2, true>), dim3(nbe + nbm), dim3(256), 0, st, src,
                         phi, (double2*)E, zero_next, md, nx, ny, nz, dx, rf, nbm);
    else
      hipLaunchKernelGGL((field_out_kernel<double2, false>), dim3(nbe + nbm), dim3(256), 0, st,
                         src, phi, (double2*)E, zero_next, md, nx, ny, nz, dx, rf, nbm);
  } else {
    if (psi)
      hipLaunchKernelGGL((field_out_kernel<float4, true>), dim3(nbe + nbm), dim3(256), 0, st, src,
                         phi, (float4*)E, zero_next, md, nx, ny, nz, dx, rf, nbm);
    else
      hipLaunchKernelGGL((field_out_kernel<float4, false>), dim3(nbe + nbm), dim3(256), 0, st, src,
                         phi, (float4*)E, zero_next, md, nx, ny, nz, dx, rf, nbm);
  }
}

void launch_collide_f64(const PartF64& P, const SpeciesStep& S, const WorkLists& L,
                        hipStream_t st) {
  if (L.ngrid > 0)
    hipLaunchKernelGGL(collide_kernel<PartF64>, dim3(L.ngrid), dim3(64), 0, st, P, S, L, 1);
}

void launch_collide_f32r(const PartF32R& P, const SpeciesStep& S, const WorkLists& L,
                         hipStream_t st) {
  if (L.ngrid > 0)
    hipLaunchKernelGGL(collide_kernel<PartF32R>, dim3(L.ngrid / push_span(L)), dim3(64), 0, st, P,
                       S, L, push_span(L));
}

void launch_lists_f64(const PartF64 P[2], const double* E, double* rho, const MdTables& md,
                      const SpeciesStep S[2], unsigned long long* gc, const WorkLists L[2],
                      int do_mcc, hipStream_t st) {
  if (L[0].ngrid <= 0) return;
  SpeciesPair<PartF64> pr{{P[0], P[1]}, {S[0], S[1]}, {L[0], L[1]}, L[0].ngrid, 1};
  hipLaunchKernelGGL(outlier_f64_kernel, dim3(2 * pr.nb), dim3(64), 0, st, pr, (const double2*)E,
                     rho, do_mcc);
  if (md.n_grains > 0) {
    pr.nb = kMdBlocks;
    hipLaunchKernelGGL((md_kernel<PartF64, double2, double>), dim3(2 * kMdBlocks), dim3(kMdThreads),
                       0, st, pr, P[0], P[1], (const double2*)E, rho, md, gc);
    if (do_mcc)
      hipLaunchKernelGGL(md_collide_kernel<PartF64>, dim3(2 * kMdBlocks), dim3(kMdThreads), 0, st,
                         pr, P[0], P[1], 0, 1, -1);
  }
}

void launch_md_scan_f32r(const PartF32R P[2], const WorkLists L[2], const MdTables& md,
                         const SpeciesStep S[2], int nx, int ny, int nz, hipStream_t st) {
  if (md.n_grains == 0 || L[0].ngrid <= 0) return;
  const int span = push_span(L[0]), npb = L[0].ngrid / span;
  hipLaunchKernelGGL(md_scan_kernel, dim3(2 * npb), dim3(256), 0, st, P[0], P[1], L[0], L[1], md,
                     nx, ny, nz, S[0].margin, S[1].margin, span, npb);
}

void launch_md_move_f32r(const PartF32R P[2], const PartF32R D[2], const float* E,
                         long long* rho, const MdTables& md, const SpeciesStep S[2],
                         unsigned long long* gc, const WorkLists L[2], hipStream_t st) {
  if (md.n_grains == 0 || L[0].ngrid <= 0) return;
  SpeciesPair<PartF32R> pr{{P[0], P[1]}, {S[0], S[1]}, {L[0], L[1]}, kMdBlocks, push_span(L[0])};
  hipLaunchKernelGGL((md_kernel<PartF32R, float4, long long>), dim3(2 * kMdBlocks),
                     dim3(kMdThreads), 0, st, pr, D[0], D[1], (const float4*)E, rho, md, gc);
}

void launch_species_lists_f32r(const PartF32R P[2], const PartF32R D[2], const float* E,
                               long long* rho, const MdTables& md, const SpeciesStep S[2],
                               const WorkLists L[2], int do_mcc, int sp, hipStream_t st) {
  if (L[0].ngrid <= 0) return;
  const int span = push_span(L[0]), npb = L[0].ngrid / span;
  SpeciesPair<PartF32R> pr{{P[0], P[1]}, {S[0], S[1]}, {L[0], L[1]}, npb, span};
  const int md_on = md.n_grains > 0 ? 1 : 0;
  hipLaunchKernelGGL(species_lists_f32r_kernel, dim3(npb + md_on * kMdListBlocks), dim3(64), 0,
                     st, pr, D[sp], (const float4*)E, rho, do_mcc, sp, npb, md_on);
}

void launch_lists_f32r(const PartF32R P[2], const PartF32R D[2], const float* E, long long* rho,
                       const MdTables& md, const SpeciesStep S[2], const WorkLists L[2],
                       int do_mcc, int sp_only, hipStream_t st) {
  if (L[0].ngrid <= 0) return;
  const int span = push_span(L[0]);
  const int ns = sp_only >= 0 ? 1 : 2;
  SpeciesPair<PartF32R> pr{{P[0], P[1]}, {S[0], S[1]}, {L[0], L[1]}, L[0].ngrid / span, span};
  hipLaunchKernelGGL(outlier_f32r_kernel, dim3(ns * pr.nb), dim3(64), 0, st, pr, (const float4*)E,
                     rho, do_mcc, sp_only);
  if (md.n_grains > 0) {
    pr.nb = kMdBlocks;
    hipLaunchKernelGGL(md_collide_kernel<PartF32R>, dim3(ns * kMdBlocks), dim3(kMdThreads), 0, st,
                       pr, D[0], D[1], 1, do_mcc, sp_only);
  }
}

void launch_init_f64(const PartF64& P, int n, int ppc, int nx, int ny, int sp, uint32_t k0,
                     uint32_t k1, double vth, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(init_f64_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, P, n, ppc, nx, ny, sp,
                     k0, k1, vth);
}

void launch_init_f32r(const PartF32R& P, int n, int ppc, int nx, int ny, int sp, uint32_t k0,
                      uint32_t k1, double vth, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(init_f32r_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, P, n, ppc, nx, ny, sp,
                     k0, k1, vth);
}

void launch_deposit_f64(const PartF64& P, double* rho, const MdTables& md, const SpeciesStep& S,
                        const WorkLists& L, hipStream_t st) {
  if (L.ngrid <= 0) return;
  hipLaunchKernelGGL(push_f64_kernel<false>, dim3(L.ngrid), dim3(kBlock), 0, st, P, nullptr, rho,
                     md, S, L, push_chunk(L, 1));
}

void launch_deposit_f32r(const PartF32R& P, long long* rho, const MdTables& md,
                         const SpeciesStep& S, const WorkLists& L, hipStream_t st) {
  if (L.ngrid <= 0) return;
  const int span = push_span(L);
  hipLaunchKernelGGL(push_f32r_kernel<false>, dim3(L.ngrid / span), dim3(kBlock), 0, st, P,
                     nullptr, rho, md, S, L, span, push_chunk(L, span));
}

void launch_moments(const PartF64* P64, const PartF32R* P32, const SpeciesStep& S,
                    const WorkLists& L, double* mom, long nn, const AvgBins& avg,
                    hipStream_t st) {
  if (L.ngrid <= 0) return;
  if (P64)
    hipLaunchKernelGGL(moments_kernel<PartF64>, dim3(L.ngrid), dim3(256), 0, st, *P64, S, L, mom,
                       nn, avg);
  else
    hipLaunchKernelGGL(moments_kernel<PartF32R>, dim3(L.ngrid), dim3(256), 0, st, *P32, S, L, mom,
                       nn, avg);
}

void launch_fine_moments(const PartF64* P64, const PartF32R* P32, const WorkLists& L,
                         const FineBox& fb, double* mom, const AvgBins& avg, long capacity,
                         hipStream_t st) {
  const int blocks = (int)std::min<long>(nblk(capacity, 256), 4096);
  if (blocks <= 0) return;
  if (P64)
    hipLaunchKernelGGL(fine_moments_kernel<PartF64>, dim3(blocks), dim3(256), 0, st, *P64, L, fb,
                       mom, avg);
  else
    hipLaunchKernelGGL(fine_moments_kernel<PartF32R>, dim3(blocks), dim3(256), 0, st, *P32, L, fb,
                       mom, avg);
}

void launch_ionize(const PartF64* Pe64, const PartF64* Pi64, const PartF32R* Pe32,
                   const PartF32R* Pi32, const WorkLists& Le, const WorkLists& Li,
                   const SpeciesStep& Se, uint32_t* next_id, long room_e, long room_i,
                   unsigned long long* dropped, hipStream_t st) {
  if (Pe64)
    hipLaunchKernelGGL(ionize_kernel<PartF64>, dim3(1), dim3(kIzThreads), 0, st, *Pe64, *Pi64, Le,
                       Li, Se, next_id, room_e, room_i, dropped);
  else
    hipLaunchKernelGGL(ionize_kernel<PartF32R>, dim3(1), dim3(kIzThreads), 0, st, *Pe32, *Pi32, Le,
                       Li, Se, next_id, room_e, room_i, dropped);
}

int energy_blocks() { return kEnergyBlocks; }

void launch_energy(const PartF64* P64, const PartF32R* P32, const WorkLists& L, double* out,
                   hipStream_t st) {
  if (P64)
    hipLaunchKernelGGL(kinetic_kernel<PartF64>, dim3(kEnergyBlocks), dim3(kBlock), 0, st, *P64,
                       L.cnt, out);
  else
    hipLaunchKernelGGL(kinetic_kernel<PartF32R>, dim3(kEnergyBlocks), dim3(kBlock), 0, st, *P32,
                       L.cnt, out);
}

void launch_field_energy(const void* E, int e_f64, long nxy, int nz, double* out, hipStream_t st) {
  if (e_f64)
    hipLaunchKernelGGL(field_energy_kernel<double2>, dim3(kEnergyBlocks), dim3(kBlock), 0, st,
                       (const double2*)E, nxy, nz, out);
  else
    hipLaunchKernelGGL(field_energy_kernel<float4>, dim3(kEnergyBlocks), dim3(kBlock), 0, st,
                       (const float4*)E, nxy, nz, out);
}

void launch_fill_int(int* a, long n, int v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_int_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, a, n, v);
}

long sort_keys(int ngrid) { return 2L * ngrid + 1; }

template <typename PT>
static void sort_impl(const PT& src, const PT& dst, const WorkLists& L, int* hist, int* sums,
                      long capacity, hipStream_t st) {
  const TileOrder o{L.ntx, L.nty};
  const int ng = L.ngrid;
  int* tcount = hist;            // [ngrid + 1]
  int* cursor = hist + ng + 1;   // [ngrid]
  launch_fill_int(hist, 2L * ng + 1, 0, st);
  hipLaunchKernelGGL(bin_count_kernel<PT>, dim3(nblk(capacity, kSortSlots)), dim3(256), 0, st, src,
                     L.cnt, tcount, o);
  const int n = ng + 1;
  hipLaunchKernelGGL(tile_size_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, tcount, L.tstart, ng);
  const int nb = nblk(n, kScanBlock);
  hipLaunchKernelGGL(scan_block_sums, dim3(nb), dim3(kScanBlock), 0, st, L.tstart, n, sums);
  hipLaunchKernelGGL(scan_sums_serial, dim3(1), dim3(kScanBlock), 0, st, sums, nb, L.cnt + 4);
  hipLaunchKernelGGL(scan_apply, dim3(nb), dim3(kScanBlock), 0, st, L.tstart, n, sums, L.tstart);
  hipLaunchKernelGGL(tile_pad_kernel<PT>, dim3(nblk(ng, 256)), dim3(256), 0, st, tcount, L.tstart,
                     cursor, dst, ng);
  hipLaunchKernelGGL(bin_scatter_kernel<PT>, dim3(nblk(capacity, 256 * scatter_rounds<PT>())),
                     dim3(256), 0, st,
                     src, dst, L.cnt, cursor, o);
  hipLaunchKernelGGL(sort_finish_kernel, dim3(1), dim3(64), 0, st, L.cnt, L.tstart, ng);
}

void launch_sort_f64(const PartF64& src, const PartF64& dst, const WorkLists& L, int* hist,
                     int* sums, long capacity, hipStream_t st) {
  if (capacity <= 0) return;
  sort_impl(src, dst, L, hist, sums, capacity, st);
}

void launch_sort_f32r(const PartF32R& src, const PartF32R& dst, const WorkLists& L, int* hist,
                      int* sums, long capacity, hipStream_t st) {
  if (capacity <= 0) return;
  sort_impl(src, dst, L, hist, sums, capacity, st);
  launch_zero_i32(L.stray, L.ngrid, st);  // every particle is in its own tile again
}

}  // namespace pic
