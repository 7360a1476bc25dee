/*
 * pic_oracle.c -- plain FP64 CPU oracle of the PIC-MCC/PPPM step.
 *
 * TEST INFRASTRUCTURE ONLY (see pic_oracle.h).  Written for a reader who
 * checks it against the paper by eye: no blocking, no fusion, no reordering
 * beyond what the method states.  Loops over particles use OpenMP only where
 * the particles are independent of each other; every reduction is serial or
 * integer, so results do not depend on the thread count.
 */
#include "pic_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018 values */
#define O_ECHARGE 1.602176634e-19
#define O_EPS0    8.8541878128e-12
#define O_KB      1.380649e-23
#define O_ME      9.1093837015e-31
#define O_AMU     1.66053906660e-27
#define O_MAR     (39.948 * O_AMU)
#define O_PI      3.14159265358979323846

/* Philox counter word 2: what a draw is for */
enum { PUR_INIT_POS = 1, PUR_INIT_VEL = 2, PUR_COLL = 3, PUR_NEUTRAL = 4, PUR_CORDER = 5,
       PUR_CPAIR = 6, PUR_GRAIN = 7, PUR_IONIZE = 8 };

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32  */
/* multiplies with the published multipliers; the key is bumped by the Weyl   */
/* constants between rounds.                                                  */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)prod1;
    uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)prod0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(const orc_config* c, uint32_t id, uint32_t step, uint32_t purpose,
                 uint32_t species, uint32_t out[4])
{
  uint32_t ctr[4] = {id, step, purpose, species};
  uint32_t key[2] = {(uint32_t)(c->seed & 0xffffffffu), (uint32_t)(c->seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* uniform on (0,1): (word + 1/2) 2^-32 */
static double unif_open(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* two standard normals by Box-Muller from two words (cosine branch first) */
static void box_muller(uint32_t wa, uint32_t wb, double* n0, double* n1)
{
  double ua = unif_open(wa), ub = unif_open(wb);
  double r = sqrt(-2.0 * log(ua));
  double th = 2.0 * O_PI * ub;
  *n0 = r * cos(th);
  *n1 = r * sin(th);
}

/* ------------------------------------------------------------------------ */
/* seeded grain placement (the paper's cluster of Sec. II is known only from  */
/* a figure): uniform in a sphere by rejection, with a minimum separation     */
/* from the grains placed before; candidate t of grain g proposes             */
/* x_a = c_a + R (2 u_a - 1) from words 0..2 of Philox(g, t, GRAIN, 0).        */
/* ------------------------------------------------------------------------ */
int orc_place_grains(uint64_t seed, int n, const double center[3], double radius, double min_sep,
                     double* out)
{
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  for (int g = 0; g < n; ++g) {
    int placed = 0;
    for (uint32_t t = 0; t < (1u << 20) && !placed; ++t) {
      uint32_t ctr[4] = {(uint32_t)g, t, PUR_GRAIN, 0u}, w[4];
      orc_philox4x32_10(ctr, key, w);
      double p[3];
      for (int a = 0; a < 3; ++a) p[a] = center[a] + radius * (2.0 * unif_open(w[a]) - 1.0);
      double r2 = 0.0;
      for (int a = 0; a < 3; ++a) r2 += (p[a] - center[a]) * (p[a] - center[a]);
      if (r2 > radius * radius) continue;
      int far = 1;
      for (int h = 0; h < g && far; ++h) {
        double q2 = 0.0;
        for (int a = 0; a < 3; ++a) q2 += (p[a] - out[3 * h + a]) * (p[a] - out[3 * h + a]);
        far = q2 >= min_sep * min_sep;
      }
      if (!far) continue;
      for (int a = 0; a < 3; ++a) out[3 * g + a] = p[a];
      placed = 1;
    }
    if (!placed) return -1;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* derived constants                                                          */
/* ------------------------------------------------------------------------ */
int orc_derive(const orc_config* c, orc_derived* d)
{
  if (c->ppc_e <= 0 || c->ppc_e != c->ppc_i) return -1;
  /* one super-particle weight for both species (Sec. III: super-particles) */
  d->w = c->n0 * c->dx * c->dx * c->dx / (double)c->ppc_e;
  /* the fixed-point deposit multiplies Qp by a 24-bit offset fraction in
     int64, so Qp must stay below 2^39 (w below 128) */
  if (!(d->w * 4294967296.0 < 549755813888.0)) return -2;
  d->Qp = llround(d->w * 4294967296.0);
  /* neutral reservoir density from the gas pressure (ideal gas) */
  d->n_gas = c->p_gas / (O_KB * c->T_gas);
  d->q[0] = -O_ECHARGE;
  d->q[1] = +O_ECHARGE;
  d->m[0] = O_ME;
  d->m[1] = O_MAR;
  d->vth[0] = sqrt(c->Te_eV * O_ECHARGE / O_ME);
  d->vth[1] = sqrt(c->Ti_eV * O_ECHARGE / O_MAR);
  double sigma[2] = {c->sigma_e, c->sigma_i};
  for (int s = 0; s < 2; ++s) {
    d->g_cap[s] = sqrt(2.0 * c->E_cap_eV * O_ECHARGE / d->m[s]);
    d->sg_max[s] = c->xs_n > 0 ? orc_xs_sgmax(c, s) : sigma[s] * d->g_cap[s];
    double nu_max = d->n_gas * d->sg_max[s];
    d->P_null[s] = -expm1(-nu_max * c->dt);
    d->T_null[s] = (uint64_t)floor(d->P_null[s] * 4294967296.0);
  }
  d->vth_gas = sqrt(O_KB * c->T_gas / O_MAR);
  return 0;
}

/* sigma(E) of a table: linear between the grid points, the end values past them */
double orc_xs_at(const orc_config* c, const double* table, double E)
{
  if (!table) return 0.0;
  const double* x = c->xs_E;
  int n = c->xs_n;
  if (E <= x[0]) return table[0];
  if (E >= x[n - 1]) return table[n - 1];
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (x[mid] <= E) lo = mid;
    else hi = mid;
  }
  double t = (E - x[lo]) / (x[hi] - x[lo]);
  return table[lo] + t * (table[hi] - table[lo]);
}

/* total cross section of a species at E */
static double xs_total(const orc_config* c, int sp, double E)
{
  if (sp == 0)
    return orc_xs_at(c, c->xs_e_el, E) + orc_xs_at(c, c->xs_e_ex, E) + orc_xs_at(c, c->xs_e_iz, E);
  return orc_xs_at(c, c->xs_i_cx, E) + orc_xs_at(c, c->xs_i_el, E);
}

/* max over 0 <= E <= E_cap of g(E) sigma_total(E), g = sqrt(2 E e / m):    */
/* on a piece where sigma = a + b E the function a sqrt(E) + b E^(3/2) has    */
/* its only stationary point at E = -a / (3 b); the maximum is there or at   */
/* a piece's end (past the grid sigma is constant and sqrt(E) increases).   */
double orc_xs_sgmax(const orc_config* c, int sp)
{
  double m = sp == 0 ? O_ME : O_MAR;
  double Ecap = c->E_cap_eV;
  double best = 0.0;
  double cand[3];
  for (int i = -1; i < c->xs_n; ++i) {
    double lo = i < 0 ? 0.0 : c->xs_E[i];
    double hi = i + 1 < c->xs_n ? c->xs_E[i + 1] : Ecap;
    if (lo > Ecap) break;
    if (hi > Ecap) hi = Ecap;
    if (hi < lo) continue;
    int nc = 0;
    cand[nc++] = lo;
    cand[nc++] = hi;
    if (i >= 0 && i + 1 < c->xs_n) {
      double s0 = xs_total(c, sp, lo), s1 = xs_total(c, sp, c->xs_E[i + 1]);
      double b = (s1 - s0) / (c->xs_E[i + 1] - lo);
      double a = s0 - b * lo;
      if (b < 0.0) {
        double Es = -a / (3.0 * b);
        if (Es > lo && Es < hi) cand[nc++] = Es;
      }
    }
    for (int q = 0; q < nc; ++q) {
      double f = xs_total(c, sp, cand[q]) * sqrt(2.0 * cand[q] * O_ECHARGE / m);
      if (f > best) best = f;
    }
  }
  return best;
}

double orc_rf_voltage(const orc_config* c, uint32_t k)
{
  double t = (double)k * c->dt;
  return c->V_dc + c->V_rf * sin(2.0 * O_PI * c->f_rf * t);
}

int64_t orc_n_nodes(const orc_config* c)
{
  return (int64_t)c->nx * c->ny * (c->nz + 1);
}

static int64_t node_index(const orc_config* c, int i, int j, int k)
{
  return (int64_t)i + (int64_t)c->nx * ((int64_t)j + (int64_t)c->ny * k);
}

static int wrap_index(int i, int n) { return ((i % n) + n) % n; }

/* ------------------------------------------------------------------------ */
/* loading: exactly ppc particles per cell, uniform offsets, Maxwellian v     */
/* taken as v_{-1/2}                                                          */
/* ------------------------------------------------------------------------ */
int orc_init_particles(const orc_config* c, orc_state* s)
{
  orc_derived d;
  if (orc_derive(c, &d)) return -1;
  int64_t ncell = (int64_t)c->nx * c->ny * c->nz;
  for (int sp = 0; sp < 2; ++sp) {
    int ppc = sp == 0 ? c->ppc_e : c->ppc_i;
    if (s->n[sp] != ncell * ppc) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < s->n[sp]; ++p) {
      int64_t cell = p / ppc;
      int i = (int)(cell % c->nx);
      int j = (int)((cell / c->nx) % c->ny);
      int k = (int)(cell / ((int64_t)c->nx * c->ny));
      uint32_t r[4];
      draw(c, (uint32_t)p, 0, PUR_INIT_POS, (uint32_t)sp, r);
      const double q24 = 1.0 / 16777216.0;
      s->pos[sp][3 * p + 0] = (double)i + (double)(r[0] >> 8) * q24;
      s->pos[sp][3 * p + 1] = (double)j + (double)(r[1] >> 8) * q24;
      s->pos[sp][3 * p + 2] = (double)k + (double)(r[2] >> 8) * q24;
      draw(c, (uint32_t)p, 0, PUR_INIT_VEL, (uint32_t)sp, r);
      double n0, n1, n2, unused;
      box_muller(r[0], r[1], &n0, &n1);
      box_muller(r[2], r[3], &n2, &unused);
      s->vel[sp][3 * p + 0] = d.vth[sp] * n0;
      s->vel[sp][3 * p + 1] = d.vth[sp] * n1;
      s->vel[sp][3 * p + 2] = d.vth[sp] * n2;
      s->id[sp][p] = (uint32_t)p;
      s->alive[sp][p] = 1;
    }
  }
  for (int sp = 0; sp < 2; ++sp) s->next_id[sp] = (uint32_t)s->n[sp];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* cloud-in-cell: the 8 corner nodes of the particle's cell, each weighted by */
/* the product of the three 1-D linear weights (Sec. III, box-like shape)     */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t node[8]; double w[8]; } cic8;

static cic8 cic_weights(const orc_config* c, double X, double Y, double Z)
{
  cic8 r;
  int i0 = (int)floor(X), j0 = (int)floor(Y), k0 = (int)floor(Z);
  double fx = X - i0, fy = Y - j0, fz = Z - k0;
  int t = 0;
  for (int cc = 0; cc < 2; ++cc)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        double wx = a ? fx : 1.0 - fx;
        double wy = b ? fy : 1.0 - fy;
        double wz = cc ? fz : 1.0 - fz;
        r.node[t] = node_index(c, wrap_index(i0 + a, c->nx), wrap_index(j0 + b, c->ny), k0 + cc);
        r.w[t] = wx * wy * wz;
        ++t;
      }
  return r;
}

/* grain charge in coulomb, taken at the start of a step */
static double grain_charge(const orc_config* c, const orc_derived* d, const orc_state* s, int g)
{
  if (c->flags & ORC_FROZEN_Q) return c->Q_frozen_e * O_ECHARGE;
  int64_t net = s->grain_count[2 * g + 1] - s->grain_count[2 * g + 0];
  return (double)net * d->w * O_ECHARGE;
}

int orc_deposit(const orc_config* c, const orc_state* s, double* rho)
{
  orc_derived d;
  if (orc_derive(c, &d)) return -1;
  int64_t nn = orc_n_nodes(c);
  memset(rho, 0, sizeof(double) * nn);
  double vol = c->dx * c->dx * c->dx;
  for (int sp = 0; sp < 2; ++sp) {
    double qw = d.q[sp] * d.w;
    for (int64_t p = 0; p < s->n[sp]; ++p) {
      if (!s->alive[sp][p]) continue;
      const double* x = &s->pos[sp][3 * p];
      cic8 W = cic_weights(c, x[0], x[1], x[2]);
      for (int t = 0; t < 8; ++t) rho[W.node[t]] += qw * W.w[t];
    }
  }
  /* grain charges act on the mesh through the same assignment */
  for (int g = 0; g < c->n_grains; ++g) {
    const double* xg = &c->grain_pos[3 * g];
    double Q = grain_charge(c, &d, s, g);
    cic8 W = cic_weights(c, xg[0], xg[1], xg[2]);
    for (int t = 0; t < 8; ++t) rho[W.node[t]] += Q * W.w[t];
  }
  for (int64_t n = 0; n < nn; ++n) rho[n] /= vol;
  return 0;
}

/* Particle moments on the nodes, the densities and fluxes of the results    */
/* section (Sec. IV): n_s = w/dx^3 sum_p W and flux_s = w/dx^3 sum_p v W, with */
/* the same cloud-in-cell weights W as the charge; v is the stored v_{k-1/2}. */
/* n is [2][nodes], flux is [2][3][nodes].                                    */
int orc_moments(const orc_config* c, const orc_state* s, double* n, double* flux)
{
  orc_derived d;
  if (orc_derive(c, &d)) return -1;
  int64_t nn = orc_n_nodes(c);
  memset(n, 0, sizeof(double) * 2 * nn);
  memset(flux, 0, sizeof(double) * 6 * nn);
  double scale = d.w / (c->dx * c->dx * c->dx);
  for (int sp = 0; sp < 2; ++sp) {
    double* ns = n + sp * nn;
    double* fs = flux + 3 * sp * nn;
    for (int64_t p = 0; p < s->n[sp]; ++p) {
      if (!s->alive[sp][p]) continue;
      const double* x = &s->pos[sp][3 * p];
      const double* v = &s->vel[sp][3 * p];
      cic8 W = cic_weights(c, x[0], x[1], x[2]);
      for (int t = 0; t < 8; ++t) {
        ns[W.node[t]] += W.w[t];
        for (int a = 0; a < 3; ++a) fs[a * nn + W.node[t]] += v[a] * W.w[t];
      }
    }
  }
  for (int64_t m = 0; m < 2 * nn; ++m) n[m] *= scale;
  for (int64_t m = 0; m < 6 * nn; ++m) flux[m] *= scale;
  return 0;
}

/* Densities and fluxes on a fine cubical grid over a sub-box: the grid of   */
/* 0.08 dx cells over the region of the grains (Sec. IV).  The box's lower    */
/* corner is origin (grid units); its cells have edge h (grid units), m[a]    */
/* cells and m[a] + 1 nodes per axis, x fastest.  A particle whose            */
/* u = (x - origin) / h lies in [0, m) on every axis is assigned to the 8     */
/* nodes of its fine cell with the cloud-in-cell weights; a particle outside  */
/* the box adds nothing.  n = w sum W / (h dx)^3, flux = w sum v W / (h dx)^3. */
int orc_fine_moments(const orc_config* c, const orc_state* s, const double origin[3], double h,
                     const int32_t m[3], double* n, double* flux)
{
  orc_derived d;
  if (orc_derive(c, &d)) return -1;
  if (!(h > 0.0) || m[0] < 1 || m[1] < 1 || m[2] < 1) return -2;
  const int64_t mx = m[0] + 1, my = m[1] + 1, mz = m[2] + 1;
  const int64_t fn = mx * my * mz;
  memset(n, 0, sizeof(double) * 2 * fn);
  memset(flux, 0, sizeof(double) * 6 * fn);
  const double hdx = h * c->dx;
  const double scale = d.w / (hdx * hdx * hdx);
  for (int sp = 0; sp < 2; ++sp) {
    double* ns = n + sp * fn;
    double* fs = flux + 3 * sp * fn;
    for (int64_t p = 0; p < s->n[sp]; ++p) {
      if (!s->alive[sp][p]) continue;
      const double* x = &s->pos[sp][3 * p];
      const double* v = &s->vel[sp][3 * p];
      double u[3];
      int inside = 1;
      for (int a = 0; a < 3; ++a) {
        u[a] = (x[a] - origin[a]) / h;
        if (!(u[a] >= 0.0 && u[a] < (double)m[a])) inside = 0;
      }
      if (!inside) continue;
      const int64_t i0 = (int64_t)floor(u[0]), j0 = (int64_t)floor(u[1]), k0 = (int64_t)floor(u[2]);
      const double fx = u[0] - (double)i0, fy = u[1] - (double)j0, fz = u[2] - (double)k0;
      for (int cc = 0; cc < 2; ++cc)
        for (int b = 0; b < 2; ++b)
          for (int a = 0; a < 2; ++a) {
            const double wt = (a ? fx : 1.0 - fx) * (b ? fy : 1.0 - fy) * (cc ? fz : 1.0 - fz);
            const int64_t node = ((k0 + cc) * my + (j0 + b)) * mx + (i0 + a);
            ns[node] += wt;
            for (int q = 0; q < 3; ++q) fs[q * fn + node] += v[q] * wt;
          }
    }
  }
  for (int64_t q = 0; q < 2 * fn; ++q) n[q] *= scale;
  for (int64_t q = 0; q < 6 * fn; ++q) flux[q] *= scale;
  return 0;
}

/* Fixed-point CIC: the macro charge Qp (2^-32 e) is split along x, then each */
/* half along y, then each quarter along z, by q1 = (Q * f24) >> 24 and        */
/* q0 = Q - q1, where f24 = floor(offset * 2^24).  The 8 parts sum to Qp.      */
static void split_fixed(int64_t Q, double fx, double fy, double fz, int64_t part[8])
{
  int64_t qx = (int64_t)floor(fx * 16777216.0);
  int64_t qy = (int64_t)floor(fy * 16777216.0);
  int64_t qz = (int64_t)floor(fz * 16777216.0);
  int64_t ax[2], axy[2][2];
  ax[1] = (Q * qx) >> 24;
  ax[0] = Q - ax[1];
  for (int a = 0; a < 2; ++a) {
    axy[a][1] = (ax[a] * qy) >> 24;
    axy[a][0] = ax[a] - axy[a][1];
  }
  int t = 0;
  for (int cc = 0; cc < 2; ++cc)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        int64_t z1 = (axy[a][b] * qz) >> 24;
        part[t++] = cc ? z1 : axy[a][b] - z1;
      }
}

int orc_deposit_fixed(const orc_config* c, const orc_state* s, int64_t* rho_fixed)
{
  orc_derived d;
  if (orc_derive(c, &d)) return -1;
  if (c->flags & ORC_FROZEN_Q) return -3;
  int64_t nn = orc_n_nodes(c);
  memset(rho_fixed, 0, sizeof(int64_t) * nn);
  for (int sp = 0; sp < 2; ++sp) {
    int64_t sign = sp == 0 ? -1 : 1;
    for (int64_t p = 0; p < s->n[sp]; ++p) {
      if (!s->alive[sp][p]) continue;
      const double* x = &s->pos[sp][3 * p];
      cic8 W = cic_weights(c, x[0], x[1], x[2]);
      int64_t part[8];
      split_fixed(d.Qp, x[0] - floor(x[0]), x[1] - floor(x[1]), x[2] - floor(x[2]), part);
      for (int t = 0; t < 8; ++t) rho_fixed[W.node[t]] += sign * part[t];
    }
  }
  for (int g = 0; g < c->n_grains; ++g) {
    const double* xg = &c->grain_pos[3 * g];
    int64_t net = s->grain_count[2 * g + 1] - s->grain_count[2 * g + 0];
    cic8 W = cic_weights(c, xg[0], xg[1], xg[2]);
    int64_t part[8];
    split_fixed(d.Qp, xg[0] - floor(xg[0]), xg[1] - floor(xg[1]), xg[2] - floor(xg[2]), part);
    for (int t = 0; t < 8; ++t) rho_fixed[W.node[t]] += net * part[t];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Poisson, Eq. (3), in the 7-point finite-difference form on the nodes:      */
/*   sum of 6 neighbours - 6 phi = -dx^2 rho / eps0  on interior z nodes,     */
/*   periodic in x,y, phi = 0 on the grounded wall, phi = V on the rf wall.   */
/* phi = V k / nz + psi (the linear lift is discrete-harmonic); psi is found  */
/* by a plain DFT in x and y and, for every Fourier mode, a tridiagonal solve */
/* along z.                                                                    */
/* ------------------------------------------------------------------------ */

/* plain O(n^2) DFT of `count` lines of length n: out[m] = sum_j in[j] e^{sign 2 pi i m j / n} */
static void dft_lines(double complex* buf, int n, int64_t count, int64_t elem_stride,
                      int64_t line_stride, int sign, double complex* scratch)
{
  double complex* tw = (double complex*)malloc(sizeof(double complex) * n);
  for (int t = 0; t < n; ++t) {
    double a = 2.0 * O_PI * (double)t / (double)n;
    tw[t] = cos(a) + sign * sin(a) * I;
  }
  for (int64_t l = 0; l < count; ++l) {
    double complex* line = buf + l * line_stride;
    for (int m = 0; m < n; ++m) {
      double complex acc = 0;
      for (int j = 0; j < n; ++j) acc += line[j * elem_stride] * tw[((int64_t)m * j) % n];
      scratch[m] = acc;
    }
    for (int m = 0; m < n; ++m) line[m * elem_stride] = scratch[m];
  }
  free(tw);
}

/* forward (sign -1) or inverse (sign +1, unnormalised) 2-D DFT of one plane */
static void dft2_plane(double complex* plane, int nx, int ny, int sign, double complex* scratch)
{
  dft_lines(plane, nx, ny, 1, nx, sign, scratch);   /* rows: along x */
  dft_lines(plane, ny, nx, nx, 1, sign, scratch);   /* columns: along y */
}

/* tridiagonal with unit off-diagonals and diagonal `diag`, Dirichlet zeros at both ends */
static void thomas_unit(double diag, double complex* d, int K, double* cp)
{
  /* forward elimination */
  cp[0] = 1.0 / diag;
  d[0] = d[0] / diag;
  for (int k = 1; k < K; ++k) {
    double den = diag - cp[k - 1];
    cp[k] = 1.0 / den;
    d[k] = (d[k] - d[k - 1]) / den;
  }
  /* back substitution */
  for (int k = K - 2; k >= 0; --k) d[k] = d[k] - cp[k] * d[k + 1];
}

int orc_poisson(const orc_config* c, const double* rho, double V, double* phi)
{
  int nx = c->nx, ny = c->ny, nz = c->nz;
  int64_t plane = (int64_t)nx * ny;
  int K = nz - 1; /* interior planes k = 1 .. nz-1 */
  if (K < 1) return -1;
  double complex* hat = (double complex*)malloc(sizeof(double complex) * plane * K);
  if (!hat) return -2;
  double scale = -c->dx * c->dx / O_EPS0;
#pragma omp parallel
  {
    double complex* scratch = (double complex*)malloc(sizeof(double complex) * (nx > ny ? nx : ny));
#pragma omp for schedule(static)
    for (int k = 1; k <= K; ++k) {
      double complex* h = hat + (int64_t)(k - 1) * plane;
      for (int64_t n = 0; n < plane; ++n) h[n] = scale * rho[k * plane + n];
      dft2_plane(h, nx, ny, -1, scratch);
    }
    free(scratch);
  }
  /* one tridiagonal system per mode (m, n) */
#pragma omp parallel
  {
    double complex* col = (double complex*)malloc(sizeof(double complex) * K);
    double* cp = (double*)malloc(sizeof(double) * K);
#pragma omp for schedule(static)
    for (int64_t mn = 0; mn < plane; ++mn) {
      int m = (int)(mn % nx), n = (int)(mn / nx);
      double sx = sin(O_PI * m / nx), sy = sin(O_PI * n / ny);
      double diag = -(2.0 + 4.0 * (sx * sx + sy * sy));
      for (int k = 0; k < K; ++k) col[k] = hat[(int64_t)k * plane + mn];
      thomas_unit(diag, col, K, cp);
      for (int k = 0; k < K; ++k) hat[(int64_t)k * plane + mn] = col[k];
    }
    free(col);
    free(cp);
  }
#pragma omp parallel
  {
    double complex* scratch = (double complex*)malloc(sizeof(double complex) * (nx > ny ? nx : ny));
#pragma omp for schedule(static)
    for (int k = 1; k <= K; ++k) {
      double complex* h = hat + (int64_t)(k - 1) * plane;
      dft2_plane(h, nx, ny, +1, scratch);
      for (int64_t n = 0; n < plane; ++n)
        phi[k * plane + n] = creal(h[n]) / (double)plane + V * (double)k / (double)nz;
    }
    free(scratch);
  }
  for (int64_t n = 0; n < plane; ++n) {
    phi[n] = 0.0;
    phi[(int64_t)nz * plane + n] = V;
  }
  free(hat);
  return 0;
}

/* E = -grad phi, Eq. (4): central differences; one-sided along z on the two  */
/* electrode planes                                                            */
int orc_efield(const orc_config* c, const double* phi, double* E)
{
  int nx = c->nx, ny = c->ny, nz = c->nz;
  int64_t nn = orc_n_nodes(c);
  double* Ex = E;
  double* Ey = E + nn;
  double* Ez = E + 2 * nn;
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t n = node_index(c, i, j, k);
        Ex[n] = -(phi[node_index(c, wrap_index(i + 1, nx), j, k)] -
                  phi[node_index(c, wrap_index(i - 1, nx), j, k)]) / (2.0 * c->dx);
        Ey[n] = -(phi[node_index(c, i, wrap_index(j + 1, ny), k)] -
                  phi[node_index(c, i, wrap_index(j - 1, ny), k)]) / (2.0 * c->dx);
        if (k == 0)
          Ez[n] = -(phi[node_index(c, i, j, 1)] - phi[n]) / c->dx;
        else if (k == nz)
          Ez[n] = -(phi[n] - phi[node_index(c, i, j, nz - 1)]) / c->dx;
        else
          Ez[n] = -(phi[node_index(c, i, j, k + 1)] - phi[node_index(c, i, j, k - 1)]) / (2.0 * c->dx);
      }
  return 0;
}

int orc_fields(const orc_config* c, const orc_state* s, double* rho, int64_t* rho_fixed,
               double* phi, double* E)
{
  int rc;
  if (rho_fixed) {
    if ((rc = orc_deposit_fixed(c, s, rho_fixed))) return rc;
    double conv = O_ECHARGE / 4294967296.0 / (c->dx * c->dx * c->dx);
    for (int64_t n = 0; n < orc_n_nodes(c); ++n) rho[n] = (double)rho_fixed[n] * conv;
  } else if ((rc = orc_deposit(c, s, rho))) {
    return rc;
  }
  if ((rc = orc_poisson(c, rho, orc_rf_voltage(c, s->step), phi))) return rc;
  return orc_efield(c, phi, E);
}

/* ------------------------------------------------------------------------ */
/* MD region: the cube of (2c+1)^3 cells centred on the grain's cell,         */
/* periodic in x,y (c = 1 is the grain's cell plus its direct neighbours)     */
/* ------------------------------------------------------------------------ */
static int periodic_delta(int a, int b, int n)
{
  int d = wrap_index(a - b, n);
  if (d > n / 2) d -= n;
  return d;
}

int orc_md_grains(const orc_config* c, int i, int j, int k, int* out, int cap)
{
  int cnt = 0;
  for (int g = 0; g < c->n_grains; ++g) {
    const double* xg = &c->grain_pos[3 * g];
    int gi = (int)floor(xg[0]), gj = (int)floor(xg[1]), gk = (int)floor(xg[2]);
    if (abs(periodic_delta(i, gi, c->nx)) <= c->cutoff &&
        abs(periodic_delta(j, gj, c->ny)) <= c->cutoff && abs(k - gk) <= c->cutoff) {
      if (cnt < cap) out[cnt] = g;
      ++cnt;
    }
  }
  return cnt;
}

static int cube_side(const orc_config* c) { return 2 * c->cutoff + 2; }

/* E_PIC^dust of a unit (1 C) grain charge: the same deposit, solver and      */
/* stencil as the plasma field, kept on the nodes of the grain's MD cube      */
int orc_unit_fields(const orc_config* c, double* U)
{
  int64_t nn = orc_n_nodes(c);
  int side = cube_side(c);
  int64_t cube = (int64_t)side * side * side;
  double* rho = (double*)malloc(sizeof(double) * nn);
  double* phi = (double*)malloc(sizeof(double) * nn);
  double* E = (double*)malloc(sizeof(double) * nn * 3);
  if (!rho || !phi || !E) return -2;
  double vol = c->dx * c->dx * c->dx;
  int rc = 0;
  for (int g = 0; g < c->n_grains && !rc; ++g) {
    const double* xg = &c->grain_pos[3 * g];
    int gi = (int)floor(xg[0]), gj = (int)floor(xg[1]), gk = (int)floor(xg[2]);
    if (gk - c->cutoff < 0 || gk + c->cutoff + 1 > c->nz) { rc = -4; break; }
    memset(rho, 0, sizeof(double) * nn);
    cic8 W = cic_weights(c, xg[0], xg[1], xg[2]);
    for (int t = 0; t < 8; ++t) rho[W.node[t]] += W.w[t] / vol;
    if ((rc = orc_poisson(c, rho, 0.0, phi))) break;
    orc_efield(c, phi, E);
    for (int comp = 0; comp < 3; ++comp)
      for (int cz = 0; cz < side; ++cz)
        for (int cy = 0; cy < side; ++cy)
          for (int cx = 0; cx < side; ++cx) {
            int64_t n = node_index(c, wrap_index(gi - c->cutoff + cx, c->nx),
                                   wrap_index(gj - c->cutoff + cy, c->ny), gk - c->cutoff + cz);
            U[(int64_t)g * 3 * cube + comp * cube + ((int64_t)cz * side + cy) * side + cx] =
                E[comp * nn + n];
          }
  }
  free(rho);
  free(phi);
  free(E);
  return rc;
}

/* phi of a unit (1 C) grain charge on the nodes of its MD cube: [g][side^3] */
int orc_unit_potentials(const orc_config* c, double* Uphi)
{
  int64_t nn = orc_n_nodes(c);
  int side = cube_side(c);
  int64_t cube = (int64_t)side * side * side;
  double* rho = (double*)malloc(sizeof(double) * nn);
  double* phi = (double*)malloc(sizeof(double) * nn);
  if (!rho || !phi) return -2;
  double vol = c->dx * c->dx * c->dx;
  int rc = 0;
  for (int g = 0; g < c->n_grains && !rc; ++g) {
    const double* xg = &c->grain_pos[3 * g];
    int gi = (int)floor(xg[0]), gj = (int)floor(xg[1]), gk = (int)floor(xg[2]);
    if (gk - c->cutoff < 0 || gk + c->cutoff + 1 > c->nz) { rc = -4; break; }
    memset(rho, 0, sizeof(double) * nn);
    cic8 W = cic_weights(c, xg[0], xg[1], xg[2]);
    for (int t = 0; t < 8; ++t) rho[W.node[t]] += W.w[t] / vol;
    if ((rc = orc_poisson(c, rho, 0.0, phi))) break;
    for (int cz = 0; cz < side; ++cz)
      for (int cy = 0; cy < side; ++cy)
        for (int cx = 0; cx < side; ++cx)
          Uphi[(int64_t)g * cube + ((int64_t)cz * side + cy) * side + cx] =
              phi[node_index(c, wrap_index(gi - c->cutoff + cx, c->nx),
                             wrap_index(gj - c->cutoff + cy, c->ny), gk - c->cutoff + cz)];
  }
  free(rho);
  free(phi);
  return rc;
}

/* The potential on the nodes of the fine grid (the paper's MD-region grid,   */
/* Sec. IV), in the PPPM split of Eq. (5)-(6) applied to the potential: the   */
/* mesh potential interpolated with the cloud-in-cell weights at the node,    */
/* plus, for every grain whose MD cube holds the node's PIC cell, Q_g times   */
/* the bare Coulomb potential 1/(4 pi eps0 r) (r at least the grain radius:   */
/* the conducting grain's own potential inside it) minus the grain's          */
/* unit-charge mesh potential interpolated the same way.  A node on the upper */
/* face of the domain belongs to the last cell.                               */
int orc_fine_phi(const orc_config* c, const orc_state* s, const double* phi,
                 const double* Uphi, const double origin[3], double h, const int32_t m[3],
                 double* out)
{
  orc_derived d;
  if (orc_derive(c, &d)) return -1;
  if (!(h > 0.0) || m[0] < 1 || m[1] < 1 || m[2] < 1) return -2;
  const int side = cube_side(c);
  const int64_t cube = (int64_t)side * side * side;
  const int64_t mx = m[0] + 1, my = m[1] + 1, mz = m[2] + 1;
  int* G = (int*)malloc(sizeof(int) * (c->n_grains > 0 ? c->n_grains : 1));
  if (!G) return -3;
  for (int64_t kk = 0; kk < mz; ++kk)
    for (int64_t jj = 0; jj < my; ++jj)
      for (int64_t ii = 0; ii < mx; ++ii) {
        const double X[3] = {origin[0] + h * (double)ii, origin[1] + h * (double)jj,
                             origin[2] + h * (double)kk};
        const int n3[3] = {c->nx, c->ny, c->nz};
        int cl[3];
        double f[3];
        for (int a = 0; a < 3; ++a) {
          cl[a] = (int)floor(X[a]);
          if (cl[a] > n3[a] - 1) cl[a] = n3[a] - 1;
          f[a] = X[a] - (double)cl[a];
        }
        double w[8];
        int64_t node[8];
        int t = 0;
        for (int cc = 0; cc < 2; ++cc)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
              w[t] = (a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1]) * (cc ? f[2] : 1.0 - f[2]);
              node[t] = node_index(c, wrap_index(cl[0] + a, c->nx), wrap_index(cl[1] + b, c->ny),
                                   cl[2] + cc);
              ++t;
            }
        double v = 0.0;
        for (t = 0; t < 8; ++t) v += w[t] * phi[node[t]];
        int nG = orc_md_grains(c, cl[0], cl[1], cl[2], G, c->n_grains);
        for (int q = 0; q < nG; ++q) {
          const int g = G[q];
          const double* xg = &c->grain_pos[3 * g];
          const int gi = (int)floor(xg[0]), gj = (int)floor(xg[1]), gk = (int)floor(xg[2]);
          double r2 = 0.0;
          for (int a = 0; a < 3; ++a) {
            double dd = X[a] - xg[a];
            if (a < 2) dd -= n3[a] * floor(dd / n3[a] + 0.5);
            r2 += dd * dd;
          }
          double r = sqrt(r2) * c->dx;
          if (r < c->grain_radius) r = c->grain_radius;
          /* the node's CIC corners in the cube's node frame */
          const int ox = periodic_delta(cl[0], gi, c->nx) + c->cutoff;
          const int oy = periodic_delta(cl[1], gj, c->ny) + c->cutoff;
          const int oz = cl[2] - gk + c->cutoff;
          double unit = 0.0;
          t = 0;
          for (int cc = 0; cc < 2; ++cc)
            for (int b = 0; b < 2; ++b)
              for (int a = 0; a < 2; ++a) {
                unit += w[t] * Uphi[(int64_t)g * cube + ((int64_t)(oz + cc) * side + (oy + b)) * side +
                                    (ox + a)];
                ++t;
              }
          v += grain_charge(c, &d, s, g) * (1.0 / (4.0 * O_PI * O_EPS0 * r) - unit);
        }
        out[(kk * my + jj) * mx + ii] = v;
      }
  free(G);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* particle motion                                                            */
/* ------------------------------------------------------------------------ */
static void gather_mesh(const orc_config* c, const double* E, double X, double Y, double Z,
                        double out[3])
{
  out[0] = out[1] = out[2] = 0.0;
  if (!E) return;
  int64_t nn = orc_n_nodes(c);
  cic8 W = cic_weights(c, X, Y, Z);
  for (int t = 0; t < 8; ++t)
    for (int comp = 0; comp < 3; ++comp) out[comp] += W.w[t] * E[comp * nn + W.node[t]];
}

/* the same CIC weights applied to a grain's unit field on its cube */
static void gather_unit(const orc_config* c, const double* U, int g, double X, double Y,
                        double Z, double out[3])
{
  int side = cube_side(c);
  int64_t cube = (int64_t)side * side * side;
  const double* xg = &c->grain_pos[3 * g];
  int gi = (int)floor(xg[0]), gj = (int)floor(xg[1]), gk = (int)floor(xg[2]);
  int i0 = (int)floor(X), j0 = (int)floor(Y), k0 = (int)floor(Z);
  double fx = X - i0, fy = Y - j0, fz = Z - k0;
  out[0] = out[1] = out[2] = 0.0;
  for (int cc = 0; cc < 2; ++cc)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        double w = (a ? fx : 1.0 - fx) * (b ? fy : 1.0 - fy) * (cc ? fz : 1.0 - fz);
        int lx = wrap_index(i0 + a - (gi - c->cutoff), c->nx);
        int ly = wrap_index(j0 + b - (gj - c->cutoff), c->ny);
        int lz = k0 + cc - (gk - c->cutoff);
        int64_t l = ((int64_t)lz * side + ly) * side + lx;
        for (int comp = 0; comp < 3; ++comp) out[comp] += w * U[(int64_t)g * 3 * cube + comp * cube + l];
      }
}

/* minimum-image separation x - x_g in cell units */
static void separation(const orc_config* c, int g, double X, double Y, double Z, double r[3])
{
  const double* xg = &c->grain_pos[3 * g];
  r[0] = X - xg[0];
  r[1] = Y - xg[1];
  r[2] = Z - xg[2];
  if (r[0] > 0.5 * c->nx) r[0] -= c->nx;
  else if (r[0] < -0.5 * c->nx) r[0] += c->nx;
  if (r[1] > 0.5 * c->ny) r[1] -= c->ny;
  else if (r[1] < -0.5 * c->ny) r[1] += c->ny;
}

static double wrap_coord(double X, int n)
{
  X = X - (double)n * floor(X / (double)n);
  if (X >= (double)n) X -= (double)n;
  return X;
}

enum { MV_ALIVE = 0, MV_WALL0 = 1, MV_WALL1 = 2, MV_GRAIN = 3 };

static double dmin(double a, double b) { return a < b ? a : b; }

/* plain PIC particle: gather, Eq. (2) kick, Eq. (1) drift, wrap, electrodes */
static int move_plain(const orc_config* c, const double* E, double qm, double* x, double* v,
                      double* margin)
{
  double Ep[3];
  gather_mesh(c, E, x[0], x[1], x[2], Ep);
  for (int a = 0; a < 3; ++a) v[a] += qm * Ep[a] * c->dt;
  for (int a = 0; a < 3; ++a) x[a] += v[a] * c->dt / c->dx;
  x[0] = wrap_coord(x[0], c->nx);
  x[1] = wrap_coord(x[1], c->ny);
  *margin = dmin(*margin, dmin(fabs(x[2]), fabs(x[2] - c->nz)));
  if (x[2] < 0.0) return MV_WALL0;
  if (x[2] >= (double)c->nz) return MV_WALL1;
  return MV_ALIVE;
}

/* MD particle: md_sub sub-steps of dt/md_sub with the PPPM field of Eq. (5)-(6) */
static int move_md(const orc_config* c, const double* E, const double* U, const double* Q,
                   double qm, double* x, double* v, double* margin, int* hit_grain)
{
  double h = c->dt / (double)c->md_sub;
  double a2 = c->grain_radius * c->grain_radius;
  int G[64];
  for (int sub = 0; sub < c->md_sub; ++sub) {
    double Ep[3];
    gather_mesh(c, E, x[0], x[1], x[2], Ep);
    int nG = orc_md_grains(c, (int)floor(x[0]), (int)floor(x[1]), (int)floor(x[2]), G, 64);
    for (int t = 0; t < nG && t < 64; ++t) {
      int g = G[t];
      if (Q[g] == 0.0) continue;
      double r[3];
      separation(c, g, x[0], x[1], x[2], r);
      for (int a = 0; a < 3; ++a) r[a] *= c->dx;
      double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      double inv = 1.0 / (4.0 * O_PI * O_EPS0 * r2 * sqrt(r2));
      double Um[3] = {0.0, 0.0, 0.0};
      if (U) gather_unit(c, U, g, x[0], x[1], x[2], Um);
      for (int a = 0; a < 3; ++a) Ep[a] += Q[g] * (r[a] * inv - Um[a]);
    }
    for (int a = 0; a < 3; ++a) v[a] += qm * Ep[a] * h;
    for (int a = 0; a < 3; ++a) x[a] += v[a] * h / c->dx;
    x[0] = wrap_coord(x[0], c->nx);
    x[1] = wrap_coord(x[1], c->ny);
    *margin = dmin(*margin, dmin(fabs(x[2]), fabs(x[2] - c->nz)));
    if (x[2] < 0.0) return MV_WALL0;
    if (x[2] >= (double)c->nz) return MV_WALL1;
    nG = orc_md_grains(c, (int)floor(x[0]), (int)floor(x[1]), (int)floor(x[2]), G, 64);
    for (int t = 0; t < nG && t < 64; ++t) {
      int g = G[t];
      double r[3];
      separation(c, g, x[0], x[1], x[2], r);
      for (int a = 0; a < 3; ++a) r[a] *= c->dx;
      double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      *margin = dmin(*margin, fabs(sqrt(r2) - c->grain_radius) / c->grain_radius);
      if (r2 <= a2) {
        *hit_grain = g;
        return MV_GRAIN;
      }
    }
  }
  return MV_ALIVE;
}

/* the same with energy-dependent cross sections: the process is picked by  */
/* u1 against the cumulative g sigma_k(E) / (g sigma)_max.  Electrons:      */
/* elastic, then excitation (only with the CM energy above E_ex: the CM     */
/* energy drops by E_ex, isotropic scattering); ions: charge exchange, then */
/* isotropic elastic scattering in the CM frame of ion and neutral.  Above  */
/* the bound (a cap violation) the collision happens and u1 splits sigma.   */
/* an electron-impact ionisation of one step, applied after every particle has
   moved: the parent's index and id, its velocity before the collision and
   the squared relative speed left to share, g^2 - 2 E_iz / mu */
typedef struct iz_event {
  int64_t p;
  uint32_t id;
  double v[3];
  double gsq;
} iz_event;

typedef struct iz_sink {
  iz_event* ev;
  int64_t n, cap;
} iz_sink;

static void collide_xs(const orc_config* c, const orc_derived* d, int sp, uint32_t id, uint32_t k,
                       const uint32_t r[4], const double* vn, double* v, double* margin,
                       int64_t* cap_viol, int64_t* ncoll, int64_t p, iz_sink* iz)
{
  double gv[3] = {v[0] - vn[0], v[1] - vn[1], v[2] - vn[2]};
  double g2 = gv[0] * gv[0] + gv[1] * gv[1] + gv[2] * gv[2];
  double g = sqrt(g2);
  double E = 0.5 * d->m[sp] * g2 / O_ECHARGE;
  double mu = d->m[0] * d->m[1] / (d->m[0] + d->m[1]);
  double s1, s2, s3 = 0.0;
  if (sp == 0) {
    s1 = orc_xs_at(c, c->xs_e_el, E);
    s2 = 0.5 * mu * g2 > c->E_ex_eV * O_ECHARGE ? orc_xs_at(c, c->xs_e_ex, E) : 0.0;
    s3 = 0.5 * mu * g2 > c->E_iz_eV * O_ECHARGE ? orc_xs_at(c, c->xs_e_iz, E) : 0.0;
  } else {
    s1 = orc_xs_at(c, c->xs_i_cx, E);
    s2 = orc_xs_at(c, c->xs_i_el, E);
  }
  double a1 = g * s1 / d->sg_max[sp], a2 = g * (s1 + s2) / d->sg_max[sp];
  double a3 = g * (s1 + s2 + s3) / d->sg_max[sp];
  double u1 = unif_open(r[1]);
  int proc; /* 0 none, 1 first process, 2 second, 3 ionisation */
  if (a3 > 1.0) {
#pragma omp atomic
    cap_viol[sp] += 1;
    double x = u1 * (s1 + s2 + s3);
    proc = x < s1 ? 1 : (x < s1 + s2 ? 2 : 3);
  } else {
    *margin = dmin(*margin, dmin(fabs(u1 - a1), fabs(u1 - a2)));
    if (s3 > 0.0) *margin = dmin(*margin, fabs(u1 - a3));
    proc = u1 < a1 ? 1 : (u1 < a2 ? 2 : (u1 < a3 ? 3 : 0));
  }
  if (proc == 0) return;
#pragma omp atomic
  ncoll[sp] += 1;
  if (sp == 1 && proc == 1) {
    for (int a = 0; a < 3; ++a) v[a] = vn[a]; /* charge exchange */
    return;
  }
  double cost = 1.0 - 2.0 * unif_open(r[2]);
  double sint = sqrt(fmax(0.0, 1.0 - cost * cost));
  double ph = 2.0 * O_PI * unif_open(r[3]);
  double nh[3] = {sint * cos(ph), sint * sin(ph), cost};
  double mt = d->m[0] + d->m[1];
  if (sp == 0) {
    /* neutral at rest: v' = (m v + M 0) / (m + M) + M / (m + M) g' n */
    double gp = g;
    if (proc == 2) gp = sqrt(g2 - 2.0 * c->E_ex_eV * O_ECHARGE / mu);
    if (proc == 3) {
      /* ionisation: the centre-of-mass energy less E_iz is shared, a fraction
         s (uniform, Philox(id, k, IONIZE, 0) word 0) to the ejected electron,
         1 - s to the scattered one; the ejected electron and the new ion are
         made after the step (ionize_apply) */
      double gsq = g2 - 2.0 * c->E_iz_eV * O_ECHARGE / mu;
      uint32_t w[4];
      draw(c, id, k, PUR_IONIZE, 0u, w);
      double share = unif_open(w[0]);
      int64_t slot;
#pragma omp atomic capture
      slot = iz->n++;
      if (slot < iz->cap) {
        iz->ev[slot].p = p;
        iz->ev[slot].id = id;
        for (int a = 0; a < 3; ++a) iz->ev[slot].v[a] = v[a];
        iz->ev[slot].gsq = gsq;
      }
      gp = sqrt((1.0 - share) * gsq);
    }
    for (int a = 0; a < 3; ++a) v[a] = (d->m[0] / mt) * v[a] + (d->m[1] / mt) * gp * nh[a];
  } else {
    /* ion and neutral of equal mass: v' = (v + v_n) / 2 + (g / 2) n */
    for (int a = 0; a < 3; ++a) v[a] = 0.5 * (v[a] + vn[a]) + 0.5 * g * nh[a];
  }
}

/* binary collision with a neutral drawn from the reservoir, null-collision form */
static void collide(const orc_config* c, const orc_derived* d, int sp, uint32_t id, uint32_t k,
                    double* v, double* margin, int64_t* cap_viol, int64_t* ncoll, int64_t p,
                    iz_sink* iz)
{
  uint32_t r[4];
  draw(c, id, k, PUR_COLL, (uint32_t)sp, r);
  if ((uint64_t)r[0] >= d->T_null[sp]) return; /* not a candidate */
  double vn[3] = {0.0, 0.0, 0.0};
  if (sp == 1) {
    uint32_t rn[4];
    double unused;
    draw(c, id, k, PUR_NEUTRAL, (uint32_t)sp, rn);
    box_muller(rn[0], rn[1], &vn[0], &vn[1]);
    box_muller(rn[2], rn[3], &vn[2], &unused);
    for (int a = 0; a < 3; ++a) vn[a] *= d->vth_gas;
  }
  if (c->xs_n > 0) {
    collide_xs(c, d, sp, id, k, r, vn, v, margin, cap_viol, ncoll, p, iz);
    return;
  }
  double gv[3] = {v[0] - vn[0], v[1] - vn[1], v[2] - vn[2]};
  double g = sqrt(gv[0] * gv[0] + gv[1] * gv[1] + gv[2] * gv[2]);
  double u1 = unif_open(r[1]);
  double ratio = g / d->g_cap[sp];
  int accept;
  if (ratio > 1.0) {
#pragma omp atomic
    cap_viol[sp] += 1;
    accept = 1;
  } else {
    *margin = dmin(*margin, fabs(u1 - ratio));
    accept = u1 < ratio;
  }
  if (!accept) return;
#pragma omp atomic
  ncoll[sp] += 1;
  if (sp == 0) {
    /* e-Ar elastic: isotropic in the centre-of-mass frame, neutral at rest */
    double cost = 1.0 - 2.0 * unif_open(r[2]);
    double sint = sqrt(fmax(0.0, 1.0 - cost * cost));
    double ph = 2.0 * O_PI * unif_open(r[3]);
    double nh[3] = {sint * cos(ph), sint * sin(ph), cost};
    double mt = d->m[0] + d->m[1];
    for (int a = 0; a < 3; ++a) v[a] = (d->m[0] / mt) * v[a] + (d->m[1] / mt) * g * nh[a];
  } else {
    /* Ar+-Ar charge exchange: the ion leaves with the neutral's velocity */
    for (int a = 0; a < 3; ++a) v[a] = vn[a];
  }
}

/* ------------------------------------------------------------------------ */
/* Coulomb collisions (Table I: e-e, e-Ar+, Ar+-Ar+), the binary model of      */
/* Takizuka and Abe cited with the collision set: the particles of a cell are  */
/* paired at random; each pair's relative velocity u turns by an angle theta   */
/* with delta = tan(theta/2) normal of variance                                */
/*   q_a^2 q_b^2 n_L lnL dtc / (8 pi eps0^2 mu^2 |u|^3)                        */
/* (mu the reduced mass, n_L the density of the less numerous species of the   */
/* pair, the species' own density for like particles) and a uniform azimuth   */
/* phi about u; both velocities change so that momentum and energy are kept.  */
/* ------------------------------------------------------------------------ */
double orc_coulomb_var(const orc_config* c, int sa, int sb, double u, double nL, double dtc)
{
  orc_derived d;
  if (orc_derive(c, &d)) return NAN;
  double mu = d.m[sa] * d.m[sb] / (d.m[sa] + d.m[sb]);
  double qq = d.q[sa] * d.q[sb];
  return qq * qq * nL * c->coulomb_lnL * dtc / (8.0 * O_PI * O_EPS0 * O_EPS0 * mu * mu * u * u * u);
}

void orc_coulomb_pair(const orc_config* c, int sa, int sb, double* va, double* vb, double delta,
                      double phi)
{
  orc_derived d;
  if (orc_derive(c, &d)) return;
  double u[3] = {va[0] - vb[0], va[1] - vb[1], va[2] - vb[2]};
  double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  double up = sqrt(u[0] * u[0] + u[1] * u[1]);
  double sn = 2.0 * delta / (1.0 + delta * delta);        /* sin theta */
  double omc = 2.0 * delta * delta / (1.0 + delta * delta); /* 1 - cos theta */
  double cp = cos(phi), sp = sin(phi);
  double du[3];
  if (up > 0.0) {
    du[0] = (u[0] / up) * u[2] * sn * cp - (u[1] / up) * um * sn * sp - u[0] * omc;
    du[1] = (u[1] / up) * u[2] * sn * cp + (u[0] / up) * um * sn * sp - u[1] * omc;
    du[2] = -up * sn * cp - u[2] * omc;
  } else {
    /* u along z: the same rotation with the azimuth measured from x */
    du[0] = um * sn * cp;
    du[1] = um * sn * sp;
    du[2] = -u[2] * omc;
  }
  double mu = d.m[sa] * d.m[sb] / (d.m[sa] + d.m[sb]);
  for (int a = 0; a < 3; ++a) {
    va[a] += (mu / d.m[sa]) * du[a];
    vb[a] -= (mu / d.m[sb]) * du[a];
  }
}

/* one collision of the pass: draws from Philox(id of the pair's first      */
/* particle, k, PUR_CPAIR, kind), kind 0 e-e, 1 Ar+-Ar+, 2 + a for unlike    */
/* pairs whose more numerous species is a; delta from the Box-Muller cosine */
/* branch of words 0 and 1, phi = 2 pi u(word 2)                            */
static void coulomb_one(const orc_config* c, int sa, int sb, double* va, double* vb, double nL,
                        double dtc, uint32_t id, uint32_t k, uint32_t kind)
{
  double u[3] = {va[0] - vb[0], va[1] - vb[1], va[2] - vb[2]};
  double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  if (!(um > 0.0)) return;
  uint32_t r[4];
  draw(c, id, k, PUR_CPAIR, kind, r);
  double n0, n1;
  box_muller(r[0], r[1], &n0, &n1);
  double delta = sqrt(orc_coulomb_var(c, sa, sb, um, nL, dtc)) * n0;
  orc_coulomb_pair(c, sa, sb, va, vb, delta, 2.0 * O_PI * unif_open(r[2]));
}

typedef struct {
  int64_t cell;
  uint64_t key; /* Philox(id, k, PUR_CORDER, species) word 0, then id */
  int64_t p;
} ckey;

static int cmp_ckey(const void* a, const void* b)
{
  const ckey* x = (const ckey*)a;
  const ckey* y = (const ckey*)b;
  if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return 0;
}

/* Pairing in a cell.  Each species' particles are put in the order of their */
/* keys.  Like particles: consecutive pairs (p0,p1), (p2,p3), ...; an odd     */
/* count of three or more starts with the triplet (p0,p1), (p1,p2), (p2,p0),  */
/* each at half the time step.  Unlike particles: with N_a >= N_b (electrons  */
/* on a tie) particle j of a collides with particle j mod N_b of b, in order  */
/* of j, at density n_L = N_b w / dx^3.  Order: e-e, Ar+-Ar+, then e-Ar+.    */
int64_t orc_coulomb(const orc_config* c, orc_state* s)
{
  orc_derived d;
  if (orc_derive(c, &d)) return -1;
  if (c->coulomb_interval <= 0) return 0;
  const uint32_t k = s->step;
  const double dtc = c->coulomb_interval * c->dt;
  const double vol = c->dx * c->dx * c->dx;
  ckey* L[2] = {NULL, NULL};
  int64_t n[2] = {0, 0};
  for (int sp = 0; sp < 2; ++sp) {
    L[sp] = (ckey*)malloc(sizeof(ckey) * (size_t)(s->n[sp] > 0 ? s->n[sp] : 1));
    if (!L[sp]) {
      free(L[0]);
      return -2;
    }
    for (int64_t p = 0; p < s->n[sp]; ++p) {
      if (!s->alive[sp][p]) continue;
      const double* x = &s->pos[sp][3 * p];
      int64_t i = (int64_t)floor(x[0]), j = (int64_t)floor(x[1]), kk = (int64_t)floor(x[2]);
      uint32_t r[4];
      draw(c, s->id[sp][p], k, PUR_CORDER, (uint32_t)sp, r);
      ckey e = {(kk * c->ny + j) * c->nx + i, ((uint64_t)r[0] << 32) | s->id[sp][p], p};
      L[sp][n[sp]++] = e;
    }
    qsort(L[sp], (size_t)n[sp], sizeof(ckey), cmp_ckey);
  }
  int64_t ncoll = 0;
  int64_t a0[2] = {0, 0};
  while (a0[0] < n[0] || a0[1] < n[1]) {
    /* the next cell holding a particle of either species */
    int64_t cell = INT64_MAX;
    for (int sp = 0; sp < 2; ++sp)
      if (a0[sp] < n[sp] && L[sp][a0[sp]].cell < cell) cell = L[sp][a0[sp]].cell;
    int64_t a1[2];
    for (int sp = 0; sp < 2; ++sp) {
      a1[sp] = a0[sp];
      while (a1[sp] < n[sp] && L[sp][a1[sp]].cell == cell) ++a1[sp];
    }
#define VEL(sp, q) (&s->vel[sp][3 * L[sp][q].p])
#define PID(sp, q) (s->id[sp][L[sp][q].p])
    for (int sp = 0; sp < 2; ++sp) {
      int64_t N = a1[sp] - a0[sp], b = a0[sp];
      if (N < 2) continue;
      double ns = (double)N * d.w / vol;
      int64_t q = b;
      if (N % 2 == 1) {
        coulomb_one(c, sp, sp, VEL(sp, b), VEL(sp, b + 1), ns, 0.5 * dtc, PID(sp, b), k, sp);
        coulomb_one(c, sp, sp, VEL(sp, b + 1), VEL(sp, b + 2), ns, 0.5 * dtc, PID(sp, b + 1), k, sp);
        coulomb_one(c, sp, sp, VEL(sp, b + 2), VEL(sp, b), ns, 0.5 * dtc, PID(sp, b + 2), k, sp);
        ncoll += 3;
        q = b + 3;
      }
      for (; q + 1 < a1[sp]; q += 2) {
        coulomb_one(c, sp, sp, VEL(sp, q), VEL(sp, q + 1), ns, dtc, PID(sp, q), k, sp);
        ncoll += 1;
      }
    }
    int64_t Ne = a1[0] - a0[0], Ni = a1[1] - a0[1];
    if (Ne > 0 && Ni > 0) {
      int sa = Ne >= Ni ? 0 : 1, sb = 1 - sa;
      int64_t Na = sa == 0 ? Ne : Ni, Nb = sa == 0 ? Ni : Ne;
      double nL = (double)Nb * d.w / vol;
      for (int64_t j = 0; j < Na; ++j) {
        coulomb_one(c, sa, sb, VEL(sa, a0[sa] + j), VEL(sb, a0[sb] + j % Nb), nL, dtc,
                    PID(sa, a0[sa] + j), k, 2 + (uint32_t)sa);
        ncoll += 1;
      }
    }
#undef VEL
#undef PID
    a0[0] = a1[0];
    a0[1] = a1[1];
  }
  free(L[0]);
  free(L[1]);
  return ncoll;
}

static int cmp_iz(const void* a, const void* b)
{
  uint32_t x = ((const iz_event*)a)->id, y = ((const iz_event*)b)->id;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* The ionisations of step k, in order of the parent electron's id: each makes
   an electron and an ion at the parent's new position x_{k+1}, with ids
   next_id[s]++ (s: species).  The ejected electron takes the share s of the
   available centre-of-mass energy: relative speed g_e = sqrt(s gsq), an
   isotropic direction from Philox(id, k, IONIZE, 0) words 1 and 2, and
   v = V_cm + M / (m + M) g_e n with V_cm = m v_parent / (m + M) (the neutral
   at rest, as for the other electron collisions); the ion takes a Maxwellian
   velocity of the gas temperature from Philox(id, k, IONIZE, 1) (Box-Muller,
   cosine branch first).  Both join the next step with these as v_{k+1/2}. */
static int ionize_apply(const orc_config* c, const orc_derived* d, orc_state* s, uint32_t k,
                        iz_sink* iz)
{
  if (iz->n == 0) return 0;
  if (iz->n > iz->cap) return -7;
  qsort(iz->ev, (size_t)iz->n, sizeof(iz_event), cmp_iz);
  if (s->n[0] + iz->n > s->cap[0] || s->n[1] + iz->n > s->cap[1]) return -8;
  double mt = d->m[0] + d->m[1];
  for (int64_t q = 0; q < iz->n; ++q) {
    const iz_event* e = &iz->ev[q];
    uint32_t w0[4], w1[4];
    draw(c, e->id, k, PUR_IONIZE, 0u, w0);
    draw(c, e->id, k, PUR_IONIZE, 1u, w1);
    double share = unif_open(w0[0]);
    double ge = sqrt(share * e->gsq);
    double cost = 1.0 - 2.0 * unif_open(w0[1]);
    double sint = sqrt(fmax(0.0, 1.0 - cost * cost));
    double ph = 2.0 * O_PI * unif_open(w0[2]);
    double nh[3] = {sint * cos(ph), sint * sin(ph), cost};
    int64_t pe = s->n[0]++, pi = s->n[1]++;
    for (int a = 0; a < 3; ++a) {
      s->pos[0][3 * pe + a] = s->pos[0][3 * e->p + a];
      s->pos[1][3 * pi + a] = s->pos[0][3 * e->p + a];
      s->vel[0][3 * pe + a] = (d->m[0] / mt) * e->v[a] + (d->m[1] / mt) * ge * nh[a];
    }
    double n0, n1, n2, unused;
    box_muller(w1[0], w1[1], &n0, &n1);
    box_muller(w1[2], w1[3], &n2, &unused);
    s->vel[1][3 * pi + 0] = d->vth_gas * n0;
    s->vel[1][3 * pi + 1] = d->vth_gas * n1;
    s->vel[1][3 * pi + 2] = d->vth_gas * n2;
    s->id[0][pe] = s->next_id[0]++;
    s->id[1][pi] = s->next_id[1]++;
    s->alive[0][pe] = s->alive[1][pi] = 1;
    if (s->margin[0]) s->margin[0][pe] = INFINITY;
    if (s->margin[1]) s->margin[1][pi] = INFINITY;
  }
  s->n_ionizations += iz->n;
  return 0;
}

static int move_all(const orc_config* c, orc_state* s, const double* E, const double* U)
{
  orc_derived d;
  if (orc_derive(c, &d)) return -1;
  if (c->n_grains > 64) return -5;
  double Q[64];
  for (int g = 0; g < c->n_grains; ++g) Q[g] = grain_charge(c, &d, s, g);
  const double* Uuse = (c->flags & ORC_NO_MESH) ? NULL : U;
  const double* Euse = (c->flags & ORC_NO_MESH) ? NULL : E;
  uint32_t k = s->step;
  /* Coulomb collisions on (x_k, v_{k-1/2}) at the start of every interval-th step */
  if (c->coulomb_interval > 0 && k % (uint32_t)c->coulomb_interval == 0 && orc_coulomb(c, s) < 0)
    return -6;
  /* a plain push at least this fast crosses cutoff cells in one step: it could
     reach a grain from outside the grain's MD cube, where no grain test is made */
  const double vfast = c->cutoff * c->dx / c->dt;
  /* ionisation events of this step (at most one per electron) */
  iz_sink iz = {NULL, 0, 0};
  if (c->xs_n > 0 && c->xs_e_iz && !(c->flags & ORC_NO_MCC) && s->n[0] > 0) {
    iz.cap = s->n[0];
    iz.ev = (iz_event*)malloc(sizeof(iz_event) * (size_t)iz.cap);
    if (!iz.ev) return -2;
  }
  for (int sp = 0; sp < 2; ++sp) {
    double qm = d.q[sp] / d.m[sp];
    int64_t wall[2] = {0, 0}, fast = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : wall[:2], fast)
    for (int64_t p = 0; p < s->n[sp]; ++p) {
      if (!s->alive[sp][p]) continue;
      if (sp == 1 && (c->flags & ORC_IMMOBILE_IONS)) continue;
      double* x = &s->pos[sp][3 * p];
      double* v = &s->vel[sp][3 * p];
      double margin = INFINITY;
      int G[1];
      int nG = (c->flags & ORC_NO_MD) ? 0
                                      : orc_md_grains(c, (int)floor(x[0]), (int)floor(x[1]),
                                                      (int)floor(x[2]), G, 1);
      int hit = -1, st;
      if (nG == 0) {
        st = move_plain(c, Euse, qm, x, v, &margin);
        if (c->n_grains > 0 && !(c->flags & ORC_NO_MD) &&
            v[0] * v[0] + v[1] * v[1] + v[2] * v[2] >= vfast * vfast)
          fast += 1;
      } else
        st = move_md(c, Euse, Uuse, Q, qm, x, v, &margin, &hit);
      if (st == MV_WALL0 || st == MV_WALL1) {
        wall[st - 1] += 1;
        s->alive[sp][p] = 0;
      } else if (st == MV_GRAIN) {
#pragma omp atomic
        s->grain_count[2 * hit + sp] += 1;
        s->alive[sp][p] = 0;
      } else if (!(c->flags & ORC_NO_MCC)) {
        collide(c, &d, sp, s->id[sp][p], k, v, &margin, s->cap_violation, s->n_collisions, p, &iz);
      }
      if (s->margin[sp]) s->margin[sp][p] = margin;
    }
    s->wall_count[0][sp] += wall[0];
    s->wall_count[1][sp] += wall[1];
    s->md_margin[sp] += fast;
  }
  int rc = ionize_apply(c, &d, s, k, &iz);
  free(iz.ev);
  if (rc) return rc;
  s->step = k + 1;
  return 0;
}

/* Test mode for the orbit-motion-limited (OML) pin of grain charging
 * (Sec. IV.B): test particles of species sp start at pos/vel (cell units,
 * m/s; n of them) and move in the field of grain 0 alone -- charge
 * c->Q_frozen_e e, no mesh field, no collisions -- by the MD sub-step of
 * Eq. (5)-(6) (move_md with the configuration's dt and md_sub), with its
 * grain test, until the grain absorbs them or they are farther than R_c
 * cells from it; outside that sphere the grain's field counts as zero, so a
 * particle that leaves does not come back.  The caller takes md_sub = 1 so
 * that the sphere is tested after every sub-step.  A particle still inside
 * after max_calls calls of move_md counts in *n_open.  Returns the number
 * absorbed, *n_out those that left, or a negative error.  pos/vel end with
 * the final states. */
int64_t orc_oml_collect(const orc_config* c, int sp, double R_c, int64_t n, double* pos,
                        double* vel, int64_t max_calls, int64_t* n_out, int64_t* n_open)
{
  orc_derived d;
  if (orc_derive(c, &d) || c->n_grains < 1 || sp < 0 || sp > 1) return -1;
  double Q[64];
  for (int g = 0; g < c->n_grains && g < 64; ++g) Q[g] = g == 0 ? c->Q_frozen_e * O_ECHARGE : 0.0;
  const double qm = d.q[sp] / d.m[sp];
  int64_t hits = 0, outs = 0, open = 0, bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : hits, outs, open, bad)
  for (int64_t p = 0; p < n; ++p) {
    double* x = &pos[3 * p];
    double* v = &vel[3 * p];
    int64_t call = 0;
    int fate = 0; /* 0 inside, 1 absorbed, 2 left */
    for (; call < max_calls && fate == 0; ++call) {
      double margin = INFINITY;
      int hit = -1;
      int st = move_md(c, NULL, NULL, Q, qm, x, v, &margin, &hit);
      if (st == MV_GRAIN) {
        fate = hit == 0 ? 1 : 3;
      } else if (st != MV_ALIVE) {
        fate = 3;
      } else {
        double r[3];
        separation(c, 0, x[0], x[1], x[2], r);
        if (r[0] * r[0] + r[1] * r[1] + r[2] * r[2] > R_c * R_c) fate = 2;
      }
    }
    if (fate == 1) hits += 1;
    else if (fate == 2) outs += 1;
    else if (fate == 0) open += 1;
    else bad += 1;
  }
  if (bad) return -2;
  if (n_out) *n_out = outs;
  if (n_open) *n_open = open;
  return hits;
}

int orc_step_in_field(const orc_config* c, orc_state* s, const double* E, const double* U)
{
  return move_all(c, s, E, U);
}

int orc_step(const orc_config* c, orc_state* s, const double* U)
{
  if (c->flags & ORC_NO_MESH) return move_all(c, s, NULL, NULL);
  int64_t nn = orc_n_nodes(c);
  double* rho = (double*)malloc(sizeof(double) * nn);
  double* phi = (double*)malloc(sizeof(double) * nn);
  double* E = (double*)malloc(sizeof(double) * nn * 3);
  int64_t* rf = (c->flags & ORC_FIXED_POINT) ? (int64_t*)malloc(sizeof(int64_t) * nn) : NULL;
  int rc = -2;
  if (rho && phi && E)
    rc = orc_fields(c, s, rho, rf, phi, E);
  if (!rc) rc = move_all(c, s, E, U);
  free(rho);
  free(phi);
  free(E);
  free(rf);
  return rc;
}
