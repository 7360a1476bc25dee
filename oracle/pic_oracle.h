/*
 * pic_oracle.h -- plain FP64 CPU oracle of the PIC-MCC/PPPM time step of
 * Schleede et al., "Plasma flow around and charge distribution of a dust
 * cluster in a rf discharge" (arXiv:1801.00972).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or constant
 * generator with the HIP path.
 *
 * Every function follows the method section of the paper (Sec. III):
 *   - super-particles, kinetic e- and Ar+, neutral Ar reservoir (Sec. III, first paragraphs)
 *   - leapfrog push, Eq. (1)-(2)
 *   - Poisson on cell corners, Eq. (3)-(4), CIC charge assignment and field gather
 *   - PPPM near-grain field, Eq. (5)-(6), with dt_MD = dt/40
 *   - perfect absorbers: electrodes and grains; grain charge in quanta of the
 *     super-particle charge (Sec. IV.B)
 *   - binary Monte-Carlo collisions against the neutral reservoir (Table I), in
 *     the null-collision form with constant cross sections.
 * Where the paper is silent, the reading taken is the one listed in the
 * design notes of the repository (leapfrog start, step order, Philox usage,
 * wall-node stencil, MD-region extent, ...).
 *
 * Units: SI, except particle positions which are in cell units (x / dx).
 * Species index: 0 = electron, 1 = Ar+.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* test-mode flags */
#define ORC_NO_MESH      1  /* no deposit / Poisson: mesh field identically 0 */
#define ORC_NO_MCC       2  /* no collisions */
#define ORC_FIXED_POINT  4  /* CIC deposit in int64 fixed point (2^-32 e units) */
#define ORC_FROZEN_Q     8  /* grain charges do not change when particles hit */
#define ORC_IMMOBILE_IONS 16 /* ions are deposited but never moved or collided */
#define ORC_NO_MD       32  /* grains act only as CIC charges on the mesh: no MD
                               region, no sub-cycling, no absorption */

typedef struct orc_config {
  int32_t nx, ny, nz;        /* cells; x,y periodic, z bounded by two electrodes */
  int32_t ppc_e, ppc_i;      /* macro-particles per cell at load */
  int32_t n_grains;
  int32_t cutoff;            /* MD cube half-width c, in cells */
  int32_t md_sub;            /* sub-steps per step in the MD region (40) */
  int32_t flags;             /* ORC_* test modes */
  int32_t coulomb_interval;  /* Coulomb collisions every this many steps (0: none) */
  double dx, dt;             /* m, s */
  double n0;                 /* plasma density setting the macro-particle weight */
  double Te_eV, Ti_eV;       /* load temperatures, kT in eV */
  double p_gas, T_gas;       /* neutral reservoir: Pa, K */
  double sigma_e, sigma_i;   /* e-Ar elastic, Ar+-Ar charge exchange, m^2 */
  double V_dc, V_rf, f_rf;   /* phi(z=L_z, t) = V_dc + V_rf sin(2 pi f_rf t) */
  double grain_radius;       /* m */
  double E_cap_eV;           /* null-collision cap on the relative kinetic energy */
  double Q_frozen_e;         /* grain charge in e when ORC_FROZEN_Q is set */
  double coulomb_lnL;        /* Coulomb logarithm of the charged-particle collisions */
  /* energy-dependent cross sections (xs_n = 0: the constant sigma_e, sigma_i
     above, e-Ar elastic and Ar+-Ar charge exchange only).  One energy grid,
     the projectile's energy with the target at rest (eV), increasing;
     sigma(E) linear between the points and constant past the ends. */
  int32_t xs_n;
  int32_t pad1;
  const double* xs_E;        /* [xs_n] eV */
  const double* xs_e_el;     /* [xs_n] e-Ar elastic, m^2 */
  const double* xs_e_ex;     /* [xs_n] e-Ar excitation, m^2, nullable */
  const double* xs_i_cx;     /* [xs_n] Ar+-Ar charge exchange, m^2 */
  const double* xs_i_el;     /* [xs_n] Ar+-Ar elastic (isotropic), m^2, nullable */
  double E_ex_eV;            /* excitation energy */
  uint64_t seed;             /* Philox key */
  const double* grain_pos;   /* [n_grains][3], cell units */
  /* electron-impact ionisation (Table I: e + Ar -> Ar+ + 2e), with the tables
     above: sigma on the same energy grid (nullable: none) and the threshold */
  const double* xs_e_iz;     /* [xs_n] m^2, nullable */
  double E_iz_eV;            /* ionisation energy */
} orc_config;

typedef struct orc_derived {
  double w;                  /* real particles per macro-particle */
  int64_t Qp;                /* macro-particle charge in units of 2^-32 e */
  double n_gas;              /* neutral density */
  double q[2], m[2];
  double vth[2];             /* per-component thermal speed sqrt(kT/m) at load */
  double g_cap[2];           /* relative-speed cap of the null-collision method */
  double P_null[2];          /* candidate probability per step */
  uint64_t T_null[2];        /* integer candidate threshold floor(P * 2^32) */
  double vth_gas;            /* sqrt(kB T_gas / M_Ar) */
  double sg_max[2];          /* tables: max over g <= g_cap of g sigma_total */
} orc_derived;

typedef struct orc_state {
  int64_t n[2];              /* particles per species (array lengths) */
  double* pos[2];            /* [n][3] cell units */
  double* vel[2];            /* [n][3] m/s, at the half step k-1/2 */
  uint32_t* id[2];           /* Philox counter word 0 */
  uint8_t* alive[2];         /* 1 alive, 0 removed */
  double* margin[2];         /* nullable: smallest margin of a discrete decision */
  int64_t* grain_count;      /* [n_grains][2] absorbed macro-particles */
  int64_t wall_count[2][2];  /* [wall: 0 grounded z=0, 1 rf z=L_z][species] */
  int64_t cap_violation[2];  /* relative speed above g_cap */
  int64_t n_collisions[2];   /* accepted collisions */
  uint32_t step;             /* k: the state holds x_k and v_{k-1/2} */
  uint32_t pad0;
  int64_t md_margin[2];      /* plain pushes with |v_{k+1/2}| dt >= cutoff dx (with grains) */
  int64_t cap[2];            /* array capacity per species (>= n): room for new particles */
  uint32_t next_id[2];       /* id of the next particle an ionisation creates, per species */
  int64_t n_ionizations;     /* ionisations (pairs created) */
} orc_state;

/* ---- building blocks (exposed for the pins) ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int  orc_derive(const orc_config* c, orc_derived* d);
double orc_rf_voltage(const orc_config* c, uint32_t k);
int64_t orc_n_nodes(const orc_config* c);

/* seeded grain placement: n grains uniform in the sphere of `radius` around
 * `center` (cell units) by rejection, each at least min_sep from the grains
 * placed before it; candidate t of grain g proposes c + R (2u - 1) from words
 * 0..2 of Philox(g, t, 7, 0) under `seed`.  out: [n][3]; -1 if a grain finds
 * no room in 2^20 candidates. */
int orc_place_grains(uint64_t seed, int n, const double center[3], double radius, double min_sep,
                     double* out);

/* particle loading: fills pos/vel/id for n = nx*ny*nz*ppc particles per species */
int orc_init_particles(const orc_config* c, orc_state* s);

/* CIC deposit of the alive particles and of the grain charges.
 * FP64 mode: rho in C/m^3.  Fixed-point mode: rho_fixed in 2^-32 e per node. */
int orc_deposit(const orc_config* c, const orc_state* s, double* rho);
int orc_deposit_fixed(const orc_config* c, const orc_state* s, int64_t* rho_fixed);
/* densities n [2][nodes] (m^-3) and fluxes [2][3][nodes] (m^-2 s^-1) */
int orc_moments(const orc_config* c, const orc_state* s, double* n, double* flux);
int orc_fine_moments(const orc_config* c, const orc_state* s, const double origin[3], double h,
                     const int32_t m[3], double* n, double* flux);

/* cross-section tables: sigma of one table at energy E (eV), and the bound
 * max over g <= g_cap of g sigma_total(E(g)) of a species */
double orc_xs_at(const orc_config* c, const double* table, double E_eV);
double orc_xs_sgmax(const orc_config* c, int sp);

/* Coulomb collisions of the charged particles (Table I; binary model of
 * Takizuka and Abe): one pass over all cells at the state's step k, with
 * time step coulomb_interval * dt.  orc_step applies it at the start of
 * every step k with k % coulomb_interval == 0.  Returns the number of
 * binary collisions performed (>= 0) or a negative error. */
int64_t orc_coulomb(const orc_config* c, orc_state* s);
/* one binary collision of the model on the velocities va (species sa) and vb
 * (species sb) with the given rotation draws: delta = tan(theta/2), phi */
void orc_coulomb_pair(const orc_config* c, int sa, int sb, double* va, double* vb, double delta,
                      double phi);
/* the variance of delta = tan(theta/2) for relative speed u, density nL of
 * the partner species and time step dtc */
double orc_coulomb_var(const orc_config* c, int sa, int sb, double u, double nL, double dtc);

/* Poisson: phi on all nodes, Dirichlet phi(k=0)=0, phi(k=nz)=V */
int orc_poisson(const orc_config* c, const double* rho, double V, double* phi);
/* E = -grad phi; E is [3][nodes] */
int orc_efield(const orc_config* c, const double* phi, double* E);
/* fields at the state's step: rho (C/m^3), phi, E; rho_fixed nullable */
int orc_fields(const orc_config* c, const orc_state* s, double* rho, int64_t* rho_fixed,
               double* phi, double* E);
/* unit-charge mesh field of each grain on its (2c+2)^3 node cube: [g][3][(2c+2)^3] */
int orc_unit_fields(const orc_config* c, double* U);
/* phi of a unit (1 C) grain charge on its MD cube's nodes: [g][(2c+2)^3] */
int orc_unit_potentials(const orc_config* c, double* Uphi);
/* the potential on the fine grid of orc_fine_moments (the mesh potential phi
 * interpolated, plus the grains' Coulomb potential minus their unit mesh
 * potential, as in the PPPM field) */
int orc_fine_phi(const orc_config* c, const orc_state* s, const double* phi,
                 const double* Uphi, const double origin[3], double h, const int32_t m[3],
                 double* out);
/* grains whose MD cube contains cell (i,j,k): writes indices, returns the count */
int orc_md_grains(const orc_config* c, int i, int j, int k, int* out, int cap);

/* OML test mode (grain charging, Sec. IV.B): test particles of species sp
 * moved in the field of grain 0 alone (charge Q_frozen_e e, no mesh, no
 * collisions) by the MD sub-step until absorbed or farther than R_c cells from
 * the grain; returns the number absorbed, *n_out those that left, *n_open
 * those still inside after max_calls sub-step calls (see pic_oracle.c) */
int64_t orc_oml_collect(const orc_config* c, int sp, double R_c, int64_t n, double* pos,
                        double* vel, int64_t max_calls, int64_t* n_out, int64_t* n_open);

/* one full time step k -> k+1 (deposit, solve, field, move, absorb, collide);
 * U: the grains' unit fields from orc_unit_fields (nullable without grains) */
int orc_step(const orc_config* c, orc_state* s, const double* U);
/* move particles through a given mesh field E_k ([3][nodes], nullable = 0)
 * without solving, then collide; grains and walls as in orc_step. */
int orc_step_in_field(const orc_config* c, orc_state* s, const double* E, const double* U);

#ifdef __cplusplus
}
#endif
#endif
