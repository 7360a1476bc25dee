/*
 * pic.h -- C ABI of the MI355X (gfx950) PIC-MCC/PPPM hot path.
 *
 * The library advances electrons and Ar+ ions of a capacitively coupled rf
 * argon discharge around a fixed cluster of absorbing dust grains, following
 * the method of Schleede et al., "Plasma flow around and charge distribution
 * of a dust cluster in a rf discharge" (arXiv:1801.00972), Sec. III:
 *   - super-particles of one weight for both kinetic species (Sec. III);
 *   - CIC (box-shape) charge assignment on the cell corners, Poisson's
 *     equation Eq. (3) in 7-point finite-difference form, E = -grad phi by
 *     finite differences, Eq. (4), and the field at the particle by the same
 *     weights (Sec. III);
 *   - leapfrog, Eq. (1)-(2), electric field only;
 *   - PPPM correction near the grains, Eq. (5)-(6), with dt_MD = dt/40;
 *   - electrodes and grains as perfect absorbers, the grain charge changing in
 *     quanta of the super-particle charge (Sec. III end, Sec. IV.B);
 *   - binary Monte-Carlo collisions against a neutral argon reservoir
 *     (Table I: e-Ar elastic, Ar+-Ar charge exchange), null-collision form.
 * Geometry: x,y periodic; z from a grounded electrode (z = 0, phi = 0) to the
 * rf electrode (z = L_z, phi = V_dc + V_rf sin(2 pi f_rf t)) -- the paper's
 * discharge axis y is called z here.
 *
 * Conventions of every call:
 *   - returns PIC_OK (0) or a negative PIC_E* code; no exception or abort
 *     crosses the ABI; pic_last_error() describes the last failure;
 *   - an asynchronous device fault becomes a sticky PIC_EDEVICE;
 *   - the context owns all device memory; callers own every buffer they pass;
 *   - all device work is ordered on the stream given to pic_init (NULL: the
 *     default stream); calls that return host data synchronise that stream;
 *   - a context is not thread-safe; several contexts may coexist;
 *   - SI units; temperatures as kT in eV; particle positions in cell units
 *     (x / dx); node arrays are x-fastest: n = i + nx (j + ny k), k = 0..nz.
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_OK        0
#define PIC_EINVAL   -1  /* bad argument or configuration value */
#define PIC_ECONFIG  -2  /* configuration that cannot be realised (grain placement, sizes) */
#define PIC_ENOMEM   -3  /* device or host allocation failed */
#define PIC_EDEVICE  -4  /* HIP runtime or kernel fault (sticky) */
#define PIC_ENUMERIC -5  /* non-finite or out-of-range particle data */
#define PIC_ESTATE   -6  /* call not valid in the context's state */

/* arithmetic forms */
#define PIC_FP64  0  /* FP64 positions (cell units), velocities, fields and deposit */
#define PIC_FP32R 1  /* int32 cell + FP32 offset, FP32 velocity and field, int64
                        fixed-point deposit (2^-32 e), FP32 Poisson solve with FP64
                        residual refinement */

/* pic_fields selection bits */
#define PIC_PHI       1u  /* double [nodes]                     V        */
#define PIC_E         2u  /* double [3][nodes]                  V/m      */
#define PIC_RHO       4u  /* double [nodes]  plasma + grains    C/m^3    */
#define PIC_RHO_FIXED 8u  /* int64  [nodes]  PIC_FP32R only     2^-32 e  */
#define PIC_N        16u  /* double [2][nodes] e, Ar+           m^-3     */
#define PIC_FLUX     32u  /* double [2][3][nodes] e, Ar+; x,y,z m^-2 s^-1 */
#define PIC_FINE_N   64u  /* double [2][fine nodes]               m^-3     */
#define PIC_FINE_FLUX 128u /* double [2][3][fine nodes]           m^-2 s^-1 */
#define PIC_FINE_PHI 256u /* double [fine nodes]                   V        */

/*
 * One replica.  Read-only; copied by pic_init.
 *   weight w = n0 dx^3 / ppc real particles per macro-particle (both species);
 *   phi(z = nz dx, t_k) = V_dc + V_rf sin(2 pi f_rf k dt), phi(z = 0) = 0;
 *   grain_pos: [n_grains][3] in cell units, each at least cutoff+1 cells from
 *   both electrodes; the MD region of a grain is the cube of (2 cutoff + 1)^3
 *   cells centred on its cell (cutoff 1: the grain's cell and its direct
 *   neighbours, Sec. III);  md_subcycles sub-steps of dt / md_subcycles are taken
 *   inside it (40 in the paper);
 *   E_cap_eV caps the relative kinetic energy used by the null-collision
 *   method (a particle above the cap collides and is counted);
 *   coulomb_interval > 0 switches on the Coulomb collisions between the
 *   charged particles (Table I: e-e, e-Ar+, Ar+-Ar+; the binary model of
 *   Takizuka and Abe cited there): at the start of every step k with
 *   k % coulomb_interval == 0 the particles of each cell are paired at random
 *   and each pair's relative velocity turns by a random angle theta about
 *   itself, delta = tan(theta/2) normal with variance
 *   q_a^2 q_b^2 n_L coulomb_lnL dt_c / (8 pi eps0^2 mu^2 |u|^3), dt_c =
 *   coulomb_interval dt, n_L the density of the less numerous species of
 *   the pair (the species' own for like particles), mu the reduced mass;
 *   momentum and energy are kept.  The pairing: each species' particles in
 *   the order of their Philox keys; like particles in consecutive pairs, an
 *   odd count of three or more starting with a triplet (three collisions at
 *   dt_c / 2); unlike particles j of the more numerous species (electrons on
 *   a tie) with particle j mod N_b of the other, in order of j; e-e, then
 *   Ar+-Ar+, then e-Ar+.  With Coulomb collisions on, steps are launched
 *   directly (no graph replay).
 */
typedef struct pic_config {
  int32_t nx, ny, nz;
  int32_t ppc;                 /* macro-particles per cell per species at load */
  int32_t n_grains;
  int32_t pp_cutoff_cells;
  int32_t md_subcycles;
  int32_t precision;           /* PIC_FP64 or PIC_FP32R */
  int32_t max_refine;          /* FP32R: most residual-refinement sweeps per solve (1..16) */
  int32_t sort_interval;       /* steps between re-binnings of the electrons (0: never; see pic_tuning) */
  double dx, dt;
  double n0;
  double Te_eV, Ti_eV;
  double p_gas_Pa, T_gas_K;
  double sigma_e_el, sigma_i_cx;
  double V_dc, V_rf, f_rf;
  double grain_radius;
  double E_cap_eV;
  double refine_tol;           /* FP32R: the refinement stops once ||b - A phi|| <= refine_tol ||b||
                                  (b with the electrode lift; 0: always max_refine sweeps) */
  uint64_t seed;               /* Philox key of the replica */
  const double* grain_pos;     /* host pointer, [n_grains][3], cell units; NULL: seeded
                                  placement (cluster_center, cluster_radius, grain_min_sep) */
  int32_t coulomb_interval;    /* steps between Coulomb-collision passes (0: none) */
  int32_t reserved0;           /* 0 */
  double coulomb_lnL;          /* Coulomb logarithm (> 0 when coulomb_interval > 0) */
  /* energy-dependent cross sections (xs_n = 0: the constant sigma_e_el and
   * sigma_i_cx above).  Host arrays of xs_n points, copied by pic_init: one
   * energy grid, the projectile's kinetic energy with the target at rest
   * (eV, increasing, >= 0); sigma(E) is linear between the points and
   * constant past the ends.  The null-collision rate bound is the maximum of
   * g sigma_total(E(g)) for relative speeds up to the E_cap_eV speed; the
   * process of a candidate is picked by a uniform draw against the
   * cumulative g sigma_k / bound: electrons elastic, then excitation (only
   * with a centre-of-mass energy above E_ex_eV, which it removes; isotropic
   * scattering in the centre-of-mass frame, neutral at rest); ions charge
   * exchange, then isotropic elastic scattering in the centre-of-mass frame
   * of ion and drawn neutral (Table I's e + Ar elastic, excitation,
   * Ar+ + Ar charge exchange and elastic; ionisation is not provided). */
  int32_t xs_n;                /* 0, or 2 .. PIC_MAX_XS points */
  int32_t reserved1;           /* 0 */
  const double* xs_E;          /* [xs_n] eV */
  const double* xs_e_el;       /* [xs_n] e-Ar elastic, m^2 */
  const double* xs_e_ex;       /* [xs_n] e-Ar excitation, m^2, nullable (none) */
  const double* xs_i_cx;       /* [xs_n] Ar+-Ar charge exchange, m^2 */
  const double* xs_i_el;       /* [xs_n] Ar+-Ar elastic, m^2, nullable (none) */
  double E_ex_eV;              /* excitation energy (>= 0) */
  /* seeded grain placement, used when grain_pos is NULL and n_grains > 0 (the
   * paper's 44 measured positions exist only in a figure): the grains are
   * uniform in the sphere of cluster_radius around cluster_center (cell
   * units), drawn by rejection with every grain at least grain_min_sep (cell
   * units) from the grains placed before it; candidate t of grain g takes
   * the uniforms u_a = (w_a + 1/2) 2^-32 of Philox4x32-10 words 0..2 of the
   * counter (g, t, 7, 0) under `seed` and proposes x_a = c_a + R (2 u_a - 1)
   * (FP64, no fused multiply-adds).  pic_grain_positions returns them.
   * PIC_ECONFIG if a grain finds no room in 2^20 candidates; the placed grains
   * must satisfy the grain_pos rules above. */
  double cluster_center[3];
  double cluster_radius;
  double grain_min_sep;
  /* electron-impact ionisation (Table I: e + Ar -> Ar+ + 2e), in the
   * null-collision method with the tables above (xs_n > 0): sigma on the same
   * energy grid (m^2; NULL: no ionisation) and the ionisation energy E_iz_eV.
   * An electron whose centre-of-mass energy exceeds E_iz can ionise (the third
   * electron process after elastic and excitation); the energy left,
   * (mu/2) g^2 - E_iz, is shared: a fraction s, uniform from Philox(id, k, 8,
   * 0) word 0, goes to a new electron (isotropic, words 1 and 2), 1 - s to the
   * scattered one (isotropic, as for elastic scattering), both in the
   * centre-of-mass frame with the neutral at rest; a new ion takes a
   * Maxwellian velocity of T_gas_K (Philox(id, k, 8, 1), Box-Muller).  Both
   * new particles start at the parent's position x_{k+1} with these as
   * v_{k+1/2}; the ionisations of a step take new ids in the order of their
   * parents' ids (from the loaded count, or max id + 1 after pic_set_state).
   * max_particles: slots per species (0: the loaded count, plus a quarter
   * with ionisation); ionisations that find no room are counted in
   * pic_counters.iz_dropped (a run with drops is not valid). */
  const double* xs_e_iz;
  double E_iz_eV;
  int64_t max_particles;
} pic_config;
#define PIC_MAX_XS 4096

typedef struct pic_ctx pic_ctx;

/* Host view of one replica's particle state (for pic_get_state/pic_set_state). */
typedef struct pic_state_view {
  int64_t capacity[2];   /* get: length of the arrays below per species */
  int64_t n[2];          /* get: particles written; set: particles given */
  double* pos[2];        /* [n][3] cell units, x,y in [0,n), z in [0,nz) */
  double* vel[2];        /* [n][3] m/s at the half step k - 1/2 */
  uint32_t* id[2];       /* Philox particle ids, unique per species */
  int64_t* grain_count;  /* [n_grains][2] absorbed (electrons, ions); nullable */
  int64_t wall_count[2][2]; /* [wall 0: z=0, 1: z=L_z][species] */
  uint32_t step;         /* k */
  uint32_t pad0;
} pic_state_view;

typedef struct pic_counters {
  int64_t n_alive[2];
  int64_t wall_count[2][2];
  int64_t cap_violation[2];   /* collisions whose relative speed exceeded g_cap */
  int64_t n_collisions[2];    /* accepted collisions */
  int64_t md_particles[2];    /* particle-steps moved by the sub-cycled MD path */
  uint32_t step;
  int32_t refine_sweeps;      /* FP32R: sweeps in the last solve */
  double refine_residual;     /* FP32R: ||b - A phi|| / ||b|| after the last solve */
  int64_t numeric_bad;        /* particles removed for a non-finite position (0 for valid input) */
  int64_t tile_fallback;      /* particle-steps outside their tile's LDS window (global-memory path) */
  int64_t n_coulomb;          /* binary Coulomb collisions (pairings) performed */
  int64_t refine_unconverged; /* FP32R: solves that ended after max_refine sweeps above refine_tol */
  int64_t md_margin[2];       /* plain (not sub-cycled) particle-steps with |v_{k+1/2}| dt >=
                                 pp_cutoff_cells dx: moves long enough to reach a grain from
                                 outside its MD cube, where no grain test is made (0 without
                                 grains) */
  int64_t n_ionizations;      /* electron-ion pairs created by ionisation */
  int64_t iz_dropped;         /* ionisations that found no room (0 in a valid run) */
} pic_counters;

/*
 * pic_init -- validate and copy n_replicas configurations (n_replicas > 1 is
 * the batched ensemble form), allocate every device buffer, load the
 * particles (ppc per cell, uniform offsets, Maxwellian velocities taken as
 * v_{-1/2}, Philox keyed by the seed), precompute the tridiagonal factors
 * and each grain's unit-charge mesh field, and deposit rho_0.
 * hip_stream: a hipStream_t (NULL: default stream).  *out receives the
 * context (NULL on failure; pic_last_error(NULL) then describes it).
 * Errors: PIC_EINVAL (bad values), PIC_ECONFIG (grains too close to an
 * electrode or cube wider than the box), PIC_ENOMEM, PIC_EDEVICE.
 */
int pic_init(const pic_config* cfgs, int n_replicas, void* hip_stream, pic_ctx** out);

/*
 * pic_step -- advance every replica by n_steps time steps, asynchronously on
 * the context's stream.  One step k -> k+1: solve Eq. (3) for phi_k with the
 * grains' charges on the mesh and phi(L_z) = V(t_k), E_k by Eq. (4), move
 * every particle (Eq. (1)-(2) or the sub-cycled PPPM path of Eq. (5)-(6)),
 * absorb at electrodes and grains, collide with the neutral gas, deposit
 * rho_{k+1}.  Errors: PIC_EINVAL (n_steps < 0), PIC_EDEVICE.
 */
int pic_step(pic_ctx* ctx, int n_steps);

/*
 * pic_grain_charges -- exact absorbed macro-particle counts per grain,
 * counts[g][0] electrons, counts[g][1] ions (host buffer of 2 n_grains
 * int64), and, if Q_C is not NULL, the grain charges Q_g = (C_i - C_e) w e in
 * coulomb (host buffer of n_grains doubles).  Synchronises the stream.
 */
int pic_grain_charges(pic_ctx* ctx, int replica, int64_t* counts, double* Q_C);

/*
 * pic_energy -- FP64 energy diagnostic of a replica at the current step k
 * (solving for E_k if needed): out[0], out[1] the kinetic energies
 * sum_p (1/2) m_s w |v_p|^2 of the electrons and ions (J; v at k - 1/2, as
 * stored), out[2] the field energy (eps0 / 2) sum_n |E_n|^2 V_n (J; E_k as
 * stored, V_n = dx^3, half on the two electrode planes), out[3] their sum.
 * Summed in FP64 in a fixed order (repeatable).  Synchronises the stream.
 */
int pic_energy(pic_ctx* ctx, int replica, double out[4]);

/* pic_grain_positions -- the grains of a replica, [n_grains][3] in cell units
 * (host buffer): grain_pos as given, or the seeded placement's result. */
int pic_grain_positions(pic_ctx* ctx, int replica, double* pos);

/*
 * pic_fields -- the mesh quantities at the current step k for the current
 * particle state (solving if needed): out[b] receives the quantity of the
 * b-th set bit of `what`, in the order PHI, E, RHO, RHO_FIXED, N, FLUX,
 * FINE_N, FINE_FLUX, FINE_PHI (the last three on the fine grid of pic_set_fine_grid).
 * Buffers are host pointers (out_on_device = 0, the call synchronises) or
 * device pointers on the context's device (out_on_device = 1,
 * stream-ordered).  Every array is x-fastest over the nx ny (nz+1) nodes.
 * N and FLUX are the particle densities and fluxes of the paper's results
 * (Sec. IV, densities and ion and electron fluxes): per species s and node,
 * n_s = (w / dx^3) sum_p W_p and flux_s = (w / dx^3) sum_p v_p W_p, with W_p
 * the particle's cloud-in-cell weight for the node (the charge assignment of
 * Sec. III) at x_k, and v_p the stored half-step velocity v_{k-1/2}.  They
 * are computed on request (summed in FP64 with atomics, so the last bits
 * depend on the order of additions) and are not part of pic_step.
 * Errors: PIC_EINVAL (bad replica, NULL buffer, RHO_FIXED without FP32R,
 * unknown bits), PIC_ESTATE (FINE bits without a fine grid).
 */
int pic_fields(pic_ctx* ctx, int replica, unsigned what, void* const* out, int out_on_device);

/*
 * pic_fields_static -- pic_fields for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same quantities, order and layouts, but staged in a
 * fixed device array of the library (48 MiB, 6 Mi doubles, one per GPU, held
 * until the process ends) instead of context buffers allocated on first use;
 * the call itself allocates nothing.  Only PIC_PHI, PIC_E, PIC_RHO,
 * PIC_RHO_FIXED, PIC_N and PIC_FLUX are accepted; the selection must fit
 * the array: 4 doubles per node with N or FLUX, else 3 with E, 2 with RHO or
 * RHO_FIXED (N or FLUX up to 1,572,864 nodes).  Every call on a GPU uses
 * that GPU's one array, so calls that overlap on one GPU (several streams,
 * threads or contexts) race; calls ordered on one stream do not.  With
 * out_on_device = 1 the call is stream-ordered and does not synchronise.
 * Errors: as pic_fields, plus PIC_EINVAL (a bit outside the list, or a
 * selection larger than the array) and PIC_ESTATE (the array's address could
 * not be resolved at pic_init).
 */
int pic_fields_static(pic_ctx* ctx, int replica, unsigned what, void* const* out,
                      int out_on_device);

/*
 * Time- and rf-phase-averaged diagnostics (the averaged densities, fluxes and
 * potential of the paper's results, Sec. IV: ion fluxes averaged over rf
 * periods, electron fluxes resolved in rf phase).
 *
 * pic_average -- interval > 0 clears the averages of every replica and
 * starts sampling: at the start of the next step k and then of every
 * interval-th step, phi_k and the moments of PIC_N and PIC_FLUX (at x_k with
 * v_{k-1/2}, as pic_fields gives them) are added to the sums of rf-phase bin
 * b = floor(phase_bins frac(f_rf k dt)), and the bin's sample count is
 * incremented.  interval = 0 stops sampling and keeps the sums.  Samples
 * run inside pic_step (captured with the step when graphs are on).  Device
 * memory: 9 nodes doubles per bin and replica.
 * Errors: PIC_EINVAL (interval < 0, phase_bins outside 1..PIC_MAX_PHASE_BINS),
 * PIC_ENOMEM.
 *
 * pic_average_read -- the averages of bin `bin` (or over all bins for
 * bin = -1): out[b] receives the quantity of the b-th set bit of `what` (a
 * subset of PIC_PHI | PIC_N | PIC_FLUX, with PIC_FINE_N | PIC_FINE_FLUX |
 * PIC_FINE_PHI when the fine grid was sampled, layouts as in pic_fields), each the
 * sum over samples divided by their number (zeros with no sample).
 * samples (nullable host pointer) receives that number.  Buffers as in
 * pic_fields.  Errors: PIC_EINVAL (bad replica, bin, bits or buffer),
 * PIC_ESTATE (pic_average never started, or FINE bits without fine sums).
 */
#define PIC_MAX_PHASE_BINS 64
int pic_average(pic_ctx* ctx, int interval, int phase_bins);
int pic_average_read(pic_ctx* ctx, int replica, int bin, unsigned what, void* const* out,
                     int out_on_device, int64_t* samples);

/*
 * Fine diagnostic grid (the paper's results, Sec. IV: densities and fluxes
 * over the region of the grains on a cubical grid of 0.08 dx cells, much
 * finer than the PIC cells).
 *
 * pic_set_fine_grid -- sets (g != NULL) or removes (NULL) the fine grid of
 * a replica.  g->origin is the box's lower corner in grid units (cells of
 * dx), g->h the fine cell edge in grid units (> 0), g->cells[a] >= 1 the
 * cells per axis; the fine nodes are origin + h (i, j, k), cells[a] + 1 per
 * axis, x fastest, at most PIC_MAX_FINE_NODES.  The box lies inside the
 * domain: 0 <= origin[a] and origin[a] + cells[a] h <= nx, ny, nz (no
 * periodic wrap).  A particle at x (grid units) whose u = (x - origin) / h
 * lies in [0, cells[a]) on every axis adds its cloud-in-cell weights W for
 * the 8 nodes of its fine cell; other particles add nothing.  Per species:
 * n = (w / (h dx)^3) sum W and flux = (w / (h dx)^3) sum v W, with x_k and
 * v_{k-1/2} as for PIC_N and PIC_FLUX (FP64 sums with atomics).  PIC_FINE_PHI
 * is the potential phi_k at the fine nodes in the split of Eq. (5)-(6): the
 * mesh potential with the node's cloud-in-cell weights (a node on the
 * domain's upper face in the last cell), plus for every grain whose MD cube
 * holds the node's cell Q_g (1 / (4 pi eps0 max(r, a)) - the grain's
 * unit-charge mesh potential at the node).
 * With a fine grid set, pic_fields accepts PIC_FINE_N, PIC_FINE_FLUX and
 * PIC_FINE_PHI (in that order after the PIC quantities), and
 * a later pic_average also samples the fine grid, after which
 * pic_average_read accepts the same bits (their output buffers follow the
 * PIC quantities' in out[]).  Setting or removing the grid drops the fine
 * sums of earlier averaging.  Device memory: 9 doubles per fine node for
 * pic_fields, and 9 per fine node and phase bin while averaging.
 * Errors: PIC_EINVAL (bad replica, h, cells, or a box outside the domain),
 * PIC_ESTATE (averaging is running: stop it with interval 0 first).
 */
typedef struct pic_fine_grid {
  double origin[3];  /* lower corner, grid units */
  double h;          /* fine cell edge, grid units */
  int32_t cells[3];  /* fine cells per axis */
  int32_t reserved;  /* 0 */
} pic_fine_grid;
#define PIC_MAX_FINE_NODES (1L << 26)
int pic_set_fine_grid(pic_ctx* ctx, int replica, const pic_fine_grid* g);

/* pic_destroy -- free the context and all its device memory (NULL is a no-op). */
void pic_destroy(pic_ctx* ctx);

/* pic_last_error -- text of the last failure on ctx (or of the last failed
 * pic_init when ctx is NULL); owned by the library, valid until the next call. */
const char* pic_last_error(const pic_ctx* ctx);

/*
 * Test and checkpoint hooks.
 * pic_get_state copies one replica's particles (device order, not sorted by
 * id), counts and step to host arrays of the given capacities; PIC_EINVAL if
 * a capacity is too small.  pic_set_state replaces them (FP32R: positions are
 * split into cell + FP32 offset and velocities rounded to FP32) and deposits
 * rho for the new state; PIC_ENUMERIC for non-finite data or positions
 * outside the box; PIC_EINVAL if n exceeds the replica's particle capacity.
 */
int pic_get_state(pic_ctx* ctx, int replica, pic_state_view* view);
int pic_set_state(pic_ctx* ctx, int replica, const pic_state_view* view);

/*
 * Checkpoints (exact resume of the long runs of hundreds of rf periods that
 * the paper's results average over, Sec. IV.A).
 * pic_save writes every replica's state to the file `path` (written to
 * path.tmp, then renamed): the particles as pic_get_state gives them, the
 * step k, grain and electrode counts, the event counters, and in the FP32R
 * form the potential the next field solve starts from, together with each
 * replica's configuration.  pic_load replaces every replica's state with a
 * checkpoint's; the context must come from pic_init with the same
 * configurations (same order).  Counters continue from the saved values.
 * Philox draws depend on (seed, id, step) only, so a run of 2n steps and a
 * run of n steps, saved, loaded into a new context and continued for n
 * steps give the same particles: bit for bit in the FP32R form, to round-off
 * in the FP64 form (its deposit adds in floating point in an order that
 * depends on the particles' array order).  Launch settings, the time
 * averages and the fine grid are not part of a checkpoint.
 * pic_load reads and checks the whole file before it changes any replica.
 * Errors: PIC_EINVAL (NULL path, unreadable or unwritable file, not a
 * checkpoint, truncated), PIC_ECONFIG (another number of replicas or a
 * configuration that differs), PIC_ESTATE (pic_load while averaging runs),
 * PIC_EDEVICE.
 */
int pic_save(pic_ctx* ctx, const char* path);
int pic_load(pic_ctx* ctx, const char* path);

/* pic_get_counters -- per-replica diagnostics; synchronises the stream. */
int pic_get_counters(pic_ctx* ctx, int replica, pic_counters* out);

/* pic_derived -- constants the library derived for a replica, for checking:
 * out[0] weight w, out[1] Qp (2^-32 e, as double), out[2] n_gas,
 * out[3..4] g_cap e/i, out[5..6] candidate thresholds e/i (as double). */
int pic_derived(pic_ctx* ctx, int replica, double out[7]);

/*
 * Launch settings.  None of them changes what a step computes: in the FP32R
 * form the particle state (as a set of records) and every count after n steps
 * are bitwise the same under any settings, because each particle's update is
 * a function of its own record and the field alone and the fixed-point
 * deposit is order-free; in the FP64 form the deposit's rounding depends on
 * the particle order.  The array order of the particles depends on them.
 * The particles are kept binned by tiles of 4x4x4 cells; the push stages the
 * field of each tile plus a margin of cells (its window) in LDS.
 *   sort_interval      steps between re-binnings of the electrons (0: never
 *                      after loading); initially pic_config.sort_interval of
 *                      replica 0
 *   ion_sort_interval  the same for the ions; initially 64
 *   tile_margin        the electrons' window margin in cells (0..3; particles
 *                      beyond it take the global-memory path); initially 2
 *   ion_tile_margin    the same for the ions; initially 1
 *   batch_push         1: the pushes of every replica and species run as one
 *                      persistent launch (all replicas FP32R only); initially
 *                      1 for an FP32R ensemble, else 0
 *   batch_blocks       the persistent grid, a multiple of 8 (the XCD count);
 *                      initially 4 per compute unit
 *   use_graphs         1: a step is the replay of a captured HIP graph; 0:
 *                      direct launches; initially 1
 */
typedef struct pic_tuning {
  int32_t sort_interval;
  int32_t ion_sort_interval;
  int32_t tile_margin;
  int32_t ion_tile_margin;
  int32_t batch_push;
  int32_t batch_blocks;
  int32_t use_graphs;
} pic_tuning;

/* pic_get_tuning / pic_set_tuning -- read or replace the settings
 * (synchronises the stream; captured graphs are dropped).  PIC_EINVAL for a
 * value out of range or batch_push on a context that cannot batch. */
int pic_get_tuning(pic_ctx* ctx, pic_tuning* out);
int pic_set_tuning(pic_ctx* ctx, const pic_tuning* t);

/*
 * pic_autotune -- choose the settings by measurement on live steps: starting
 * from the current settings, a coordinate search over sort_interval in
 * {4, 6, 8, 12, 16}, then tile_margin in {1, 2, 3}, then (FP32R contexts)
 * batch_push off or on with batch_blocks of 2, 3, 4 or 6 per compute unit,
 * then use_graphs on or off (the ion settings are kept).  Each trial takes 2
 * untimed steps, then trial_steps steps, each bracketed by HIP events after
 * any graph capture (a multiple of 48 gives every interval the same share of
 * re-binnings).  As the plasma evolves during the search, each candidate is
 * timed between two timings of the incumbent and wins only against their
 * mean.  The best settings are applied.  Every step taken is a real step of
 * the simulation (see the invariance above).  If tried and ms_per_step are
 * given, the first `capacity` trials are written there (incumbent re-timings
 * included); *n_tried (nullable) receives the number of trials.
 * Errors: PIC_EINVAL, PIC_ESTATE (kernel timing enabled), PIC_EDEVICE.
 */
int pic_autotune(pic_ctx* ctx, int trial_steps, pic_tuning* tried, double* ms_per_step,
                 int capacity, int* n_tried);

/*
 * Kernel timing.  pic_profile_enable(ctx, 1) clears the record and brackets
 * every following launch of the selected kernel class with HIP events on the
 * context's stream; pic_profile_read synchronises and returns the summed
 * elapsed time (ms) and the number of launches measured since enabling.
 *   PIC_PROF_PUSH   the streaming gather / push / electrode / candidate / deposit
 *                   kernel (one launch per species and step)
 *   PIC_PROF_FIELD  the whole field stage of a step (RHS, Poisson, E)
 *   PIC_PROF_SORT   the periodic cell sort of both species
 *   PIC_PROF_LISTS  the listed particles of one species: sub-cycled near-grain
 *                   motion and the collisions of the candidates
 *   PIC_PROF_COULOMB  one Coulomb-collision pass of a replica (steps launched
 *                   one replica at a time; in the batched step it is part of
 *                   PIC_PROF_FIELD)
 */
#define PIC_PROF_PUSH  0
#define PIC_PROF_FIELD 1
#define PIC_PROF_SORT  2
#define PIC_PROF_LISTS 3
#define PIC_PROF_COULOMB 4
int pic_profile_enable(pic_ctx* ctx, int on);
int pic_profile_read(pic_ctx* ctx, int kernel_class, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif
