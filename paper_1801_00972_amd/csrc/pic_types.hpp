// pic_types.hpp -- plain-data structures shared by the library's host code and
// its HIP kernels (passed to kernels by value).
#pragma once
#include <cstdint>

namespace pic {

// CODATA 2018
constexpr double kCharge = 1.602176634e-19;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kBoltz = 1.380649e-23;
constexpr double kMassE = 9.1093837015e-31;
constexpr double kAmu = 1.66053906660e-27;
constexpr double kMassAr = 39.948 * kAmu;
constexpr double kPi = 3.14159265358979323846;

// Philox counter word 2: what a draw is for
enum Purpose : uint32_t {
  kInitPos = 1, kInitVel = 2, kColl = 3, kNeutral = 4, kGrain = 7, kIonize = 8
};

// an electron-impact ionisation of the current step, made into particles after
// every particle has moved: the parent's id and slot, its velocity before the
// collision (m/s) and the squared relative speed left to share,
// g^2 - 2 E_iz / mu (m^2/s^2)
struct IzEvent {
  uint32_t id;
  int32_t slot;
  double v[3];
  double gsq;
};

// particle arrays of one species, structure of arrays
struct PartF64 {
  double *x, *y, *z;      // cell units
  double *vx, *vy, *vz;   // m/s
  uint32_t* id;
};
struct PartF32R {
  int32_t* cell;          // i + nx (j + ny k)
  float *ox, *oy, *oz;    // offsets in [0, 1)
  float *vx, *vy, *vz;    // m/s
  uint32_t* id;
};

// phi on the rf electrode at t_k = k dt: V_dc + V_rf sin(2 pi f_rf t_k), with k
// read from device memory so a captured step needs no new arguments
struct RfDrive {
  double V_dc, V_rf, f_rf, dt;
  const uint32_t* step;
};

// per-species work lists and counters of one step (device)
// The particle arrays are binned by tiles of 4x4x4 cells (tiles x fastest,
// then y, then z): tile t owns slots [tstart[t], tstart[t+1]), a multiple of 4
// long, ordered by cell inside the tile and padded with empty slots.  The
// grid of tiles is padded to a multiple of 16 (twice the XCD count) with empty tiles.
// coll and out are segmented the same way: tile t's entries start at tstart[t].
struct WorkLists {
  int32_t* md;        // dense list: slots of particles that start the step in an MD cube
  int32_t* coll;      // slots of collision candidates (tile segments)
  int32_t* out;       // slots of particles outside their tile's LDS window (tile segments)
  int32_t* coll_cnt;  // [ngrid] entries in coll
  int32_t* out_cnt;   // [ngrid] entries in out
  int32_t* tstart;    // [ngrid + 1] first slot of each tile (set by the sort)
  unsigned long long* tally;  // [ngrid + MD blocks][TL_N] accumulated event counts (see
                              // TallyKind); one row per tile, then one per MD block
  int32_t* cnt;       // [0] slots in use, [2] entries in md, [4] scan total of the sort
  int32_t* stray;     // [ngrid] per push block (at its first tile), FP32R: nonzero once a
                      // particle of the block's slots has ended a push outside the block's
                      // window since the last sort (cleared by the sort)
  int ntx, nty, ntz;  // tiles along x, y, z
  int ngrid;          // tiles rounded up to a multiple of 8
};

// per-tile event counts, accumulated since loading; TL_DEAD counts removed
// particles; TL_FAST counts plain (not sub-cycled) pushes with |v| dt >= cutoff dx
// TL_BORN particles created by ionisation (first tile row; one writer)
enum TallyKind {
  TL_W0 = 0, TL_W1, TL_BAD, TL_MD, TL_FALL, TL_COLL, TL_CAP, TL_DEAD, TL_FAST, TL_BORN, TL_N
};

// near-grain (MD) tables of one replica
struct MdTables {
  int n_grains;
  int cutoff;
  int side;                // 2 cutoff + 2 nodes per cube edge
  int bx0, by0, bz0;       // periodic bounding box of all MD cubes (cells)
  int bsx, bsy, bsz;
  const uint32_t* cell_list;  // [bsz][bsy][bsx]: (start << 8) | count
  const int32_t* grain_idx;   // grain indices referenced by cell_list
  const double* gpos;         // [g][3] cell units
  const int32_t* gcell;       // [g][3] floor of gpos
  const double* Q;            // [g] grain charge (C) frozen at the start of the step
  const double* U;            // [g][3][side^3] unit-charge mesh field on the cube
  double* ecorr;              // [bsz][bsy][bsx][8][3] per box cell, rebuilt every step:
                              // E_k - sum_g Q_g U_g on the cell's 8 nodes (V/m), the sum
                              // over the grains whose cube holds the cell
  double a2;                  // grain radius^2 (m^2)
};

// everything the particle kernels need for one species of one replica
struct SpeciesStep {
  int nx, ny, nz, nxy;
  int sp;                  // 0 electron, 1 ion
  int md_sub;
  int margin;              // cells of drift around a tile staged in the LDS window
  double dx;
  double coul_c;           // 1 / (4 pi eps0 dx^2): Coulomb field per charge at one cell
  double qm_dt, dt_dx;     // (q/m) dt, dt/dx
  double qm_h, h_dx;       // the same for the MD sub-step h = dt / md_sub
  double qm;               // q/m
  float qm_dt_f, dt_dx_f;
  // a plain push with |v|^2 >= vfast2 ((cutoff dx / dt)^2; +inf without
  // grains) moves far enough to cross a grain outside its MD cube
  double vfast2;
  float vfast2_f;
  // null-collision MCC
  uint64_t T_null;         // candidate iff Philox word 0 < T_null
  double g_cap;            // relative-speed cap
  double vth_gas;
  double mass_ratio_e;     // m_e / (m_e + M)
  double mass_ratio_n;     // M / (m_e + M)
  // energy-dependent cross sections (xs_n > 0): [6][xs_n] doubles: energy
  // grid (eV), e-Ar elastic, e-Ar excitation, Ar+-Ar charge exchange, Ar+-Ar
  // elastic, e-Ar ionisation (m^2); sg_max bounds g sigma_total; an
  // excitation needs g^2 > ex_g2 = 2 E_ex / mu and leaves g'^2 = g^2 - ex_g2
  const double* xs;
  int xs_n;
  double sg_max;
  double ex_g2;
  // ionisation (electrons with an ionisation table): needs g^2 > iz_g2 =
  // 2 E_iz / mu; events go to iz_ev (iz_cap entries, iz_cnt counts them,
  // including those beyond the capacity); iz_ev == nullptr: none
  double iz_g2;
  IzEvent* iz_ev;
  int* iz_cnt;
  int iz_cap;
  uint32_t key0, key1;
  const uint32_t* step;    // device: the step index k of the replica
  // deposit
  int64_t Qp;              // macro charge, 2^-32 e
  double sign;             // -1 electrons, +1 ions
  long long isign;
};

// both species of one replica for the kernels that follow the push: blocks
// [0, nb) of a launch work on species 0, [nb, 2 nb) on species 1; a tile
// kernel's block b takes the lists of tile b * span (the push blocks' spans)
template <typename PT>
struct SpeciesPair {
  PT P[2];
  SpeciesStep S[2];
  WorkLists L[2];
  int nb;
  int span;
};

// rf-phase binning of the time averages: sums of step k go to bin
// phase_bin(k), `stride` doubles apart; step == nullptr means no binning
struct AvgBins {
  const uint32_t* step;
  double f_rf, dt;
  int nbins;
  long stride;
};

// fine diagnostic grid over a sub-box: lower corner o and cell edge h in
// grid units, m cells per axis; PIC cells lo <= cell < hi can hold a particle
// inside; mx, my nodes along x, y and fn nodes in all (x fastest)
struct FineBox {
  double o[3];
  double h;
  int m[3];
  int lo[3], hi[3];
  long mx, my, fn;
};

// one (replica, species) of a batched push launch
struct PushDescF32 {
  PartF32R P;
  const float4* E;
  long long* rho;
  MdTables md;
  SpeciesStep S;
  WorkLists L;
  int span;   // tiles per push block (push_span)
  int chunk;  // z-layer chunk of the XCD interleaving (push_chunk)
};

// tiles per FP32R push block: pairs along x where the rows of tiles split into
// pairs (the tile grid, a multiple of 16, then still gives a multiple of 8
// blocks); the kernels that read the push's lists use the same span
__host__ __device__ inline int push_span(const WorkLists& L) { return L.ntx % 2 == 0 ? 2 : 1; }

// the chunk of the push blocks' XCD interleaving for a grid of ngrid / span
// blocks: one z-layer of tile spans, cut down to a divisor of the blocks per
// XCD
inline int push_chunk(const WorkLists& L, int span) {
  const int per_xcd = L.ngrid / span / 8;
  int c = L.ntx * L.nty / span;
  c = c < per_xcd ? c : per_xcd;
  if (c < 1) c = 1;
  while (c > 1 && per_xcd % c) --c;
  return c;
}

}  // namespace pic
