// launch.hpp -- host-side entry points of the library's kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "pic_types.hpp"

namespace pic {

// the fixed device scratch array of pic_fields_static (scratch.hip): doubles
// per GPU, 48 MiB; scratch_setup resolves its address on the current device
// (once per device, returns 0 on success), scratch_address returns the kept
// address of a device (nullptr before its set-up)
constexpr size_t kScratchDoubles = size_t(6) << 20;
int scratch_setup(int* device_out, void** addr_out);
void* scratch_address(int device);

// factorisation of the FFT line lengths and lines per block
struct FftPlanHost {
  int nfac_x, fac_x[12];
  int nfac_y, fac_y[12];
  int L_x, L_y;
};

// particles: arrays binned by 4x4x4-cell tile and updated in place (see
// WorkLists); one push block per tile or pair of tiles, the grid padded to a
// multiple of 16
// tiles (plus `extra` padding tiles) rounded up to a multiple of 16
int tile_grid(int nx, int ny, int nz, int extra);
// blocks of the MD kernel; each owns a tally row after the ngrid tile rows
constexpr int kMdTallyRows = 4096;
long sort_keys(int ngrid);                  // ints of sort workspace (tile counts and cursors)
// the streaming kernel of one species (gather, push, walls, candidate test, deposit)
void launch_push_f64(const PartF64& P, const double* E, double* rho, const MdTables& md,
                     const SpeciesStep& S, const WorkLists& L, hipStream_t st);
void launch_push_f32r(const PartF32R& P, const float* E, long long* rho, const MdTables& md,
                      const SpeciesStep& S, const WorkLists& L, hipStream_t st);
// the push of every (replica, species) of an FP32R ensemble in one persistent launch;
// start[d] is the first work item (tile) of descriptor d, start[ndesc] the total;
// queue: 8 ints of device scratch, cleared by the launcher (items dealt per XCD)
void launch_push_batch_f32r(const PushDescF32* descs, const int32_t* start, int ndesc, int grid,
                            int* queue, hipStream_t st);
// the collisions of one species' push candidates (right after its push)
void launch_collide_f64(const PartF64& P, const SpeciesStep& S, const WorkLists& L,
                        hipStream_t st);
void launch_collide_f32r(const PartF32R& P, const SpeciesStep& S, const WorkLists& L,
                         hipStream_t st);
// the listed particles of both species of an FP64 replica, after both
// pushes: outliers and sub-cycled MD motion (each with its collision and
// deposit); each kernel covers both species in one launch
void launch_lists_f64(const PartF64 P[2], const double* E, double* rho, const MdTables& md,
                      const SpeciesStep S[2], unsigned long long* gc, const WorkLists L[2],
                      int do_mcc, hipStream_t st);
// FP32R MD particles: their list (before the push, md_scan_kernel), their
// sub-cycled motion from P into the other record buffers D (beside the push),
// then, with the outliers, their states copied back into P and their
// collisions (after the push): of both species (sp_only -1) or of one
void launch_md_scan_f32r(const PartF32R P[2], const WorkLists L[2], const MdTables& md,
                         const SpeciesStep S[2], int nx, int ny, int nz, hipStream_t st);
void launch_md_move_f32r(const PartF32R P[2], const PartF32R D[2], const float* E,
                         long long* rho, const MdTables& md, const SpeciesStep S[2],
                         unsigned long long* gc, const WorkLists L[2], hipStream_t st);
void launch_lists_f32r(const PartF32R P[2], const PartF32R D[2], const float* E, long long* rho,
                       const MdTables& md, const SpeciesStep S[2], const WorkLists L[2],
                       int do_mcc, int sp_only, hipStream_t st);
// all of that for species sp in one launch, its collision candidates included
// (in place of launch_collide_f32r and launch_lists_f32r for that species)
void launch_species_lists_f32r(const PartF32R P[2], const PartF32R D[2], const float* E,
                               long long* rho, const MdTables& md, const SpeciesStep S[2],
                               const WorkLists L[2], int do_mcc, int sp, hipStream_t st);
// The fields of a step in one launch: phi (from the refined solve's psi,
// lifted with the electrode voltages, when psi is given; otherwise phi is read
// as stored), E = -grad phi into E (FP64 double2 pairs or FP32 float4), the
// MD cells' corrected node fields, and zero_next (nn 8-byte words, may be
// null) cleared for the next deposit.
void launch_field_out(const double* psi, double* phi, void* E, int e_f64,
                      unsigned long long* zero_next, const MdTables& md, int nx, int ny, int nz,
                      double dx, RfDrive rf, hipStream_t st);
void launch_init_f64(const PartF64& P, int n, int ppc, int nx, int ny, int sp, uint32_t k0,
                     uint32_t k1, double vth, hipStream_t st);
void launch_init_f32r(const PartF32R& P, int n, int ppc, int nx, int ny, int sp, uint32_t k0,
                      uint32_t k1, double vth, hipStream_t st);
// deposit of the current positions through the tile windows (arrays freshly sorted)
void launch_deposit_f64(const PartF64& P, double* rho, const MdTables& md, const SpeciesStep& S,
                        const WorkLists& L, hipStream_t st);
void launch_deposit_f32r(const PartF32R& P, long long* rho, const MdTables& md,
                         const SpeciesStep& S, const WorkLists& L, hipStream_t st);
// density and flux moments of one species: mom [4][nn] gets W, v W summed per
// node (added to what it holds, in the rf-phase bin of the step if avg.step
// is set); exactly one of P64, P32 is non-null
void launch_moments(const PartF64* P64, const PartF32R* P32, const SpeciesStep& S,
                    const WorkLists& L, double* mom, long nn, const AvgBins& avg,
                    hipStream_t st);
// fine-grid moments of one species: mom [4][fb.fn] gets W, v W of the
// particles inside the box summed per fine node (added as in launch_moments);
// capacity bounds the slots in use
void launch_fine_moments(const PartF64* P64, const PartF32R* P32, const WorkLists& L,
                         const FineBox& fb, double* mom, const AvgBins& avg, long capacity,
                         hipStream_t st);
// Coulomb collisions (coulomb.hip).  Work buffers of a replica: per species
// the per-cell counts turned into range starts [ncell + 1], fill cursors
// [ncell], each tile's own particles per cell [ncell] (the counting kernel's
// histograms, for the scatter), the (order key, slot) entries [cap] and the
// slots in key order [cap]; the scan's block sums [coulomb_scan_sums(ncell)];
// the pairings performed (accumulated).
struct CoulombBufs {
  int* start[2];
  int* fill[2];
  int* thist[2];
  unsigned long long* key[2];
  int* slot[2];
  int* ord[2];
  int* sums;
  unsigned long long* count;
};
// constants of a pass: pair kinds 0 e-e, 1 Ar+-Ar+, 2 e-Ar+; the variance of
// delta is c_var[kind] n_L / |u|^3 with n_L = (particles) w_vol; species s of
// a pair changes by +- frac[kind][s] du; ncell counts the cells in the tile
// order of the particle bins (64 a tile, the start arrays hold ncell + 1)
struct CoulombConst {
  int ncell;
  uint32_t key0, key1;
  const uint32_t* step;
  double w_vol;
  double c_var[3];
  double frac[3][2];
};
long coulomb_scan_sums(long ncell);
// one pass over both species of a replica; exactly one of P64, P32 is non-null
// (each then points to the two species' arrays); cap bounds the slots in use
void launch_coulomb(const PartF64* P64, const PartF32R* P32, const WorkLists L[2],
                    const CoulombBufs& B, const CoulombConst& C, const long cap[2],
                    hipStream_t st);
// time averages: phi added to its rf-phase bin (avg.stride apart), and one
// sample counted in cnt[bin]
void launch_avg_phi(const double* phi, double* acc, long nn, const AvgBins& avg,
                    unsigned long long* cnt, hipStream_t st);
// out[u] = (sum over bins b0..b1-1 of acc[b stride + u]) / (samples in those
// bins), times wv for u >= n_plain (the moments), for u < total
void launch_avg_out(const double* acc, int b0, int b1, long stride, long total, long n_plain,
                    const unsigned long long* cnt, double wv, double* out, hipStream_t st);
// counting sort of the slots in use into dst (dropping empty slots, padding
// every tile to a multiple of 4); capacity bounds the slots in use
void launch_sort_f64(const PartF64& src, const PartF64& dst, const WorkLists& L, int* hist,
                     int* sums, long capacity, hipStream_t st);
void launch_sort_f32r(const PartF32R& src, const PartF32R& dst, const WorkLists& L, int* hist,
                      int* sums, long capacity, hipStream_t st);
void launch_fill_int(int* a, long n, int v, hipStream_t st);
// the step's ionisations made into particles (one block; see ionize_kernel):
// exactly one of the FP64 and FP32R pointer pairs is non-null
void launch_ionize(const PartF64* Pe64, const PartF64* Pi64, const PartF32R* Pe32,
                   const PartF32R* Pi32, const WorkLists& Le, const WorkLists& Li,
                   const SpeciesStep& Se, uint32_t* next_id, long room_e, long room_i,
                   unsigned long long* dropped, hipStream_t st);
// FP64 energy diagnostic: per-block sums (energy_blocks() of them) of |v|^2
// over a species' live particles, and of |E|^2 times each node's share of a
// cell volume over the mesh (E as stored: double pairs if e_f64, else float4)
int energy_blocks();
void launch_energy(const PartF64* P64, const PartF32R* P32, const WorkLists& L, double* out,
                   hipStream_t st);
void launch_field_energy(const void* E, int e_f64, long nxy, int nz, double* out, hipStream_t st);
// the step counter advances and the dense MD lists of both species start
// empty for the next step
void launch_advance_step(uint32_t* step, int32_t* cnt0, int32_t* cnt1, hipStream_t st);

// mesh
void launch_solve_f64(const FftPlanHost& P, int nx, int ny, int nz, const double* b, void* work,
                      const void* tw_x, const void* tw_y, const void* inv, double* phi, RfDrive rf,
                      hipStream_t st);
void launch_solve_refined(const FftPlanHost& P, int nx, int ny, int nz, const double* b,
                          double* psi, double* r, void* work32, const void* tw_x32,
                          const void* tw_y32, const void* inv, RfDrive rf, int sweeps,
                          double tol, double* norms, int* ctl, hipStream_t st,
                          bool have_r0 = false);
// one grain's share of the FP32R right-hand side: interior node `node` (the
// index into b), grain g, the fixed-point part of its charge quantum at that
// corner; a replica's table is sorted by node, then by grain and corner
struct GrainShare {
  long long part;
  int node;
  int g;
};
// the FP32R right-hand side (fixed-point rho and the grains' shares, tab)
// and the first residual with its norm partials (partials = norms + 2 of the
// refined solve, which then runs with have_r0); also freezes Q_g
void launch_rhs_residual(const long long* rho, double scale, const GrainShare* tab, int ntab,
                         const unsigned long long* counts, int ng, double we, double* Q,
                         double* b, const double* psi, double* r, int nx, int ny, int nz,
                         double* partials, hipStream_t st);
// the arguments of the FP32R right-hand side (launch_rhs_residual's)
struct RhsArgs {
  const long long* rho;
  double scale;
  const GrainShare* tab;
  int ntab;
  const unsigned long long* counts;
  int ng;
  double we;
  double* Q;
};
// launch_rhs_residual + launch_solve_refined(..., have_r0 = true) in fewer
// kernels where the plane transforms fit in LDS (same phi, psi and Q; the
// norms' partial sums are grouped differently).  With defer_final the
// residual after the last sweep and its test are left to the caller where that
// path applies (returns 1; launch_refine_final), else returns 0.  first_done
// (may be null) is recorded on st after the right-hand side's kernel; -1 if
// that record fails.
int launch_rhs_solve_refined(const RhsArgs& a, const FftPlanHost& P, int nx, int ny, int nz,
                             double* b, double* psi, double* r, void* work32,
                             const void* tw_x32, const void* tw_y32, const void* inv, RfDrive rf,
                             int sweeps, double tol, double* norms, int* ctl, hipStream_t st,
                             bool defer_final, hipEvent_t first_done);
// the residual after the last of `sweeps` refinement sweeps and its stopping
// test (norms, ctl as launch_solve_refined); psi and b unchanged since the solve
void launch_refine_final(int nx, int ny, int nz, const double* b, const double* psi, double* r,
                         int sweeps, double tol, double* norms, int* ctl, hipStream_t st);
void launch_rhs_f64(const double* rho, double scale, double* b, int nx, int ny, int nz,
                    hipStream_t st);
void launch_grain_rhs(const unsigned long long* counts, const double* gpos, int ng, int nx, int ny,
                      int nz, double we, double* Q, double* b, double scale, int mode,
                      long long Qp, hipStream_t st);
void launch_unit_rhs(const double* gpos, int g, int nx, int ny, int nz, double scale, double* b,
                     hipStream_t st);
void launch_extract_cube(const double* E, const int* gcell, int g, int c, int nx, int ny, double* U,
                         hipStream_t st);
// phi of the unit-charge solve on grain g's MD cube into Uphi[g][(2c+2)^3]
void launch_extract_cube_phi(const double* phi, const int* gcell, int g, int c, int nx, int ny,
                             double* Uphi, hipStream_t st);
// the potential on the fine grid's nodes (stored, or added to the rf-phase
// bin of the step when avg.step is set); Uphi may be null without grains
void launch_fine_phi(const double* phi, const MdTables& md, const double* Uphi, const FineBox& fb,
                     int nx, int ny, int nz, double dx, double radius, double* out,
                     const AvgBins& avg, hipStream_t st);
void launch_efield_f64(const double* phi, double* E, int nx, int ny, int nz, double dx,
                       hipStream_t st);
void launch_e_out(const double* E64, const float* E32, double* out, long nn, hipStream_t st);
void launch_rho_total(const double* acc64, const long long* accfx, double* tot64, long long* totfx,
                      const unsigned long long* counts, const double* gpos, int ng, int nx, int ny,
                      long nn, long long Qp, hipStream_t st);
void launch_scale(const double* in, const long long* infx, double conv, double* out, long nn,
                  hipStream_t st);
void launch_zero_f64(double* a, long n, hipStream_t st);
void launch_zero_i64(long long* a, long n, hipStream_t st);
void launch_zero_i32(int* a, long n, hipStream_t st);

}  // namespace pic
