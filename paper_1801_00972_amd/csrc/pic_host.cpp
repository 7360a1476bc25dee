// pic_host.cpp -- the C ABI of include/pic.h: configuration checks, derived
// constants, device memory, the per-step launch sequence, readouts and the
// state hooks.  All arithmetic of the step runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "launch.hpp"
#include "pic.h"

using namespace pic;

namespace {

thread_local std::string g_init_error;

struct DevMem {
  std::vector<void*> blocks;
  ~DevMem() {
    for (void* p : blocks) (void)hipFree(p);
  }
};

struct Replica {
  pic_config cfg{};
  std::vector<double> gpos;  // [g][3] cell units
  int nx = 0, ny = 0, nz = 0;
  long nxy = 0, ncell = 0, nn = 0, n_int = 0;
  int prec = PIC_FP64;
  // derived constants
  double w = 0, n_gas = 0, we = 0;
  long long Qp = 0;
  double q[2]{}, m[2]{}, vth[2]{}, g_cap[2]{}, P_null[2]{};
  uint64_t T_null[2]{};
  // energy-dependent cross sections: host copy [5][n] (grid, e elastic,
  // e excitation, ion charge exchange, ion elastic), device copy, the bounds
  std::vector<double> xs;
  double* d_xs = nullptr;
  // electron-impact ionisation (an ionisation table given): the step's
  // events, their count, the next ids per species, events lost (no room)
  bool ionize = false;
  IzEvent* d_iz = nullptr;
  int* d_iz_cnt = nullptr;
  int iz_cap = 0;
  uint32_t* d_next_id = nullptr;
  unsigned long long* d_iz_drop = nullptr;
  int64_t iz_base = 0;  // ionisations before the last pic_set_state / pic_load
  double sg_max[2]{};
  double vth_gas = 0;
  long n_load = 0;     // particles per species at load
  long cap[2]{};       // slots per species buffer (a multiple of 1024)
  long n_base[2]{};    // particles at load or pic_set_state (alive = n_base - removed)
  // particles: [species][buffer]; updated in place, the other buffer receives the sort
  PartF64 p64[2][2]{};
  PartF32R p32[2][2]{};
  int cur[2]{};        // buffer of each species in use
  int ntiles = 0, ngrid = 0;
  int* d_cnt = nullptr;  // [species][8]: see WorkLists
  WorkLists lists[2]{};
  // mesh
  void* rho[2]{};      // accumulators: double (units w e) or int64 (2^-32 e)
  int rho_cur = 0;
  double* b = nullptr;
  double* phi = nullptr;
  void* E = nullptr;   // double pairs (FP64) or float4 (FP32R)
  double* psi = nullptr;
  double* r = nullptr;
  void* work = nullptr;
  void* tw_x = nullptr;
  void* tw_y = nullptr;
  void* inv = nullptr;
  FftPlanHost fft{};
  double* norms = nullptr;
  int* refine_ctl = nullptr;  // FP32R refinement: [0] converged, [1] sweeps, [2] unconverged solves
  double* tot64 = nullptr;
  long long* totfx = nullptr;
  double* eout = nullptr;
  double* mom = nullptr;  // [species][4][nn] moments for pic_fields
  double* energy = nullptr;  // [3][energy_blocks()] partial sums of pic_energy
  // time averages (pic_average): per rf-phase bin [9][nn] sums of phi, then
  // W, v W of electrons and of ions; samples per bin; the read-out buffer
  double* avg = nullptr;
  unsigned long long* d_avg_cnt = nullptr;
  int avg_cap = 0;  // bins allocated
  double* avg_out = nullptr;
  // fine diagnostic grid (pic_set_fine_grid): moments for pic_fields [2][4][fn],
  // per-bin sums while averaging [bins][2][4][fn] (fine_avg_on: the sums
  // belong to the current box), the read-out buffer
  bool fine_on = false, fine_avg_on = false;
  FineBox fine{};
  double* fine_mom = nullptr;
  double* fine_phi = nullptr;  // [fn] the potential for pic_fields
  double* Uphi = nullptr;      // [g][side^3] unit-charge potentials on the MD cubes
  double* fine_avg = nullptr;
  int fine_cap = 0;
  double* fine_out = nullptr;
  // Coulomb collisions (cfg.coulomb_interval > 0): work buffers of a pass
  CoulombBufs coul{};
  // near-grain tables
  MdTables md{};
  double* d_Q = nullptr;
  GrainShare* d_gtab = nullptr;  // FP32R: the grains' right-hand-side shares (sorted)
  int n_gtab = 0;
  // grain counts; event tallies live per chunk in lists[sp].tally
  unsigned long long* d_gc = nullptr;
  int64_t wall_base[2][2]{};  // electrode counts handed over by pic_set_state
  // sort
  int* d_hist = nullptr;
  int* d_sums = nullptr;
  uint32_t step = 0;       // host mirror of *d_step
  uint32_t* d_step = nullptr;
  int margin[2]{2, 1};     // LDS window margin of the push per species (cells)
  DevMem mem;
};

}  // namespace

struct pic_ctx {
  std::vector<std::unique_ptr<Replica>> reps;
  hipStream_t stream = nullptr;
  std::string err;
  int sticky = 0;
  // kernel timing: event pairs per kernel class
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pairs[5];
  // launch settings (pic_set_tuning)
  pic_tuning tune{};
  int since_sort[2]{};
  // captured steps, by phase (see step_all)
  hipStream_t capture_stream = nullptr;
  // a second stream for the ions' push and collisions in a one-replica step
  // (fork and join events around them on the step's stream)
  hipStream_t species_stream = nullptr;
  hipEvent_t species_fork = nullptr, species_join = nullptr;
  // FP32R MD particles beside the field solve and the push (one replica)
  hipStream_t md_stream = nullptr;
  hipEvent_t md_fork = nullptr, md_join = nullptr;
  hipEvent_t md_scanned = nullptr, md_fields = nullptr;
  // replicas stepped one by one are spread over worker streams (default
  // priority), forked from and joined back into the caller's stream
  std::vector<hipStream_t> workers;
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
  hipGraphExec_t graph[64] = {};
  // time averages: a sample every avg_interval steps (0: off) into avg_bins
  // rf-phase bins; since_avg counts the steps since the last sample
  int avg_interval = 0, avg_bins = 0, since_avg = 0;
  // some replica has Coulomb collisions on
  bool coulomb = false;
  // batched push: descriptors of every (replica, species) for each phase of
  // the buffers (electron, ion, rho), and the first tile of each descriptor
  bool batchable = false;
  int ndesc = 0;
  PushDescF32* d_desc = nullptr;
  int32_t* d_start = nullptr;
  int* d_queue = nullptr;  // the persistent push's 8 work queues
  int n_cu = 256;
  // device of the context, and whether the fixed scratch array of
  // pic_fields_static has its address resolved there
  int device = -1;
  bool scratch_ok = false;
  // per-step GPU timing of the autotuner: events around each step's launches
  std::vector<hipEvent_t>* step_ev = nullptr;
  size_t step_ev_used = 0;
  void drop_graphs() {
    for (hipGraphExec_t& g : graph)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  }
  ~pic_ctx() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    drop_graphs();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    if (species_stream) (void)hipStreamDestroy(species_stream);
    if (species_fork) (void)hipEventDestroy(species_fork);
    if (species_join) (void)hipEventDestroy(species_join);
    if (md_stream) (void)hipStreamDestroy(md_stream);
    if (md_fork) (void)hipEventDestroy(md_fork);
    if (md_join) (void)hipEventDestroy(md_join);
    if (md_scanned) (void)hipEventDestroy(md_scanned);
    if (md_fields) (void)hipEventDestroy(md_fields);
    for (hipStream_t w : workers) (void)hipStreamDestroy(w);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    for (hipEvent_t e : join_ev) (void)hipEventDestroy(e);
    if (d_desc) (void)hipFree(d_desc);
    if (d_start) (void)hipFree(d_start);
    if (d_queue) (void)hipFree(d_queue);
  }
};

namespace {

int fail(pic_ctx* ctx, int code, const std::string& msg) {
  if (ctx) {
    ctx->err = msg;
    if (code == PIC_EDEVICE) ctx->sticky = PIC_EDEVICE;
  } else {
    g_init_error = msg;
  }
  return code;
}

#define HIPCHK(ctx, call)                                                                \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, e_ == hipErrorOutOfMemory ? PIC_ENOMEM : PIC_EDEVICE,             \
                  std::string(#call) + ": " + hipGetErrorString(e_));                    \
  } while (0)

#define CHECK_LAUNCH(ctx) HIPCHK(ctx, hipGetLastError())

template <typename T>
int dalloc(pic_ctx* ctx, Replica& R, T** p, size_t count) {
  void* q = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, PIC_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  R.mem.blocks.push_back(q);
  *p = static_cast<T*>(q);
  return PIC_OK;
}

template <typename T>
void dfree(Replica& R, T*& p) {
  if (!p) return;
  auto& v = R.mem.blocks;
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i] == (void*)p) {
      (void)hipFree(v[i]);
      v.erase(v.begin() + (long)i);
      break;
    }
  p = nullptr;
}

#define TRY(x)               \
  do {                       \
    int rc_ = (x);           \
    if (rc_ != PIC_OK) return rc_; \
  } while (0)

bool factor_len(int N, int* fac, int* nfac) {
  int n = N, k = 0;
  while (n % 4 == 0 && k < 12) { fac[k++] = 4; n /= 4; }
  while (n % 2 == 0 && k < 12) { fac[k++] = 2; n /= 2; }
  while (n % 3 == 0 && k < 12) { fac[k++] = 3; n /= 3; }
  while (n % 5 == 0 && k < 12) { fac[k++] = 5; n /= 5; }
  *nfac = k;
  return n == 1;
}

int lines_per_block(int N, int lines) {
  int L = 1;
  while (L * 2 * N <= 1024 && lines % (L * 2) == 0) L *= 2;
  return L;
}


int periodic_delta(int a, int b, int n) {
  int d = ((a - b) % n + n) % n;
  if (d > n / 2) d -= n;
  return d;
}

// smallest periodic interval [origin, origin + size) covering every marked cell
void periodic_bbox(const std::vector<char>& cov, int n, int* origin, int* size) {
  int best_len = 0, best_end = 0;
  bool any = false;
  for (int i = 0; i < n; ++i) any |= cov[i] != 0;
  if (!any) { *origin = 0; *size = 0; return; }
  // longest circular run of uncovered cells
  for (int s = 0; s < n; ++s) {
    if (cov[s] || !cov[(s - 1 + n) % n]) continue;  // run starts right after a covered cell
    int len = 0;
    while (len < n && !cov[(s + len) % n]) ++len;
    if (len > best_len) { best_len = len; best_end = (s + len) % n; }
  }
  *origin = best_len ? best_end : 0;
  *size = n - best_len;
}

// Seeded grain placement (pic_config.grain_pos == NULL): uniform in the
// sphere of cluster_radius around cluster_center (cell units) by rejection,
// each candidate at least grain_min_sep from every grain placed before it.
// Candidate t of grain g takes three uniforms u_a = (w_a + 1/2) 2^-32 from
// Philox4x32-10 words 0..2 of the counter (g, t, purpose 7, 0) under the
// replica's seed, and proposes x_a = c_a + R (2 u_a - 1).  The arithmetic is
// kept free of fused multiply-adds so that any FP64 implementation of the
// same steps gives the same bits.
int place_grains(const pic_config& c, std::vector<double>& out, std::string& why) {
#pragma clang fp contract(off)
  const int ng = c.n_grains;
  const double R = c.cluster_radius, R2 = R * R, d2 = c.grain_min_sep * c.grain_min_sep;
  const uint32_t k0 = (uint32_t)(c.seed & 0xffffffffu), k1 = (uint32_t)(c.seed >> 32);
  out.assign(3 * (size_t)ng, 0.0);
  for (int g = 0; g < ng; ++g) {
    bool placed = false;
    for (uint32_t t = 0; t < (1u << 20) && !placed; ++t) {
      const uint4 w = philox4x32_10((uint32_t)g, t, kGrain, 0u, k0, k1);
      const uint32_t word[3] = {w.x, w.y, w.z};
      double p[3];
      for (int a = 0; a < 3; ++a) {
        const double u = ((double)word[a] + 0.5) * 2.3283064365386962890625e-10;
        const double s = 2.0 * u - 1.0;
        const double off = R * s;
        p[a] = c.cluster_center[a] + off;
      }
      double r2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        const double d = p[a] - c.cluster_center[a];
        r2 += d * d;
      }
      if (r2 > R2) continue;
      bool far = true;
      for (int h = 0; h < g && far; ++h) {
        double q2 = 0.0;
        for (int a = 0; a < 3; ++a) {
          const double d = p[a] - out[3 * (size_t)h + a];
          q2 += d * d;
        }
        far = q2 >= d2;
      }
      if (!far) continue;
      for (int a = 0; a < 3; ++a) out[3 * (size_t)g + a] = p[a];
      placed = true;
    }
    if (!placed) {
      why = "grain placement failed: no room for grain " + std::to_string(g) +
            " at the minimum separation";
      return PIC_ECONFIG;
    }
  }
  return PIC_OK;
}

int validate(const pic_config& c, std::string& why) {
  auto bad = [&](const std::string& s) { why = s; return PIC_EINVAL; };
  if (c.nx < 2 || c.ny < 2 || c.nz < 2) return bad("nx, ny, nz must be >= 2");
  if (c.nx > 1024 || c.ny > 1024 || c.nz > 2047) return bad("nx, ny <= 1024 and nz <= 2047");
  int f[12], nf;
  if (!factor_len(c.nx, f, &nf) || !factor_len(c.ny, f, &nf))
    return bad("nx and ny must factor into 2, 3 and 5");
  if (c.ppc < 1) return bad("ppc must be >= 1");
  const double np = (double)c.nx * c.ny * c.nz * c.ppc;
  if (np > 2147483647.0) return bad("more than 2^31-1 particles per species");
  if (!(c.dx > 0) || !(c.dt > 0) || !(c.n0 > 0)) return bad("dx, dt and n0 must be > 0");
  if (!(c.Te_eV >= 0) || !(c.Ti_eV >= 0) || !(c.p_gas_Pa >= 0) || !(c.T_gas_K > 0))
    return bad("temperatures and pressure out of range");
  if (!(c.sigma_e_el >= 0) || !(c.sigma_i_cx >= 0) || !(c.E_cap_eV > 0))
    return bad("cross sections must be >= 0 and E_cap > 0");
  if (!std::isfinite(c.V_dc) || !std::isfinite(c.V_rf) || !std::isfinite(c.f_rf))
    return bad("rf drive must be finite");
  if (c.precision != PIC_FP64 && c.precision != PIC_FP32R) return bad("unknown precision");
  if (c.precision == PIC_FP32R && (c.max_refine < 1 || c.max_refine > 16))
    return bad("max_refine must be 1..16");
  if (c.precision == PIC_FP32R && !(std::isfinite(c.refine_tol) && c.refine_tol >= 0))
    return bad("refine_tol must be >= 0");
  if (c.md_subcycles < 1) return bad("md_subcycles must be >= 1");
  if (c.pp_cutoff_cells < 0) return bad("pp_cutoff_cells must be >= 0");
  if (c.n_grains < 0 || c.n_grains > 4096) return bad("n_grains out of range");
  if (c.n_grains > 0 && !c.grain_pos) {
    // seeded placement: the cluster must be a sphere inside the box
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(c.cluster_center[a])) return bad("cluster_center must be finite");
    if (!(std::isfinite(c.cluster_radius) && c.cluster_radius > 0))
      return bad("cluster_radius must be > 0 (grain_pos is NULL)");
    if (!(std::isfinite(c.grain_min_sep) && c.grain_min_sep >= 0))
      return bad("grain_min_sep must be >= 0");
  }
  if (c.n_grains > 0 && !(c.grain_radius > 0)) return bad("grain_radius must be > 0");
  if (c.sort_interval < 0) return bad("sort_interval must be >= 0");
  if (c.xs_n != 0) {
    if (c.xs_n < 2 || c.xs_n > PIC_MAX_XS) return bad("xs_n must be 0 or 2..PIC_MAX_XS");
    if (!c.xs_E || !c.xs_e_el || !c.xs_i_cx) return bad("cross-section tables missing");
    if (!(std::isfinite(c.E_ex_eV) && c.E_ex_eV >= 0)) return bad("E_ex_eV must be >= 0");
    for (int i = 0; i < c.xs_n; ++i) {
      if (!(std::isfinite(c.xs_E[i]) && c.xs_E[i] >= 0) || (i > 0 && !(c.xs_E[i] > c.xs_E[i - 1])))
        return bad("xs_E must be finite, >= 0 and increasing");
      for (const double* t : {c.xs_e_el, c.xs_e_ex, c.xs_i_cx, c.xs_i_el, c.xs_e_iz})
        if (t && !(std::isfinite(t[i]) && t[i] >= 0)) return bad("cross sections must be >= 0");
    }
  }
  if (c.xs_e_iz && (c.xs_n == 0 || !(std::isfinite(c.E_iz_eV) && c.E_iz_eV > 0)))
    return bad("ionisation needs the cross-section tables and E_iz_eV > 0");
  if (c.max_particles < 0 || c.max_particles > 2147483647L - 4L * 1048576L)
    return bad("max_particles out of range");
  if (c.coulomb_interval < 0) return bad("coulomb_interval must be >= 0");
  if (c.coulomb_interval > 0 && !(std::isfinite(c.coulomb_lnL) && c.coulomb_lnL > 0))
    return bad("coulomb_lnL must be > 0");
  // The fixed-point deposit forms Qp * f24 in int64 (f24 < 2^24), so the
  // macro charge Qp = w 2^32 must stay below 2^39: a weight w below 128.
  const double w = c.n0 * c.dx * c.dx * c.dx / (double)c.ppc;
  if (!(std::isfinite(w) && w * 4294967296.0 < 549755813888.0)) {
    why = "weight n0 dx^3 / ppc must be below 128 (fixed-point macro charge below 2^39)";
    return PIC_ECONFIG;
  }
  return PIC_OK;
}

// The FP32R grains' shares of the right-hand side: for each grain its 8 CIC
// nodes (those on interior planes) and the exact fixed-point split of one
// macro charge Qp at its offsets, the split the particle deposit makes, sorted
// by node and then by (grain, corner), the order in which the separate grain
// kernel adds them.  Each step adds scale (net_g part) at the node.
std::vector<GrainShare> grain_shares(const Replica& R) {
  struct Key {
    long node;
    int p;
    GrainShare s;
  };
  std::vector<Key> v;
  const long plane = (long)R.nx * R.ny;
  for (int g = 0; g < R.cfg.n_grains; ++g) {
    const double X = R.gpos[3 * g], Y = R.gpos[3 * g + 1], Z = R.gpos[3 * g + 2];
    const int i0 = (int)std::floor(X), j0 = (int)std::floor(Y), k0 = (int)std::floor(Z);
    const int i1 = i0 + 1 == R.nx ? 0 : i0 + 1, j1 = j0 + 1 == R.ny ? 0 : j0 + 1;
    const int ii[2] = {i0, i1}, jj[2] = {j0, j1};
    const long long qx = (long long)std::floor((X - std::floor(X)) * 16777216.0);
    const long long qy = (long long)std::floor((Y - std::floor(Y)) * 16777216.0);
    const long long qz = (long long)std::floor((Z - std::floor(Z)) * 16777216.0);
    long long part[8], ax[2];
    ax[1] = (R.Qp * qx) >> 24;
    ax[0] = R.Qp - ax[1];
    for (int a = 0; a < 2; ++a) {
      const long long y1 = (ax[a] * qy) >> 24;
      const long long yy[2] = {ax[a] - y1, y1};
      for (int b = 0; b < 2; ++b) {
        const long long z1 = (yy[b] * qz) >> 24;
        part[a + 2 * b] = yy[b] - z1;
        part[a + 2 * b + 4] = z1;
      }
    }
    for (int t = 0; t < 8; ++t) {
      const int a = t & 1, b = (t >> 1) & 1, c = t >> 2;
      const long n = ii[a] + (long)R.nx * (jj[b] + (long)R.ny * (k0 + c));
      const long k = n / plane;
      if (k < 1 || k > R.nz - 1) continue;
      v.push_back(Key{n - plane, 8 * g + t, GrainShare{part[t], (int)(n - plane), g}});
    }
  }
  std::sort(v.begin(), v.end(), [](const Key& x, const Key& y) {
    return x.node != y.node ? x.node < y.node : x.p < y.p;
  });
  std::vector<GrainShare> out;
  for (const Key& k : v) out.push_back(k.s);
  return out;
}

int setup_md(pic_ctx* ctx, Replica& R) {
  const pic_config& c = R.cfg;
  const int ng = c.n_grains, cc = c.pp_cutoff_cells;
  MdTables& md = R.md;
  md.n_grains = ng;
  md.cutoff = cc;
  md.side = 2 * cc + 2;
  md.a2 = c.grain_radius * c.grain_radius;
  TRY(dalloc(ctx, R, &R.d_Q, std::max(ng, 1)));
  md.Q = R.d_Q;
  if (ng == 0) return PIC_OK;
  if (2 * cc + 1 > R.nx || 2 * cc + 1 > R.ny)
    return fail(ctx, PIC_ECONFIG, "MD cube wider than the periodic box");
  std::vector<int> gcell(3 * ng);
  std::vector<char> covx(R.nx, 0), covy(R.ny, 0);
  int zmin = R.nz, zmax = -1;
  for (int g = 0; g < ng; ++g) {
    const double* x = &R.gpos[3 * g];
    if (!(x[0] >= 0 && x[0] < R.nx && x[1] >= 0 && x[1] < R.ny && x[2] >= 0 && x[2] < R.nz))
      return fail(ctx, PIC_ECONFIG, "grain " + std::to_string(g) + " outside the box");
    for (int a = 0; a < 3; ++a) gcell[3 * g + a] = (int)std::floor(x[a]);
    const int gk = gcell[3 * g + 2];
    if (gk - cc < 0 || gk + cc + 1 > R.nz || gk < 1 || gk > R.nz - 2)
      return fail(ctx, PIC_ECONFIG, "grain " + std::to_string(g) + " too close to an electrode");
    for (int d = -cc; d <= cc; ++d) {
      covx[((gcell[3 * g] + d) % R.nx + R.nx) % R.nx] = 1;
      covy[((gcell[3 * g + 1] + d) % R.ny + R.ny) % R.ny] = 1;
    }
    zmin = std::min(zmin, gk - cc);
    zmax = std::max(zmax, gk + cc);
  }
  periodic_bbox(covx, R.nx, &md.bx0, &md.bsx);
  periodic_bbox(covy, R.ny, &md.by0, &md.bsy);
  md.bz0 = zmin;
  md.bsz = zmax - zmin + 1;
  std::vector<uint32_t> cell_list((size_t)md.bsx * md.bsy * md.bsz, 0u);
  std::vector<int32_t> idx;
  for (int z = 0; z < md.bsz; ++z)
    for (int y = 0; y < md.bsy; ++y)
      for (int x = 0; x < md.bsx; ++x) {
        const int i = (md.bx0 + x) % R.nx, j = (md.by0 + y) % R.ny, k = md.bz0 + z;
        const size_t start = idx.size();
        for (int g = 0; g < ng; ++g)
          if (std::abs(periodic_delta(i, gcell[3 * g], R.nx)) <= cc &&
              std::abs(periodic_delta(j, gcell[3 * g + 1], R.ny)) <= cc &&
              std::abs(k - gcell[3 * g + 2]) <= cc)
            idx.push_back(g);
        const size_t cnt = idx.size() - start;
        if (cnt > 255) return fail(ctx, PIC_ECONFIG, "more than 255 grains share an MD cell");
        if (start >= (1u << 24)) return fail(ctx, PIC_ECONFIG, "MD tables too large");
        cell_list[((size_t)z * md.bsy + y) * md.bsx + x] = (uint32_t)(start << 8) | (uint32_t)cnt;
      }
  uint32_t* d_cl;
  int32_t* d_idx;
  double* d_gpos;
  int32_t* d_gcell;
  double* d_U;
  const long cube = (long)md.side * md.side * md.side;
  TRY(dalloc(ctx, R, &d_cl, cell_list.size()));
  TRY(dalloc(ctx, R, &d_idx, std::max<size_t>(idx.size(), 1)));
  TRY(dalloc(ctx, R, &d_gpos, 3 * ng));
  TRY(dalloc(ctx, R, &d_gcell, 3 * ng));
  TRY(dalloc(ctx, R, &d_U, (size_t)ng * 3 * cube));
  TRY(dalloc(ctx, R, &md.ecorr, cell_list.size() * 24));
  HIPCHK(ctx, hipMemcpy(d_cl, cell_list.data(), cell_list.size() * 4, hipMemcpyHostToDevice));
  if (!idx.empty())
    HIPCHK(ctx, hipMemcpy(d_idx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(ctx, hipMemcpy(d_gpos, R.gpos.data(), 3 * ng * 8, hipMemcpyHostToDevice));
  HIPCHK(ctx, hipMemcpy(d_gcell, gcell.data(), 3 * ng * 4, hipMemcpyHostToDevice));
  md.cell_list = d_cl;
  md.grain_idx = d_idx;
  md.gpos = d_gpos;
  md.gcell = d_gcell;
  md.U = d_U;
  if (R.prec != PIC_FP64) {
    const std::vector<GrainShare> tab = grain_shares(R);
    R.n_gtab = (int)tab.size();
    TRY(dalloc(ctx, R, &R.d_gtab, std::max<size_t>(tab.size(), 1)));
    if (!tab.empty())
      HIPCHK(ctx, hipMemcpy(R.d_gtab, tab.data(), tab.size() * sizeof(GrainShare),
                            hipMemcpyHostToDevice));
  }
  return PIC_OK;
}

// FFT twiddles in T and the tridiagonal factors in double (the tridiagonal
// solves run in double in both forms)
template <typename T>
int setup_solver_tables(pic_ctx* ctx, Replica& R, void** tw_x, void** tw_y, void** inv) {
  auto twiddles = [&](int N, void** out) -> int {
    std::vector<T> h(2 * N);
    for (int t = 0; t < N; ++t) {
      const double a = 2.0 * kPi * (double)t / (double)N;
      h[2 * t] = (T)std::cos(a);
      h[2 * t + 1] = (T)std::sin(a);
    }
    T* d;
    TRY(dalloc(ctx, R, &d, 2 * N));
    HIPCHK(ctx, hipMemcpy(d, h.data(), 2 * N * sizeof(T), hipMemcpyHostToDevice));
    *out = d;
    return PIC_OK;
  };
  TRY(twiddles(R.nx, tw_x));
  TRY(twiddles(R.ny, tw_y));
  const int K = R.nz - 1;
  std::vector<double> h((size_t)K * R.nxy);
  for (long mn = 0; mn < R.nxy; ++mn) {
    const int m = (int)(mn % R.nx), n = (int)(mn / R.nx);
    const double sx = std::sin(kPi * m / R.nx), sy = std::sin(kPi * n / R.ny);
    const double diag = -(2.0 + 4.0 * (sx * sx + sy * sy));
    double cprev = 0.0;
    for (int k = 0; k < K; ++k) {
      const double f = 1.0 / (diag - cprev);
      h[(size_t)k * R.nxy + mn] = f;
      cprev = f;
    }
  }
  double* d;
  TRY(dalloc(ctx, R, &d, h.size()));
  HIPCHK(ctx, hipMemcpy(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  *inv = d;
  return PIC_OK;
}

SpeciesStep species_step(const Replica& R, int sp) {
  SpeciesStep S{};
  const pic_config& c = R.cfg;
  S.nx = R.nx;
  S.ny = R.ny;
  S.nz = R.nz;
  S.nxy = (int)R.nxy;
  S.sp = sp;
  S.md_sub = c.md_subcycles;
  S.margin = R.margin[sp];
  S.dx = c.dx;
  S.coul_c = 1.0 / (4.0 * kPi * kEps0 * c.dx * c.dx);
  const double qm = R.q[sp] / R.m[sp];
  const double h = c.dt / (double)c.md_subcycles;
  S.qm = qm;
  S.qm_dt = qm * c.dt;
  S.dt_dx = c.dt / c.dx;
  S.qm_h = qm * h;
  S.h_dx = h / c.dx;
  S.qm_dt_f = (float)S.qm_dt;
  S.dt_dx_f = (float)S.dt_dx;
  {
    const double vf = c.pp_cutoff_cells * c.dx / c.dt;
    S.vfast2 = c.n_grains > 0 ? vf * vf : HUGE_VAL;
    S.vfast2_f = (float)S.vfast2;
  }
  S.T_null = R.T_null[sp];
  S.g_cap = R.g_cap[sp];
  S.vth_gas = R.vth_gas;
  S.mass_ratio_e = R.m[0] / (R.m[0] + R.m[1]);
  S.mass_ratio_n = R.m[1] / (R.m[0] + R.m[1]);
  S.xs = R.d_xs;
  S.xs_n = c.xs_n;
  S.sg_max = R.sg_max[sp];
  S.ex_g2 = 2.0 * c.E_ex_eV * kCharge / (R.m[0] * R.m[1] / (R.m[0] + R.m[1]));
  if (sp == 0 && R.ionize) {
    S.iz_g2 = 2.0 * c.E_iz_eV * kCharge / (R.m[0] * R.m[1] / (R.m[0] + R.m[1]));
    S.iz_ev = R.d_iz;
    S.iz_cnt = R.d_iz_cnt;
    S.iz_cap = R.iz_cap;
  }
  S.key0 = (uint32_t)(c.seed & 0xffffffffu);
  S.key1 = (uint32_t)(c.seed >> 32);
  S.step = R.d_step;
  S.Qp = R.Qp;
  S.sign = sp == 0 ? -1.0 : 1.0;
  S.isign = sp == 0 ? -1 : 1;
  return S;
}

int alloc_particles(pic_ctx* ctx, Replica& R) {
  for (int sp = 0; sp < 2; ++sp)
    for (int bsel = 0; bsel < 2; ++bsel) {
      const long n = R.cap[sp];
      if (R.prec == PIC_FP64) {
        PartF64& P = R.p64[sp][bsel];
        TRY(dalloc(ctx, R, &P.x, n));
        TRY(dalloc(ctx, R, &P.y, n));
        TRY(dalloc(ctx, R, &P.z, n));
        TRY(dalloc(ctx, R, &P.vx, n));
        TRY(dalloc(ctx, R, &P.vy, n));
        TRY(dalloc(ctx, R, &P.vz, n));
        TRY(dalloc(ctx, R, &P.id, n));
      } else {
        PartF32R& P = R.p32[sp][bsel];
        TRY(dalloc(ctx, R, &P.cell, n));
        TRY(dalloc(ctx, R, &P.ox, n));
        TRY(dalloc(ctx, R, &P.oy, n));
        TRY(dalloc(ctx, R, &P.oz, n));
        TRY(dalloc(ctx, R, &P.vx, n));
        TRY(dalloc(ctx, R, &P.vy, n));
        TRY(dalloc(ctx, R, &P.vz, n));
        TRY(dalloc(ctx, R, &P.id, n));
      }
    }
  TRY(dalloc(ctx, R, &R.d_cnt, 16));
  TRY(dalloc(ctx, R, &R.d_step, 1));
  HIPCHK(ctx, hipMemsetAsync(R.d_step, 0, 4, ctx->stream));
  for (int sp = 0; sp < 2; ++sp) {
    WorkLists& L = R.lists[sp];
    L.ntx = (R.nx + 3) / 4;
    L.nty = (R.ny + 3) / 4;
    L.ntz = (R.nz + 3) / 4;
    L.ngrid = R.ngrid;
    TRY(dalloc(ctx, R, &L.md, R.cap[sp]));
    TRY(dalloc(ctx, R, &L.coll, R.cap[sp]));
    TRY(dalloc(ctx, R, &L.out, R.cap[sp]));
    TRY(dalloc(ctx, R, &L.coll_cnt, R.ngrid));
    TRY(dalloc(ctx, R, &L.out_cnt, R.ngrid));
    TRY(dalloc(ctx, R, &L.tstart, R.ngrid + 1));
    TRY(dalloc(ctx, R, &L.tally, TL_N * (R.ngrid + kMdTallyRows)));
    TRY(dalloc(ctx, R, &L.stray, R.ngrid));
    L.cnt = R.d_cnt + 8 * sp;
    HIPCHK(ctx, hipMemsetAsync(L.tally, 0, 8 * TL_N * (R.ngrid + kMdTallyRows), ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(L.tstart, 0, 4 * (R.ngrid + 1), ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(L.stray, 0, 4 * R.ngrid, ctx->stream));
  }
  return PIC_OK;
}

// records an event on the stream when profiling (nullptr otherwise)
hipEvent_t prof_event(pic_ctx* ctx) {
  if (!ctx->prof) return nullptr;
  if (ctx->ev_used == ctx->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->ev_pool.push_back(e);
  }
  hipEvent_t e = ctx->ev_pool[ctx->ev_used++];
  if (hipEventRecord(e, ctx->stream) != hipSuccess) return nullptr;
  return e;
}

void prof_pair(pic_ctx* ctx, int cls, hipEvent_t a, hipEvent_t b) {
  if (a && b) ctx->ev_pairs[cls].push_back({a, b});
}

// rho_cur <- deposit of the current particles (used after loading or set_state)
int deposit_current(pic_ctx* ctx, Replica& R) {
  hipStream_t st = ctx->stream;
  if (R.prec == PIC_FP64) {
    launch_zero_f64((double*)R.rho[R.rho_cur], R.nn, st);
    for (int sp = 0; sp < 2; ++sp)
      launch_deposit_f64(R.p64[sp][R.cur[sp]], (double*)R.rho[R.rho_cur], R.md,
                         species_step(R, sp), R.lists[sp], st);
  } else {
    launch_zero_i64((long long*)R.rho[R.rho_cur], R.nn, st);
    for (int sp = 0; sp < 2; ++sp)
      launch_deposit_f32r(R.p32[sp][R.cur[sp]], (long long*)R.rho[R.rho_cur], R.md,
                          species_step(R, sp), R.lists[sp], st);
  }
  CHECK_LAUNCH(ctx);
  return PIC_OK;
}

// phi_k and E_k from rho_k, the grains' charges and V(t_k); also freezes Q_g.
// zero_next: the same launch clears the other charge accumulator for the
// step's deposit of rho_{k+1}
// final_pending (FP32R): when given, the residual after the last refinement
// sweep and its test may be left to the caller (*final_pending tells), who
// launches them with launch_refine_final on another stream.  first_done
// (FP32R, may be null): recorded on the stream after the right-hand side's
// kernel, so that other work can start beside the rest of the solve.
int solve_fields(pic_ctx* ctx, Replica& R, bool zero_next = false,
                 bool* final_pending = nullptr, hipEvent_t first_done = nullptr) {
  hipStream_t st = ctx->stream;
  const pic_config& c = R.cfg;
  const RfDrive rf{c.V_dc, c.V_rf, c.f_rf, c.dt, R.d_step};
  const double vol = c.dx * c.dx * c.dx;
  unsigned long long* next =
      zero_next ? (unsigned long long*)R.rho[1 - R.rho_cur] : nullptr;  // 8-byte words, 0 = 0.0
  if (R.prec == PIC_FP64) {
    const double scale = -c.dx * c.dx / kEps0 * (R.we / vol);
    launch_rhs_f64((const double*)R.rho[R.rho_cur], scale, R.b, R.nx, R.ny, R.nz, st);
    launch_grain_rhs(R.d_gc, R.md.gpos, c.n_grains, R.nx, R.ny, R.nz, R.we, R.d_Q, R.b, scale, 0,
                     R.Qp, st);
    launch_solve_f64(R.fft, R.nx, R.ny, R.nz, R.b, R.work, R.tw_x, R.tw_y, R.inv, R.phi, rf, st);
    launch_field_out(nullptr, R.phi, R.E, 1, next, R.md, R.nx, R.ny, R.nz, c.dx, rf, st);
  } else {
    const double scale = -c.dx * c.dx / kEps0 * (kCharge / 4294967296.0 / vol);
    const RhsArgs ra{(const long long*)R.rho[R.rho_cur], scale, R.d_gtab, R.n_gtab, R.d_gc,
                     c.n_grains, R.we, R.d_Q};
    const int deferred = launch_rhs_solve_refined(
        ra, R.fft, R.nx, R.ny, R.nz, R.b, R.psi, R.r, R.work, R.tw_x, R.tw_y, R.inv, rf,
        c.max_refine, c.refine_tol, R.norms, R.refine_ctl, st, final_pending != nullptr,
        first_done);
    if (deferred < 0) return fail(ctx, PIC_EDEVICE, "event record in the field solve failed");
    if (final_pending) *final_pending = deferred != 0;
    launch_field_out(R.psi, R.phi, R.E, 0, next, R.md, R.nx, R.ny, R.nz, c.dx, rf, st);
  }
  CHECK_LAUNCH(ctx);
  return PIC_OK;
}

// counting sort of one species into its other buffer (drops empty slots,
// restores the tile order), launched on ctx->stream; the caller flips cur
int enqueue_sort(pic_ctx* ctx, Replica& R, int sp) {
  const int c = R.cur[sp], o = 1 - c;
  if (R.prec == PIC_FP64)
    launch_sort_f64(R.p64[sp][c], R.p64[sp][o], R.lists[sp], R.d_hist, R.d_sums, R.cap[sp],
                    ctx->stream);
  else
    launch_sort_f32r(R.p32[sp][c], R.p32[sp][o], R.lists[sp], R.d_hist, R.d_sums, R.cap[sp],
                     ctx->stream);
  CHECK_LAUNCH(ctx);
  return PIC_OK;
}

// sorts both species now (loading, pic_set_state)
int resort(pic_ctx* ctx, Replica& R) {
  for (int sp = 0; sp < 2; ++sp) {
    TRY(enqueue_sort(ctx, R, sp));
    R.cur[sp] = 1 - R.cur[sp];
  }
  return PIC_OK;
}

// event tallies of one species summed over the tiles
int read_tallies(pic_ctx* ctx, Replica& R, int sp, unsigned long long out[TL_N]) {
  std::vector<unsigned long long> h((size_t)TL_N * (R.ngrid + kMdTallyRows));
  HIPCHK(ctx, hipMemcpy(h.data(), R.lists[sp].tally, h.size() * 8, hipMemcpyDeviceToHost));
  for (int w = 0; w < TL_N; ++w) out[w] = 0;
  for (long c = 0; c < R.ngrid + kMdTallyRows; ++c)
    for (int w = 0; w < TL_N; ++w) out[w] += h[(size_t)TL_N * c + w];
  return PIC_OK;
}

// Buffer phase of a replica: which particle buffer each species uses and
// which rho buffer holds rho_k.  A step is fully described by the phase and
// the species sorted at its end (bit sp of `sorts`).
int phase_of(const Replica& R) { return R.cur[0] | (R.cur[1] << 1) | (R.rho_cur << 2); }

AvgBins avg_bins_of(const pic_ctx* ctx, const Replica& R) {
  return AvgBins{R.d_step, R.cfg.f_rf, R.cfg.dt, ctx->avg_bins, 9 * R.nn};
}

// fine-grid moments of both species added to mom [2][4][fn] (in the
// rf-phase bin of the step when avg.step is set)
int enqueue_fine(pic_ctx* ctx, Replica& R, double* mom, const AvgBins& avg) {
  for (int sp = 0; sp < 2; ++sp) {
    double* m = mom + 4 * R.fine.fn * sp;
    if (R.prec == PIC_FP64)
      launch_fine_moments(&R.p64[sp][R.cur[sp]], nullptr, R.lists[sp], R.fine, m, avg, R.cap[sp],
                          ctx->stream);
    else
      launch_fine_moments(nullptr, &R.p32[sp][R.cur[sp]], R.lists[sp], R.fine, m, avg, R.cap[sp],
                          ctx->stream);
  }
  CHECK_LAUNCH(ctx);
  return PIC_OK;
}

// Coulomb collisions at the start of step k when k % coulomb_interval == 0
bool coulomb_due(const Replica& R) {
  return R.cfg.coulomb_interval > 0 && R.step % (uint32_t)R.cfg.coulomb_interval == 0;
}

int enqueue_coulomb(pic_ctx* ctx, Replica& R) {
  const pic_config& c = R.cfg;
  CoulombConst C{};
  C.ncell = 64 * R.ngrid;
  C.key0 = (uint32_t)(c.seed & 0xffffffffu);
  C.key1 = (uint32_t)(c.seed >> 32);
  C.step = R.d_step;
  C.w_vol = R.w / (c.dx * c.dx * c.dx);
  const double m[2] = {kMassE, kMassAr}, q[2] = {-kCharge, kCharge};
  const double dtc = (double)c.coulomb_interval * c.dt;
  const int kinds[3][2] = {{0, 0}, {1, 1}, {0, 1}};
  for (int t = 0; t < 3; ++t) {
    const int a = kinds[t][0], b = kinds[t][1];
    const double mu = m[a] * m[b] / (m[a] + m[b]);
    const double qq = q[a] * q[b];
    C.c_var[t] = qq * qq * c.coulomb_lnL * dtc / (8.0 * kPi * kEps0 * kEps0 * mu * mu);
    C.frac[t][a] = mu / m[a];
    C.frac[t][b] = mu / m[b];
  }
  const WorkLists L[2] = {R.lists[0], R.lists[1]};
  if (R.prec == PIC_FP64) {
    const PartF64 P[2] = {R.p64[0][R.cur[0]], R.p64[1][R.cur[1]]};
    launch_coulomb(P, nullptr, L, R.coul, C, R.cap, ctx->stream);
  } else {
    const PartF32R P[2] = {R.p32[0][R.cur[0]], R.p32[1][R.cur[1]]};
    launch_coulomb(nullptr, P, L, R.coul, C, R.cap, ctx->stream);
  }
  CHECK_LAUNCH(ctx);
  return PIC_OK;
}

// one sample of the time averages at the start of a step: phi_k and the
// moments of x_k, v_{k-1/2}, into the rf-phase bin of step k
int enqueue_sample(pic_ctx* ctx, Replica& R) {
  hipStream_t st = ctx->stream;
  const AvgBins ab = avg_bins_of(ctx, R);
  launch_avg_phi(R.phi, R.avg, R.nn, ab, R.d_avg_cnt, st);
  for (int sp = 0; sp < 2; ++sp) {
    const SpeciesStep S = species_step(R, sp);
    double* m = R.avg + (1 + 4 * sp) * R.nn;
    if (R.prec == PIC_FP64)
      launch_moments(&R.p64[sp][R.cur[sp]], nullptr, S, R.lists[sp], m, R.nn, ab, st);
    else
      launch_moments(nullptr, &R.p32[sp][R.cur[sp]], S, R.lists[sp], m, R.nn, ab, st);
  }
  if (R.fine_avg_on) {
    // per bin: the potential, then W and v W per species (9 fine-node arrays)
    const AvgBins fb{R.d_step, R.cfg.f_rf, R.cfg.dt, ctx->avg_bins, 9 * R.fine.fn};
    launch_fine_phi(R.phi, R.md, R.Uphi, R.fine, R.nx, R.ny, R.nz, R.cfg.dx, R.cfg.grain_radius,
                    R.fine_avg, fb, ctx->stream);
    TRY(enqueue_fine(ctx, R, R.fine_avg + R.fine.fn, fb));
  }
  CHECK_LAUNCH(ctx);
  return PIC_OK;
}

// slots in use a species may reach with the particles of ionisation, so that
// the next re-binning (each tile padded to a multiple of 4) still fits
long iz_room(const Replica& R) { return R.cap[0] - 4L * R.ngrid; }

// The two species' push and collision kernels depend on each other only
// through the atomically summed charge: in a one-replica context (and not
// while kernels are timed one by one) the ions' go to a second stream,
// forked after the field solve and joined before the list kernels, so that
// one species' latency-bound kernels and launch tails overlap the other's
// streaming.  *forked tells whether the ions' kernels go to ctx->species_stream.
int species_fork(pic_ctx* ctx, bool* forked) {
  *forked = ctx->reps.size() == 1 && !ctx->prof;
  if (!*forked) return PIC_OK;
  if (!ctx->species_stream) {
    HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->species_stream, hipStreamNonBlocking));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->species_fork, hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->species_join, hipEventDisableTiming));
  }
  HIPCHK(ctx, hipEventRecord(ctx->species_fork, ctx->stream));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->species_stream, ctx->species_fork, 0));
  return PIC_OK;
}
int species_join(pic_ctx* ctx, bool forked) {
  if (!forked) return PIC_OK;
  HIPCHK(ctx, hipEventRecord(ctx->species_join, ctx->species_stream));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->species_join, 0));
  return PIC_OK;
}

// The FP32R MD particles of a one-replica step on a stream of their own
// (md_streams makes the stream and its events): md_fork, recorded after the
// field solve's first kernel, starts the scan of their list beside the rest of
// the solve from the cells the previous step left (the pushes, which rewrite
// the cells in place, wait for the scan: md_scanned); their sub-cycled motion
// follows once the fields (and any Coulomb pass) are in place (md_fields) and
// runs beside the pushes; md_done marks the end of that work, which each
// species' stream waits for before its lists kernels copy the states back.
// *forked tells whether ctx->md_stream is used.
int md_streams(pic_ctx* ctx, bool* forked) {
  *forked = ctx->reps.size() == 1 && !ctx->prof;
  if (!*forked) return PIC_OK;
  if (!ctx->md_stream) {
    HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->md_stream, hipStreamNonBlocking));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->md_fork, hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->md_join, hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->md_scanned, hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->md_fields, hipEventDisableTiming));
  }
  return PIC_OK;
}
int md_done(pic_ctx* ctx, bool forked) {
  if (!forked) return PIC_OK;
  HIPCHK(ctx, hipEventRecord(ctx->md_join, ctx->md_stream));
  return PIC_OK;
}
int md_wait(pic_ctx* ctx, bool forked, hipStream_t s) {
  if (!forked) return PIC_OK;
  HIPCHK(ctx, hipStreamWaitEvent(s, ctx->md_join, 0));
  return PIC_OK;
}

// the species' current and other record buffers of an FP32R replica
static void f32_buffers(const Replica& R, PartF32R P[2], PartF32R D[2]) {
  for (int sp = 0; sp < 2; ++sp) {
    P[sp] = R.p32[sp][R.cur[sp]];
    D[sp] = R.p32[sp][1 - R.cur[sp]];
  }
}

// launches one step of a replica on ctx->stream from the host state at the
// start of the step (buffer phases); advance_host then moves the host mirrors
int enqueue_step(pic_ctx* ctx, Replica& R, int sorts, int sample) {
  hipStream_t st = ctx->stream;
  // FP32R: the MD list scan must read the particles' cells as the previous
  // step left them (the pushes rewrite them in place).  With the MD stream it
  // runs first, beside the field solve, and the pushes wait for it; otherwise
  // it runs in line before them.
  bool mdf = false;
  if (R.prec != PIC_FP64) TRY(md_streams(ctx, &mdf));
  hipEvent_t f0 = prof_event(ctx);
  // with the MD stream, the refinement's last residual and test go there too
  // (nothing in the step reads them), off the path to the pushes.  The scan
  // starts once the solve's first kernel is done (md_fork): beside the large
  // plane-transform blocks of that kernel its blocks slowed it by half.
  bool fin = false;
  TRY(solve_fields(ctx, R, true, mdf ? &fin : nullptr, mdf ? ctx->md_fork : nullptr));
  if (mdf) {
    PartF32R P[2], D[2];
    f32_buffers(R, P, D);
    const SpeciesStep S[2] = {species_step(R, 0), species_step(R, 1)};
    HIPCHK(ctx, hipStreamWaitEvent(ctx->md_stream, ctx->md_fork, 0));
    launch_md_scan_f32r(P, R.lists, R.md, S, R.nx, R.ny, R.nz, ctx->md_stream);
    HIPCHK(ctx, hipEventRecord(ctx->md_scanned, ctx->md_stream));
  }
  if (sample) TRY(enqueue_sample(ctx, R));
  prof_pair(ctx, PIC_PROF_FIELD, f0, prof_event(ctx));
  if (coulomb_due(R)) {
    hipEvent_t c0 = prof_event(ctx);
    TRY(enqueue_coulomb(ctx, R));
    prof_pair(ctx, PIC_PROF_COULOMB, c0, prof_event(ctx));
  }
  const int rnx = 1 - R.rho_cur;
  const int do_mcc = 1;
  const SpeciesStep S[2] = {species_step(R, 0), species_step(R, 1)};
  bool forked = false;
  if (R.prec == PIC_FP64) {
    const PartF64 P[2] = {R.p64[0][R.cur[0]], R.p64[1][R.cur[1]]};
    TRY(species_fork(ctx, &forked));
    for (int sp = 0; sp < 2; ++sp) {
      hipStream_t ss = forked && sp == 1 ? ctx->species_stream : st;
      hipEvent_t a = prof_event(ctx);
      launch_push_f64(P[sp], (const double*)R.E, (double*)R.rho[rnx], R.md, S[sp], R.lists[sp], ss);
      hipEvent_t b = prof_event(ctx);
      launch_collide_f64(P[sp], S[sp], R.lists[sp], ss);
      prof_pair(ctx, PIC_PROF_PUSH, a, b);
      prof_pair(ctx, PIC_PROF_LISTS, b, prof_event(ctx));
    }
    TRY(species_join(ctx, forked));
    hipEvent_t b = prof_event(ctx);
    launch_lists_f64(P, (const double*)R.E, (double*)R.rho[rnx], R.md, S, R.d_gc, R.lists, do_mcc,
                     st);
    if (R.ionize)
      launch_ionize(&P[0], &P[1], nullptr, nullptr, R.lists[0], R.lists[1], S[0], R.d_next_id,
                    iz_room(R), iz_room(R), R.d_iz_drop, st);
    prof_pair(ctx, PIC_PROF_LISTS, b, prof_event(ctx));
  } else {
    PartF32R P[2], D[2];
    f32_buffers(R, P, D);
    {
      hipStream_t ms = mdf ? ctx->md_stream : st;
      if (mdf) {
        // the MD kernel needs the fields (and any Coulomb pass); the pushes
        // need the scan done
        HIPCHK(ctx, hipEventRecord(ctx->md_fields, st));
        HIPCHK(ctx, hipStreamWaitEvent(ms, ctx->md_fields, 0));
        HIPCHK(ctx, hipStreamWaitEvent(st, ctx->md_scanned, 0));
      }
      if (fin)
        launch_refine_final(R.nx, R.ny, R.nz, R.b, R.psi, R.r, R.cfg.max_refine,
                            R.cfg.refine_tol, R.norms, R.refine_ctl, ms);
      hipEvent_t m0 = prof_event(ctx);
      if (!mdf) launch_md_scan_f32r(P, R.lists, R.md, S, R.nx, R.ny, R.nz, ms);
      launch_md_move_f32r(P, D, (const float*)R.E, (long long*)R.rho[rnx], R.md, S, R.d_gc,
                          R.lists, ms);
      TRY(md_done(ctx, mdf));
      prof_pair(ctx, PIC_PROF_LISTS, m0, prof_event(ctx));
    }
    TRY(species_fork(ctx, &forked));
    for (int sp = 0; sp < 2; ++sp) {
      hipStream_t ss = forked && sp == 1 ? ctx->species_stream : st;
      hipEvent_t a = prof_event(ctx);
      launch_push_f32r(P[sp], (const float*)R.E, (long long*)R.rho[rnx], R.md, S[sp], R.lists[sp],
                       ss);
      hipEvent_t b = prof_event(ctx);
      // this species' collisions, outliers, and MD particles' states back
      // (once the MD kernel is done) in one launch, while the other species
      // may still stream
      TRY(md_wait(ctx, mdf, ss));
      launch_species_lists_f32r(P, D, (const float*)R.E, (long long*)R.rho[rnx], R.md, S, R.lists,
                                do_mcc, sp, ss);
      prof_pair(ctx, PIC_PROF_PUSH, a, b);
      prof_pair(ctx, PIC_PROF_LISTS, b, prof_event(ctx));
    }
    TRY(species_join(ctx, forked));
    hipEvent_t b = prof_event(ctx);
    if (R.ionize)
      launch_ionize(nullptr, nullptr, &P[0], &P[1], R.lists[0], R.lists[1], S[0], R.d_next_id,
                    iz_room(R), iz_room(R), R.d_iz_drop, st);
    prof_pair(ctx, PIC_PROF_LISTS, b, prof_event(ctx));
  }
  launch_advance_step(R.d_step, R.lists[0].cnt, R.lists[1].cnt, st);
  CHECK_LAUNCH(ctx);
  if (sorts) {
    hipEvent_t s0 = prof_event(ctx);
    for (int sp = 0; sp < 2; ++sp)
      if (sorts & (1 << sp)) TRY(enqueue_sort(ctx, R, sp));
    prof_pair(ctx, PIC_PROF_SORT, s0, prof_event(ctx));
  }
  return PIC_OK;
}

constexpr int kWorkers = 4;  // worker streams for the replicas of an ensemble

// the caller's stream waits for every worker stream (after for_replicas)
int join_replicas(pic_ctx* ctx) {
  const int nw = std::min<int>(kWorkers, (int)ctx->reps.size());
  if (nw <= 1 || ctx->prof) return PIC_OK;
  for (int w = 0; w < nw; ++w) {
    HIPCHK(ctx, hipEventRecord(ctx->join_ev[w], ctx->workers[w]));
    HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->join_ev[w], 0));
  }
  return PIC_OK;
}

// Runs fn(R) for every replica: replica r on worker stream r % kWorkers, after
// an event on the caller's stream, which then waits for every worker (a fork
// and join that graph capture records as dependencies).  The replicas share
// no memory, so their kernels may overlap.  With kernel timing on, or one
// replica, everything stays on the caller's stream.
// With join false the caller's stream does not wait yet: join_replicas()
// does it later, so that work enqueued on the caller's stream meanwhile runs
// beside the replicas' kernels.
template <typename Fn>
int for_replicas(pic_ctx* ctx, Fn fn, bool join = true) {
  const int nw = std::min<int>(kWorkers, (int)ctx->reps.size());
  if (nw <= 1 || ctx->prof) {
    for (auto& R : ctx->reps) TRY(fn(*R));
    return PIC_OK;
  }
  if (ctx->workers.empty()) {
    ctx->workers.assign(nw, nullptr);
    ctx->join_ev.assign(nw, nullptr);
    for (int w = 0; w < nw; ++w) {
      HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->workers[w], hipStreamNonBlocking));
      HIPCHK(ctx, hipEventCreateWithFlags(&ctx->join_ev[w], hipEventDisableTiming));
    }
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
  }
  hipStream_t caller = ctx->stream;
  HIPCHK(ctx, hipEventRecord(ctx->fork_ev, caller));
  for (int w = 0; w < nw; ++w) HIPCHK(ctx, hipStreamWaitEvent(ctx->workers[w], ctx->fork_ev, 0));
  int rc = PIC_OK;
  for (size_t r = 0; r < ctx->reps.size() && rc == PIC_OK; ++r) {
    ctx->stream = ctx->workers[r % nw];
    rc = fn(*ctx->reps[r]);
  }
  ctx->stream = caller;
  if (rc == PIC_OK && join) rc = join_replicas(ctx);
  return rc;
}

// one step of every replica of an FP32R context with the push of all
// replicas and species in one persistent launch (replicas in the same phase)
int enqueue_batch(pic_ctx* ctx, int sorts, int sample) {
  hipStream_t st = ctx->stream;
  const Replica& R0 = *ctx->reps[0];
  hipEvent_t f0 = prof_event(ctx);
  TRY(for_replicas(ctx, [&](Replica& R) -> int {
    // the MD list scan reads the cells as the previous step left them: on the
    // replica's worker stream, joined before the push launch
    {
      PartF32R P[2], D[2];
      f32_buffers(R, P, D);
      const SpeciesStep S[2] = {species_step(R, 0), species_step(R, 1)};
      launch_md_scan_f32r(P, R.lists, R.md, S, R.nx, R.ny, R.nz, ctx->stream);
    }
    TRY(solve_fields(ctx, R, true));
    if (sample) TRY(enqueue_sample(ctx, R));
    if (coulomb_due(R)) TRY(enqueue_coulomb(ctx, R));
    return PIC_OK;
  }));
  CHECK_LAUNCH(ctx);
  prof_pair(ctx, PIC_PROF_FIELD, f0, prof_event(ctx));
  // every replica's MD kernel on the worker streams beside the one push
  // launch (enqueued first, so their waves are resident before the push's
  // blocks fill the rest; the push's items are dealt dynamically)
  TRY(for_replicas(
      ctx,
      [&](Replica& R) -> int {
        PartF32R P[2], D[2];
        f32_buffers(R, P, D);
        const SpeciesStep S[2] = {species_step(R, 0), species_step(R, 1)};
        launch_md_move_f32r(P, D, (const float*)R.E, (long long*)R.rho[1 - R.rho_cur], R.md, S,
                            R.d_gc, R.lists, ctx->stream);
        return PIC_OK;
      },
      false));
  hipEvent_t a = prof_event(ctx);
  launch_push_batch_f32r(ctx->d_desc + (size_t)phase_of(R0) * ctx->ndesc, ctx->d_start, ctx->ndesc,
                         ctx->tune.batch_blocks, ctx->d_queue, st);
  CHECK_LAUNCH(ctx);
  hipEvent_t b = prof_event(ctx);
  TRY(join_replicas(ctx));
  TRY(for_replicas(ctx, [&](Replica& R) -> int {
    hipStream_t ws = ctx->stream;
    const int rnx = 1 - R.rho_cur;
    PartF32R P[2], D[2];
    f32_buffers(R, P, D);
    const SpeciesStep S[2] = {species_step(R, 0), species_step(R, 1)};
    for (int sp = 0; sp < 2; ++sp) launch_collide_f32r(P[sp], S[sp], R.lists[sp], ws);
    launch_lists_f32r(P, D, (const float*)R.E, (long long*)R.rho[rnx], R.md, S, R.lists, 1, -1,
                      ws);
    if (R.ionize)
      launch_ionize(nullptr, nullptr, &P[0], &P[1], R.lists[0], R.lists[1], S[0], R.d_next_id,
                    iz_room(R), iz_room(R), R.d_iz_drop, ws);
    launch_advance_step(R.d_step, R.lists[0].cnt, R.lists[1].cnt, ws);
    return PIC_OK;
  }));
  CHECK_LAUNCH(ctx);
  prof_pair(ctx, PIC_PROF_PUSH, a, b);
  prof_pair(ctx, PIC_PROF_LISTS, b, prof_event(ctx));
  if (sorts) {
    hipEvent_t s0 = prof_event(ctx);
    TRY(for_replicas(ctx, [&](Replica& R) -> int {
      for (int sp = 0; sp < 2; ++sp)
        if (sorts & (1 << sp)) TRY(enqueue_sort(ctx, R, sp));
      return PIC_OK;
    }));
    prof_pair(ctx, PIC_PROF_SORT, s0, prof_event(ctx));
  }
  return PIC_OK;
}

bool replicas_aligned(const pic_ctx* ctx) {
  const int p0 = phase_of(*ctx->reps[0]);
  for (auto& R : ctx->reps)
    if (phase_of(*R) != p0) return false;
  return true;
}

// one step of every replica, launched on ctx->stream
int enqueue_all(pic_ctx* ctx, int sorts, int sample) {
  if (ctx->batchable && ctx->tune.batch_push && replicas_aligned(ctx))
    return enqueue_batch(ctx, sorts, sample);
  return for_replicas(ctx, [&](Replica& R) { return enqueue_step(ctx, R, sorts, sample); });
}

// (re)builds the descriptors of the batched push: for buffer phase ph,
// descriptor 2 r + sp pushes species sp of replica r from its buffer in ph
// and deposits into the rho buffer that ph does not hold
int build_batch(pic_ctx* ctx) {
  ctx->batchable = false;
  for (auto& R : ctx->reps)
    if (R->prec != PIC_FP32R) return PIC_OK;
  const int nd = 2 * (int)ctx->reps.size();
  std::vector<PushDescF32> h((size_t)8 * nd);
  std::vector<int32_t> start(nd + 1, 0);
  for (int ph = 0; ph < 8; ++ph)
    for (int r = 0; r < (int)ctx->reps.size(); ++r) {
      const Replica& R = *ctx->reps[r];
      for (int sp = 0; sp < 2; ++sp) {
        PushDescF32& d = h[(size_t)ph * nd + 2 * r + sp];
        d.P = R.p32[sp][(ph >> sp) & 1];
        d.E = (const float4*)R.E;
        d.rho = (long long*)R.rho[1 - ((ph >> 2) & 1)];
        d.md = R.md;
        d.S = species_step(R, sp);
        d.L = R.lists[sp];
        d.span = push_span(R.lists[sp]);
        d.chunk = push_chunk(R.lists[sp], d.span);
        if (ph == 0) {
          const long total = (long)start[2 * r + sp] + R.ngrid / d.span;
          if (total > 0x7fffffffL) return PIC_OK;  // beyond the int32 item index
          start[2 * r + sp + 1] = (int32_t)total;
        }
      }
    }
  if (!ctx->d_desc) {
    HIPCHK(ctx, hipMalloc(&ctx->d_desc, h.size() * sizeof(PushDescF32)));
    HIPCHK(ctx, hipMalloc(&ctx->d_start, start.size() * sizeof(int32_t)));
    HIPCHK(ctx, hipMalloc(&ctx->d_queue, 8 * sizeof(int)));
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  HIPCHK(ctx, hipMemcpy(ctx->d_desc, h.data(), h.size() * sizeof(PushDescF32),
                        hipMemcpyHostToDevice));
  HIPCHK(ctx, hipMemcpy(ctx->d_start, start.data(), start.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice));
  ctx->ndesc = nd;
  ctx->batchable = true;
  return PIC_OK;
}

void advance_host(Replica& R, int sorts) {
  R.rho_cur = 1 - R.rho_cur;
  R.step += 1;
  for (int sp = 0; sp < 2; ++sp)
    if (sorts & (1 << sp)) R.cur[sp] = 1 - R.cur[sp];
}

// captures the step of `key` = buffer phase | sorts << 3 | sample << 5 into ctx->graph[key]
// without running it: the host phases of the replicas are set to the key for
// the capture and restored after
int capture_step(pic_ctx* ctx, int key) {
  if (ctx->graph[key]) return PIC_OK;
  if (!ctx->capture_stream)
    HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
  std::vector<std::array<int, 3>> saved;
  for (auto& R : ctx->reps) {
    saved.push_back({R->cur[0], R->cur[1], R->rho_cur});
    R->cur[0] = key & 1;
    R->cur[1] = (key >> 1) & 1;
    R->rho_cur = (key >> 2) & 1;
  }
  hipStream_t user = ctx->stream;
  ctx->stream = ctx->capture_stream;
  hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
  int rc = PIC_OK;
  hipGraph_t g = nullptr;
  if (e == hipSuccess) {
    rc = enqueue_all(ctx, (key >> 3) & 3, key >> 5);
    e = hipStreamEndCapture(ctx->stream, &g);
  }
  ctx->stream = user;
  for (size_t r = 0; r < saved.size(); ++r) {
    ctx->reps[r]->cur[0] = saved[r][0];
    ctx->reps[r]->cur[1] = saved[r][1];
    ctx->reps[r]->rho_cur = saved[r][2];
  }
  if (rc != PIC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(ctx, PIC_EDEVICE, "graph capture failed");
  const hipError_t ei = hipGraphInstantiate(&ctx->graph[key], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    ctx->graph[key] = nullptr;
    return fail(ctx, PIC_EDEVICE, "graph instantiation failed");
  }
  return PIC_OK;
}

// the species whose sort falls due at the end of the next step, given the
// steps since each species' last sort
int sorts_due(const pic_ctx* ctx, const int since[2]) {
  const int iv[2] = {ctx->tune.sort_interval, ctx->tune.ion_sort_interval};
  int sorts = 0;
  for (int sp = 0; sp < 2; ++sp)
    if (iv[sp] > 0 && since[sp] + 1 >= iv[sp]) sorts |= 1 << sp;
  return sorts;
}
int due_sorts(const pic_ctx* ctx) { return sorts_due(ctx, ctx->since_sort); }

// The graph keys of the coming steps in the order they fall due, from the
// host state as it is: buffer phases, sorts and samples run ahead (as
// step_all and advance_host move them) over four periods of the schedule,
// which covers every key it reaches.
std::vector<int> upcoming_keys(const pic_ctx* ctx) {
  const Replica& R = *ctx->reps[0];
  int cur[2] = {R.cur[0], R.cur[1]}, rho = R.rho_cur;
  int since[2] = {ctx->since_sort[0], ctx->since_sort[1]}, since_avg = ctx->since_avg;
  long period = 2;
  for (int v : {ctx->tune.sort_interval, ctx->tune.ion_sort_interval, ctx->avg_interval})
    if (v > 1 && period < (1L << 20)) period = std::lcm(period, (long)v);
  const long n = 4 * std::min(period, 1L << 20);
  std::vector<int> keys;
  bool seen[64] = {};
  for (long t = 0; t < n; ++t) {
    const int sorts = sorts_due(ctx, since);
    const int sample = ctx->avg_interval > 0 && since_avg == 0;
    const int key = (cur[0] | (cur[1] << 1) | (rho << 2)) | (sorts << 3) | (sample << 5);
    if (!seen[key]) {
      seen[key] = true;
      keys.push_back(key);
    }
    rho = 1 - rho;
    for (int sp = 0; sp < 2; ++sp) {
      if (sorts & (1 << sp)) cur[sp] = 1 - cur[sp];
      since[sp] = (sorts & (1 << sp)) ? 0 : since[sp] + 1;
    }
    if (ctx->avg_interval > 0) since_avg = (since_avg + 1) % ctx->avg_interval;
  }
  return keys;
}

// one step of every replica: direct launches when profiling (the events must
// bracket single kernels) or when the replicas are in different buffer
// phases, otherwise the replay of the captured graph of the whole step for
// the current phase and sorts, on the caller's stream
int step_all(pic_ctx* ctx) {
  const int sorts = due_sorts(ctx);
  const int sample = ctx->avg_interval > 0 && ctx->since_avg == 0;
  // with step timing on, an event pair brackets the step's launches (after
  // any capture, so host-side capture time is not counted)
  std::vector<hipEvent_t>* ev = ctx->step_ev;
  const bool timed = ev && ctx->step_ev_used + 2 <= ev->size();
  // Coulomb passes fall on some steps only: those contexts launch directly
  if (ctx->prof || !ctx->tune.use_graphs || ctx->coulomb || !replicas_aligned(ctx)) {
    if (timed) HIPCHK(ctx, hipEventRecord((*ev)[ctx->step_ev_used], ctx->stream));
    TRY(enqueue_all(ctx, sorts, sample));
  } else {
    const int key = phase_of(*ctx->reps[0]) | (sorts << 3) | (sample << 5);
    if (!ctx->graph[key]) {
      // the capture stream is not ordered after the caller's stream: the
      // graph's first launch must not overtake work queued there.  Every
      // key the schedule will reach is captured now, so that later steps
      // neither wait for the stream to drain nor for a capture.
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      for (int k : upcoming_keys(ctx)) TRY(capture_step(ctx, k));
      TRY(capture_step(ctx, key));
    }
    if (timed) HIPCHK(ctx, hipEventRecord((*ev)[ctx->step_ev_used], ctx->stream));
    HIPCHK(ctx, hipGraphLaunch(ctx->graph[key], ctx->stream));
  }
  if (timed) {
    HIPCHK(ctx, hipEventRecord((*ev)[ctx->step_ev_used + 1], ctx->stream));
    ctx->step_ev_used += 2;
  }
  for (auto& R : ctx->reps) advance_host(*R, sorts);
  for (int sp = 0; sp < 2; ++sp)
    ctx->since_sort[sp] = (sorts & (1 << sp)) ? 0 : ctx->since_sort[sp] + 1;
  if (ctx->avg_interval > 0) ctx->since_avg = (ctx->since_avg + 1) % ctx->avg_interval;
  return PIC_OK;
}

int check_tuning(const pic_ctx* ctx, const pic_tuning& t, std::string& why) {
  if (t.sort_interval < 0 || t.sort_interval > 1000000) why = "sort_interval out of range";
  else if (t.ion_sort_interval < 0 || t.ion_sort_interval > 1000000)
    why = "ion_sort_interval out of range";
  else if (t.tile_margin < 0 || t.tile_margin > 3) why = "tile_margin must be in 0..3";
  else if (t.ion_tile_margin < 0 || t.ion_tile_margin > 3) why = "ion_tile_margin must be in 0..3";
  else if (t.batch_push != 0 && t.batch_push != 1) why = "batch_push must be 0 or 1";
  else if (t.batch_push && !ctx->batchable) why = "batch_push needs an all-FP32R context";
  else if (t.batch_blocks < 8 || t.batch_blocks % 8 || t.batch_blocks > 65536)
    why = "batch_blocks must be a multiple of 8 in 8..65536";
  else if (t.use_graphs != 0 && t.use_graphs != 1) why = "use_graphs must be 0 or 1";
  return why.empty() ? PIC_OK : PIC_EINVAL;
}

int apply_tuning(pic_ctx* ctx, const pic_tuning& t) {
  std::string why;
  if (check_tuning(ctx, t, why) != PIC_OK) return fail(ctx, PIC_EINVAL, why);
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  const bool margin_changed =
      t.tile_margin != ctx->tune.tile_margin || t.ion_tile_margin != ctx->tune.ion_tile_margin;
  ctx->tune = t;
  for (auto& R : ctx->reps) {
    R->margin[0] = t.tile_margin;
    R->margin[1] = t.ion_tile_margin;
    // the stray flags refer to the old windows: every push block counts as
    // stray until the next sort (the MD list's scan then covers all slots)
    if (margin_changed && R->prec != PIC_FP64)
      for (int sp = 0; sp < 2; ++sp) launch_fill_int(R->lists[sp].stray, R->ngrid, 1, ctx->stream);
  }
  if (margin_changed && ctx->batchable) TRY(build_batch(ctx));
  ctx->drop_graphs();
  return PIC_OK;
}

int unit_fields(pic_ctx* ctx, Replica& R) {
  const pic_config& c = R.cfg;
  const int ng = c.n_grains;
  if (ng == 0) return PIC_OK;
  hipStream_t st = ctx->stream;
  // FP64 solver resources for the unit-charge solves (the FP32R form uses them only here)
  void *tw_x = R.tw_x, *tw_y = R.tw_y, *inv = R.inv, *work = R.work;
  double* E = (double*)R.E;
  if (R.prec != PIC_FP64) {
    TRY(setup_solver_tables<double>(ctx, R, &tw_x, &tw_y, &inv));
    double2* w2;
    TRY(dalloc(ctx, R, &w2, R.n_int));
    work = w2;
    TRY(dalloc(ctx, R, &E, 2 * 2 * R.nn));
  }
  const double scale = -c.dx * c.dx / kEps0 / (c.dx * c.dx * c.dx);
  const long side = 2L * c.pp_cutoff_cells + 2;
  TRY(dalloc(ctx, R, &R.Uphi, (size_t)ng * side * side * side));
  for (int g = 0; g < ng; ++g) {
    launch_zero_f64(R.b, R.n_int, st);
    launch_unit_rhs(R.md.gpos, g, R.nx, R.ny, R.nz, scale, R.b, st);
    launch_solve_f64(R.fft, R.nx, R.ny, R.nz, R.b, work, tw_x, tw_y, inv, R.phi,
                     RfDrive{0.0, 0.0, 0.0, 0.0, R.d_step}, st);
    launch_extract_cube_phi(R.phi, R.md.gcell, g, c.pp_cutoff_cells, R.nx, R.ny, R.Uphi, st);
    launch_efield_f64(R.phi, E, R.nx, R.ny, R.nz, c.dx, st);
    launch_extract_cube(E, R.md.gcell, g, c.pp_cutoff_cells, R.nx, R.ny,
                        const_cast<double*>(R.md.U), st);
  }
  CHECK_LAUNCH(ctx);
  HIPCHK(ctx, hipStreamSynchronize(st));
  return PIC_OK;
}

// sigma of column k of the [5][n] table at E (eV): linear inside the grid,
// the end values outside
double xs_value(const std::vector<double>& xs, int n, int k, double E) {
  const double* x = xs.data();
  const double* t = xs.data() + (long)k * n;
  if (E <= x[0]) return t[0];
  if (E >= x[n - 1]) return t[n - 1];
  const long hi = std::upper_bound(x, x + n, E) - x;  // x[hi - 1] <= E < x[hi]
  const double f = (E - x[hi - 1]) / (x[hi] - x[hi - 1]);
  return t[hi - 1] + f * (t[hi] - t[hi - 1]);
}

// bound of the null-collision method: the maximum over 0 <= E <= E_cap of
// g(E) sigma_total(E), g = sqrt(2 E e / m).  Between grid points sigma_total
// is a + b E, and a sqrt(E) + b E^1.5 is stationary only at E = -a / (3 b);
// past the grid sigma is constant and g increases, so the candidates are the
// grid points, E_cap and those stationary points.
double xs_bound(const std::vector<double>& xs, int n, int sp, double E_cap, double m) {
  const int c0 = sp == 0 ? 1 : 3;
  auto total = [&](double E) {
    return xs_value(xs, n, c0, E) + xs_value(xs, n, c0 + 1, E) + (sp == 0 ? xs_value(xs, n, 5, E) : 0.0);
  };
  auto f = [&](double E) { return total(E) * std::sqrt(2.0 * E * kCharge / m); };
  std::vector<double> cand{0.0, E_cap};
  for (int i = 0; i < n; ++i)
    if (xs[i] <= E_cap) cand.push_back(xs[i]);
  for (int i = 0; i + 1 < n; ++i) {
    const double e0 = xs[i], e1 = xs[i + 1];
    const double b = (total(e1) - total(e0)) / (e1 - e0), a = total(e0) - b * e0;
    if (b < 0) {
      const double Es = -a / (3.0 * b);
      if (Es > e0 && Es < e1 && Es <= E_cap) cand.push_back(Es);
    }
  }
  double best = 0.0;
  for (double E : cand) best = std::max(best, f(E));
  return best;
}

int init_replica(pic_ctx* ctx, Replica& R, const pic_config& cin) {
  std::string why;
  const int vrc = validate(cin, why);
  if (vrc != PIC_OK) return fail(ctx, vrc, why);
  R.cfg = cin;
  if (cin.n_grains > 0 && !cin.grain_pos) {
    const int prc = place_grains(cin, R.gpos, why);
    if (prc != PIC_OK) return fail(ctx, prc, why);
  } else {
    R.gpos.assign(cin.grain_pos, cin.grain_pos + 3 * (size_t)cin.n_grains);
  }
  R.cfg.grain_pos = nullptr;
  pic_config& c = R.cfg;
  R.nx = c.nx;
  R.ny = c.ny;
  R.nz = c.nz;
  R.nxy = (long)c.nx * c.ny;
  R.ncell = R.nxy * c.nz;
  R.nn = R.nxy * (c.nz + 1);
  R.n_int = R.nxy * (c.nz - 1);
  R.prec = c.precision;
  // derived constants (Sec. III: one super-particle weight for both species)
  R.w = c.n0 * c.dx * c.dx * c.dx / (double)c.ppc;
  R.Qp = std::llround(R.w * 4294967296.0);
  R.we = R.w * kCharge;
  R.n_gas = c.p_gas_Pa / (kBoltz * c.T_gas_K);
  R.q[0] = -kCharge;
  R.q[1] = kCharge;
  R.m[0] = kMassE;
  R.m[1] = kMassAr;
  R.vth[0] = std::sqrt(c.Te_eV * kCharge / kMassE);
  R.vth[1] = std::sqrt(c.Ti_eV * kCharge / kMassAr);
  const double sigma[2] = {c.sigma_e_el, c.sigma_i_cx};
  if (c.xs_n > 0) {
    const int n = c.xs_n;
    R.xs.assign(6L * n, 0.0);
    const double* cols[6] = {c.xs_E, c.xs_e_el, c.xs_e_ex, c.xs_i_cx, c.xs_i_el, c.xs_e_iz};
    R.ionize = c.xs_e_iz != nullptr;
    for (int k = 0; k < 6; ++k)
      if (cols[k]) std::copy(cols[k], cols[k] + n, R.xs.begin() + (long)k * n);
    // the caller's arrays are not kept
    c.xs_E = c.xs_e_el = c.xs_e_ex = c.xs_i_cx = c.xs_i_el = c.xs_e_iz = nullptr;
  }
  for (int s = 0; s < 2; ++s) {
    R.g_cap[s] = std::sqrt(2.0 * c.E_cap_eV * kCharge / R.m[s]);
    R.sg_max[s] = c.xs_n > 0 ? xs_bound(R.xs, c.xs_n, s, c.E_cap_eV, R.m[s])
                             : sigma[s] * R.g_cap[s];
    const double nu_max = R.n_gas * R.sg_max[s];
    R.P_null[s] = -std::expm1(-nu_max * c.dt);
    R.T_null[s] = (uint64_t)std::floor(R.P_null[s] * 4294967296.0);
  }
  R.vth_gas = std::sqrt(kBoltz * c.T_gas_K / kMassAr);
  if (R.ionize) {
    R.iz_cap = (int)std::min<long>(std::max<long>(4096, (long)c.nx * c.ny * c.nz * c.ppc / 64), 1L << 24);
    TRY(dalloc(ctx, R, &R.d_iz, R.iz_cap));
    TRY(dalloc(ctx, R, &R.d_iz_cnt, 1));
    TRY(dalloc(ctx, R, &R.d_next_id, 2));
    TRY(dalloc(ctx, R, &R.d_iz_drop, 1));
    HIPCHK(ctx, hipMemsetAsync(R.d_iz_cnt, 0, 4, ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(R.d_iz_drop, 0, 8, ctx->stream));
    const uint32_t nid[2] = {(uint32_t)((long)c.nx * c.ny * c.nz * c.ppc),
                             (uint32_t)((long)c.nx * c.ny * c.nz * c.ppc)};
    HIPCHK(ctx, hipMemcpyAsync(R.d_next_id, nid, 8, hipMemcpyHostToDevice, ctx->stream));
  }
  if (c.xs_n > 0) {
    TRY(dalloc(ctx, R, &R.d_xs, R.xs.size()));
    HIPCHK(ctx, hipMemcpyAsync(R.d_xs, R.xs.data(), R.xs.size() * sizeof(double),
                               hipMemcpyHostToDevice, ctx->stream));
  }
  R.n_load = R.ncell * c.ppc;
  // tiles of 4x4x4 cells; each tile's slot range is padded to a multiple of 4
  R.ntiles = ((R.nx + 3) / 4) * ((R.ny + 3) / 4) * ((R.nz + 3) / 4);
  // with ionisation the grid keeps a padding tile at its end, whose slot range
  // takes the particles made since the last re-binning
  R.ngrid = tile_grid(R.nx, R.ny, R.nz, R.ionize ? 1 : 0);
  {
    long most = R.n_load;
    if (c.max_particles > 0) most = std::max<long>(most, (long)c.max_particles);
    else if (R.ionize) most = R.n_load + R.n_load / 4;
    R.cap[0] = R.cap[1] = (most + 4L * R.ngrid + 1023) / 1024 * 1024;
  }
  if (!factor_len(R.nx, R.fft.fac_x, &R.fft.nfac_x) || !factor_len(R.ny, R.fft.fac_y, &R.fft.nfac_y))
    return fail(ctx, PIC_EINVAL, "FFT length not supported");
  R.fft.L_x = lines_per_block(R.nx, R.ny);
  R.fft.L_y = lines_per_block(R.ny, R.nx);

  hipStream_t st = ctx->stream;
  TRY(alloc_particles(ctx, R));
  if (R.prec == PIC_FP64) {
    double *r0, *r1;
    TRY(dalloc(ctx, R, &r0, R.nn));
    TRY(dalloc(ctx, R, &r1, R.nn));
    R.rho[0] = r0;
    R.rho[1] = r1;
    double* E;
    TRY(dalloc(ctx, R, &E, 4 * R.nn));
    R.E = E;
    double2* w;
    TRY(dalloc(ctx, R, &w, R.n_int));
    R.work = w;
    TRY(setup_solver_tables<double>(ctx, R, &R.tw_x, &R.tw_y, &R.inv));
  } else {
    long long *r0, *r1;
    TRY(dalloc(ctx, R, &r0, R.nn));
    TRY(dalloc(ctx, R, &r1, R.nn));
    R.rho[0] = r0;
    R.rho[1] = r1;
    float* E;
    TRY(dalloc(ctx, R, &E, 4 * R.nn));
    R.E = E;
    float2* w;
    TRY(dalloc(ctx, R, &w, R.n_int));
    R.work = w;
    TRY(setup_solver_tables<float>(ctx, R, &R.tw_x, &R.tw_y, &R.inv));
    TRY(dalloc(ctx, R, &R.psi, R.n_int));
    launch_zero_f64(R.psi, R.n_int, st);  // the first solve starts from psi = 0
    TRY(dalloc(ctx, R, &R.r, R.n_int));
  }
  TRY(dalloc(ctx, R, &R.b, R.n_int));
  TRY(dalloc(ctx, R, &R.phi, R.nn));
  // two sums and a partial pair per residual block (blocks of 256 nodes per plane)
  TRY(dalloc(ctx, R, &R.norms, 2 + 2 * ((R.nxy + 255) / 256) * (R.nz - 1)));
  TRY(dalloc(ctx, R, &R.d_gc, 2 * std::max(c.n_grains, 1)));
  const long nkey = sort_keys(R.ngrid);
  TRY(dalloc(ctx, R, &R.d_hist, nkey));
  TRY(dalloc(ctx, R, &R.d_sums, (nkey + 1023) / 1024 + 1));
  HIPCHK(ctx, hipMemsetAsync(R.d_gc, 0, 16 * std::max(c.n_grains, 1), st));
  HIPCHK(ctx, hipMemsetAsync(R.norms, 0, 16, st));
  TRY(dalloc(ctx, R, &R.refine_ctl, 4));
  HIPCHK(ctx, hipMemsetAsync(R.refine_ctl, 0, 16, st));
  if (c.coulomb_interval > 0) {
    for (int sp = 0; sp < 2; ++sp) {
      // cells in the tile order of the particle bins, 64 a tile
      TRY(dalloc(ctx, R, &R.coul.start[sp], 64L * R.ngrid + 1));
      TRY(dalloc(ctx, R, &R.coul.fill[sp], 64L * R.ngrid));
      TRY(dalloc(ctx, R, &R.coul.thist[sp], 64L * R.ngrid));
      TRY(dalloc(ctx, R, &R.coul.key[sp], R.cap[sp]));
      TRY(dalloc(ctx, R, &R.coul.slot[sp], R.cap[sp]));
      TRY(dalloc(ctx, R, &R.coul.ord[sp], R.cap[sp]));
    }
    TRY(dalloc(ctx, R, &R.coul.sums, coulomb_scan_sums(64L * R.ngrid)));
    TRY(dalloc(ctx, R, &R.coul.count, 1));
    launch_zero_i64((long long*)R.coul.count, 1, st);
    ctx->coulomb = true;
  }
  TRY(setup_md(ctx, R));
  TRY(unit_fields(ctx, R));

  // load: ppc particles per cell, Maxwellian, Philox keyed by the seed
  const uint32_t k0 = (uint32_t)(c.seed & 0xffffffffu), k1 = (uint32_t)(c.seed >> 32);
  for (int sp = 0; sp < 2; ++sp) {
    const int n = (int)R.n_load;
    if (R.prec == PIC_FP64)
      launch_init_f64(R.p64[sp][0], n, c.ppc, R.nx, R.ny, sp, k0, k1, R.vth[sp], st);
    else
      launch_init_f32r(R.p32[sp][0], n, c.ppc, R.nx, R.ny, sp, k0, k1, R.vth[sp], st);
  }
  CHECK_LAUNCH(ctx);
  int counts[16] = {0};
  counts[0] = counts[8] = (int)R.n_load;
  HIPCHK(ctx, hipMemcpyAsync(R.d_cnt, counts, sizeof(counts), hipMemcpyHostToDevice, st));
  R.cur[0] = R.cur[1] = 0;
  R.rho_cur = 0;
  R.step = 0;
  R.n_base[0] = R.n_base[1] = R.n_load;
  TRY(resort(ctx, R));
  TRY(deposit_current(ctx, R));
  HIPCHK(ctx, hipStreamSynchronize(st));
  return PIC_OK;
}

Replica* get_rep(pic_ctx* ctx, int replica) {
  if (!ctx || replica < 0 || replica >= (int)ctx->reps.size()) return nullptr;
  return ctx->reps[replica].get();
}

// Where pic_fields stages what it hands out: the context's buffers, allocated
// on first use (sc == nullptr), or slices of a caller-given device array of
// sc->cap doubles (pic_fields_static), reused quantity by quantity.
struct FieldStage {
  double* base;
  size_t cap;
};

int fields_impl(pic_ctx* ctx, Replica* R, unsigned what, void* const* out, int out_on_device,
                const FieldStage* sc) {
  if (!out || (what & ~511u)) return fail(ctx, PIC_EINVAL, "bad selection or out");
  if ((what & PIC_RHO_FIXED) && R->prec != PIC_FP32R)
    return fail(ctx, PIC_EINVAL, "PIC_RHO_FIXED needs the FP32R form");
  if ((what & (PIC_FINE_N | PIC_FINE_FLUX | PIC_FINE_PHI)) && !R->fine_on)
    return fail(ctx, PIC_ESTATE, "no fine grid: call pic_set_fine_grid");
  {
    int slot = 0;
    for (unsigned bit = 1; bit <= PIC_FINE_PHI; bit <<= 1)
      if ((what & bit) && !out[slot++]) return fail(ctx, PIC_EINVAL, "NULL output buffer");
  }
  hipStream_t st = ctx->stream;
  TRY(solve_fields(ctx, *R));
  const long nn = R->nn;
  double* tot64 = nullptr;
  long long* totfx = nullptr;
  double* eout = nullptr;
  if (sc) {
    tot64 = sc->base;
    totfx = (long long*)(sc->base + nn);
    eout = sc->base;
  } else {
    if (!R->tot64) TRY(dalloc(ctx, *R, &R->tot64, nn));
    if (!R->totfx) TRY(dalloc(ctx, *R, &R->totfx, nn));
    if (!R->eout) TRY(dalloc(ctx, *R, &R->eout, 3 * nn));
    tot64 = R->tot64;
    totfx = R->totfx;
    eout = R->eout;
  }
  const hipMemcpyKind kind = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const double vol = R->cfg.dx * R->cfg.dx * R->cfg.dx;
  // densities and fluxes of one species into mom [4][nn] (W, then v W), scaled
  auto moments_of = [&](int sp, double* mom) {
    launch_zero_f64(mom, 4 * nn, st);
    const SpeciesStep S = species_step(*R, sp);
    if (R->prec == PIC_FP64)
      launch_moments(&R->p64[sp][R->cur[sp]], nullptr, S, R->lists[sp], mom, nn, AvgBins{}, st);
    else
      launch_moments(nullptr, &R->p32[sp][R->cur[sp]], S, R->lists[sp], mom, nn, AvgBins{}, st);
    launch_scale(mom, nullptr, R->w / vol, mom, 4 * nn, st);
  };
  if ((what & (PIC_N | PIC_FLUX)) && !sc) {
    if (!R->mom) TRY(dalloc(ctx, *R, &R->mom, 8 * nn));
    for (int sp = 0; sp < 2; ++sp) moments_of(sp, R->mom + 4 * nn * sp);
    CHECK_LAUNCH(ctx);
  }
  const long fn = R->fine.fn;
  if (what & (PIC_FINE_N | PIC_FINE_FLUX)) {
    if (!R->fine_mom) TRY(dalloc(ctx, *R, &R->fine_mom, 8 * fn));
    launch_zero_f64(R->fine_mom, 8 * fn, st);
    TRY(enqueue_fine(ctx, *R, R->fine_mom, AvgBins{}));
    const double hdx = R->fine.h * R->cfg.dx;
    launch_scale(R->fine_mom, nullptr, R->w / (hdx * hdx * hdx), R->fine_mom, 8 * fn, st);
    CHECK_LAUNCH(ctx);
  }
  if (what & PIC_FINE_PHI) {
    if (!R->fine_phi) TRY(dalloc(ctx, *R, &R->fine_phi, fn));
    launch_fine_phi(R->phi, R->md, R->Uphi, R->fine, R->nx, R->ny, R->nz, R->cfg.dx,
                    R->cfg.grain_radius, R->fine_phi, AvgBins{}, st);
    CHECK_LAUNCH(ctx);
  }
  int slot = 0, slot_n = -1, slot_flux = -1;
  for (unsigned bit = 1; bit <= PIC_FINE_PHI; bit <<= 1) {
    if (!(what & bit)) continue;
    if (bit == PIC_N) slot_n = slot;
    if (bit == PIC_FLUX) slot_flux = slot;
    ++slot;
  }
  slot = 0;
  for (unsigned bit = 1; bit <= PIC_FINE_PHI; bit <<= 1) {
    if (!(what & bit)) continue;
    void* dst = out[slot++];
    if (bit == PIC_FINE_PHI) {
      HIPCHK(ctx, hipMemcpyAsync(dst, R->fine_phi, fn * 8, kind, st));
    } else if (bit == PIC_FINE_N || bit == PIC_FINE_FLUX) {
      const long len = bit == PIC_FINE_FLUX ? 3 * fn : fn;
      for (int sp = 0; sp < 2; ++sp)
        HIPCHK(ctx, hipMemcpyAsync((char*)dst + sp * len * 8,
                                   R->fine_mom + (4 * sp + (bit == PIC_FINE_FLUX ? 1 : 0)) * fn,
                                   len * 8, kind, st));
    } else if (bit == PIC_PHI) {
      HIPCHK(ctx, hipMemcpyAsync(dst, R->phi, nn * 8, kind, st));
    } else if ((bit == PIC_N || bit == PIC_FLUX) && sc) {
      // one species at a time through the scratch, both quantities at once
      if (bit == PIC_FLUX && slot_n >= 0) continue;  // already handed out with N
      for (int sp = 0; sp < 2; ++sp) {
        moments_of(sp, sc->base);
        if (slot_n >= 0)
          HIPCHK(ctx, hipMemcpyAsync((char*)out[slot_n] + sp * nn * 8, sc->base, nn * 8, kind,
                                     st));
        if (slot_flux >= 0)
          HIPCHK(ctx, hipMemcpyAsync((char*)out[slot_flux] + 3 * sp * nn * 8, sc->base + nn,
                                     3 * nn * 8, kind, st));
      }
    } else if (bit == PIC_N) {
      for (int sp = 0; sp < 2; ++sp)
        HIPCHK(ctx, hipMemcpyAsync((char*)dst + sp * nn * 8, R->mom + 4 * nn * sp, nn * 8, kind, st));
    } else if (bit == PIC_FLUX) {
      for (int sp = 0; sp < 2; ++sp)
        HIPCHK(ctx, hipMemcpyAsync((char*)dst + 3 * sp * nn * 8, R->mom + (4 * sp + 1) * nn,
                                   3 * nn * 8, kind, st));
    } else if (bit == PIC_E) {
      launch_e_out(R->prec == PIC_FP64 ? (const double*)R->E : nullptr,
                   R->prec == PIC_FP64 ? nullptr : (const float*)R->E, eout, nn, st);
      HIPCHK(ctx, hipMemcpyAsync(dst, eout, 3 * nn * 8, kind, st));
    } else {
      if (R->prec == PIC_FP64) {
        launch_rho_total((const double*)R->rho[R->rho_cur], nullptr, tot64, nullptr, R->d_gc,
                         R->md.gpos, R->cfg.n_grains, R->nx, R->ny, nn, R->Qp, st);
        launch_scale(tot64, nullptr, R->we / vol, tot64, nn, st);
      } else {
        launch_rho_total(nullptr, (const long long*)R->rho[R->rho_cur], nullptr, totfx,
                         R->d_gc, R->md.gpos, R->cfg.n_grains, R->nx, R->ny, nn, R->Qp, st);
        launch_scale(nullptr, totfx, kCharge / 4294967296.0 / vol, tot64, nn, st);
      }
      if (bit == PIC_RHO)
        HIPCHK(ctx, hipMemcpyAsync(dst, tot64, nn * 8, kind, st));
      else
        HIPCHK(ctx, hipMemcpyAsync(dst, totfx, nn * 8, kind, st));
    }
    CHECK_LAUNCH(ctx);
  }
  if (!out_on_device) HIPCHK(ctx, hipStreamSynchronize(st));
  return PIC_OK;
}


// ---------------------------------------------------------------- checkpoints
// Binary, native byte order: "PICCKPT1", n_replicas, then per replica its
// configuration (the scalars below, the grain positions and the cross-section
// tables, which a loading context must match), the step, grain and electrode
// counts, the event-counter totals, and per species the particles as
// pic_get_state gives them; FP32R adds the potential the next solve starts
// from (psi), so a resumed run repeats the uninterrupted one bit for bit.
struct CkptConfig {
  int32_t nx, ny, nz, ppc, n_grains, cutoff, md_sub, precision, max_refine, coulomb_interval,
      xs_n, pad;
  double dx, dt, n0, Te, Ti, p_gas, T_gas, sig_e, sig_i, V_dc, V_rf, f_rf, radius, E_cap,
      refine_tol, lnL, E_ex, E_iz;
  uint64_t seed;
  int64_t max_particles;
};

CkptConfig ckpt_config(const Replica& R) {
  const pic_config& c = R.cfg;
  CkptConfig k;
  std::memset(&k, 0, sizeof(k));
  k.nx = c.nx;
  k.ny = c.ny;
  k.nz = c.nz;
  k.ppc = c.ppc;
  k.n_grains = c.n_grains;
  k.cutoff = c.pp_cutoff_cells;
  k.md_sub = c.md_subcycles;
  k.precision = c.precision;
  k.max_refine = c.max_refine;
  k.coulomb_interval = c.coulomb_interval;
  k.xs_n = c.xs_n;
  k.dx = c.dx;
  k.dt = c.dt;
  k.n0 = c.n0;
  k.Te = c.Te_eV;
  k.Ti = c.Ti_eV;
  k.p_gas = c.p_gas_Pa;
  k.T_gas = c.T_gas_K;
  k.sig_e = c.sigma_e_el;
  k.sig_i = c.sigma_i_cx;
  k.V_dc = c.V_dc;
  k.V_rf = c.V_rf;
  k.f_rf = c.f_rf;
  k.radius = c.grain_radius;
  k.E_cap = c.E_cap_eV;
  k.refine_tol = c.refine_tol;
  k.lnL = c.coulomb_lnL;
  k.E_ex = c.E_ex_eV;
  k.E_iz = R.ionize ? c.E_iz_eV : 0.0;
  k.seed = c.seed;
  k.max_particles = c.max_particles;
  return k;
}

constexpr char kCkptMagic[8] = {'P', 'I', 'C', 'C', 'K', 'P', 'T', '2'};
constexpr int kCkptTallies[] = {TL_MD, TL_FALL, TL_COLL, TL_CAP, TL_BAD, TL_FAST};

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) std::fclose(f);
  }
};

template <typename T>
bool put(FILE* f, const T* p, size_t n) {
  return n == 0 || std::fwrite(p, sizeof(T), n, f) == n;
}
template <typename T>
bool get(FILE* f, T* p, size_t n) {
  return n == 0 || std::fread(p, sizeof(T), n, f) == n;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

int pic_init(const pic_config* cfgs, int n_replicas, void* hip_stream, pic_ctx** out) {
  if (!out) return fail(nullptr, PIC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfgs || n_replicas < 1) return fail(nullptr, PIC_EINVAL, "no configuration given");
  std::unique_ptr<pic_ctx> ctx(new (std::nothrow) pic_ctx());
  if (!ctx) return fail(nullptr, PIC_ENOMEM, "host allocation failed");
  ctx->stream = (hipStream_t)hip_stream;
  for (int r = 0; r < n_replicas; ++r) {
    std::unique_ptr<Replica> R(new (std::nothrow) Replica());
    if (!R) return fail(nullptr, PIC_ENOMEM, "host allocation failed");
    int rc = init_replica(ctx.get(), *R, cfgs[r]);
    if (rc != PIC_OK) {
      g_init_error = "replica " + std::to_string(r) + ": " + ctx->err;
      return rc;
    }
    ctx->reps.push_back(std::move(R));
  }
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      ncu > 0)
    ctx->n_cu = ncu;
  // the address of the fixed scratch array on this device (once per device);
  // without it only pic_fields_static is unavailable
  ctx->scratch_ok = scratch_setup(&ctx->device, nullptr) == 0;
  if (build_batch(ctx.get()) != PIC_OK) {
    g_init_error = ctx->err;
    return PIC_EDEVICE;
  }
  pic_tuning& t = ctx->tune;
  t.sort_interval = ctx->reps[0]->cfg.sort_interval;
  t.ion_sort_interval = 64;
  t.tile_margin = 2;
  t.ion_tile_margin = 1;
  t.batch_push = ctx->batchable && n_replicas > 1 ? 1 : 0;
  t.batch_blocks = (4 * ctx->n_cu + 7) / 8 * 8;
  t.use_graphs = 1;
  *out = ctx.release();
  return PIC_OK;
}

int pic_step(pic_ctx* ctx, int n_steps) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  if (n_steps < 0) return fail(ctx, PIC_EINVAL, "n_steps < 0");
  for (int s = 0; s < n_steps; ++s) TRY(step_all(ctx));
  return PIC_OK;
}

int pic_grain_charges(pic_ctx* ctx, int replica, int64_t* counts, double* Q_C) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  Replica* R = get_rep(ctx, replica);
  if (!R) return fail(ctx, PIC_EINVAL, "bad replica index");
  const int ng = R->cfg.n_grains;
  if (ng == 0) return PIC_OK;
  if (!counts) return fail(ctx, PIC_EINVAL, "counts is NULL");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  HIPCHK(ctx, hipMemcpy(counts, R->d_gc, 16 * ng, hipMemcpyDeviceToHost));
  if (Q_C)
    for (int g = 0; g < ng; ++g) Q_C[g] = (double)(counts[2 * g + 1] - counts[2 * g]) * R->we;
  return PIC_OK;
}

int pic_energy(pic_ctx* ctx, int replica, double out[4]) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  Replica* R = get_rep(ctx, replica);
  if (!R || !out) return fail(ctx, PIC_EINVAL, "bad replica or out");
  const int nb = energy_blocks();
  if (!R->energy) TRY(dalloc(ctx, *R, &R->energy, 3 * (size_t)nb));
  TRY(solve_fields(ctx, *R));
  for (int sp = 0; sp < 2; ++sp) {
    if (R->prec == PIC_FP64)
      launch_energy(&R->p64[sp][R->cur[sp]], nullptr, R->lists[sp], R->energy + sp * nb,
                    ctx->stream);
    else
      launch_energy(nullptr, &R->p32[sp][R->cur[sp]], R->lists[sp], R->energy + sp * nb,
                    ctx->stream);
  }
  launch_field_energy(R->E, R->prec == PIC_FP64, R->nxy, R->nz, R->energy + 2 * nb, ctx->stream);
  CHECK_LAUNCH(ctx);
  std::vector<double> h(3 * (size_t)nb);
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  HIPCHK(ctx, hipMemcpy(h.data(), R->energy, h.size() * 8, hipMemcpyDeviceToHost));
  double sum[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < 3; ++q)
    for (int b = 0; b < nb; ++b) sum[q] += h[(size_t)q * nb + b];
  const double vol = R->cfg.dx * R->cfg.dx * R->cfg.dx;
  out[0] = 0.5 * R->m[0] * R->w * sum[0];
  out[1] = 0.5 * R->m[1] * R->w * sum[1];
  out[2] = 0.5 * kEps0 * vol * sum[2];
  out[3] = out[0] + out[1] + out[2];
  return PIC_OK;
}

int pic_grain_positions(pic_ctx* ctx, int replica, double* pos) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  Replica* R = get_rep(ctx, replica);
  if (!R) return fail(ctx, PIC_EINVAL, "bad replica index");
  if (R->cfg.n_grains == 0) return PIC_OK;
  if (!pos) return fail(ctx, PIC_EINVAL, "pos is NULL");
  std::copy(R->gpos.begin(), R->gpos.end(), pos);
  return PIC_OK;
}

int pic_fields(pic_ctx* ctx, int replica, unsigned what, void* const* out, int out_on_device) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  Replica* R = get_rep(ctx, replica);
  if (!R) return fail(ctx, PIC_EINVAL, "bad replica index");
  return fields_impl(ctx, R, what, out, out_on_device, nullptr);
}

int pic_fields_static(pic_ctx* ctx, int replica, unsigned what, void* const* out,
                      int out_on_device) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  Replica* R = get_rep(ctx, replica);
  if (!R) return fail(ctx, PIC_EINVAL, "bad replica index");
  const unsigned allowed = PIC_PHI | PIC_E | PIC_RHO | PIC_RHO_FIXED | PIC_N | PIC_FLUX;
  if (what & ~allowed)
    return fail(ctx, PIC_EINVAL, "pic_fields_static: only PHI, E, RHO, RHO_FIXED, N and FLUX");
  const size_t nn = (size_t)R->nn;
  size_t need = 0;
  if (what & (PIC_N | PIC_FLUX)) need = std::max(need, 4 * nn);
  if (what & PIC_E) need = std::max(need, 3 * nn);
  if (what & (PIC_RHO | PIC_RHO_FIXED)) need = std::max(need, 2 * nn);
  if (need > kScratchDoubles)
    return fail(ctx, PIC_EINVAL,
                "pic_fields_static: the selection needs " + std::to_string(need) +
                    " doubles of scratch, the fixed array holds " +
                    std::to_string(kScratchDoubles) + " (at most " +
                    std::to_string(kScratchDoubles / 4) + " nodes with N or FLUX)");
  void* base = ctx->scratch_ok ? scratch_address(ctx->device) : nullptr;
  if (!base)
    return fail(ctx, PIC_ESTATE, "pic_fields_static: the scratch array's address is unknown");
  const FieldStage sc{(double*)base, kScratchDoubles};
  return fields_impl(ctx, R, what, out, out_on_device, &sc);
}

int pic_average(pic_ctx* ctx, int interval, int phase_bins) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  if (interval < 0) return fail(ctx, PIC_EINVAL, "interval must be >= 0");
  if (interval == 0) {
    ctx->avg_interval = 0;
    return PIC_OK;
  }
  if (phase_bins < 1 || phase_bins > PIC_MAX_PHASE_BINS)
    return fail(ctx, PIC_EINVAL, "phase_bins out of range");
  hipStream_t st = ctx->stream;
  HIPCHK(ctx, hipStreamSynchronize(st));
  for (auto& R : ctx->reps) {
    if (R->avg_cap < phase_bins) {
      TRY(dalloc(ctx, *R, &R->avg, (size_t)9 * R->nn * phase_bins));
      TRY(dalloc(ctx, *R, &R->d_avg_cnt, (size_t)phase_bins));
      R->avg_cap = phase_bins;
    }
    launch_zero_f64(R->avg, 9 * R->nn * phase_bins, st);
    launch_zero_i64((long long*)R->d_avg_cnt, phase_bins, st);
    R->fine_avg_on = R->fine_on;
    if (R->fine_on) {
      const long fn = R->fine.fn;
      if (R->fine_cap < phase_bins) {
        dfree(*R, R->fine_avg);
        R->fine_cap = 0;
        TRY(dalloc(ctx, *R, &R->fine_avg, (size_t)9 * fn * phase_bins));
        R->fine_cap = phase_bins;
      }
      launch_zero_f64(R->fine_avg, 9 * fn * phase_bins, st);
    }
  }
  CHECK_LAUNCH(ctx);
  ctx->avg_interval = interval;
  ctx->avg_bins = phase_bins;
  ctx->since_avg = 0;
  ctx->drop_graphs();  // the captured samples hold the bin count and buffers
  return PIC_OK;
}

int pic_average_read(pic_ctx* ctx, int replica, int bin, unsigned what, void* const* out,
                     int out_on_device, int64_t* samples) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  Replica* R = get_rep(ctx, replica);
  if (!R) return fail(ctx, PIC_EINVAL, "bad replica index");
  if (!R->avg || ctx->avg_bins == 0) return fail(ctx, PIC_ESTATE, "no averages: call pic_average");
  const unsigned fine_bits = PIC_FINE_N | PIC_FINE_FLUX | PIC_FINE_PHI;
  if ((what & ~(PIC_PHI | PIC_N | PIC_FLUX | fine_bits)) || (what && !out))
    return fail(ctx, PIC_EINVAL, "bad selection or out");
  if ((what & fine_bits) && !R->fine_avg_on)
    return fail(ctx, PIC_ESTATE, "no fine-grid averages: set the fine grid before pic_average");
  if (bin < -1 || bin >= ctx->avg_bins) return fail(ctx, PIC_EINVAL, "bad bin");
  hipStream_t st = ctx->stream;
  const long nn = R->nn;
  const int b0 = bin < 0 ? 0 : bin, b1 = bin < 0 ? ctx->avg_bins : bin + 1;
  if (!R->avg_out) TRY(dalloc(ctx, *R, &R->avg_out, 9 * nn));
  const double vol = R->cfg.dx * R->cfg.dx * R->cfg.dx;
  launch_avg_out(R->avg, b0, b1, 9 * nn, 9 * nn, nn, R->d_avg_cnt, R->w / vol, R->avg_out, st);
  const long fn = R->fine.fn;
  if (what & fine_bits) {
    if (!R->fine_out) TRY(dalloc(ctx, *R, &R->fine_out, 9 * fn));
    const double hdx = R->fine.h * R->cfg.dx;
    launch_avg_out(R->fine_avg, b0, b1, 9 * fn, 9 * fn, fn, R->d_avg_cnt, R->w / (hdx * hdx * hdx),
                   R->fine_out, st);
  }
  CHECK_LAUNCH(ctx);
  const hipMemcpyKind kind = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  int slot = 0;
  for (unsigned bit : {PIC_PHI, PIC_N, PIC_FLUX, PIC_FINE_N, PIC_FINE_FLUX, PIC_FINE_PHI}) {
    if (!(what & bit)) continue;
    char* dst = (char*)out[slot++];
    if (!dst) return fail(ctx, PIC_EINVAL, "NULL output buffer");
    if (bit == PIC_FINE_PHI) {
      HIPCHK(ctx, hipMemcpyAsync(dst, R->fine_out, fn * 8, kind, st));
      continue;
    }
    if (bit == PIC_FINE_N || bit == PIC_FINE_FLUX) {
      const long len = bit == PIC_FINE_FLUX ? 3 * fn : fn;
      for (int sp = 0; sp < 2; ++sp)
        HIPCHK(ctx, hipMemcpyAsync(dst + sp * len * 8,
                                   R->fine_out + fn + (4 * sp + (bit == PIC_FINE_FLUX ? 1 : 0)) * fn,
                                   len * 8, kind, st));
      continue;
    }
    for (int sp = 0; sp < (bit == PIC_PHI ? 1 : 2); ++sp) {
      const double* src = bit == PIC_PHI ? R->avg_out
                          : R->avg_out + (1 + 4 * sp + (bit == PIC_FLUX ? 1 : 0)) * nn;
      const long len = bit == PIC_FLUX ? 3 * nn : nn;
      HIPCHK(ctx, hipMemcpyAsync(dst + sp * len * 8, src, len * 8, kind, st));
    }
  }
  if (samples) {
    std::vector<unsigned long long> c(ctx->avg_bins);
    HIPCHK(ctx, hipMemcpyAsync(c.data(), R->d_avg_cnt, c.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    *samples = 0;
    for (int b = b0; b < b1; ++b) *samples += (int64_t)c[b];
  }
  if (!out_on_device) HIPCHK(ctx, hipStreamSynchronize(st));
  return PIC_OK;
}

int pic_set_fine_grid(pic_ctx* ctx, int replica, const pic_fine_grid* g) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  Replica* R = get_rep(ctx, replica);
  if (!R) return fail(ctx, PIC_EINVAL, "bad replica index");
  if (ctx->avg_interval > 0)
    return fail(ctx, PIC_ESTATE, "averaging is running: stop it before changing the fine grid");
  FineBox fb{};
  if (g) {
    const int n[3] = {R->nx, R->ny, R->nz};
    if (!(std::isfinite(g->h) && g->h > 0.0)) return fail(ctx, PIC_EINVAL, "fine grid: h must be > 0");
    long nodes = 1;
    for (int a = 0; a < 3; ++a) {
      if (g->cells[a] < 1) return fail(ctx, PIC_EINVAL, "fine grid: cells must be >= 1");
      const double top = g->origin[a] + g->h * (double)g->cells[a];
      if (!(std::isfinite(g->origin[a]) && g->origin[a] >= 0.0 && top <= (double)n[a]))
        return fail(ctx, PIC_EINVAL, "fine grid: the box must lie inside the domain");
      nodes *= (long)g->cells[a] + 1;
      if (nodes > PIC_MAX_FINE_NODES)
        return fail(ctx, PIC_EINVAL, "fine grid: more than PIC_MAX_FINE_NODES nodes");
      fb.o[a] = g->origin[a];
      fb.m[a] = g->cells[a];
      // PIC cells that can hold a particle of the box, one cell of slack for rounding
      fb.lo[a] = (int)std::floor(g->origin[a]) - 1;
      fb.hi[a] = (int)std::ceil(top) + 1;
    }
    fb.h = g->h;
    fb.mx = (long)fb.m[0] + 1;
    fb.my = (long)fb.m[1] + 1;
    fb.fn = nodes;
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  dfree(*R, R->fine_mom);
  dfree(*R, R->fine_phi);
  dfree(*R, R->fine_avg);
  dfree(*R, R->fine_out);
  R->fine_cap = 0;
  R->fine_avg_on = false;
  R->fine_on = g != nullptr;
  R->fine = fb;
  ctx->drop_graphs();  // captured samples hold the fine buffers
  return PIC_OK;
}

void pic_destroy(pic_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
}

const char* pic_last_error(const pic_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

int pic_get_state(pic_ctx* ctx, int replica, pic_state_view* v) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  Replica* R = get_rep(ctx, replica);
  if (!R || !v) return fail(ctx, PIC_EINVAL, "bad replica or view");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  int cnts[16];
  HIPCHK(ctx, hipMemcpy(cnts, R->d_cnt, sizeof(cnts), hipMemcpyDeviceToHost));
  for (int sp = 0; sp < 2; ++sp) {
    const long slots = cnts[8 * sp];
    // copy every slot in use, then keep the occupied ones
    std::vector<uint32_t> ids(slots);
    std::vector<double> a[6];
    std::vector<char> alive(slots, 0);
    if (slots > 0) {
      HIPCHK(ctx, hipMemcpy(ids.data(), R->prec == PIC_FP64 ? R->p64[sp][R->cur[sp]].id
                                                             : R->p32[sp][R->cur[sp]].id,
                            slots * 4, hipMemcpyDeviceToHost));
      for (auto& x : a) x.resize(slots);
      if (R->prec == PIC_FP64) {
        const PartF64& P = R->p64[sp][R->cur[sp]];
        double* src[6] = {P.x, P.y, P.z, P.vx, P.vy, P.vz};
        for (int q = 0; q < 6; ++q)
          HIPCHK(ctx, hipMemcpy(a[q].data(), src[q], slots * 8, hipMemcpyDeviceToHost));
        for (long i = 0; i < slots; ++i) alive[i] = a[2][i] >= 0.0;
      } else {
        const PartF32R& P = R->p32[sp][R->cur[sp]];
        std::vector<int32_t> cell(slots);
        std::vector<float> f(slots);
        HIPCHK(ctx, hipMemcpy(cell.data(), P.cell, slots * 4, hipMemcpyDeviceToHost));
        float* src[6] = {P.ox, P.oy, P.oz, P.vx, P.vy, P.vz};
        for (int q = 0; q < 6; ++q) {
          HIPCHK(ctx, hipMemcpy(f.data(), src[q], slots * 4, hipMemcpyDeviceToHost));
          for (long i = 0; i < slots; ++i) a[q][i] = (double)f[i];
        }
        for (long i = 0; i < slots; ++i) {
          const int c = cell[i];
          alive[i] = c >= 0;
          if (c < 0) continue;
          a[0][i] += (double)(c & 1023);
          a[1][i] += (double)((c >> 10) & 1023);
          a[2][i] += (double)(c >> 20);
        }
      }
    }
    long cnt = 0;
    for (long i = 0; i < slots; ++i) cnt += alive[i];
    if (cnt > v->capacity[sp]) return fail(ctx, PIC_EINVAL, "view capacity too small");
    if (cnt > 0 && (!v->pos[sp] || !v->vel[sp] || !v->id[sp]))
      return fail(ctx, PIC_EINVAL, "NULL view array");
    long o = 0;
    for (long i = 0; i < slots; ++i) {
      if (!alive[i]) continue;
      for (int q = 0; q < 3; ++q) {
        v->pos[sp][3 * o + q] = a[q][i];
        v->vel[sp][3 * o + q] = a[3 + q][i];
      }
      v->id[sp][o] = ids[i];
      ++o;
    }
    v->n[sp] = cnt;
  }
  for (int sp = 0; sp < 2; ++sp) {
    unsigned long long t[TL_N];
    TRY(read_tallies(ctx, *R, sp, t));
    v->wall_count[0][sp] = R->wall_base[0][sp] + (int64_t)t[TL_W0];
    v->wall_count[1][sp] = R->wall_base[1][sp] + (int64_t)t[TL_W1];
  }
  if (v->grain_count && R->cfg.n_grains > 0)
    HIPCHK(ctx, hipMemcpy(v->grain_count, R->d_gc, 16 * R->cfg.n_grains, hipMemcpyDeviceToHost));
  v->step = R->step;
  return PIC_OK;
}

int pic_set_state(pic_ctx* ctx, int replica, const pic_state_view* v) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  Replica* R = get_rep(ctx, replica);
  if (!R || !v) return fail(ctx, PIC_EINVAL, "bad replica or view");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  for (int sp = 0; sp < 2; ++sp) {
    const long cnt = v->n[sp];
    if (cnt < 0 || cnt > R->cap[sp] - 4L * R->ntiles)
      return fail(ctx, PIC_EINVAL, "n exceeds the capacity");
    if (cnt > 0 && (!v->pos[sp] || !v->vel[sp] || !v->id[sp]))
      return fail(ctx, PIC_EINVAL, "NULL view array");
    for (long i = 0; i < cnt; ++i) {
      const double* x = &v->pos[sp][3 * i];
      const double* u = &v->vel[sp][3 * i];
      const bool ok = x[0] >= 0 && x[0] < R->nx && x[1] >= 0 && x[1] < R->ny && x[2] >= 0 &&
                      x[2] < R->nz && std::isfinite(u[0]) && std::isfinite(u[1]) &&
                      std::isfinite(u[2]);
      if (!ok) return fail(ctx, PIC_ENUMERIC, "particle outside the box or not finite");
    }
  }
  // upload into the spare buffers; the sort below brings the particles back
  // to the current ones, so every replica keeps its buffer phase
  for (int sp = 0; sp < 2; ++sp) {
    const int up = 1 - R->cur[sp];
    R->cur[sp] = up;
    R->n_base[sp] = v->n[sp];
    const long cnt = v->n[sp];
    if (cnt == 0) continue;
    if (R->prec == PIC_FP64) {
      const PartF64& P = R->p64[sp][up];
      std::vector<double> a(cnt);
      double* dst[6] = {P.x, P.y, P.z, P.vx, P.vy, P.vz};
      for (int q = 0; q < 6; ++q) {
        const double* src = q < 3 ? v->pos[sp] : v->vel[sp];
        for (long i = 0; i < cnt; ++i) a[i] = src[3 * i + q % 3];
        HIPCHK(ctx, hipMemcpy(dst[q], a.data(), cnt * 8, hipMemcpyHostToDevice));
      }
      HIPCHK(ctx, hipMemcpy(P.id, v->id[sp], cnt * 4, hipMemcpyHostToDevice));
    } else {
      const PartF32R& P = R->p32[sp][up];
      std::vector<int32_t> cell(cnt);
      std::vector<float> a(6 * cnt);
      for (long i = 0; i < cnt; ++i) {
        int c3[3];
        for (int q = 0; q < 3; ++q) {
          const double x = v->pos[sp][3 * i + q];
          int ci = (int)std::floor(x);
          float f = (float)(x - ci);
          const int nq = q == 0 ? R->nx : (q == 1 ? R->ny : R->nz);
          if (f >= 1.0f) {  // rounding up to the next cell
            f = 0.0f;
            ci += 1;
            if (q < 2 && ci == nq) ci = 0;
            if (q == 2 && ci == nq) return fail(ctx, PIC_ENUMERIC, "particle rounds onto z = L_z");
          }
          c3[q] = ci;
          a[q * cnt + i] = f;
          a[(3 + q) * cnt + i] = (float)v->vel[sp][3 * i + q];
        }
        cell[i] = c3[0] | (c3[1] << 10) | (c3[2] << 20);
      }
      HIPCHK(ctx, hipMemcpy(P.cell, cell.data(), cnt * 4, hipMemcpyHostToDevice));
      float* dst[6] = {P.ox, P.oy, P.oz, P.vx, P.vy, P.vz};
      for (int q = 0; q < 6; ++q)
        HIPCHK(ctx, hipMemcpy(dst[q], a.data() + q * cnt, cnt * 4, hipMemcpyHostToDevice));
      HIPCHK(ctx, hipMemcpy(P.id, v->id[sp], cnt * 4, hipMemcpyHostToDevice));
    }
  }
  int counts[16] = {0};
  counts[0] = (int)v->n[0];
  counts[8] = (int)v->n[1];
  HIPCHK(ctx, hipMemcpy(R->d_cnt, counts, sizeof(counts), hipMemcpyHostToDevice));
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) R->wall_base[a][b] = v->wall_count[a][b];
  for (int sp = 0; sp < 2; ++sp)
    HIPCHK(ctx, hipMemset(R->lists[sp].tally, 0, 8 * TL_N * (R->ngrid + kMdTallyRows)));
  const int ng = R->cfg.n_grains;
  if (ng > 0) {
    std::vector<int64_t> gc(2 * ng, 0);
    if (v->grain_count) std::copy(v->grain_count, v->grain_count + 2 * ng, gc.begin());
    HIPCHK(ctx, hipMemcpy(R->d_gc, gc.data(), 16 * ng, hipMemcpyHostToDevice));
  }
  R->step = v->step;
  HIPCHK(ctx, hipMemcpy(R->d_step, &v->step, 4, hipMemcpyHostToDevice));
  if (R->ionize) {
    // ionisations continue with the ids after the largest given
    uint32_t nid[2] = {0u, 0u};
    for (int sp = 0; sp < 2; ++sp)
      for (long i = 0; i < v->n[sp]; ++i) nid[sp] = std::max(nid[sp], v->id[sp][i] + 1u);
    HIPCHK(ctx, hipMemcpy(R->d_next_id, nid, 8, hipMemcpyHostToDevice));
    const int zero = 0;
    HIPCHK(ctx, hipMemcpy(R->d_iz_cnt, &zero, 4, hipMemcpyHostToDevice));
    R->iz_base = 0;
  }
  TRY(resort(ctx, *R));
  TRY(deposit_current(ctx, *R));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return PIC_OK;
}

int pic_save(pic_ctx* ctx, const char* path) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  if (!path) return fail(ctx, PIC_EINVAL, "path is NULL");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  const std::string tmp = std::string(path) + ".tmp";
  {
    File out;
    out.f = std::fopen(tmp.c_str(), "wb");
    if (!out.f) return fail(ctx, PIC_EINVAL, std::string("cannot write ") + tmp);
    const uint32_t nrep = (uint32_t)ctx->reps.size();
    bool ok = put(out.f, kCkptMagic, 8) && put(out.f, &nrep, 1);
    for (uint32_t r = 0; ok && r < nrep; ++r) {
      Replica& R = *ctx->reps[r];
      const CkptConfig k = ckpt_config(R);
      const int ng = R.cfg.n_grains;
      ok = put(out.f, &k, 1) && put(out.f, R.gpos.data(), R.gpos.size()) &&
           put(out.f, R.xs.data(), R.xs.size());
      // particles and counts
      pic_state_view v;
      std::memset(&v, 0, sizeof(v));
      std::vector<double> pos[2], vel[2];
      std::vector<uint32_t> id[2];
      for (int sp = 0; sp < 2; ++sp) {
        v.capacity[sp] = R.cap[sp];
        pos[sp].resize(3 * (size_t)R.cap[sp]);
        vel[sp].resize(3 * (size_t)R.cap[sp]);
        id[sp].resize((size_t)R.cap[sp]);
        v.pos[sp] = pos[sp].data();
        v.vel[sp] = vel[sp].data();
        v.id[sp] = id[sp].data();
      }
      std::vector<int64_t> gc(2 * (size_t)std::max(ng, 1), 0);
      v.grain_count = gc.data();
      TRY(pic_get_state(ctx, (int)r, &v));
      ok = ok && put(out.f, &v.step, 1) && put(out.f, gc.data(), 2 * (size_t)ng) &&
           put(out.f, &v.wall_count[0][0], 4);
      for (int sp = 0; ok && sp < 2; ++sp) {
        unsigned long long t[TL_N];
        TRY(read_tallies(ctx, R, sp, t));
        for (int w : kCkptTallies) ok = ok && put(out.f, &t[w], 1);
      }
      unsigned long long n_coul = 0;
      if (R.coul.count)
        HIPCHK(ctx, hipMemcpy(&n_coul, R.coul.count, 8, hipMemcpyDeviceToHost));
      int ctl[4] = {0, 0, 0, 0};
      HIPCHK(ctx, hipMemcpy(ctl, R.refine_ctl, sizeof(ctl), hipMemcpyDeviceToHost));
      ok = ok && put(out.f, &n_coul, 1) && put(out.f, &ctl[2], 1);
      // ionisation: the next ids, the pairs made, the ones dropped
      uint32_t nid[2] = {0u, 0u};
      unsigned long long drop = 0;
      int64_t n_iz = 0;
      if (R.ionize) {
        HIPCHK(ctx, hipMemcpy(nid, R.d_next_id, 8, hipMemcpyDeviceToHost));
        HIPCHK(ctx, hipMemcpy(&drop, R.d_iz_drop, 8, hipMemcpyDeviceToHost));
        pic_counters cn;
        TRY(pic_get_counters(ctx, (int)r, &cn));
        n_iz = cn.n_ionizations;
      }
      ok = ok && put(out.f, nid, 2) && put(out.f, &n_iz, 1) && put(out.f, &drop, 1);
      for (int sp = 0; ok && sp < 2; ++sp) {
        const int64_t n = v.n[sp];
        ok = put(out.f, &n, 1) && put(out.f, pos[sp].data(), 3 * (size_t)n) &&
             put(out.f, vel[sp].data(), 3 * (size_t)n) && put(out.f, id[sp].data(), (size_t)n);
      }
      const int64_t npsi = R.prec == PIC_FP32R ? R.n_int : 0;
      std::vector<double> psi((size_t)npsi);
      if (npsi)
        HIPCHK(ctx, hipMemcpy(psi.data(), R.psi, npsi * 8, hipMemcpyDeviceToHost));
      ok = ok && put(out.f, &npsi, 1) && put(out.f, psi.data(), (size_t)npsi);
    }
    if (!ok || std::fflush(out.f) != 0) return fail(ctx, PIC_EINVAL, "writing " + tmp + " failed");
  }
  if (std::rename(tmp.c_str(), path) != 0)
    return fail(ctx, PIC_EINVAL, std::string("cannot rename the checkpoint to ") + path);
  return PIC_OK;
}

int pic_load(pic_ctx* ctx, const char* path) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  if (!path) return fail(ctx, PIC_EINVAL, "path is NULL");
  if (ctx->avg_interval > 0)
    return fail(ctx, PIC_ESTATE, "averaging is running: stop it with pic_average(ctx, 0, 0)");
  File in;
  in.f = std::fopen(path, "rb");
  if (!in.f) return fail(ctx, PIC_EINVAL, std::string("cannot read ") + path);
  char magic[8];
  uint32_t nrep = 0;
  if (!get(in.f, magic, 8) || std::memcmp(magic, kCkptMagic, 8) != 0 || !get(in.f, &nrep, 1))
    return fail(ctx, PIC_EINVAL, "not a checkpoint of this library");
  if (nrep != ctx->reps.size())
    return fail(ctx, PIC_ECONFIG, "the checkpoint holds another number of replicas");
  // the whole file is read and checked before any replica changes
  struct Saved {
    pic_state_view v;
    std::vector<int64_t> gc;
    std::vector<double> pos[2], vel[2], psi;
    std::vector<uint32_t> id[2];
    unsigned long long t[2][6];
    unsigned long long n_coul = 0;
    int unconverged = 0;
    uint32_t next_id[2] = {0u, 0u};
    int64_t n_iz = 0;
    unsigned long long drop = 0;
  };
  std::vector<Saved> saved(nrep);
  const std::string trunc = "checkpoint truncated";
  for (uint32_t r = 0; r < nrep; ++r) {
    Replica& R = *ctx->reps[r];
    Saved& S = saved[r];
    CkptConfig k;
    if (!get(in.f, &k, 1)) return fail(ctx, PIC_EINVAL, trunc);
    const CkptConfig mine = ckpt_config(R);
    if (std::memcmp(&k, &mine, sizeof(k)) != 0)
      return fail(ctx, PIC_ECONFIG, "replica " + std::to_string(r) +
                                        ": the checkpoint's configuration differs");
    std::vector<double> gpos(R.gpos.size()), xs(R.xs.size());
    if (!get(in.f, gpos.data(), gpos.size()) || !get(in.f, xs.data(), xs.size()))
      return fail(ctx, PIC_EINVAL, trunc);
    if (gpos != R.gpos || xs != R.xs)
      return fail(ctx, PIC_ECONFIG, "replica " + std::to_string(r) +
                                        ": grain positions or cross sections differ");
    const int ng = R.cfg.n_grains;
    pic_state_view& v = S.v;
    std::memset(&v, 0, sizeof(v));
    S.gc.assign(2 * (size_t)std::max(ng, 1), 0);
    if (!get(in.f, &v.step, 1) || !get(in.f, S.gc.data(), 2 * (size_t)ng) ||
        !get(in.f, &v.wall_count[0][0], 4) || !get(in.f, &S.t[0][0], 12) ||
        !get(in.f, &S.n_coul, 1) || !get(in.f, &S.unconverged, 1) ||
        !get(in.f, S.next_id, 2) || !get(in.f, &S.n_iz, 1) || !get(in.f, &S.drop, 1))
      return fail(ctx, PIC_EINVAL, trunc);
    for (int sp = 0; sp < 2; ++sp) {
      int64_t n = 0;
      if (!get(in.f, &n, 1)) return fail(ctx, PIC_EINVAL, trunc);
      if (n < 0 || n > R.cap[sp] - 4L * R.ntiles)
        return fail(ctx, PIC_EINVAL, "bad particle count in the checkpoint");
      S.pos[sp].resize(3 * (size_t)n);
      S.vel[sp].resize(3 * (size_t)n);
      S.id[sp].resize((size_t)n);
      if (!get(in.f, S.pos[sp].data(), 3 * (size_t)n) ||
          !get(in.f, S.vel[sp].data(), 3 * (size_t)n) || !get(in.f, S.id[sp].data(), (size_t)n))
        return fail(ctx, PIC_EINVAL, trunc);
      v.n[sp] = v.capacity[sp] = n;
    }
    int64_t npsi = 0;
    if (!get(in.f, &npsi, 1)) return fail(ctx, PIC_EINVAL, trunc);
    if (npsi != (R.prec == PIC_FP32R ? R.n_int : 0))
      return fail(ctx, PIC_EINVAL, "bad potential size in the checkpoint");
    S.psi.resize((size_t)npsi);
    if (!get(in.f, S.psi.data(), (size_t)npsi)) return fail(ctx, PIC_EINVAL, trunc);
  }
  char extra;
  if (std::fread(&extra, 1, 1, in.f) != 0)
    return fail(ctx, PIC_EINVAL, "trailing data in the checkpoint");
  for (uint32_t r = 0; r < nrep; ++r) {
    Replica& R = *ctx->reps[r];
    Saved& S = saved[r];
    for (int sp = 0; sp < 2; ++sp) {
      S.v.pos[sp] = S.pos[sp].data();
      S.v.vel[sp] = S.vel[sp].data();
      S.v.id[sp] = S.id[sp].data();
    }
    S.v.grain_count = R.cfg.n_grains > 0 ? S.gc.data() : nullptr;
    TRY(pic_set_state(ctx, (int)r, &S.v));
    // the event totals continue: they go to the first tile's tally row
    for (int sp = 0; sp < 2; ++sp) {
      std::vector<unsigned long long> row(TL_N, 0ull);
      for (int w = 0; w < 6; ++w) row[kCkptTallies[w]] = S.t[sp][w];
      HIPCHK(ctx, hipMemcpy(R.lists[sp].tally, row.data(), 8 * TL_N, hipMemcpyHostToDevice));
    }
    if (R.coul.count) HIPCHK(ctx, hipMemcpy(R.coul.count, &S.n_coul, 8, hipMemcpyHostToDevice));
    const int ctl[4] = {0, 0, S.unconverged, 0};
    HIPCHK(ctx, hipMemcpy(R.refine_ctl, ctl, sizeof(ctl), hipMemcpyHostToDevice));
    if (!S.psi.empty())
      HIPCHK(ctx, hipMemcpy(R.psi, S.psi.data(), S.psi.size() * 8, hipMemcpyHostToDevice));
    if (R.ionize) {
      HIPCHK(ctx, hipMemcpy(R.d_next_id, S.next_id, 8, hipMemcpyHostToDevice));
      HIPCHK(ctx, hipMemcpy(R.d_iz_drop, &S.drop, 8, hipMemcpyHostToDevice));
      R.iz_base = S.n_iz;
    }
  }
  return PIC_OK;
}

int pic_get_counters(pic_ctx* ctx, int replica, pic_counters* out) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  Replica* R = get_rep(ctx, replica);
  if (!R || !out) return fail(ctx, PIC_EINVAL, "bad replica or out");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  double norms[2] = {0, 0};
  int ctl[4] = {0, 0, 0, 0};
  HIPCHK(ctx, hipMemcpy(norms, R->norms, sizeof(norms), hipMemcpyDeviceToHost));
  HIPCHK(ctx, hipMemcpy(ctl, R->refine_ctl, sizeof(ctl), hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof(*out));
  for (int sp = 0; sp < 2; ++sp) {
    unsigned long long t[TL_N];
    TRY(read_tallies(ctx, *R, sp, t));
    out->n_alive[sp] = R->n_base[sp] - (int64_t)t[TL_DEAD] + (int64_t)t[TL_BORN];
    if (sp == 0) out->n_ionizations = R->iz_base + (int64_t)t[TL_BORN];
    out->cap_violation[sp] = (int64_t)t[TL_CAP];
    out->n_collisions[sp] = (int64_t)t[TL_COLL];
    out->md_particles[sp] = (int64_t)t[TL_MD];
    out->wall_count[0][sp] = R->wall_base[0][sp] + (int64_t)t[TL_W0];
    out->wall_count[1][sp] = R->wall_base[1][sp] + (int64_t)t[TL_W1];
    out->numeric_bad += (int64_t)t[TL_BAD];
    out->tile_fallback += (int64_t)t[TL_FALL];
    out->md_margin[sp] = (int64_t)t[TL_FAST];
  }
  out->step = R->step;
  out->refine_sweeps = R->prec == PIC_FP32R ? ctl[1] : 0;
  out->refine_unconverged = R->prec == PIC_FP32R ? ctl[2] : 0;
  if (R->d_iz_drop) {
    unsigned long long dr = 0;
    HIPCHK(ctx, hipMemcpy(&dr, R->d_iz_drop, 8, hipMemcpyDeviceToHost));
    out->iz_dropped = (int64_t)dr;
  }
  out->refine_residual = norms[1] > 0 ? std::sqrt(norms[0] / norms[1]) : std::sqrt(norms[0]);
  if (R->coul.count) {
    unsigned long long nc = 0;
    HIPCHK(ctx, hipMemcpy(&nc, R->coul.count, sizeof(nc), hipMemcpyDeviceToHost));
    out->n_coulomb = (int64_t)nc;
  }
  return PIC_OK;
}

int pic_profile_enable(pic_ctx* ctx, int on) {
  if (!ctx) return PIC_EINVAL;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->prof = on != 0;
  ctx->ev_used = 0;
  for (auto& v : ctx->ev_pairs) v.clear();
  return PIC_OK;
}

int pic_profile_read(pic_ctx* ctx, int cls, double* total_ms, int64_t* launches) {
  if (!ctx) return PIC_EINVAL;
  if (cls < 0 || cls > PIC_PROF_COULOMB || !total_ms || !launches) return fail(ctx, PIC_EINVAL, "bad arguments");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  for (auto& p : ctx->ev_pairs[cls]) {
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, p.first, p.second));
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)ctx->ev_pairs[cls].size();
  return PIC_OK;
}

int pic_get_tuning(pic_ctx* ctx, pic_tuning* out) {
  if (!ctx || !out) return PIC_EINVAL;
  *out = ctx->tune;
  return PIC_OK;
}

int pic_set_tuning(pic_ctx* ctx, const pic_tuning* t) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  if (!t) return fail(ctx, PIC_EINVAL, "tuning is NULL");
  return apply_tuning(ctx, *t);
}

int pic_autotune(pic_ctx* ctx, int trial_steps, pic_tuning* tried, double* ms_per_step,
                 int capacity, int* n_tried) {
  if (!ctx) return PIC_EINVAL;
  if (ctx->sticky) return ctx->sticky;
  if (trial_steps < 1) return fail(ctx, PIC_EINVAL, "trial_steps < 1");
  if (capacity < 0 || (capacity > 0 && (!tried || !ms_per_step)))
    return fail(ctx, PIC_EINVAL, "bad trial record buffers");
  if (ctx->prof) return fail(ctx, PIC_ESTATE, "autotune while kernel timing is enabled");
  std::vector<hipEvent_t> ev(2 * (size_t)trial_steps, nullptr);
  for (hipEvent_t& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
      return fail(ctx, PIC_EDEVICE, "hipEventCreate failed");
    }
  int count = 0;
  // GPU time per step under t: two untimed steps, then trial_steps steps each
  // bracketed by events
  auto measure = [&](const pic_tuning& t, double* ms) -> int {
    TRY(apply_tuning(ctx, t));
    for (int k = 0; k < 2; ++k) TRY(step_all(ctx));
    ctx->step_ev = &ev;
    ctx->step_ev_used = 0;
    int rc = PIC_OK;
    for (int k = 0; k < trial_steps && rc == PIC_OK; ++k) rc = step_all(ctx);
    ctx->step_ev = nullptr;
    TRY(rc);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    double tot = 0.0;
    for (size_t k = 0; k + 1 < ctx->step_ev_used; k += 2) {
      float f = 0.f;
      HIPCHK(ctx, hipEventElapsedTime(&f, ev[k], ev[k + 1]));
      tot += f;
    }
    *ms = tot / trial_steps;
    if (count < capacity) {
      tried[count] = t;
      ms_per_step[count] = *ms;
    }
    ++count;
    return PIC_OK;
  };
  pic_tuning best = ctx->tune;
  double best_ms = 0.0;
  int rc = measure(best, &best_ms);
  // coordinate search: sort interval, tile margin, the batched push, graphs
  std::vector<pic_tuning> cands;
  for (int axis = 0; axis < 4 && rc == PIC_OK; ++axis) {
    cands.clear();
    if (axis == 0) {
      for (int si : {4, 6, 8, 12, 16}) {
        pic_tuning t = best;
        t.sort_interval = si;
        cands.push_back(t);
      }
    } else if (axis == 1) {
      for (int m : {1, 2, 3}) {
        pic_tuning t = best;
        t.tile_margin = m;
        cands.push_back(t);
      }
    } else if (axis == 2 && ctx->batchable) {
      pic_tuning t = best;
      t.batch_push = 0;
      cands.push_back(t);
      for (int k : {2, 3, 4, 6}) {
        t = best;
        t.batch_push = 1;
        t.batch_blocks = (k * ctx->n_cu + 7) / 8 * 8;
        cands.push_back(t);
      }
    } else if (axis == 3) {
      pic_tuning t = best;
      t.use_graphs = 1 - best.use_graphs;
      cands.push_back(t);
    }
    // the state evolves under the trials (the plasma keeps moving), so each
    // candidate is compared with the incumbent timed just before and just
    // after it, which cancels a drift that is linear in time
    for (const pic_tuning& t : cands) {
      if (std::memcmp(&t, &best, sizeof(t)) == 0) continue;
      double ms = 0.0, again = 0.0;
      rc = measure(t, &ms);
      if (rc == PIC_OK) rc = measure(best, &again);
      if (rc != PIC_OK) break;
      if (ms < 0.5 * (best_ms + again)) {
        best = t;
        best_ms = ms;
      } else {
        best_ms = again;
      }
    }
  }
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  if (n_tried) *n_tried = count;
  if (rc != PIC_OK) return rc;
  return apply_tuning(ctx, best);
}

int pic_derived(pic_ctx* ctx, int replica, double out[7]) {
  if (!ctx) return PIC_EINVAL;
  Replica* R = get_rep(ctx, replica);
  if (!R || !out) return fail(ctx, PIC_EINVAL, "bad replica or out");
  out[0] = R->w;
  out[1] = (double)R->Qp;
  out[2] = R->n_gas;
  out[3] = R->g_cap[0];
  out[4] = R->g_cap[1];
  out[5] = (double)R->T_null[0];
  out[6] = (double)R->T_null[1];
  return PIC_OK;
}

}  // extern "C"
