// Internal declarations of the gfx950 linewidth library: context, device
// buffers, physical constants and kernel launchers.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/kaldo.h"

namespace kaldo {

// ---- physical constants (CODATA 2018) -------------------------------------
constexpr double kHbar = 6.582119569e-4;                  // eV ps
constexpr double kBoltzmann = 8.617333262e-5;             // eV / K
constexpr double kElectronVolt = 1.602176634e-19;         // J
constexpr double kAmu = 1.66053906660e-27;                // kg
// 1 eV in amu A^2 / ps^2
constexpr double kEvUnit = kElectronVolt / (kAmu * 1e-20 / 1e-24);
// eV / (K A ps) -> W / (m K)
constexpr double kKappaSI = kElectronVolt / (1e-10 * 1e-12);
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.141592653589793238462643383279;
constexpr double kNuMinThz = 0.01;       // modes below are excluded
// Internal delta kind: Gaussian whose width is set per process from the
// velocities of its two partner modes (kaldo_adaptive_width)
constexpr int kDeltaGaussAdaptive = 3;
constexpr double kNuUnstableThz = -0.05; // below: imaginary mode error
constexpr double kDegenerateThz = 1e-5;  // chained gap for degenerate sets

// ---- device buffer ----------------------------------------------------------
// A caller's workspace (kaldo_set_workspace): buffers are carved from it front
// to back, 256-byte aligned, and never handed back one by one.
struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
  size_t short_by = 0;  // bytes missing at the last failed carve
};
// The workspace of the context whose library call is running on this thread
// (null: buffers come from hipMalloc).  Set for the duration of a call by ArenaScope.
extern thread_local Arena* g_arena;
struct ArenaScope {
  Arena* prev;
  explicit ArenaScope(Arena* a) : prev(g_arena) { g_arena = a && a->base ? a : nullptr; }
  ~ArenaScope() { g_arena = prev; }
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool ext = false;  // carved from a caller's workspace (not ours to free)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p && !ext) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    ext = false;
  }
  // (Re)allocate to at least n bytes; contents are not preserved.
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    if (n == 0) n = 16;
    if (g_arena) {
      const size_t off = (g_arena->used + 255) & ~(size_t)255;
      if (off > g_arena->size || n > g_arena->size - off) {
        g_arena->short_by = off + n - g_arena->size;
        return hipErrorOutOfMemory;
      }
      p = g_arena->base + off;
      g_arena->used = off + n;
      bytes = n;
      ext = true;
      return hipSuccess;
    }
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    else p = nullptr;
    return e;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

struct Fc3Layout {
  int64_t n_blocks = 0;
  int n_delta = 0;
  int n_dpair = 0;  // leading slot pairs (2m, 2m + 1) holding Delta and -Delta
  std::vector<int> delta;            // [nD][3]
  // Blocks sorted by (delta, j, l); groups (delta, j, l) -> [start, end).
  DevBuf d_group;                    // int2 [nD * N * N]
  DevBuf d_blk_i;                    // int  [nb]
  DevBuf d_blk_R2;                   // int  [nb][3]
  DevBuf d_blk_val;                  // double [nb][27], divided by sqrt(m_i m_j m_l)
  DevBuf d_delta;                    // int  [nD][3]
  // Raw block list (same order as above).
  DevBuf d_blk_j, d_blk_l;           // int [nb]
  // Crystal layout for many branches: the non-empty (Delta, j, l) groups, and
  // per atom pair (j, l) the list of its groups (sorted by Delta).
  int n_cgroups = 0, n_cpairs = 0;
  DevBuf d_cg_block;                 // int2 [ng] block range (in the (Delta, j, l) order)
  DevBuf d_cg_delta;                 // int [ng] Delta index
  DevBuf d_cg_order;                 // int [ng] group indices sorted by (j, l, Delta)
  DevBuf d_cpair;                    // int4 [np] (j, l, first, last+1) into d_cg_order
  DevBuf d_cpairmap;                 // int [N * N] pair (j, l) -> index into d_cpair, or -1
  // Gamma-point layout: blocks sorted by the atom pair (j, l), all cells merged.
  int n_pairs = 0;
  DevBuf d_gpair_start;              // int [npairs + 1] -> block range of each pair
  DevBuf d_gpair_l;                  // int [npairs] atom l of each pair
  DevBuf d_grow_start;               // int [N + 1] -> pair range of each row atom j
  std::vector<int> grow_start;       // host copy of the above
  DevBuf d_gblk_i;                   // int [nb]
  DevBuf d_gblk_val;                 // double [nb][27], divided by sqrt(m_i m_j m_l)
};

}  // namespace kaldo

namespace kaldo {
// Device pointers and sizes of a planned many-branch linewidth run of one
// crystal (recorded by the planning pass; the persistent batch kernel runs the
// crystal from them).  Plain data, copied to the device as is.
struct CrystalPlan {
  int valid, precision;
  int n, N, nk, ng, nd, nT, ldk, mrows, zb, G0, G1, G2, klo, khi;
  int m_tiles2;     // row tiles of both GEMMs in the persistent kernel
  unsigned char rt_fm[32];  // row tile i: 32 rt_fm[i] rows from row 32 rt_u0[i]
  unsigned char rt_u0[32];
  long long xy_elems;  // elements of X (and of Y) for one partner batch
  double C, rs;     // linewidth prefactor / N_k with the delta's normalisation; 1 / delta scale
  void *Z, *Xh, *Xl, *Yh, *Yl;
  const void *Ach, *Acl, *Aph, *Apl;
  const void *E, *cgb, *bi, *bR2, *bval, *PH, *cg_delta, *cg_order, *cpair, *pairmap;
  const int* kmap;
  const double *OM, *IW, *OCC;
  double *partial, *gacc, *graw, *gamma;
  const int* setid;
};

// How a stage runs: kRun launches everything; kPlan sizes every buffer, builds
// the mode tables and settles the tile shape of each GEMM problem, but skips
// the heavy launches; kCapture launches everything with no allocation, no
// memset node, no timing and no host synchronisation (stream capture).
enum RunMode { kRun = 0, kPlan = 1, kCapture = 2 };
}  // namespace kaldo

struct kaldo_ctx_s {
  int mode = kaldo::kRun;

  // kernel timing instrumentation
  bool prof = false;
  struct ProfEntry {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    double total_ms = 0.0;
    int64_t launches = 0;
  };
  std::map<std::string, ProfEntry> prof_tab;
  hipEvent_t prof_open = nullptr;
  kaldo::DevBuf d_prof_flops;        // unsigned long long: MFMA flops of the projection tiles that ran
  double prof_dense = 0.0;           // MFMA flops of every projection tile launched

  // tile shapes chosen by the autotuner, per problem key (kept by tune_owner
  // when set: the crystals of a batch share their parent's choices)
  int tuning = KALDO_TUNE_AUTO;
  std::map<std::string, int> tuned;
  kaldo_ctx_s* tune_owner = nullptr;

  // batch of crystals: resident sub-contexts and the captured linewidth graph
  std::vector<kaldo_ctx_s*> batch;
  hipGraphExec_t batch_exec = nullptr;
  std::vector<double> batch_key;     // parameters the graph was captured with

  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  rocblas_handle blas = nullptr;
  std::string err;

  // structure
  bool have_structure = false;
  int n_atoms = 0;
  double cell[9] = {0};
  std::vector<double> positions, masses;
  kaldo::DevBuf d_positions, d_masses;

  // fc2, blocks sorted by (i, j)
  bool have_fc2 = false;
  int64_t nb2 = 0;
  kaldo::DevBuf d_fc2_pair;          // int2 [N*N] -> [start, end)
  kaldo::DevBuf d_fc2_rows;          // int [N + 1]: the coupled pairs of atom i are [rows[i], rows[i + 1])
  kaldo::DevBuf d_fc2_plist;         // int4 per coupled pair: i, j, first block, end block
  int n_fc2_pairs = 0;
  kaldo::DevBuf d_fc2_R;             // int [nb][3]
  kaldo::DevBuf d_fc2_val;           // double [nb][9]
  kaldo::DevBuf d_fc2_i, d_fc2_j;    // int [nb]

  // phonons
  bool have_phonons = false;
  int grid[3] = {1, 1, 1};
  int nk = 0, nm = 0;
  kaldo::DevBuf d_dyn;               // complex double [Nk][n][n] (column major per k)
  kaldo::DevBuf d_lambda;            // double [Nk][n]
  kaldo::DevBuf d_evec;              // complex double [Nk][n(s)][n(a)]: eta_ks[a]
  kaldo::DevBuf d_omega;             // double [Nk][n] (signed)
  kaldo::DevBuf d_setid;             // int [Nk][n] first mode of the degenerate set
  kaldo::DevBuf d_vv;                // double [Nk][n][9]
  kaldo::DevBuf d_vel;               // double [Nk][n][3]
  kaldo::DevBuf d_info;              // int [Nk]
  kaldo::DevBuf d_work;              // scratch

  // fc3
  bool have_fc3 = false;
  kaldo::Fc3Layout fc3;

  // linewidths
  bool have_gamma = false;
  int nT = 0;
  double T[KALDO_MAX_T] = {0};
  int stats = 0;
  int delta = KALDO_DELTA_GAUSS;
  double sigma_thz = 0.0;               // delta width of the last linewidths
  bool gamma_external = false;          // the resident gamma came from kaldo_set_gamma / kaldo_gamma_interpolate
  double adaptive_scale = 0.0;          // kaldo_adaptive_width: scale of the per-process width (0: off)
  bool gamma_adaptive = false;          // the resident gamma was computed with adaptive widths
  double qhgk_bandwidth = 0.0;          // kaldo_qhgk_options: every linewidth in tau_{mu mu'} (0: off)
  double qhgk_threshold = 0.0;          // kaldo_qhgk_options: tau = 0 beyond this |w - w'| (0: off)
  kaldo::Arena arena;                   // caller's workspace (kaldo_set_workspace), if any
  int k_begin = 0, k_end = 0x7fffffff;  // first-mode grid points computed (kaldo_set_k_range)
  int g_lo = 0, g_hi = 0;                // the points the resident gamma covers
  kaldo::DevBuf d_gamma;             // double [nT][Nk][n]
  kaldo::DevBuf d_tabs;              // per-call mode tables
  kaldo::DevBuf d_phase;             // phase space: mode tables and g [nT][Nk][n]
  kaldo::DevBuf d_A;                 // step-A intermediate
  kaldo::DevBuf d_partial;           // partial sums
  kaldo::DevBuf d_kappa;             // double [nT][9]
  kaldo::DevBuf d_diff;              // double [nT][n][3] mode diffusivity (Gamma)
  kaldo::DevBuf d_scratch2;
  kaldo::DevBuf d_bte;               // full BTE: scattering operator pieces, set tables, solve
  kaldo::DevBuf d_klist;             // first-mode points a linewidth run computes (int)
  kaldo::DevBuf d_interp;            // gamma interpolation: source modes, bins, knots, raw values
  kaldo::DevBuf d_adapt;             // adaptive widths: scaled velocity projections [n][3][Nk]
  kaldo::CrystalPlan cplan{};        // the last planning pass of the many-branch path
  size_t xy_budget = (size_t)256 << 20;  // bytes of step-B and GEMM-1 outputs per partner batch
  bool xy_shared = false;                // planning a batch: X and Y come from the parent's shared pool
  // persistent batch kernel: plans, rounds and barrier state (parent context)
  kaldo::DevBuf d_batch;
  kaldo::DevBuf d_batch_xy;          // the persistent kernel's shared X and Y pool
  int batch_grid = 0, batch_nplans = 0, batch_nrounds = 0, batch_precision = -1, batch_nt = 1;
  size_t batch_rounds_off = 0, batch_sync_off = 0, batch_times_off = 0;
  std::vector<int> batch_round_handle;  // batch handle of each round's crystal (per-crystal timing)
  double batch_dense = 0.0;          // MFMA flops of every tile of one launch of the persistent kernel
  double prof_batch_executed = 0.0;  // tallied flops of persistent launches since profiling was enabled
  std::vector<int> klist_host;       // its host copy (kept alive for the stream-ordered upload)
};

namespace kaldo {

// error helpers ---------------------------------------------------------------
kaldo_status fail(kaldo_ctx ctx, kaldo_status s, const std::string& msg);
kaldo_status hip_fail(kaldo_ctx ctx, hipError_t e, const char* what);

#define KALDO_HIP(ctx, call)                                          \
  do {                                                                \
    hipError_t _e = (call);                                           \
    if (_e != hipSuccess) return ::kaldo::hip_fail((ctx), _e, #call); \
  } while (0)

// timing instrumentation around a launch (no-ops unless enabled)
void prof_begin(kaldo_ctx ctx);
void prof_end(kaldo_ctx ctx, const char* name);
void prof_clear(kaldo_ctx ctx);

// zero device memory with a fill kernel (capturable, unlike a memset node)
kaldo_status fill_zero(kaldo_ctx ctx, void* p, size_t bytes);

inline bool planning(kaldo_ctx ctx) { return ctx->mode == kPlan; }

// first-mode grid points [k_lo, k_hi) of the next linewidth run, clamped to the grid
inline int k_lo(const kaldo_ctx_s* c) { return c->k_begin < c->nk ? c->k_begin : c->nk; }
inline int k_hi(const kaldo_ctx_s* c) { return c->k_end < c->nk ? c->k_end : c->nk; }
inline bool k_partial(const kaldo_ctx_s* c) { return k_lo(c) > 0 || k_hi(c) < c->nk; }

// First-mode grid points of the next linewidth run.  The linewidth is even
// under time reversal, gamma(-k, s) = gamma(k, s) (D(-q) = conj D(q): the same
// frequencies, conjugate eigenvectors, and the momentum-conserving triples of
// -k are those of k reversed), so only one point of each pair (k, -k) is
// computed, the one with the smaller index, and its values go to both points
// of the pair that lie in the k range (kaldo_set_k_range; the whole grid by
// default).  A shard thus computes exactly what the whole run computes for
// its points.  Returns the sorted representatives.
std::vector<int> linewidth_points(const kaldo_ctx_s* c);
// the same list uploaded to ctx->d_klist (stream ordered; under capture the
// list uploaded by the planning pass is used); returns its length
kaldo_status upload_linewidth_points(kaldo_ctx ctx, int* npts);

// copy a device result into a caller pointer that may be host or device memory
kaldo_status copy_out(kaldo_ctx ctx, void* dst, const void* src, size_t bytes);

template <typename R>
struct cplx;

// FP64 tables of the few-branch path: OM, IW [n][nk], OCC [nT][n][nk],
// PH [nDelta][nk] = e^{2 pi i q_p.Delta}, ET [n][n][nk] = eta (in d_tabs)
struct SmallTables {
  double *OM, *IW, *OCC;
  cplx<double>* PH;
  cplx<double>* ET;
};
kaldo_status small_tables_fp64(kaldo_ctx ctx, SmallTables* t);
kaldo_status small_step_a_fp64(kaldo_ctx ctx, cplx<double>* A, int k0, int kc);

// stages ------------------------------------------------------------------------
kaldo_status run_phonons(kaldo_ctx ctx, bool want_velocity);
kaldo_status run_linewidths(kaldo_ctx ctx, double sigma_thz, int precision);
kaldo_status run_linewidths_gamma(kaldo_ctx ctx, double sigma_thz, int precision);
kaldo_status run_linewidths_crystal(kaldo_ctx ctx, double sigma_thz, int precision);
kaldo_status run_phase_space(kaldo_ctx ctx, const double* T, int nT, double sigma_thz, int delta, int stats,
                             double** g_dev);
kaldo_status run_kappa_rta(kaldo_ctx ctx);
// allocation-free RTA: the device address of the static scratch array of the
// current device (once per device), and the entry point's work
hipError_t noalloc_setup(int device);
kaldo_status run_kappa_rta_noalloc(kaldo_ctx ctx, double* kappa_out);
kaldo_status run_kappa_qhgk(kaldo_ctx ctx);
// the scaled velocity projections of the adaptive widths, UT[s][a][k] (see k_adapt_table)
kaldo_status adaptive_table(kaldo_ctx ctx, double sigma_omega, const double** UT);
kaldo_status run_gamma_interpolate(kaldo_ctx ctx, const double* omega_src, const double* gamma_src, int64_t n_src,
                                   int n_bins);
// gamma[t][k][s] = mean of graw over the degenerate set of (k, s), on the context's stream
kaldo_status launch_set_average(kaldo_ctx ctx, double* gamma, const double* graw, int nT);
kaldo_status copy_in(kaldo_ctx ctx, void* dst, const void* src, size_t bytes);
kaldo_status run_mode_diffusivity(kaldo_ctx ctx);
kaldo_status run_kappa_bte(kaldo_ctx ctx, int method, int max_terms, double tol, double* kappa_out, int* terms_out);
// persistent batch kernel over the crystals of `subs` planned for `precision`:
// prepare (before capture: plans and rounds to the device) and launch (on the
// parent's stream, capturable); check reads its barrier flag after a launch
kaldo_status batch_persistent_prepare(kaldo_ctx parent, const std::vector<kaldo_ctx>& subs, int precision);
kaldo_status batch_persistent_launch(kaldo_ctx parent);
kaldo_status batch_persistent_check(kaldo_ctx parent);

}  // namespace kaldo
