/*
 * kaldo.h -- C ABI of the MI355X (gfx950) three-phonon linewidth library.
 *
 * The library computes, on one GPU, the hot path of anharmonic lattice
 * dynamics (Barbalinardo et al., arXiv:2009.01967):
 *
 *   kaldo_phonons     harmonic modes on a Gamma-centred q grid
 *                     (Sec. II.A: D = phi''/sqrt(m m'), eq. eigenvectors_crystal;
 *                      Sec. II.B eq. velocity_crystal for group velocities)
 *   kaldo_linewidths  three-phonon projection and scattering-rate sum
 *                     (Sec. II.B: eq. projection_plus, gamma_operators,
 *                      phase_space, delta_deconstructed, and Gamma^0), giving
 *                     the linewidth gamma of every mode
 *   kaldo_kappa_rta   RTA conductivity of a crystal (Sec. II.B, eq. RTA)
 *   kaldo_mode_diffusivity  mode diffusivity at Gamma (Sec. II.C)
 *   kaldo_kappa_qhgk  QHGK conductivity at Gamma (Sec. II.C,
 *                     eq. conductivity_amorphous .. lorentzian_amorphous),
 *                     with the bandwidth and threshold options of Appendix A
 *                     (kaldo_qhgk_options)
 *   kaldo_kappa_bte   full linearised BTE (Sec. II.B), inverse or
 *                     self-consistent
 *   kaldo_gamma_interpolate  gamma(omega) from a smaller cell by cubic
 *                     splines (Sec. II.C, Sec. IV.B)
 *
 * Units: length A, mass amu, energy eV (fc2 in eV/A^2, fc3 in eV/A^3),
 * temperature K, frequency nu in THz, angular frequency and linewidth in
 * rad/ps, velocity in A/ps, conductivity in W/(m K).
 *
 * Conventions (the same as the paper's, with its open points read as follows):
 *  - fc2 block (i, j, R): d2E / du(i, home cell) du(j, cell R); R integer
 *    lattice coordinates; Cartesian offset R . cell (cell rows are lattice
 *    vectors).  fc3 block (i, j, R1, l, R2): d3E / du(i,0) du(j,R1) du(l,R2).
 *    Blocks with equal keys are summed.  The Bloch phase uses the lattice
 *    vector only: chi = exp(-2 pi i q.R).
 *  - The q grid is Gamma centred: q_k = (m1/G1, m2/G2, m3/G3) in reduced
 *    reciprocal coordinates with k = (m1 G2 + m2) G3 + m3.
 *  - omega = sign(lambda) sqrt(|lambda|).  Modes with nu < 0.01 THz take no
 *    part anywhere (gamma = 0, no kappa contribution).
 *  - gamma_mu = Gamma^0_mu = (1/N_k) [sum Gamma+ + 1/2 sum Gamma-] is the
 *    half width (rad/ps); tau = 1 / (2 gamma).  The energy delta is a Gaussian
 *    of standard deviation 2 pi sigma_thz in angular frequency, or a
 *    Lorentzian or triangle of that width (kaldo_delta).
 *  - gamma is averaged over each set of degenerate modes at one k (chained
 *    frequency gaps below 1e-5 THz); only set averages are basis independent.
 *
 * Memory and ownership:
 *  - Input arrays passed in the structs below are HOST memory owned by the
 *    caller; they are read during the call, copied into device memory owned
 *    by the context, and never retained.
 *  - Output arrays may be host memory or device memory of the context's GPU
 *    (HIP unified addressing decides).  Device outputs are written in order
 *    on the context's stream; host outputs are complete when the call returns.
 *  - Passing NULL for a structure, fc2 or fc3 argument reuses the copy already
 *    resident on the device from the previous call on the same context (no
 *    host-to-device transfer).  It is an error (KALDO_ESTATE) when none exists.
 *
 * Errors: every call returns a kaldo_status; nothing aborts or throws across
 * the ABI.  kaldo_last_error() gives a text for the last failing call.  A
 * context is not thread safe.  Calls are ordered phonons -> linewidths ->
 * kappa; a call whose prerequisites are missing returns KALDO_ESTATE.
 */
#ifndef KALDO_H
#define KALDO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kaldo_ctx_s* kaldo_ctx;

typedef enum {
  KALDO_OK = 0,
  KALDO_EINVAL = -1,    /* bad argument: shape, index, NULL pointer, value range */
  KALDO_ENOMEM = -2,    /* device allocation failed */
  KALDO_EDEVICE = -3,   /* HIP / rocSOLVER runtime error */
  KALDO_ESTATE = -4,    /* call out of order (no phonons / linewidths yet) */
  KALDO_EUNSTABLE = -5, /* imaginary mode below -0.05 THz (offending k, s in error text) */
  KALDO_ENOCONV = -6    /* the self-consistent series of kaldo_kappa_bte did not converge */
} kaldo_status;

typedef enum {
  KALDO_FP64 = 0,      /* projection and epilogue in FP64 (reference GPU path) */
  KALDO_FP32 = 1,      /* projection in FP32, FP32 partial sums, FP64 accumulation */
  KALDO_BF16X3 = 2     /* projection GEMMs as BF16 hi+lo split (3 MFMAs), FP32 accumulate */
} kaldo_precision;

/* Finite-width energy delta of eq. delta_deconstructed (the three kinds the
 * paper's appendix names).  Each has unit area in angular frequency with the
 * width s = 2 pi sigma_thz: Gaussian of standard deviation s; Lorentzian of
 * half width at half maximum s; triangle of half base s. */
typedef enum {
  KALDO_DELTA_GAUSS = 0,
  KALDO_DELTA_LORENTZ = 1,
  KALDO_DELTA_TRIANGLE = 2
} kaldo_delta;

typedef enum {
  KALDO_QUANTUM = 0,    /* Bose-Einstein occupations (eq. bose_einstein) */
  KALDO_CLASSICAL = 1   /* n = k_B T / (hbar omega) (Sec. II.D) */
} kaldo_stats;

typedef enum {
  KALDO_TUNE_AUTO = 0,  /* time the candidate tile shapes of each GEMM problem once, keep the fastest */
  KALDO_TUNE_FIXED = 1, /* fixed tile shapes: results bitwise reproducible across contexts */
  KALDO_TUNE_SHAPE0 = 2 /* KALDO_TUNE_SHAPE0 + v: tile shape v (0 .. 15) of every GEMM (for tests) */
} kaldo_tuning;

/* How kaldo_kappa_bte solves the full linearised BTE (paper Sec. II.B):
 * direct inversion of the scattering operator (eqs. inversemeanfreepath,
 * full_conductivity) or the self-consistent series (eqs.
 * mfp_from_scattering_inv, self-consistent). */
typedef enum {
  KALDO_BTE_INVERSE = 0,
  KALDO_BTE_SELF_CONSISTENT = 1
} kaldo_bte_method;

/* At most this many temperatures per kaldo_linewidths call. */
#define KALDO_MAX_T 8

typedef struct {
  double cell[9];            /* rows = lattice vectors [A] */
  int32_t n_atoms;           /* N >= 1; number of modes n = 3N */
  const double* positions;   /* [N][3] Cartesian [A] */
  const double* masses;      /* [N] [amu], > 0 */
} kaldo_structure;

typedef struct {
  int64_t n_blocks;
  const int32_t* i;          /* [nb], 0 <= i < N */
  const int32_t* j;          /* [nb] */
  const int32_t* R;          /* [nb][3], |R_c| <= 15 */
  const double* blocks;      /* [nb][3][3] eV/A^2 */
} kaldo_fc2;

typedef struct {
  int64_t n_blocks;
  const int32_t* i;          /* [nb] home-cell atom */
  const int32_t* j;          /* [nb] */
  const int32_t* l;          /* [nb] */
  const int32_t* R1;         /* [nb][3] cell of atom j, |R_c| <= 7 */
  const int32_t* R2;         /* [nb][3] cell of atom l, |R_c| <= 7 */
  const double* blocks;      /* [nb][3][3][3] eV/A^3 */
} kaldo_fc3;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * run on (NULL: the context creates and owns its own stream). */
kaldo_status kaldo_create(kaldo_ctx* out, int device, void* hip_stream);

/* Release all device memory of the context.  NULL is accepted. */
void kaldo_destroy(kaldo_ctx ctx);

/* Device memory from the caller (for instance one torch.empty(bytes,
 * dtype=uint8, device='cuda') tensor) instead of the library's own hipMalloc
 * (memory plumbing, not a step of the method).  From this call on, every device
 * buffer of the context, and of the crystals it batches, is carved from
 * [dev_ptr, dev_ptr + bytes), front to back, 256-byte aligned; a buffer that
 * grows takes a new piece and the old one is not reused, so size the workspace
 * generously.  The caller keeps the memory allocated and leaves it alone until
 * kaldo_destroy.  The rocBLAS/rocSOLVER handle keeps its own small workspace.
 *   dev_ptr  device memory on the context's device (NULL with bytes 0: back to
 *            the library's allocations)
 * A call that needs more than what is left returns KALDO_ENOMEM; its error text
 * says how many bytes were missing.  Errors: KALDO_ESTATE unless the context
 * holds no data yet (no phonons, fc3 or batch), KALDO_EINVAL for memory that is
 * not device memory of the context's device. */
kaldo_status kaldo_set_workspace(kaldo_ctx ctx, void* dev_ptr, size_t bytes);

/* Text of the last error on this context ("" if none); valid until the next
 * call on the context. */
const char* kaldo_last_error(kaldo_ctx ctx);

/* Harmonic modes (paper Sec. II.A-B).  Builds D(q_k) = sum_R fc2 / sqrt(m m')
 * exp(-2 pi i q_k.R) for every grid point, diagonalises it in FP64 on the GPU,
 * and keeps frequencies, eigenvectors and velocity data resident for the later
 * calls.
 *   grid     [3] grid sizes, each >= 1, product <= 2^22
 *   nu_out   [Nk][n] frequencies nu = omega / 2 pi [THz], or NULL
 *   vel_out  [Nk][n][3] group velocities [A/ps] (basis dependent inside a
 *            degenerate set), or NULL.  Not computed for grid {1,1,1}.
 * Returns KALDO_EUNSTABLE if some nu < -0.05 THz. */
kaldo_status kaldo_phonons(kaldo_ctx ctx, const kaldo_structure* structure, const kaldo_fc2* fc2,
                           const int32_t grid[3], double* nu_out, double* vel_out);

/* Three-phonon linewidths (paper Sec. II.B) of every mode on the grid of the
 * last kaldo_phonons call, for each of nT temperatures.
 *   T          [nT] temperatures [K] (> 0 unless classical), 1 <= nT <= KALDO_MAX_T
 *   sigma_thz  width of the energy delta in THz (see kaldo_delta), > 0
 *   delta      kind of energy delta; the GPU drops a 16 x 16 tile of GEMM
 *              products whose Gaussian arguments all exceed 6 sigma (mixed
 *              precisions) or 8.9 sigma (FP64), or that all lie outside the
 *              triangle, and never runs a GEMM block tile all of whose
 *              products would be dropped (frequencies ascend within a grid
 *              point, so the test uses interval bounds); the FP32 few-branch
 *              kernel skips a column s'' for a wavefront of 64 partners when
 *              all of its elements lie beyond the same cut; Lorentzian tails
 *              are kept
 *   gamma_out  [nT][Nk][n] linewidths [rad/ps], set averaged, or NULL (kept
 *              resident for kaldo_kappa_*)
 * Every precision is accepted on every grid.  Cells with n = 3 or 6 branches
 * and grid != {1,1,1} use a few-branch VALU kernel for FP64 and FP32 (in
 * FP32 it sums each (Delta, -Delta) pair of fc3 cell offsets through the sum
 * and difference of their two terms, whose phases are conjugate); all
 * other cases run the projection as MFMA GEMMs (Gamma: real, else complex). */
kaldo_status kaldo_linewidths(kaldo_ctx ctx, const kaldo_fc3* fc3, const double* T, int32_t nT,
                              double sigma_thz, kaldo_delta delta, kaldo_stats stats,
                              kaldo_precision precision, double* gamma_out);

/* Normalised three-phonon phase space per mode (paper Sec. II.B, eq.
 * phase_space and the per-mode sum that follows it) of every mode on the grid
 * of the last kaldo_phonons call, for each of nT temperatures:
 *   g_mu = (1/N_k) [ sum (n' - n'') delta(w + w' - w'')  over k'' = k + k'
 *                  + 1/2 sum (1 + n' + n'') delta(w - w' - w'')  over k'' = k - k' ]
 * summed over k', s', s'': the linewidth sum with the matrix-element factor
 * (hbar pi / 8) |phi|^2 / (w w' w'') replaced by 1, hence the same 1/N_k and
 * 1/2 on decay.  Needs frequencies only (no fc3); runs in FP64.
 *   T, sigma_thz, delta, stats  as for kaldo_linewidths
 *   g_out      [nT][Nk][n] phase space [ps/rad] (host or device), required;
 *              0 for masked modes (nu < 0.01 THz).  Nothing is kept resident
 *              and the state used by kaldo_kappa_* is not touched.
 * Errors: KALDO_ESTATE before kaldo_phonons, KALDO_EINVAL for bad arguments or
 * g_out == NULL. */
kaldo_status kaldo_phase_space(kaldo_ctx ctx, const double* T, int32_t nT, double sigma_thz, kaldo_delta delta,
                               kaldo_stats stats, double* g_out);

/* RTA conductivity (paper eq. RTA) from the last linewidths:
 *   kappa_out [nT][3][3] W/(m K).  Degenerate sets enter through the basis
 *   invariant Re Tr(W_a W_b) / (4 omega^2), W = E_set^H dD/dq E_set.
 * Requires a grid other than {1,1,1}. */
kaldo_status kaldo_kappa_rta(kaldo_ctx ctx, double* kappa_out);

/* Conductivity of the full linearised BTE (paper Sec. II.B) with the
 * off-diagonal scattering operator, for the temperatures, delta, statistics
 * and grid of the last kaldo_linewidths call (its fc3 resident):
 *   Gamma^1_mu nu = (w_nu / w_mu) (1/N_k) sum_mu'' [Gamma+_mu nu mu'' - Gamma+_mu mu'' nu
 *                   - 1/2 Gamma-_mu nu mu'' - 1/2 Gamma-_mu mu'' nu],
 * the coefficients of the linearised scattering term of Sec. II.B (with the
 * 1/N_k and the 1/2 on creation that the linewidth Gamma^0 carries), and
 *   kappa = 1/(N_k V) sum c_mu v_mu [2 (Gamma^0 + Gamma^1)]^-1_mu nu v_nu,
 * the factor 2 making Gamma^1 = 0 the RTA of kaldo_kappa_rta (tau = 1/(2 gamma)).
 * Within each degenerate set only set sums of the operator are basis
 * independent: it acts on the set means of the deviation (block sums over
 * the row and column sets) and the rest of each set relaxes with its linewidth
 * (RTA); heat capacity and Gamma^0 are set averages.  The set means are solved
 * on the vectors odd under k -> -k (the velocity is odd; this halves the system
 * and leaves out the near-zero mode of uniform deviations).
 *   method     KALDO_BTE_INVERSE: LU factorisation (rocSOLVER), or
 *              KALDO_BTE_SELF_CONSISTENT: partial sums of
 *              sum_n (-Gamma^1 / Gamma^0)^n v / (2 Gamma^0) until the last term
 *              is at most tol times the sum (largest entries), at most
 *              max_terms terms (>= 1)
 *   kappa_out  [nT][3][3] W/(m K), host or device memory, required
 *   terms_out  terms of the series (the most over the temperatures), 0 for
 *              the inverse; may be NULL
 * The operator is computed in FP64 whatever the precision of the last
 * linewidths; it takes 3 N_k^2 n^2 doubles per temperature.  Cells with 1 or
 * 2 atoms (n = 3 or 6) on grids other than {1,1,1}, without a k range.
 * Errors: KALDO_ESTATE before kaldo_linewidths; KALDO_EINVAL for other cells,
 * a k range, bad arguments; KALDO_EUNSTABLE for a singular operator;
 * KALDO_ENOCONV when the series has not converged after max_terms terms
 * (kappa_out then holds the last partial sum). */
kaldo_status kaldo_kappa_bte(kaldo_ctx ctx, kaldo_bte_method method, int32_t max_terms, double tol,
                             double* kappa_out, int32_t* terms_out);

/* kaldo_kappa_rta without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same result as kaldo_kappa_rta, computed by the same
 * kernels, but the partial sums and the reduced kappa live in a static device
 * array of the library (KALDO_MAX_T * 65 * 9 doubles, 37 KB, one per device,
 * held until the process ends) instead of context buffers; nothing is
 * allocated or freed and no context buffer is touched.
 *   kappa_out [nT][3][3] W/(m K), host or device memory, required.
 * Every call on one GPU shares that GPU's array, so calls that overlap on one
 * GPU (several host threads, or several streams in flight) race; calls in
 * order on one stream do not.  Each call writes every entry it later reads.
 * Errors: KALDO_ESTATE before kaldo_linewidths, KALDO_EINVAL for a grid
 * {1,1,1}, kappa_out == NULL or more scratch than the array holds,
 * KALDO_EDEVICE if the array's device address could not be obtained. */
kaldo_status kaldo_kappa_rta_noalloc(kaldo_ctx ctx, double* kappa_out);

/* QHGK conductivity (paper Sec. II.C) at Gamma from the last linewidths:
 *   kappa_out [nT][3][3] W/(m K).  Requires grid {1,1,1}; V is the cell volume.
 * Generalised heat capacity with the sign that makes it positive,
 * (hbar w w'/T)(n' - n)/(w - w'); generalised velocity summed over fc2 blocks
 * with the displacement x_i - (x_j + R.cell). */
kaldo_status kaldo_kappa_qhgk(kaldo_ctx ctx, double* kappa_out);

/* Mode diffusivity at Gamma (paper Sec. II.C, eq. diffusivity_per_mode) from
 * the last linewidths, per Cartesian direction a:
 *   d_out [nT][n][3]  D_{mu,a} = sum_mu' |v_{mu mu' a}|^2 tau_{mu mu'} in mm^2/s,
 * with the generalised velocity and Lorentzian lifetime of kaldo_kappa_qhgk.
 * The printed prefactor 1/(N_k V) is not applied (with it the result would
 * not have a diffusivity's units); in the classical limit
 * k_B sum_mu D_{mu,a} = V kappa_aa.  Masked modes get 0.  d_out is a host or
 * device pointer owned by the caller.
 * Errors: KALDO_ESTATE before kaldo_linewidths, KALDO_EINVAL for a grid other
 * than {1,1,1} or d_out == NULL. */
kaldo_status kaldo_mode_diffusivity(kaldo_ctx ctx, double* d_out);

/* Adaptive widths of the energy delta (paper Appendix A: in crystals the width
 * can be estimated from the phonon velocities) for the later kaldo_linewidths
 * calls on this context.  scale a > 0: every process gets its own Gaussian of
 * standard deviation
 *   max(a sigma_grid, 2 pi sigma_thz),
 *   sigma_grid = sqrt(sum_a ((v' -+ v'') . b_a / G_a)^2 / 12),
 * the spread of the energy mismatch w +- w' - w'' when the partner q' moves
 * over one cell of the q grid (reciprocal vectors b_a = 2 pi cell^-T rows,
 * grid divisions G_a; - for absorption, + for decay in the partners (p, k+p)
 * of one V); v are the mean group velocities of the modes' degenerate sets
 * (basis independent), and sigma_thz of the kaldo_linewidths call is the
 * smallest width.  0 turns it off (the default).  With adaptive widths
 * kaldo_linewidths needs the Gaussian delta and a grid other than {1,1,1}
 * (KALDO_EINVAL otherwise), and no tile is skipped by the delta window;
 * kaldo_kappa_bte takes the fixed width and refuses such linewidths; the
 * batch calls and kaldo_phase_space keep fixed widths.
 * Errors: KALDO_EINVAL for a negative or non-finite scale. */
kaldo_status kaldo_adaptive_width(kaldo_ctx ctx, double scale);

/* Options of the QHGK conductivity (paper Appendix A, the "QHGK" engine) for
 * the later kaldo_kappa_qhgk and kaldo_mode_diffusivity calls on this context:
 *   bandwidth  eta [rad/ps] > 0: every mode's linewidth in the Lorentzian
 *              lifetime is eta, tau_{mu mu'} = 2 eta / ((w - w')^2 + 4 eta^2)
 *              (the broadened delta of the Allen-Feldman model); 0: the
 *              resident linewidths (the default)
 *   threshold  w_thr [rad/ps] > 0: tau_{mu mu'} = 0 when |w - w'| > w_thr
 *              (the paper prints the inequality reversed, which would drop
 *              the diagonal); the kernels then read only the band of
 *              frequency-close pairs of V_d; 0: every pair (the default)
 * Errors: KALDO_EINVAL for negative or non-finite values. */
kaldo_status kaldo_qhgk_options(kaldo_ctx ctx, double bandwidth, double threshold);

/* Installs linewidths computed elsewhere as the resident gamma of the modes
 * of the last kaldo_phonons call, with the temperatures and statistics the
 * conductivity calls use (paper Sec. II.C: QHGK needs only gamma_mu; with a
 * bandwidth (kaldo_qhgk_options) it needs none, the Allen-Feldman model).
 *   T       [nT] temperatures [K], host memory, 1 <= nT <= KALDO_MAX_T
 *   gamma   [nT][Nk][n] linewidths [rad/ps], finite and >= 0, host or device
 *           memory; NULL installs zeros
 * The resident gamma then serves kaldo_kappa_rta, kaldo_kappa_qhgk and
 * kaldo_mode_diffusivity; kaldo_kappa_bte still needs kaldo_linewidths.
 * Errors: KALDO_ESTATE before kaldo_phonons, KALDO_EINVAL for bad arguments. */
kaldo_status kaldo_set_gamma(kaldo_ctx ctx, const double* T, int32_t nT, kaldo_stats stats, const double* gamma);

/* Linewidths interpolated in frequency (paper Sec. II.C and Sec. IV.B: gamma
 * of a smaller cell, interpolated with third-order splines, for a larger
 * one), installed as the resident gamma of this context's modes as
 * kaldo_set_gamma does.  From the source modes with nu >= 0.01 THz:
 *   1. n_bins bins of equal width between their lowest and highest omega,
 *      bin floor((w - w_lo) / (w_hi - w_lo) n_bins) (the highest mode in the
 *      last bin); each non-empty bin is one knot, (mean omega, mean gamma);
 *   2. the natural cubic spline through the knots (second derivative 0 at
 *      both ends; one knot: a constant, two: a line), per temperature;
 *   3. every mode of this context gets the spline at its omega, the end
 *      knot's gamma outside the knots, at least the smallest knot gamma;
 *      masked modes 0; averaged over each degenerate set.
 *   T          [nT] temperatures [K], host memory, 1 <= nT <= KALDO_MAX_T
 *   omega_src  [n_src] source angular frequencies [rad/ps] (2 pi nu), host
 *              or device memory
 *   gamma_src  [nT][n_src] source linewidths [rad/ps], host or device memory
 *   n_bins     1 <= n_bins <= 4096
 *   gamma_out  [nT][Nk][n] the interpolated linewidths [rad/ps], host or
 *              device memory, or NULL (kept resident either way)
 * Runs on the GPU (binning, spline solve, evaluation) on the context's stream.
 * Errors: KALDO_ESTATE before kaldo_phonons; KALDO_EINVAL for bad arguments
 * or no source mode with nu >= 0.01 THz (found on the GPU: reported after a
 * synchronisation of the stream). */
kaldo_status kaldo_gamma_interpolate(kaldo_ctx ctx, const double* T, int32_t nT, kaldo_stats stats,
                                     const double* omega_src, const double* gamma_src, int64_t n_src,
                                     int32_t n_bins, double* gamma_out);

/* Batches: the linewidths of many crystals (uneven cell sizes and grids) in
 * one HIP graph launch.
 *
 * kaldo_batch_add computes the harmonic modes of one crystal on its grid
 * (paper Sec. II.A-B, as kaldo_phonons) and keeps them with its fc3 (as
 * kaldo_linewidths would) in a crystal context owned by ctx; *handle receives
 * the crystal's index in the batch (0, 1, ...).  All four inputs are required
 * host data, copied and not retained.  Errors as kaldo_phonons; adding a
 * crystal drops a captured graph.
 *
 * kaldo_batch_run computes the linewidths (paper Sec. II.B, as
 * kaldo_linewidths with the Gaussian delta) of every mode of every crystal for
 * nT temperatures.  The first call with a given (T, sigma, statistics,
 * precision) plans the batch (sizes every device buffer, builds the static
 * operands), then captures on the context's stream into one HIP graph: one
 * persistent kernel for every crystal that takes the MFMA GEMM path, working
 * through a table of rounds (crystal, first-mode point k, range of partners)
 * with the crystals in order of decreasing cost (points x N_k x n^4) and the
 * stages of each round (step A of a new k, step B, the two GEMMs with the
 * fused linewidth epilogue, the collection) separated by grid barriers; the
 * few-branch crystals (1 or 2 atoms, FP32 or FP64) add their own kernels.  The
 * persistent grid holds the workgroups that fit on the device at once; a
 * barrier that waits for more than about a second returns KALDO_EDEVICE (and
 * leaves the results incomplete) instead of hanging.  That and later calls with
 * the same arguments launch the graph once and wait for it.
 * The context's stream must not be the null stream (pass NULL to kaldo_create
 * to get an owned one).  gamma_out, if not NULL, holds one pointer per crystal
 * in handle order, each to [nT][Nk_i][n_i] doubles (host or device memory) or
 * NULL to skip that crystal.  Returns KALDO_ESTATE for an empty batch, and for
 * arguments other than those the batch's graph was captured with (a context
 * captures one graph per batch: kaldo_batch_clear and add the crystals again,
 * or use a second context, for other arguments); the first failing crystal's
 * status otherwise.
 *
 * kaldo_batch_clear releases every crystal of the batch and the graph. */
kaldo_status kaldo_batch_add(kaldo_ctx ctx, const kaldo_structure* structure, const kaldo_fc2* fc2,
                             const kaldo_fc3* fc3, const int32_t grid[3], int32_t* handle);
kaldo_status kaldo_batch_run(kaldo_ctx ctx, const double* T, int32_t nT, double sigma_thz, kaldo_stats stats,
                             kaldo_precision precision, double* const* gamma_out);
/* kaldo_batch_plan does the planning and capture of kaldo_batch_run for these
 * arguments (when the batch holds no graph yet) without launching it; errors
 * as kaldo_batch_run. */
kaldo_status kaldo_batch_plan(kaldo_ctx ctx, const double* T, int32_t nT, double sigma_thz, kaldo_stats stats,
                              kaldo_precision precision);
kaldo_status kaldo_batch_clear(kaldo_ctx ctx);

/* One GPU's share of a run sharded over first-mode grid points.  The
 * linewidth of every mode is a sum of its own (paper Sec. II.B, Gamma^0), and
 * the RTA conductivity (eq. RTA) is a sum over modes, so both split over
 * disjoint ranges of first-mode points k.
 *
 * kaldo_set_k_range restricts later kaldo_linewidths calls on ctx to the
 * points k_begin <= k < k_end of the grid (clamped to N_k; a call whose
 * clamped range is empty returns KALDO_EINVAL).  gamma of the other points is
 * returned as 0, and kaldo_kappa_rta then sums the covered modes only: the
 * kappa of the shards [0, K1), [K1, K2), ... add up to the kappa of the full
 * grid.  (0, INT32_MAX) is the default, the whole grid.  QHGK (grid {1,1,1})
 * has the single point k = 0.  Errors: KALDO_EINVAL unless
 * 0 <= k_begin < k_end.
 *
 * kaldo_batch_set_k_range does the same for crystal `handle` of the batch
 * (0 <= k_begin < N_k of that crystal), and drops a captured graph. */
kaldo_status kaldo_set_k_range(kaldo_ctx ctx, int32_t k_begin, int32_t k_end);
kaldo_status kaldo_batch_set_k_range(kaldo_ctx ctx, int32_t handle, int32_t k_begin, int32_t k_end);

/* Tile-shape selection for the MFMA GEMMs (not a step of the method).  With
 * KALDO_TUNE_AUTO (the default) the first call that meets a GEMM shape times
 * each candidate tile shape once and keeps the fastest for the context; the
 * results of different tile shapes agree to rounding, not bitwise.
 * KALDO_TUNE_FIXED uses one fixed shape per problem.  KALDO_TUNE_SHAPE0 + v
 * forces candidate v of every GEMM problem (shape 0 where a problem has fewer
 * candidates), so that tests can reach every tile shape.  Returns KALDO_EINVAL for
 * an unknown mode. */
kaldo_status kaldo_set_tuning(kaldo_ctx ctx, kaldo_tuning mode);

/* Kernel timing instrumentation (not a step of the method).  While enabled,
 * the library records a pair of HIP events on the context's stream around
 * every launch of its main kernels, named
 *   "dyn_assemble", "eigensolve", "step_a", "step_b", "gamma_sparse",
 *   "project", "finalize", "kappa_rta", "kappa_qhgk", "diffusivity" and "batch_graph"
 *   around a kaldo_batch_run graph launch, and the phases of the persistent
 *   batch kernel as workgroup 0 sees them (its own work in each stage, summed
 *   over the rounds): "batch_a_collect" (step A, collection, Y padding),
 *   "batch_step_b", "batch_gemm1", "batch_gemm2", "batch_barrier_wait" (its
 *   waits at grid barriers; "batch_wait_gemm1_phase" and
 *   "batch_wait_gemm2_phase" split them by the phase they end) and
 *   "batch_set_average"; and each crystal's share of the launch,
 *   "batch_crystal_<handle>" (workgroup 0's clock over the crystal's rounds).
 * kaldo_profile_enable(ctx, 1) enables and clears the totals, 0 disables
 * and clears them.
 * kaldo_profile_read synchronises the stream and returns, for one kernel
 * name, the summed duration (ms) and the number of launches since enabling;
 * an unknown name gives 0 and 0.
 * kaldo_profile_flops synchronises the stream and returns the matrix-core
 * flops of the projection GEMMs (those timed as "project": GEMM 1 and GEMM 2 of
 * the many-branch path, the Gamma-point GEMM) since enabling: `executed` counts the block tiles that ran (BF16X3
 * counts its three bf16 products), `dense` every tile launched, including the
 * tiles skipped because all their outputs lie beyond the delta cut.  The
 * persistent kernel of kaldo_batch_run counts its GEMM tiles the same way
 * (read after each launch); the few-branch kernel is not counted.  Either
 * pointer may be NULL.  Enabling allocates the 8-byte device counter with
 * hipMalloc, outside any workspace set by kaldo_set_workspace. */
kaldo_status kaldo_profile_enable(kaldo_ctx ctx, int enable);
kaldo_status kaldo_profile_read(kaldo_ctx ctx, const char* kernel, double* total_ms, int64_t* launches);
kaldo_status kaldo_profile_flops(kaldo_ctx ctx, double* executed, double* dense);

#ifdef __cplusplus
}
#endif

#endif /* KALDO_H */
