// Full linearised BTE (paper Sec. II.B): the off-diagonal scattering operator
// Gamma^1, the conductivity by direct inversion (eqs. inversemeanfreepath,
// full_conductivity) and by the self-consistent series (eqs.
// mfp_from_scattering_inv, self-consistent), for cells with few branches.
//
// The operator follows the linearised scattering term of Sec. II.B, whose
// coefficient of the deviation of mode nu in the row of mode mu is
//   Gamma^1_mu nu = (w_nu / w_mu) (1/N_k) sum_mu'' [ Gamma+_mu nu mu'' - Gamma+_mu mu'' nu
//                   - 1/2 Gamma-_mu nu mu'' - 1/2 Gamma-_mu mu'' nu ]
// when that of mu itself is the linewidth Gamma^0_mu.  The projection is that
// of the few-branch linewidth kernel: for first mode (k, s) and partner p,
// V[s'][s''] is phi+ of (k,s),(p,s'),(k+p,s''), and the same V (summed over a
// degenerate set of s') is phi- of (k,s),(-p,s'),(k+p,s'').  Instead of
// reducing the rates to one number per mode, the scatter kernel keeps three
// sums per (k, s, p) and branch (FP64, no atomics, every element written once):
//   X1[k][s][s'][p]  = sum_s'' Gamma+      -> column (p, s'),     weight +1
//   X2[k][s][s'][p]  = sum_s'' Gamma-      -> column (-p, s'),    weight -1/2
//   X3[k][s][s''][p] = sum_s' (Gamma+ + 1/2 Gamma-) -> column (k+p, s''), weight -1
// (rates without the common factor hbar pi / 8 / N_k / w_mu, applied later).
//
// Degenerate modes: only sums over a set are independent of the eigenvector
// basis, so the operator is reduced to the vectors that are constant on each
// set (block sums over the row and column sets, divided by sqrt(|A| |B|)); on
// the vectors that sum to zero within a set only Gamma^0 acts (RTA).  Time
// reversal: the velocity is odd under k -> -k, so the set-mean problem is
// solved on the odd vectors (e_A - e_A') / sqrt(2), A' the set at -k that
// mirrors A.  This halves the system and leaves out the even vectors, among
// them the near-zero mode of uniform deviations that energy conservation
// creates.  The problem 2 (Gamma^0 + Gamma^1) L = v on those vectors is solved
// by LU (rocSOLVER) or summed as the series L = sum_n (-Gamma^1 / Gamma^0)^n
// v / (2 Gamma^0); the factor 2 makes Gamma^1 = 0 reproduce the RTA lifetime
// tau = 1 / (2 Gamma^0).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "internal.h"
#include "mfma.h"

namespace kaldo {

struct ScatterArgs {
  int G0, G1, G2;
  int nk, nd;
  int k0;
  double rc;  // 1 / (scale of the delta)
};

// One lane per partner p, one block per (k, 256 partners); FP64 throughout.
// OCC is the occupation table of one temperature, [s][k].
template <int NM, bool LDS_A, int DK>
__global__ void __launch_bounds__(256)
    k_scatter_small(const cplx<double>* __restrict__ A, const cplx<double>* __restrict__ PH,
                    const cplx<double>* __restrict__ ET, const double* __restrict__ OM,
                    const double* __restrict__ IW, const double* __restrict__ OCC, ScatterArgs P,
                    double* __restrict__ X1, double* __restrict__ X2, double* __restrict__ X3) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int kl = (int)blockIdx.y;
  const int k = P.k0 + kl;
  const int nk = P.nk;
  const size_t a_per_k = (size_t)NM * P.nd * NM * NM;
  const cplx<double>* Ablk = A + (size_t)kl * a_per_k;
  if constexpr (LDS_A) {
    cplx<double>* As = reinterpret_cast<cplx<double>*>(smem);
    for (size_t i = threadIdx.x; i < a_per_k; i += blockDim.x) As[i] = Ablk[i];
    Ablk = As;
  }
  __syncthreads();
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= nk) return;
  const int km0 = k / (P.G1 * P.G2), km1 = (k / P.G2) % P.G1, km2 = k % P.G2;
  const int pm0 = p / (P.G1 * P.G2), pm1 = (p / P.G2) % P.G1, pm2 = p % P.G2;
  const int kk = (((km0 + pm0) % P.G0) * P.G1 + (km1 + pm1) % P.G1) * P.G2 + (km2 + pm2) % P.G2;
  cplx<double> Ep[NM][NM];
  double wp[NM], iwp[NM], np_[NM];
#pragma unroll
  for (int s1 = 0; s1 < NM; ++s1) {
#pragma unroll
    for (int a = 0; a < NM; ++a) Ep[a][s1] = ET[((size_t)s1 * NM + a) * nk + p];
    wp[s1] = OM[(size_t)s1 * nk + p] * P.rc;
    iwp[s1] = IW[(size_t)s1 * nk + p];
    np_[s1] = OCC[(size_t)s1 * nk + p];
  }
#pragma unroll 1
  for (int s = 0; s < NM; ++s) {
    const size_t row = ((size_t)k * NM + s) * NM;  // X[k][s][.][p] = X[(row + branch) * nk + p]
    const double iws = IW[(size_t)s * nk + k];
    if (iws == 0.0) {  // masked first mode (uniform across the block): zero rows
#pragma unroll
      for (int b = 0; b < NM; ++b) {
        X1[(row + b) * nk + p] = 0.0;
        X2[(row + b) * nk + p] = 0.0;
        X3[(row + b) * nk + p] = 0.0;
      }
      continue;
    }
    const double ws = OM[(size_t)s * nk + k] * P.rc;
    // step B: Phi = sum_Delta e^{2 pi i p.Delta} A_k[s][Delta]
    cplx<double> F[NM][NM];
#pragma unroll
    for (int a = 0; a < NM; ++a)
#pragma unroll
      for (int b = 0; b < NM; ++b) F[a][b] = {0.0, 0.0};
    const cplx<double>* As = Ablk + (size_t)s * P.nd * NM * NM;
    for (int d = 0; d < P.nd; ++d) {
      const cplx<double> ph = PH[(size_t)d * nk + p];
      const cplx<double>* Ad = As + (size_t)d * NM * NM;
#pragma unroll
      for (int a = 0; a < NM; ++a)
#pragma unroll
        for (int b = 0; b < NM; ++b) cfma(F[a][b], ph, Ad[a * NM + b]);
    }
    double r1[NM], r2[NM];
#pragma unroll
    for (int b = 0; b < NM; ++b) r1[b] = r2[b] = 0.0;
#pragma unroll 1
    for (int s2 = 0; s2 < NM; ++s2) {
      const size_t colk = (size_t)s2 * NM * nk + kk;
      cplx<double> Tc[NM];
#pragma unroll
      for (int a = 0; a < NM; ++a) {
        Tc[a] = {0.0, 0.0};
#pragma unroll
        for (int b = 0; b < NM; ++b) cfma_conj(Tc[a], F[a][b], ET[colk + (size_t)b * nk]);
      }
      const double w2 = OM[(size_t)s2 * nk + kk] * P.rc;
      const double iw2 = IW[(size_t)s2 * nk + kk];
      const double n2 = OCC[(size_t)s2 * nk + kk];
      const double d2 = ws - w2;
      double col = 0.0;
#pragma unroll
      for (int s1 = 0; s1 < NM; ++s1) {
        cplx<double> V = {0.0, 0.0};
#pragma unroll
        for (int a = 0; a < NM; ++a) cfma(V, Ep[a][s1], Tc[a]);
        const double v2 = (V.re * V.re + V.im * V.im) * (iwp[s1] * iw2);
        const double gp = v2 * delta_shape<double, DK>(d2 + wp[s1]) * (np_[s1] - n2);
        const double gm = v2 * delta_shape<double, DK>(d2 - wp[s1]) * (1.0 + np_[s1] + n2);
        r1[s1] += gp;
        r2[s1] += gm;
        col += gp + 0.5 * gm;
      }
      X3[(row + s2) * nk + p] = col;
    }
#pragma unroll
    for (int b = 0; b < NM; ++b) {
      X1[(row + b) * nk + p] = r1[b];
      X2[(row + b) * nk + p] = r2[b];
    }
  }
}

// Gamma^0 per mode (rad/ps, not set averaged): C / w_mu sum_{s', p} (X1 + X2 / 2).
// One block per mode, fixed-order reduction.
__global__ void __launch_bounds__(256) k_bte_gamma0(double* __restrict__ g0, const double* __restrict__ X1,
                                                    const double* __restrict__ X2, const double* __restrict__ IW,
                                                    int n, int nk, double C) {
  __shared__ double red[256];
  const int mu = (int)blockIdx.x;  // k n + s
  const int k = mu / n, s = mu % n;
  const size_t base = (size_t)mu * n * nk;
  double v = 0.0;
  for (size_t i = threadIdx.x; i < (size_t)n * nk; i += 256) v += X1[base + i] + 0.5 * X2[base + i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) g0[mu] = C * IW[(size_t)s * nk + k] * red[0];
}

__device__ __forceinline__ double bte_heat_capacity(double w, double T, int classical) {
  if (classical) return kBoltzmann;
  const double x = kHbar * w / (kBoltzmann * T);
  if (x == 0.0) return kBoltzmann;
  const double h = 0.5 * x / sinh(0.5 * x);
  return kBoltzmann * h * h;
}

// Per set A (mode index first = k n + s0, size d): set-averaged Gamma^0 and
// heat capacity, the velocity components on the set vector u_A = sum v / sqrt(d)
// and the within-set part of kappa's weight, c / (2 g0) (sum v v - u u^T).
__global__ void k_bte_sets(double* __restrict__ g0s, double* __restrict__ cs, double* __restrict__ us,
                           double* __restrict__ dev, const int* __restrict__ sfirst, const int* __restrict__ sdim,
                           const double* __restrict__ g0, const double* __restrict__ omega,
                           const double* __restrict__ vel, const double* __restrict__ vv, int nS, double T,
                           int classical) {
  const int A = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (A >= nS) return;
  const int f = sfirst[A], d = sdim[A];
  double g = 0.0, c = 0.0, u[3] = {0, 0, 0}, t[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int a = f; a < f + d; ++a) {
    g += g0[a];
    c += bte_heat_capacity(omega[a], T, classical);
    for (int x = 0; x < 3; ++x) u[x] += vel[(size_t)a * 3 + x];
    for (int x = 0; x < 9; ++x) t[x] += vv[(size_t)a * 9 + x];
  }
  g /= d;
  c /= d;
  const double rd = 1.0 / sqrt((double)d);
  for (int x = 0; x < 3; ++x) u[x] *= rd;
  g0s[A] = g;
  cs[A] = c;
  for (int x = 0; x < 3; ++x) us[(size_t)A * 3 + x] = u[x];
  const double wgt = c / (2.0 * g);
  for (int x = 0; x < 3; ++x)
    for (int y = 0; y < 3; ++y) dev[(size_t)A * 9 + 3 * x + y] = wgt * (t[3 * x + y] - u[x] * u[y]);
}

struct BteGrid {
  int G0, G1, G2, nk, n;
};

__device__ __forceinline__ int bte_kdiff(const BteGrid& g, int q, int k, int sign) {
  // index of q - sign k on the grid (sign = +1) or of -q (k = 0, sign = 0 with q negated below)
  const int q0 = q / (g.G1 * g.G2), q1 = (q / g.G2) % g.G1, q2 = q % g.G2;
  const int k0 = k / (g.G1 * g.G2), k1 = (k / g.G2) % g.G1, k2 = k % g.G2;
  const int a = imod(q0 - sign * k0, g.G0), b = imod(q1 - sign * k1, g.G1), c = imod(q2 - sign * k2, g.G2);
  return (a * g.G1 + b) * g.G2 + c;
}

// sum_{a in set A} sum_{b in set B} (w_b / w_a) / w_a [X1 - X2(-q) / 2 - X3(q - k)]
__device__ double bte_block(const BteGrid& g, const double* __restrict__ X1, const double* __restrict__ X2,
                            const double* __restrict__ X3, const double* __restrict__ omega, int fa, int da, int fb,
                            int db) {
  const int n = g.n, nk = g.nk;
  const int ka = fa / n, q = fb / n;
  const int qneg = bte_kdiff(g, 0, q, 1);   // -q
  const int qmk = bte_kdiff(g, q, ka, 1);   // q - k_a
  double acc = 0.0;
  for (int a = fa; a < fa + da; ++a) {
    const double wa = omega[a];
    const double ra = 1.0 / (wa * wa);
    double row = 0.0;
    for (int b = fb; b < fb + db; ++b) {
      const int sb = b - q * n;
      const size_t o = ((size_t)a * n + sb) * nk;
      row += omega[b] * (X1[o + q] - 0.5 * X2[o + qneg] - X3[o + qmk]);
    }
    acc += ra * row;
  }
  return acc;
}

// The operator on the odd set vectors, column major [j][i] (i, j over the
// representative sets r = reps[.], mirrored by tr[r]):
//   B_odd[i][j] = C (blk(A,B) - blk(A,B') - blk(A',B) + blk(A',B')) / (2 sqrt(d_A d_B)),
// stored as M = 2 (diag(g0) + B_odd) (inverse) or as B_odd (series).
__global__ void k_bte_operator(double* __restrict__ M, const double* __restrict__ X1, const double* __restrict__ X2,
                               const double* __restrict__ X3, const double* __restrict__ omega,
                               const int* __restrict__ reps, const int* __restrict__ tr, const int* __restrict__ sfirst,
                               const int* __restrict__ sdim, const double* __restrict__ g0s, BteGrid g, int nr,
                               double C, int with_diag) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nr * nr) return;
  const int i = (int)(idx % nr), j = (int)(idx / nr);
  const int A = reps[i], Ap = tr[A], B = reps[j], Bp = tr[B];
  const int fa = sfirst[A], fap = sfirst[Ap], fb = sfirst[B], fbp = sfirst[Bp];
  const int da = sdim[A], db = sdim[B];
  double v = bte_block(g, X1, X2, X3, omega, fa, da, fb, db) - bte_block(g, X1, X2, X3, omega, fa, da, fbp, db) -
             bte_block(g, X1, X2, X3, omega, fap, da, fb, db) + bte_block(g, X1, X2, X3, omega, fap, da, fbp, db);
  v *= C / (2.0 * sqrt((double)da * (double)db));
  if (with_diag) v = 2.0 * (v + (i == j ? g0s[A] : 0.0));
  M[idx] = v;
}

// Right-hand side on the odd vectors, column major [x][i]: (u_A - u_A') / sqrt 2.
__global__ void k_bte_rhs(double* __restrict__ U, const double* __restrict__ us, const int* __restrict__ reps,
                          const int* __restrict__ tr, int nr) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= nr) return;
  const int A = reps[i], Ap = tr[A];
  for (int x = 0; x < 3; ++x) U[(size_t)x * nr + i] = (us[(size_t)A * 3 + x] - us[(size_t)Ap * 3 + x]) * 0.7071067811865475244;
}

// One step of the series: term <- -(B term) / g0, L <- L + term; and the two
// maxima |term|, |L| for the stopping test (one block, fixed order).
__global__ void __launch_bounds__(256) k_bte_series_step(double* __restrict__ term, double* __restrict__ L,
                                                         const double* __restrict__ Bt, const double* __restrict__ g0s,
                                                         const int* __restrict__ reps, int nr, double* __restrict__ mx) {
  __shared__ double r0[256], r1[256];
  double m0 = 0.0, m1 = 0.0;
  for (int e = threadIdx.x; e < 3 * nr; e += 256) {
    const int i = e % nr;
    const double t = -Bt[e] / g0s[reps[i]];
    term[e] = t;
    const double l = L[e] + t;
    L[e] = l;
    m0 = fmax(m0, fabs(t));
    m1 = fmax(m1, fabs(l));
  }
  r0[threadIdx.x] = m0;
  r1[threadIdx.x] = m1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      r0[threadIdx.x] = fmax(r0[threadIdx.x], r0[threadIdx.x + w]);
      r1[threadIdx.x] = fmax(r1[threadIdx.x], r1[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mx[0] = r0[0];
    mx[1] = r1[0];
  }
}

// lambda^0 = U / (2 g0): the first term and the first partial sum
__global__ void k_bte_series_start(double* __restrict__ term, double* __restrict__ L, const double* __restrict__ U,
                                   const double* __restrict__ g0s, const int* __restrict__ reps, int nr) {
  const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (e >= 3 * nr) return;
  const double v = U[e] / (2.0 * g0s[reps[e % nr]]);
  term[e] = v;
  L[e] = v;
}

// kappa[x][y] = scale (sum_i c_i U[x][i] L[y][i] + sum_A dev_A[x][y]), one block, fixed order.
__global__ void __launch_bounds__(256) k_bte_kappa(double* __restrict__ kappa, const double* __restrict__ U,
                                                   const double* __restrict__ L, const double* __restrict__ cs,
                                                   const int* __restrict__ reps, const double* __restrict__ dev,
                                                   int nr, int nS, double scale) {
  __shared__ double red[256][9];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < nr; i += 256) {
    const double c = cs[reps[i]];
    for (int x = 0; x < 3; ++x)
      for (int y = 0; y < 3; ++y) acc[3 * x + y] += c * U[(size_t)x * nr + i] * L[(size_t)y * nr + i];
  }
  for (int A = threadIdx.x; A < nS; A += 256)
    for (int x = 0; x < 9; ++x) acc[x] += dev[(size_t)A * 9 + x];
  for (int x = 0; x < 9; ++x) red[threadIdx.x][x] = acc[x];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int x = 0; x < 9; ++x) red[threadIdx.x][x] += red[threadIdx.x + w][x];
    __syncthreads();
  }
  if (threadIdx.x < 9) kappa[threadIdx.x] = scale * red[0][threadIdx.x];
}

static double bte_cell_volume(const double* c) {
  const double det = c[0] * (c[4] * c[8] - c[5] * c[7]) - c[1] * (c[3] * c[8] - c[5] * c[6]) +
                     c[2] * (c[3] * c[7] - c[4] * c[6]);
  return det < 0 ? -det : det;
}

template <int NM, bool LDS_A, int DK>
static void launch_scatter_t(dim3 grid, size_t lds, hipStream_t st, const cplx<double>* A, const SmallTables& t,
                             const double* OCC, const ScatterArgs& P, double* X1, double* X2, double* X3) {
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_scatter_small<NM, LDS_A, DK>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_scatter_small<NM, LDS_A, DK>), grid, dim3(256), lds, st, A, t.PH, t.ET, t.OM, t.IW, OCC, P,
                     X1, X2, X3);
}

template <int NM>
static void launch_scatter(int kind, dim3 grid, hipStream_t st, const cplx<double>* A, const SmallTables& t,
                           const double* OCC, const ScatterArgs& P, double* X1, double* X2, double* X3) {
  const size_t lds = (size_t)NM * P.nd * NM * NM * sizeof(cplx<double>);
  const bool in_lds = lds <= 150 * 1024;
#define KALDO_KIND(DKV)                                                            \
  {                                                                                \
    if (in_lds)                                                                    \
      launch_scatter_t<NM, true, DKV>(grid, lds, st, A, t, OCC, P, X1, X2, X3);    \
    else                                                                           \
      launch_scatter_t<NM, false, DKV>(grid, 0, st, A, t, OCC, P, X1, X2, X3);     \
  }
  if (kind == KALDO_DELTA_GAUSS) KALDO_KIND(KALDO_DELTA_GAUSS)
  else if (kind == KALDO_DELTA_LORENTZ) KALDO_KIND(KALDO_DELTA_LORENTZ)
  else KALDO_KIND(KALDO_DELTA_TRIANGLE)
#undef KALDO_KIND
}

kaldo_status run_kappa_bte(kaldo_ctx ctx, int method, int max_terms, double tol, double* kappa_out, int* terms_out) {
  const int n = ctx->nm, nk = ctx->nk, nT = ctx->nT, nd = ctx->fc3.n_delta;
  hipStream_t st = ctx->stream;
  const int TB = 256;
  const size_t nmode = (size_t)nk * n;
  // ---- the sets of the unmasked modes and their mirrors at -k (host bookkeeping)
  std::vector<int> setid(nmode);
  std::vector<double> om(nmode);
  KALDO_HIP(ctx, hipMemcpyAsync(setid.data(), ctx->d_setid.p, nmode * sizeof(int), hipMemcpyDeviceToHost, st));
  KALDO_HIP(ctx, hipMemcpyAsync(om.data(), ctx->d_omega.p, nmode * sizeof(double), hipMemcpyDeviceToHost, st));
  KALDO_HIP(ctx, hipStreamSynchronize(st));
  std::vector<int> sfirst, sdim, set_of(nmode, -1);
  for (int k = 0; k < nk; ++k)
    for (int s = 0; s < n;) {
      int e = s + 1;
      while (e < n && setid[(size_t)k * n + e] == setid[(size_t)k * n + s]) ++e;
      bool on = true;
      for (int u = s; u < e; ++u) on = on && om[(size_t)k * n + u] / kTwoPi >= kNuMinThz;
      if (on) {
        for (int u = s; u < e; ++u) set_of[(size_t)k * n + u] = (int)sfirst.size();
        sfirst.push_back(k * n + s);
        sdim.push_back(e - s);
      }
      s = e;
    }
  const int nS = (int)sfirst.size();
  if (nS == 0) return fail(ctx, KALDO_EINVAL, "kaldo_kappa_bte: no unmasked modes");
  std::vector<int> tr(nS), reps;
  for (int A = 0; A < nS; ++A) {
    const int k = sfirst[A] / n, s = sfirst[A] % n;
    const int m0 = k / (ctx->grid[1] * ctx->grid[2]), m1 = (k / ctx->grid[2]) % ctx->grid[1], m2 = k % ctx->grid[2];
    const int km = (((ctx->grid[0] - m0) % ctx->grid[0]) * ctx->grid[1] + (ctx->grid[1] - m1) % ctx->grid[1]) *
                       ctx->grid[2] +
                   (ctx->grid[2] - m2) % ctx->grid[2];
    const int B = set_of[(size_t)km * n + s];
    if (B < 0 || sfirst[B] != km * n + s || sdim[B] != sdim[A])
      return fail(ctx, KALDO_EDEVICE, "kaldo_kappa_bte: the degenerate sets at k and -k differ (k = " +
                                          std::to_string(k) + ")");
    tr[A] = B;
  }
  for (int A = 0; A < nS; ++A)
    if (A < tr[A]) reps.push_back(A);
  const int nr = (int)reps.size();
  // ---- device buffers: X1 X2 X3 | step A | g0 per mode | set tables | operator | rhs, solution, series
  const size_t xn = nmode * n * nk;
  const size_t a_per_k = (size_t)n * nd * n * n;
  const size_t a_budget = ((size_t)1 << 30) / sizeof(cplx<double>);
  const int kchunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)nk, std::min<size_t>(65535, a_budget / a_per_k)));
  const size_t nrr = (size_t)std::max(nr, 1);
  const size_t doubles = 3 * xn + a_per_k * kchunk * 2 + nmode + (size_t)nS * (1 + 1 + 3 + 9) + nrr * nrr +
                         5 * 3 * nrr + 16;
  const size_t ints = 4 * (size_t)nS + nrr + nrr + 16;
  KALDO_HIP(ctx, ctx->d_bte.ensure(doubles * sizeof(double) + ints * sizeof(int) + 1024));
  double* X1 = ctx->d_bte.as<double>();
  double* X2 = X1 + xn;
  double* X3 = X2 + xn;
  cplx<double>* Abuf = reinterpret_cast<cplx<double>*>(X3 + xn);
  double* g0m = reinterpret_cast<double*>(Abuf + a_per_k * kchunk);
  double* g0s = g0m + nmode;
  double* cs = g0s + nS;
  double* us = cs + nS;
  double* dev = us + 3 * (size_t)nS;
  double* M = dev + 9 * (size_t)nS;
  double* U = M + nrr * nrr;
  double* Lsol = U + 3 * nrr;
  double* term = Lsol + 3 * nrr;
  double* Bt = term + 3 * nrr;
  double* mx = Bt + 3 * nrr;
  double* kap = mx + 4;
  int* i_first = reinterpret_cast<int*>(kap + 9 + 3);
  int* i_dim = i_first + nS;
  int* i_tr = i_dim + nS;
  int* i_reps = i_tr + nS;
  int* ipiv = i_reps + nrr;
  int* info = ipiv + nrr;
  KALDO_HIP(ctx, hipMemcpyAsync(i_first, sfirst.data(), nS * sizeof(int), hipMemcpyHostToDevice, st));
  KALDO_HIP(ctx, hipMemcpyAsync(i_dim, sdim.data(), nS * sizeof(int), hipMemcpyHostToDevice, st));
  KALDO_HIP(ctx, hipMemcpyAsync(i_tr, tr.data(), nS * sizeof(int), hipMemcpyHostToDevice, st));
  if (nr) KALDO_HIP(ctx, hipMemcpyAsync(i_reps, reps.data(), nr * sizeof(int), hipMemcpyHostToDevice, st));
  SmallTables tb;
  kaldo_status rs = small_tables_fp64(ctx, &tb);
  if (rs != KALDO_OK) return rs;
  const double sig = kTwoPi * ctx->sigma_thz;
  double dscale, dnorm;
  delta_scale(ctx->delta, sig, dscale, dnorm);
  const double C = kPi / 8.0 * kHbar * kEvUnit * kEvUnit * kEvUnit / nk * dnorm;
  ScatterArgs P;
  P.G0 = ctx->grid[0];
  P.G1 = ctx->grid[1];
  P.G2 = ctx->grid[2];
  P.nk = nk;
  P.nd = nd;
  P.rc = 1.0 / dscale;
  const BteGrid g{ctx->grid[0], ctx->grid[1], ctx->grid[2], nk, n};
  const int classical = ctx->stats == KALDO_CLASSICAL ? 1 : 0;
  const double scale = kKappaSI / (nk * bte_cell_volume(ctx->cell));
  KALDO_HIP(ctx, ctx->d_kappa.ensure((size_t)nT * 9 * sizeof(double)));
  int terms_max = 0;
  bool all_converged = true;
  for (int t = 0; t < nT; ++t) {
    // ---- the three sums per (k, s, p, branch)
    prof_begin(ctx);
    for (int k0 = 0; k0 < nk; k0 += kchunk) {
      const int kc = std::min(kchunk, nk - k0);
      rs = small_step_a_fp64(ctx, Abuf, k0, kc);
      if (rs != KALDO_OK) return rs;
      P.k0 = k0;
      const dim3 grid(blocks_for(nk, TB), kc);
      const double* OCC = tb.OCC + (size_t)t * nmode;
      if (n == 6) launch_scatter<6>(ctx->delta, grid, st, Abuf, tb, OCC, P, X1, X2, X3);
      else launch_scatter<3>(ctx->delta, grid, st, Abuf, tb, OCC, P, X1, X2, X3);
      KALDO_HIP(ctx, hipGetLastError());
    }
    prof_end(ctx, "bte_scatter");
    // ---- Gamma^0 per mode, the set tables
    prof_begin(ctx);
    hipLaunchKernelGGL(k_bte_gamma0, dim3((unsigned)nmode), dim3(256), 0, st, g0m, X1, X2, tb.IW, n, nk, C);
    KALDO_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_bte_sets, dim3(blocks_for(nS, TB)), dim3(TB), 0, st, g0s, cs, us, dev, i_first, i_dim, g0m,
                       ctx->d_omega.as<double>(), ctx->d_vel.as<double>(), ctx->d_vv.as<double>(), nS, ctx->T[t],
                       classical);
    KALDO_HIP(ctx, hipGetLastError());
    if (nr > 0) {
      hipLaunchKernelGGL(k_bte_operator, dim3(blocks_for((long long)nr * nr, TB)), dim3(TB), 0, st, M, X1, X2, X3,
                         ctx->d_omega.as<double>(), i_reps, i_tr, i_first, i_dim, g0s, g, nr, C,
                         method == KALDO_BTE_INVERSE ? 1 : 0);
      KALDO_HIP(ctx, hipGetLastError());
      hipLaunchKernelGGL(k_bte_rhs, dim3(blocks_for(nr, TB)), dim3(TB), 0, st, U, us, i_reps, i_tr, nr);
      KALDO_HIP(ctx, hipGetLastError());
    }
    prof_end(ctx, "bte_operator");
    // ---- the set-mean problem on the odd vectors
    prof_begin(ctx);
    if (nr > 0 && method == KALDO_BTE_INVERSE) {
      KALDO_HIP(ctx, hipMemcpyAsync(Lsol, U, 3 * (size_t)nr * sizeof(double), hipMemcpyDeviceToDevice, st));
      if (rocsolver_dgetrf(ctx->blas, nr, nr, M, nr, ipiv, info) != rocblas_status_success)
        return fail(ctx, KALDO_EDEVICE, "rocsolver_dgetrf failed");
      if (rocsolver_dgetrs(ctx->blas, rocblas_operation_none, nr, 3, M, nr, ipiv, Lsol, nr) != rocblas_status_success)
        return fail(ctx, KALDO_EDEVICE, "rocsolver_dgetrs failed");
      int hinfo = 0;
      KALDO_HIP(ctx, hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st));
      KALDO_HIP(ctx, hipStreamSynchronize(st));
      if (hinfo != 0)
        return fail(ctx, KALDO_EUNSTABLE, "kaldo_kappa_bte: the scattering operator is singular (pivot " +
                                              std::to_string(hinfo) + ")");
    } else if (nr > 0) {
      hipLaunchKernelGGL(k_bte_series_start, dim3(blocks_for(3 * nr, TB)), dim3(TB), 0, st, term, Lsol, U, g0s,
                         i_reps, nr);
      KALDO_HIP(ctx, hipGetLastError());
      int terms = 0;
      bool converged = false;
      const double one = 1.0, zero = 0.0;
      for (int it = 1; it <= max_terms; ++it) {
        if (rocblas_dgemm(ctx->blas, rocblas_operation_none, rocblas_operation_none, nr, 3, nr, &one, M, nr, term, nr,
                          &zero, Bt, nr) != rocblas_status_success)
          return fail(ctx, KALDO_EDEVICE, "rocblas_dgemm failed");
        hipLaunchKernelGGL(k_bte_series_step, dim3(1), dim3(256), 0, st, term, Lsol, Bt, g0s, i_reps, nr, mx);
        KALDO_HIP(ctx, hipGetLastError());
        double hm[2] = {0.0, 0.0};
        KALDO_HIP(ctx, hipMemcpyAsync(hm, mx, sizeof(hm), hipMemcpyDeviceToHost, st));
        KALDO_HIP(ctx, hipStreamSynchronize(st));
        terms = it;
        if (!(std::isfinite(hm[0]) && std::isfinite(hm[1]))) break;
        if (hm[0] <= tol * hm[1]) {
          converged = true;
          break;
        }
      }
      terms_max = std::max(terms_max, terms);
      all_converged = all_converged && converged;
    }
    if (nr == 0) {
      KALDO_HIP(ctx, hipMemsetAsync(U, 0, 3 * sizeof(double), st));
      KALDO_HIP(ctx, hipMemsetAsync(Lsol, 0, 3 * sizeof(double), st));
    }
    hipLaunchKernelGGL(k_bte_kappa, dim3(1), dim3(256), 0, st, ctx->d_kappa.as<double>() + 9 * (size_t)t, U, Lsol, cs,
                       i_reps, dev, nr, nS, scale);
    KALDO_HIP(ctx, hipGetLastError());
    prof_end(ctx, "bte_solve");
  }
  if (terms_out) *terms_out = method == KALDO_BTE_INVERSE ? 0 : terms_max;
  rs = copy_out(ctx, kappa_out, ctx->d_kappa.p, (size_t)nT * 9 * sizeof(double));
  if (rs != KALDO_OK) return rs;
  if (method != KALDO_BTE_INVERSE && !all_converged)
    return fail(ctx, KALDO_ENOCONV, "kaldo_kappa_bte: the self-consistent series did not converge in " +
                                        std::to_string(max_terms) + " terms (kappa holds the last partial sum)");
  return KALDO_OK;
}

}  // namespace kaldo
