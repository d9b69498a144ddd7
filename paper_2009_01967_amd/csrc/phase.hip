// Normalised three-phonon phase space per mode (paper Sec. II.B, eq. phase_space
// and the per-mode sum after eq. delta_deconstructed):
//   g_mu = (1/N_k) [ sum_{k's's''} (n' - n'') delta(w + w' - w'')        (k'' = k + k')
//                  + 1/2 sum_{k's's''} (1 + n' + n'') delta(w - w' - w'') ] (k'' = k - k')
// i.e. the linewidth sum with the matrix-element factor replaced by 1.  The
// sums need frequencies and occupations only; they run in FP64, one block per
// mode (k, s), the threads over (s', k') with k' fastest (coalesced table reads).
#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"
#include "mfma.h"

namespace kaldo {

// mode tables (anharmonic.hip): OM[s][k], IW[s][k] (0 for masked modes), OCC[t][s][k]
__global__ void k_tables(double* __restrict__ OM, double* __restrict__ IW, double* __restrict__ OCC,
                         const double* __restrict__ omega, int nk, int n, int nT, double4 T03, double4 T47,
                         int classical);

template <int DK>
__global__ void __launch_bounds__(256)
    k_phase_space(double* __restrict__ g, const double* __restrict__ OM, const double* __restrict__ IW,
                  const double* __restrict__ OCC, int nk, int n, int nT, int G0, int G1, int G2, double rs,
                  double scale) {
  constexpr double cut = delta_cut<KALDO_FP64>(DK);
  const long long mode = blockIdx.x;
  const int s = (int)(mode % n);
  const int k = (int)(mode / n);
  const size_t nmode = (size_t)nk * n;
  __shared__ double red[4][KALDO_MAX_T];
  double acc[KALDO_MAX_T];
#pragma unroll
  for (int t = 0; t < KALDO_MAX_T; ++t) acc[t] = 0.0;
  const bool on = IW[(size_t)s * nk + k] != 0.0;  // uniform across the block
  if (on) {
    const double w = OM[(size_t)s * nk + k] * rs;
    const int m0 = k / (G1 * G2), m1 = (k / G2) % G1, m2 = k % G2;
    for (long long j = threadIdx.x; j < (long long)nmode; j += blockDim.x) {
      if (IW[j] == 0.0) continue;
      const int s1 = (int)(j / nk);
      const int p = (int)(j - (long long)s1 * nk);
      const double w1 = OM[j] * rs;
      double n1[KALDO_MAX_T];
#pragma unroll
      for (int t = 0; t < KALDO_MAX_T; ++t) n1[t] = t < nT ? OCC[(size_t)t * nmode + j] : 0.0;
      const int p0 = p / (G1 * G2), p1 = (p / G2) % G1, p2 = p % G2;
      const int kp = (imod(m0 + p0, G0) * G1 + imod(m1 + p1, G1)) * G2 + imod(m2 + p2, G2);
      const int km = (imod(m0 - p0, G0) * G1 + imod(m1 - p1, G1)) * G2 + imod(m2 - p2, G2);
      for (int s2 = 0; s2 < n; ++s2) {
        // absorption: k'' = k + k', weight (n' - n'') delta(w + w' - w'')
        const size_t op = (size_t)s2 * nk + kp;
        if (IW[op] != 0.0) {
          const double u = w + w1 - OM[op] * rs;
          if (u * u < cut) {
            const double d = delta_shape<double, DK>(u);
#pragma unroll
            for (int t = 0; t < KALDO_MAX_T; ++t)
              if (t < nT) acc[t] += (n1[t] - OCC[(size_t)t * nmode + op]) * d;
          }
        }
        // decay: k'' = k - k', weight 1/2 (1 + n' + n'') delta(w - w' - w'')
        const size_t om = (size_t)s2 * nk + km;
        if (IW[om] != 0.0) {
          const double u = w - w1 - OM[om] * rs;
          if (u * u < cut) {
            const double d = 0.5 * delta_shape<double, DK>(u);
#pragma unroll
            for (int t = 0; t < KALDO_MAX_T; ++t)
              if (t < nT) acc[t] += (1.0 + n1[t] + OCC[(size_t)t * nmode + om]) * d;
          }
        }
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < KALDO_MAX_T; ++t) {
    double v = acc[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave][t] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < nT) {
    const int t = threadIdx.x;
    const double v = red[0][t] + red[1][t] + red[2][t] + red[3][t];
    g[((size_t)t * nk + k) * n + s] = scale * v;
  }
}

kaldo_status run_phase_space(kaldo_ctx ctx, const double* T, int nT, double sigma_thz, int delta, int stats,
                             double** g_dev) {
  const int n = ctx->nm, nk = ctx->nk;
  const size_t nmode = (size_t)nk * n;
  hipStream_t st = ctx->stream;
  KALDO_HIP(ctx, ctx->d_phase.ensure(((2 + (size_t)nT) * nmode + (size_t)nT * nmode) * sizeof(double)));
  double* OM = ctx->d_phase.as<double>();
  double* IW = OM + nmode;
  double* OCC = IW + nmode;
  double* G = OCC + (size_t)nT * nmode;
  double Ts[KALDO_MAX_T] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int t = 0; t < nT; ++t) Ts[t] = T[t];
  hipLaunchKernelGGL(k_tables, dim3(blocks_for((long long)nmode, 256)), dim3(256), 0, st, OM, IW, OCC,
                     ctx->d_omega.as<double>(), nk, n, nT, make_double4(Ts[0], Ts[1], Ts[2], Ts[3]),
                     make_double4(Ts[4], Ts[5], Ts[6], Ts[7]), stats == KALDO_CLASSICAL ? 1 : 0);
  KALDO_HIP(ctx, hipGetLastError());
  double dscale, dnorm;
  delta_scale(delta, kTwoPi * sigma_thz, dscale, dnorm);
  const double rs = 1.0 / dscale, scale = dnorm / nk;
  const dim3 grid((unsigned)nmode);
  if (delta == KALDO_DELTA_GAUSS)
    hipLaunchKernelGGL(k_phase_space<KALDO_DELTA_GAUSS>, grid, dim3(256), 0, st, G, OM, IW, OCC, nk, n, nT,
                       ctx->grid[0], ctx->grid[1], ctx->grid[2], rs, scale);
  else if (delta == KALDO_DELTA_LORENTZ)
    hipLaunchKernelGGL(k_phase_space<KALDO_DELTA_LORENTZ>, grid, dim3(256), 0, st, G, OM, IW, OCC, nk, n, nT,
                       ctx->grid[0], ctx->grid[1], ctx->grid[2], rs, scale);
  else
    hipLaunchKernelGGL(k_phase_space<KALDO_DELTA_TRIANGLE>, grid, dim3(256), 0, st, G, OM, IW, OCC, nk, n, nT,
                       ctx->grid[0], ctx->grid[1], ctx->grid[2], rs, scale);
  KALDO_HIP(ctx, hipGetLastError());
  *g_dev = G;
  return KALDO_OK;
}

}  // namespace kaldo
