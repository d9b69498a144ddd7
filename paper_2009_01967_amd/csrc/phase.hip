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

// Frequencies in units of the delta's scale, +infinity for masked modes (every
// mismatch with them is then beyond any cut, so one load serves both tests).
__global__ void k_phase_omx(double* __restrict__ OMX, const double* __restrict__ OM, const double* __restrict__ IW,
                            int nmode, double rs) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < nmode) OMX[i] = IW[i] != 0.0 ? OM[i] * rs : __builtin_inf();
}

template <int DK>
__global__ void __launch_bounds__(256)
    k_phase_space(double* __restrict__ g, const double* __restrict__ OMX, const double* __restrict__ IW,
                  const double* __restrict__ OCC, int nk, int n, int nT, int G0, int G1, int G2, double scale) {
  constexpr double cut = delta_cut<KALDO_FP64>(DK);
  const int mode = (int)blockIdx.x;
  const int s = mode % n;
  const int k = mode / n;
  const int nmode = nk * n;
  __shared__ double red[4][KALDO_MAX_T];
  double acc[KALDO_MAX_T];
#pragma unroll
  for (int t = 0; t < KALDO_MAX_T; ++t) acc[t] = 0.0;
  const bool on = IW[(size_t)s * nk + k] != 0.0;  // uniform across the block
  if (on) {
    const double w = OMX[(size_t)s * nk + k];
    const int m0 = k / (G1 * G2), m1 = (k / G2) % G1, m2 = k % G2;
    for (int j = threadIdx.x; j < nmode; j += blockDim.x) {
      const double w1 = OMX[j];
      if (!(w1 < __builtin_inf())) continue;  // masked partner
      const int s1 = j / nk;
      const int p = j - s1 * nk;
      double n1[KALDO_MAX_T];
#pragma unroll
      for (int t = 0; t < KALDO_MAX_T; ++t) n1[t] = t < nT ? OCC[(size_t)t * nmode + j] : 0.0;
      const int p0 = p / (G1 * G2), p1 = (p / G2) % G1, p2 = p % G2;
      const int kp = (imod(m0 + p0, G0) * G1 + imod(m1 + p1, G1)) * G2 + imod(m2 + p2, G2);
      const int km = (imod(m0 - p0, G0) * G1 + imod(m1 - p1, G1)) * G2 + imod(m2 - p2, G2);
      for (int s2 = 0; s2 < n; ++s2) {
        // absorption: k'' = k + k', weight (n' - n'') delta(w + w' - w'')
        // (a masked k'' mode has +infinity: u = -infinity fails the cut)
        const int op = s2 * nk + kp;
        {
          const double u = w + w1 - OMX[op];
          if (u * u < cut) {
            const double d = delta_shape<double, DK>(u);
#pragma unroll
            for (int t = 0; t < KALDO_MAX_T; ++t)
              if (t < nT) acc[t] += (n1[t] - OCC[(size_t)t * nmode + op]) * d;
          }
        }
        // decay: k'' = k - k', weight 1/2 (1 + n' + n'') delta(w - w' - w'')
        const int om = s2 * nk + km;
        {
          const double u = w - w1 - OMX[om];
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
  if (nmode >= ((size_t)1 << 31)) return fail(ctx, KALDO_EINVAL, "kaldo_phase_space: too many modes");
  KALDO_HIP(ctx, ctx->d_phase.ensure(((3 + (size_t)nT) * nmode + (size_t)nT * nmode) * sizeof(double)));
  double* OM = ctx->d_phase.as<double>();
  double* IW = OM + nmode;
  double* OCC = IW + nmode;
  double* G = OCC + (size_t)nT * nmode;
  double* OMX = G + (size_t)nT * nmode;
  double Ts[KALDO_MAX_T] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int t = 0; t < nT; ++t) Ts[t] = T[t];
  hipLaunchKernelGGL(k_tables, dim3(blocks_for((long long)nmode, 256)), dim3(256), 0, st, OM, IW, OCC,
                     ctx->d_omega.as<double>(), nk, n, nT, make_double4(Ts[0], Ts[1], Ts[2], Ts[3]),
                     make_double4(Ts[4], Ts[5], Ts[6], Ts[7]), stats == KALDO_CLASSICAL ? 1 : 0);
  KALDO_HIP(ctx, hipGetLastError());
  double dscale, dnorm;
  delta_scale(delta, kTwoPi * sigma_thz, dscale, dnorm);
  const double rs = 1.0 / dscale, scale = dnorm / nk;
  hipLaunchKernelGGL(k_phase_omx, dim3(blocks_for((long long)nmode, 256)), dim3(256), 0, st, OMX, OM, IW,
                     (int)nmode, rs);
  KALDO_HIP(ctx, hipGetLastError());
  const dim3 grid((unsigned)nmode);
  if (delta == KALDO_DELTA_GAUSS)
    hipLaunchKernelGGL(k_phase_space<KALDO_DELTA_GAUSS>, grid, dim3(256), 0, st, G, OMX, IW, OCC, nk, n, nT,
                       ctx->grid[0], ctx->grid[1], ctx->grid[2], scale);
  else if (delta == KALDO_DELTA_LORENTZ)
    hipLaunchKernelGGL(k_phase_space<KALDO_DELTA_LORENTZ>, grid, dim3(256), 0, st, G, OMX, IW, OCC, nk, n, nT,
                       ctx->grid[0], ctx->grid[1], ctx->grid[2], scale);
  else
    hipLaunchKernelGGL(k_phase_space<KALDO_DELTA_TRIANGLE>, grid, dim3(256), 0, st, G, OMX, IW, OCC, nk, n, nT,
                       ctx->grid[0], ctx->grid[1], ctx->grid[2], scale);
  KALDO_HIP(ctx, hipGetLastError());
  *g_dev = G;
  return KALDO_OK;
}

}  // namespace kaldo
