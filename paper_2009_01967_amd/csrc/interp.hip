// Linewidths interpolated in frequency (paper Sec. II.C: gamma of a smaller
// disordered cell, interpolated as a function of frequency with third-order
// splines, serves the QHGK conductivity of a larger one; Sec. IV.B).
//   1. the unmasked source modes go into n_bins bins of equal width between
//      their lowest and highest frequency; each non-empty bin is one knot
//      (mean omega, mean gamma);
//   2. the natural cubic spline through the knots, per temperature;
//   3. every target mode gets the spline at its frequency (end values outside
//      the knots, at least the smallest knot gamma), masked modes 0, then the
//      average over its degenerate set.
// Everything is FP64.  The source holds at most a few 10^5 modes and the
// target the modes of one cell, so each stage is a small latency-bound launch:
// the bins are summed by one block per (bin, temperature) scanning the source
// (n_bins x n_src reads from cache, in a fixed order), the spline by one
// thread per temperature (a tridiagonal solve over at most 4096 knots).
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"
#include "internal.h"

namespace kaldo {

constexpr int kInterpMaxBins = 4096;

// range[0..2] = lowest and highest unmasked source frequency, their count
__global__ void __launch_bounds__(1024) k_interp_range(double* __restrict__ range, const double* __restrict__ w,
                                                       long long n_src) {
  __shared__ double s_lo[1024], s_hi[1024], s_n[1024];
  double lo = INFINITY, hi = -INFINITY, cnt = 0.0;
  for (long long i = threadIdx.x; i < n_src; i += blockDim.x) {
    const double x = w[i];
    if (!(x / kTwoPi >= kNuMinThz)) continue;
    lo = fmin(lo, x);
    hi = fmax(hi, x);
    cnt += 1.0;
  }
  s_lo[threadIdx.x] = lo;
  s_hi[threadIdx.x] = hi;
  s_n[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_lo[threadIdx.x] = fmin(s_lo[threadIdx.x], s_lo[threadIdx.x + off]);
      s_hi[threadIdx.x] = fmax(s_hi[threadIdx.x], s_hi[threadIdx.x + off]);
      s_n[threadIdx.x] += s_n[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    range[0] = s_lo[0];
    range[1] = s_hi[0];
    range[2] = s_n[0];
  }
}

// bins[t][b][0..2] = count, sum of omega, sum of gamma of the unmasked source
// modes in bin b = floor((w - lo) / (hi - lo) n_bins) (the highest in the last bin)
__global__ void __launch_bounds__(256) k_interp_bins(double* __restrict__ bins, const double* __restrict__ w,
                                                     const double* __restrict__ g, long long n_src, int nb,
                                                     const double* __restrict__ range) {
  const int b = blockIdx.x, t = blockIdx.y;
  const double lo = range[0], hi = range[1];
  const double* gt = g + (size_t)t * n_src;
  double cnt = 0.0, sw = 0.0, sg = 0.0;
  for (long long i = threadIdx.x; i < n_src; i += blockDim.x) {
    const double x = w[i];
    if (!(x / kTwoPi >= kNuMinThz)) continue;
    long long bi = 0;
    if (hi > lo) {
      bi = (long long)floor((x - lo) / (hi - lo) * (double)nb);
      if (bi > nb - 1) bi = nb - 1;
    }
    if (bi != b) continue;
    cnt += 1.0;
    sw += x;
    sg += gt[i];
  }
  __shared__ double s[3][256];
  s[0][threadIdx.x] = cnt;
  s[1][threadIdx.x] = sw;
  s[2][threadIdx.x] = sg;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s[0][threadIdx.x] += s[0][threadIdx.x + off];
      s[1][threadIdx.x] += s[1][threadIdx.x + off];
      s[2][threadIdx.x] += s[2][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) bins[((size_t)t * nb + b) * 3 + threadIdx.x] = s[threadIdx.x][0];
}

// Per temperature (one thread each): the knots of the non-empty bins and the
// second derivatives M of the natural cubic spline through them, from the
// continuity of the first derivative at the interior knots,
//   h_{i-1} M_{i-1} + 2 (h_{i-1} + h_i) M_i + h_i M_{i+1}
//       = 6 ((y_{i+1} - y_i) / h_i - (y_i - y_{i-1}) / h_{i-1}),   M_0 = M_{m-1} = 0,
// solved by forward elimination and back substitution (the system is
// diagonally dominant).  knots[t] = x[nb], y[nb], M[nb], c'[nb], d'[nb];
// meta[t] = knot count m, smallest knot gamma.
__global__ void k_interp_spline(double* __restrict__ knots, double* __restrict__ meta,
                                const double* __restrict__ bins, int nb, int nT) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nT) return;
  double* x = knots + (size_t)t * 5 * nb;
  double* y = x + nb;
  double* M = y + nb;
  double* cp = M + nb;
  double* dp = cp + nb;
  int m = 0;
  double ymin = INFINITY;
  for (int b = 0; b < nb; ++b) {
    const double* e = bins + ((size_t)t * nb + b) * 3;
    if (e[0] > 0.0) {
      x[m] = e[1] / e[0];
      y[m] = e[2] / e[0];
      ymin = fmin(ymin, y[m]);
      ++m;
    }
  }
  for (int i = 0; i < m; ++i) M[i] = 0.0;
  if (m >= 3) {
    // interior unknowns M_1 .. M_{m-2}; row i: a = h_{i-1}, b = 2 (h_{i-1} + h_i), c = h_i
    for (int i = 1; i <= m - 2; ++i) {
      const double h0 = x[i] - x[i - 1], h1 = x[i + 1] - x[i];
      const double a = h0, bb = 2.0 * (h0 + h1), c = h1;
      const double r = 6.0 * ((y[i + 1] - y[i]) / h1 - (y[i] - y[i - 1]) / h0);
      if (i == 1) {
        cp[i] = c / bb;
        dp[i] = r / bb;
      } else {
        const double den = bb - a * cp[i - 1];
        cp[i] = c / den;
        dp[i] = (r - a * dp[i - 1]) / den;
      }
    }
    M[m - 2] = dp[m - 2];
    for (int i = m - 3; i >= 1; --i) M[i] = dp[i] - cp[i] * M[i + 1];
  }
  meta[2 * t] = (double)m;
  meta[2 * t + 1] = ymin;
}

// graw[t][mode] = the spline at the target mode's frequency: on the knot
// interval [x_i, x_{i+1}] holding w, with h = x_{i+1} - x_i, a = x_{i+1} - w, b = w - x_i,
//   s = (M_i a^3 + M_{i+1} b^3) / (6 h) + (y_i - M_i h^2 / 6) a / h + (y_{i+1} - M_{i+1} h^2 / 6) b / h;
// the end knot's value outside, at least the smallest knot value; 0 if masked.
__global__ void k_interp_eval(double* __restrict__ graw, const double* __restrict__ omega,
                              const double* __restrict__ knots, const double* __restrict__ meta, long long nmode,
                              int nb, int nT) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nmode * nT) return;
  const int t = (int)(idx / nmode);
  const long long mode = idx - (long long)t * nmode;
  const double w = omega[mode];
  if (!(w / kTwoPi >= kNuMinThz)) {
    graw[idx] = 0.0;
    return;
  }
  const double* x = knots + (size_t)t * 5 * nb;
  const double* y = x + nb;
  const double* M = y + nb;
  const int m = (int)meta[2 * t];
  const double ymin = meta[2 * t + 1];
  double v;
  if (m == 1 || w <= x[0]) {
    v = y[0];
  } else if (w >= x[m - 1]) {
    v = y[m - 1];
  } else {
    int lo = 0, hi = m - 1;  // x[lo] <= w < x[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (x[mid] <= w) lo = mid; else hi = mid;
    }
    const double h = x[hi] - x[lo], a = x[hi] - w, b = w - x[lo];
    v = (M[lo] * a * a * a + M[hi] * b * b * b) / (6.0 * h) + (y[lo] - M[lo] * h * h / 6.0) * a / h +
        (y[hi] - M[hi] * h * h / 6.0) * b / h;
  }
  graw[idx] = fmax(v, ymin);
}

kaldo_status run_gamma_interpolate(kaldo_ctx ctx, const double* omega_src, const double* gamma_src, int64_t n_src,
                                   int n_bins) {
  const int nT = ctx->nT;
  const long long nmode = (long long)ctx->nk * ctx->nm;
  if (n_bins < 1 || n_bins > kInterpMaxBins) return fail(ctx, KALDO_EINVAL, "n_bins must be in 1 .. 4096");
  hipStream_t st = ctx->stream;
  // doubles: source omega, source gamma, range (4), bins, knots, meta, raw values
  const size_t o_w = 0, o_g = o_w + (size_t)n_src, o_r = o_g + (size_t)nT * n_src, o_b = o_r + 4,
               o_k = o_b + (size_t)nT * n_bins * 3, o_m = o_k + (size_t)nT * 5 * n_bins, o_raw = o_m + 2 * (size_t)nT,
               total = o_raw + (size_t)nT * nmode;
  KALDO_HIP(ctx, ctx->d_interp.ensure(total * sizeof(double)));
  double* base = ctx->d_interp.as<double>();
  kaldo_status s;
  if ((s = copy_in(ctx, base + o_w, omega_src, (size_t)n_src * sizeof(double))) != KALDO_OK) return s;
  if ((s = copy_in(ctx, base + o_g, gamma_src, (size_t)nT * n_src * sizeof(double))) != KALDO_OK) return s;
  prof_begin(ctx);
  hipLaunchKernelGGL(k_interp_range, dim3(1), dim3(1024), 0, st, base + o_r, base + o_w, (long long)n_src);
  KALDO_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL(k_interp_bins, dim3(n_bins, nT), dim3(256), 0, st, base + o_b, base + o_w, base + o_g,
                     (long long)n_src, n_bins, base + o_r);
  KALDO_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL(k_interp_spline, dim3(1), dim3(64), 0, st, base + o_k, base + o_m, base + o_b, n_bins, nT);
  KALDO_HIP(ctx, hipGetLastError());
  double count = 0.0;
  KALDO_HIP(ctx, hipMemcpyAsync(&count, base + o_r + 2, sizeof(double), hipMemcpyDeviceToHost, st));
  KALDO_HIP(ctx, hipStreamSynchronize(st));
  if (!(count > 0.0)) return fail(ctx, KALDO_EINVAL, "kaldo_gamma_interpolate: no source mode with nu >= 0.01 THz");
  KALDO_HIP(ctx, ctx->d_gamma.ensure((size_t)nT * nmode * sizeof(double)));
  hipLaunchKernelGGL(k_interp_eval, dim3(blocks_for(nmode * nT, 256)), dim3(256), 0, st, base + o_raw,
                     ctx->d_omega.as<double>(), base + o_k, base + o_m, nmode, n_bins, nT);
  KALDO_HIP(ctx, hipGetLastError());
  if ((s = launch_set_average(ctx, ctx->d_gamma.as<double>(), base + o_raw, nT)) != KALDO_OK) return s;
  prof_end(ctx, "gamma_interpolate");
  return KALDO_OK;
}

}  // namespace kaldo
