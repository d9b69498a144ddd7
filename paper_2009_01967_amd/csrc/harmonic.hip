// Harmonic stage on the GPU (paper Sec. II.A-B):
//   D(q_k) = sum_R fc2(i,j,R) / sqrt(m_i m_j) exp(-2 pi i q_k.R)   (eq. eigenvectors_crystal)
//   FP64 Hermitian eigensolve (rocSOLVER), omega = sign(lambda) sqrt|lambda|
//   velocity matrices W_a = E^H dD/dq_a E inside degenerate sets (eq. velocity_crystal)
#include <rocsolver/rocsolver.h>

#include "common.h"
#include "internal.h"

namespace kaldo {

using zc = cplx<double>;

// Column-major Hermitian D(q_k): element (a, b) at D[k][b * n + a], in ps^-2.
__global__ void k_dyn_assemble(zc* __restrict__ D, const int2* __restrict__ pair, const int* __restrict__ R,
                               const double* __restrict__ val, const double* __restrict__ mass, int N, int G0,
                               int G1, int G2, int nk) {
  const int n = 3 * N;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nk * n * n) return;
  const int a = (int)(idx % n);
  const int b = (int)((idx / n) % n);
  const int k = (int)(idx / ((long long)n * n));
  const int i = a / 3, al = a % 3, j = b / 3, be = b % 3;
  const int m0 = k / (G1 * G2), m1 = (k / G2) % G1, m2 = k % G2;
  const long long Gt = (long long)G0 * G1 * G2;
  const int2 pr = pair[i * N + j];
  double re = 0.0, im = 0.0;
  for (int q = pr.x; q < pr.y; ++q) {
    const long long num = (long long)m0 * R[3 * q] * (G1 * G2) + (long long)m1 * R[3 * q + 1] * (G0 * G2) +
                          (long long)m2 * R[3 * q + 2] * (G0 * G1);
    double c, s;
    unit_phase(-num, Gt, c, s);  // exp(-2 pi i q.R)
    const double v = val[9 * q + 3 * al + be];
    re += v * c;
    im += v * s;
  }
  const double scale = kEvUnit / sqrt(mass[i] * mass[j]);
  D[(size_t)k * n * n + (size_t)b * n + a] = {re * scale, im * scale};
}

// Real symmetric D at Gamma for the real eigensolver.
__global__ void k_dyn_assemble_real(double* __restrict__ D, const int2* __restrict__ pair,
                                    const double* __restrict__ val, const double* __restrict__ mass, int N) {
  const int n = 3 * N;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * n) return;
  const int a = (int)(idx % n), b = (int)(idx / n);
  const int i = a / 3, al = a % 3, j = b / 3, be = b % 3;
  const int2 pr = pair[i * N + j];
  double s = 0.0;
  for (int q = pr.x; q < pr.y; ++q) s += val[9 * q + 3 * al + be];
  D[(size_t)b * n + a] = s * kEvUnit / sqrt(mass[i] * mass[j]);
}

__global__ void k_real_to_complex(zc* __restrict__ out, const double* __restrict__ in, long long count) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) out[idx] = {in[idx], 0.0};
}

// Per k: omega, frequencies in THz, degenerate sets, unstable-mode and solver checks.
// flag[0] = first unstable (k * n + s) + 1, flag[1] = first failed k + 1 (0 = none).
__global__ void k_modes(const double* __restrict__ lambda, const int* __restrict__ info, double* __restrict__ omega,
                        double* __restrict__ nu, int* __restrict__ setid, int* __restrict__ flag, int nk, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  if (info[k] != 0) atomicCAS(&flag[1], 0, k + 1);
  int first = 0;
  double prev = 0.0;
  for (int s = 0; s < n; ++s) {
    const double lam = lambda[(size_t)k * n + s];
    const double w = lam >= 0.0 ? sqrt(lam) : -sqrt(-lam);
    const double f = w / kTwoPi;
    omega[(size_t)k * n + s] = w;
    nu[(size_t)k * n + s] = f;
    if (f < kNuUnstableThz) atomicCAS(&flag[0], 0, k * n + s + 1);
    if (s == 0 || fabs(f - prev) >= kDegenerateThz) first = s;
    setid[(size_t)k * n + s] = first;
    prev = f;
  }
}

// dD/dq_a (Cartesian, 1/A), row-major per k and direction: G[k][a][r][c], ps^-2 A.
__global__ void k_dyn_gradient(zc* __restrict__ G, const int2* __restrict__ pair, const int* __restrict__ R,
                               const double* __restrict__ val, const double* __restrict__ mass,
                               const double* __restrict__ cell, int N, int G0, int G1, int G2, int nk) {
  const int n = 3 * N;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nk * n * n) return;
  const int c = (int)(idx % n);
  const int r = (int)((idx / n) % n);
  const int k = (int)(idx / ((long long)n * n));
  const int i = r / 3, al = r % 3, j = c / 3, be = c % 3;
  const int m0 = k / (G1 * G2), m1 = (k / G2) % G1, m2 = k % G2;
  const long long Gt = (long long)G0 * G1 * G2;
  const int2 pr = pair[i * N + j];
  double acc[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  for (int q = pr.x; q < pr.y; ++q) {
    const int R0 = R[3 * q], R1 = R[3 * q + 1], R2 = R[3 * q + 2];
    const long long num = (long long)m0 * R0 * (G1 * G2) + (long long)m1 * R1 * (G0 * G2) + (long long)m2 * R2 * (G0 * G1);
    double cs, sn;
    unit_phase(-num, Gt, cs, sn);
    const double v = val[9 * q + 3 * al + be];
    for (int d = 0; d < 3; ++d) {
      const double Rc = R0 * cell[d] + R1 * cell[3 + d] + R2 * cell[6 + d];
      // (-i Rc) (cs + i sn) = Rc sn - i Rc cs
      acc[d][0] += v * Rc * sn;
      acc[d][1] -= v * Rc * cs;
    }
  }
  const double scale = kEvUnit / sqrt(mass[i] * mass[j]);
  for (int d = 0; d < 3; ++d)
    G[(((size_t)k * 3 + d) * n + r) * n + c] = {acc[d][0] * scale, acc[d][1] * scale};
}

// W_a[s][t] = eta_s^H dD_a eta_t for modes s, t of the same degenerate set.
__global__ void k_velocity_matrix(zc* __restrict__ W, const zc* __restrict__ G, const zc* __restrict__ E,
                                  const int* __restrict__ setid, int nk, int n) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nk * 3 * n * n) return;
  const int t = (int)(idx % n);
  const int s = (int)((idx / n) % n);
  const int d = (int)((idx / ((long long)n * n)) % 3);
  const int k = (int)(idx / (3LL * n * n));
  if (setid[(size_t)k * n + s] != setid[(size_t)k * n + t]) return;
  const zc* es = E + ((size_t)k * n + s) * n;
  const zc* et = E + ((size_t)k * n + t) * n;
  const zc* g = G + ((size_t)k * 3 + d) * n * n;
  double re = 0.0, im = 0.0;
  for (int r = 0; r < n; ++r) {
    double xr = 0.0, xi = 0.0;  // (dD eta_t)[r]
    for (int c = 0; c < n; ++c) {
      const zc gv = g[(size_t)r * n + c];
      const zc ev = et[c];
      xr += gv.re * ev.re - gv.im * ev.im;
      xi += gv.re * ev.im + gv.im * ev.re;
    }
    const zc e = es[r];
    re += e.re * xr + e.im * xi;  // conj(e) * x
    im += e.re * xi - e.im * xr;
  }
  W[(((size_t)k * 3 + d) * n + s) * n + t] = {re, im};
}

// Per mode: v = Re W_a[s][s] / (2 w) and the set product Re Tr(W_a W_b) / (4 w^2) / |set|.
__global__ void k_velocity_products(double* __restrict__ vel, double* __restrict__ vv, const zc* __restrict__ W,
                                    const double* __restrict__ omega, const int* __restrict__ setid, int nk, int n) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nk * n) return;
  const int s = (int)(idx % n);
  const int k = (int)(idx / n);
  const double* om = omega + (size_t)k * n;
  const int* sid = setid + (size_t)k * n;
  const double w = om[s];
  double* vo = vel + idx * 3;
  double* vvo = vv + idx * 9;
  if (w / kTwoPi < kNuMinThz) {
    for (int d = 0; d < 3; ++d) vo[d] = 0.0;
    for (int d = 0; d < 9; ++d) vvo[d] = 0.0;
    return;
  }
  for (int d = 0; d < 3; ++d) vo[d] = W[(((size_t)k * 3 + d) * n + s) * n + s].re / (2.0 * w);
  const int first = sid[s];
  int last = first;
  while (last + 1 < n && sid[last + 1] == first) ++last;
  double wm = 0.0;
  for (int t = first; t <= last; ++t) wm += om[t];
  wm /= (last - first + 1);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double tr = 0.0;
      for (int t = first; t <= last; ++t)
        for (int u = first; u <= last; ++u) {
          const zc x = W[(((size_t)k * 3 + a) * n + t) * n + u];
          const zc y = W[(((size_t)k * 3 + b) * n + u) * n + t];
          tr += x.re * y.re - x.im * y.im;
        }
      vvo[3 * a + b] = tr / (4.0 * wm * wm) / (last - first + 1);
    }
}

kaldo_status run_phonons(kaldo_ctx ctx, bool want_velocity) {
  const int N = ctx->n_atoms, n = ctx->nm, nk = ctx->nk;
  const size_t nn = (size_t)n * n;
  hipStream_t st = ctx->stream;
  const int T = 256;
  KALDO_HIP(ctx, ctx->d_evec.ensure(nn * nk * sizeof(zc)));
  KALDO_HIP(ctx, ctx->d_lambda.ensure((size_t)nk * n * sizeof(double)));
  KALDO_HIP(ctx, ctx->d_omega.ensure((size_t)nk * n * sizeof(double)));
  KALDO_HIP(ctx, ctx->d_setid.ensure((size_t)nk * n * sizeof(int)));
  KALDO_HIP(ctx, ctx->d_info.ensure(((size_t)nk + 2) * sizeof(int)));
  KALDO_HIP(ctx, ctx->d_work.ensure(std::max<size_t>((size_t)nk * n * sizeof(double), 2 * n * sizeof(double))));
  const int2* pair = ctx->d_fc2_pair.as<int2>();
  int* info = ctx->d_info.as<int>();
  int* flag = info + nk;
  KALDO_HIP(ctx, hipMemsetAsync(flag, 0, 2 * sizeof(int), st));
  if (nk == 1) {
    KALDO_HIP(ctx, ctx->d_dyn.ensure(nn * sizeof(double) + 2 * n * sizeof(double)));
    double* Dr = ctx->d_dyn.as<double>();
    double* offd = Dr + nn;
    hipLaunchKernelGGL(k_dyn_assemble_real, dim3(blocks_for((long long)nn, T)), dim3(T), 0, st, Dr, pair,
                       ctx->d_fc2_val.as<double>(), ctx->d_masses.as<double>(), N);
    KALDO_HIP(ctx, hipGetLastError());
    prof_begin(ctx);
    rocblas_status rs = rocsolver_dsyevd(ctx->blas, rocblas_evect_original, rocblas_fill_upper, n, Dr, n,
                                         ctx->d_lambda.as<double>(), offd, info);
    if (rs != rocblas_status_success) return fail(ctx, KALDO_EDEVICE, "rocsolver_dsyevd failed");
    prof_end(ctx, "eigensolve");
    hipLaunchKernelGGL(k_real_to_complex, dim3(blocks_for((long long)nn, T)), dim3(T), 0, st,
                       ctx->d_evec.as<zc>(), Dr, (long long)nn);
    KALDO_HIP(ctx, hipGetLastError());
  } else {
    zc* D = ctx->d_evec.as<zc>();
    prof_begin(ctx);
    hipLaunchKernelGGL(k_dyn_assemble, dim3(blocks_for((long long)nn * nk, T)), dim3(T), 0, st, D, pair,
                       ctx->d_fc2_R.as<int>(), ctx->d_fc2_val.as<double>(), ctx->d_masses.as<double>(), N,
                       ctx->grid[0], ctx->grid[1], ctx->grid[2], nk);
    KALDO_HIP(ctx, hipGetLastError());
    prof_end(ctx, "dyn_assemble");
    KALDO_HIP(ctx, ctx->d_dyn.ensure((size_t)nk * n * sizeof(double)));
    prof_begin(ctx);
    rocblas_status rs = rocsolver_zheevd_strided_batched(
        ctx->blas, rocblas_evect_original, rocblas_fill_upper, n, reinterpret_cast<rocblas_double_complex*>(D), n,
        (rocblas_stride)nn, ctx->d_lambda.as<double>(), (rocblas_stride)n, ctx->d_dyn.as<double>(),
        (rocblas_stride)n, info, nk);
    if (rs != rocblas_status_success) return fail(ctx, KALDO_EDEVICE, "rocsolver_zheevd_strided_batched failed");
    prof_end(ctx, "eigensolve");
  }
  hipLaunchKernelGGL(k_modes, dim3(blocks_for(nk, T)), dim3(T), 0, st, ctx->d_lambda.as<double>(), info,
                     ctx->d_omega.as<double>(), ctx->d_work.as<double>(), ctx->d_setid.as<int>(), flag, nk, n);
  KALDO_HIP(ctx, hipGetLastError());
  if (want_velocity) {
    KALDO_HIP(ctx, ctx->d_vel.ensure((size_t)nk * n * 3 * sizeof(double)));
    KALDO_HIP(ctx, ctx->d_vv.ensure((size_t)nk * n * 9 * sizeof(double)));
    KALDO_HIP(ctx, ctx->d_scratch2.ensure(2 * (size_t)nk * 3 * nn * sizeof(zc)));
    KALDO_HIP(ctx, ctx->d_tabs.ensure(9 * sizeof(double)));
    KALDO_HIP(ctx, hipMemcpyAsync(ctx->d_tabs.p, ctx->cell, 9 * sizeof(double), hipMemcpyHostToDevice, st));
    zc* G = ctx->d_scratch2.as<zc>();
    zc* W = G + (size_t)nk * 3 * nn;
    KALDO_HIP(ctx, hipMemsetAsync(W, 0, (size_t)nk * 3 * nn * sizeof(zc), st));
    hipLaunchKernelGGL(k_dyn_gradient, dim3(blocks_for((long long)nn * nk, T)), dim3(T), 0, st, G, pair,
                       ctx->d_fc2_R.as<int>(), ctx->d_fc2_val.as<double>(), ctx->d_masses.as<double>(),
                       ctx->d_tabs.as<double>(), N, ctx->grid[0], ctx->grid[1], ctx->grid[2], nk);
    KALDO_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_velocity_matrix, dim3(blocks_for((long long)nn * 3 * nk, T)), dim3(T), 0, st, W, G,
                       ctx->d_evec.as<zc>(), ctx->d_setid.as<int>(), nk, n);
    KALDO_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_velocity_products, dim3(blocks_for((long long)n * nk, T)), dim3(T), 0, st,
                       ctx->d_vel.as<double>(), ctx->d_vv.as<double>(), W, ctx->d_omega.as<double>(),
                       ctx->d_setid.as<int>(), nk, n);
    KALDO_HIP(ctx, hipGetLastError());
  }
  int hflag[2] = {0, 0};
  KALDO_HIP(ctx, hipMemcpyAsync(hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, st));
  KALDO_HIP(ctx, hipStreamSynchronize(st));
  if (hflag[1]) return fail(ctx, KALDO_EDEVICE, "eigensolver did not converge at k = " + std::to_string(hflag[1] - 1));
  if (hflag[0]) {
    const int ks = hflag[0] - 1;
    return fail(ctx, KALDO_EUNSTABLE,
                "imaginary mode below -0.05 THz at k = " + std::to_string(ks / n) + ", s = " + std::to_string(ks % n));
  }
  return KALDO_OK;
}

}  // namespace kaldo
