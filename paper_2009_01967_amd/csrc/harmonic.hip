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

// Batched FP64 Hermitian eigensolver for small n (<= kJacobiMaxN): cyclic
// two-sided Jacobi with the round-robin ordering, one block per k, matrix in
// LDS.  Each rotation first turns the (p, q) element real with a phase, then
// applies the real symmetric Jacobi rotation; the n/2 rotations of a round act
// on disjoint index pairs and are applied together.  On exit D[k] holds the
// eigenvectors (column s = eta_s, contiguous) and lambda[k] the ascending
// eigenvalues.  info[k] = 1 if the sweep limit was reached.
constexpr int kJacobiMaxN = 32;

template <int kJacobiMaxN>
__global__ void __launch_bounds__(64) k_jacobi_hermitian(zc* __restrict__ D, double* __restrict__ lambda,
                                                         int* __restrict__ info, int n) {
  __shared__ zc A[kJacobiMaxN * kJacobiMaxN];
  __shared__ zc V[kJacobiMaxN * kJacobiMaxN];
  __shared__ double rc[kJacobiMaxN / 2], rs[kJacobiMaxN / 2];
  __shared__ zc ru[kJacobiMaxN / 2];
  __shared__ int rp[kJacobiMaxN / 2], rq[kJacobiMaxN / 2];
  __shared__ double red[64];
  __shared__ int done;
  const int k = blockIdx.x, tid = threadIdx.x;
  const int m = (n + 1) & ~1;  // even size for the round-robin schedule (index n is a dummy)
  zc* Dk = D + (size_t)k * n * n;
  for (int e = tid; e < n * n; e += 64) {
    const int a = e % n, b = e / n;  // column major input, Hermitian part (D + D^H) / 2
    const zc x = Dk[e], y = Dk[(size_t)a * n + b];
    A[a * kJacobiMaxN + b] = {0.5 * (x.re + y.re), 0.5 * (x.im - y.im)};
    V[a * kJacobiMaxN + b] = {a == b ? 1.0 : 0.0, 0.0};
  }
  if (tid == 0) done = 0;
  __syncthreads();
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    // convergence test on the off-diagonal norm
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += 64) {
      const int a = e / n, b = e % n;
      const zc v = A[a * kJacobiMaxN + b];
      const double x = v.re * v.re + v.im * v.im;
      tot += x;
      if (a != b) off += x;
    }
    red[tid] = off;
    __syncthreads();
    if (tid == 0) {
      double so = 0.0;
      for (int t = 0; t < 64; ++t) so += red[t];
      red[0] = so;
    }
    __syncthreads();
    const double soff = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    if (tid == 0) {
      double st = 0.0;
      for (int t = 0; t < 64; ++t) st += red[t];
      const double eps = 4.0 * n * 2.220446049250313e-16;  // relative off-diagonal norm target
      done = soff <= eps * eps * st;
    }
    __syncthreads();
    if (done) break;
    for (int round = 0; round < m - 1; ++round) {
      // round-robin pairs: position 0 fixed, the others rotate
      if (tid < m / 2) {
        auto slot = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (m - 1); };
        int p = slot(tid), q = slot(m - 1 - tid);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        rp[tid] = p;
        rq[tid] = q;
        double c = 1.0, s = 0.0;
        zc u = {1.0, 0.0};
        if (q < n) {
          const zc apq = A[p * kJacobiMaxN + q];
          const double mag = sqrt(apq.re * apq.re + apq.im * apq.im);
          if (mag > 0.0) {
            u = {apq.re / mag, apq.im / mag};
            const double app = A[p * kJacobiMaxN + p].re, aqq = A[q * kJacobiMaxN + q].re;
            const double theta = (aqq - app) / (2.0 * mag);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        rc[tid] = c;
        rs[tid] = s;
        ru[tid] = u;
      }
      __syncthreads();
      // columns: col_p <- c col_p - s conj(u) col_q ; col_q <- s col_p + c conj(u) col_q  (A and V)
      for (int e = tid; e < (m / 2) * n; e += 64) {
        const int pr = e / n, r = e % n;
        const int p = rp[pr], q = rq[pr];
        if (q >= n) continue;
        const double c = rc[pr], s = rs[pr];
        const zc ub = {ru[pr].re, -ru[pr].im};
        for (int w = 0; w < 2; ++w) {
          zc* M = w == 0 ? A : V;
          const zc xp = M[r * kJacobiMaxN + p], xq = M[r * kJacobiMaxN + q];
          const zc uq = cmul(ub, xq);
          M[r * kJacobiMaxN + p] = {c * xp.re - s * uq.re, c * xp.im - s * uq.im};
          M[r * kJacobiMaxN + q] = {s * xp.re + c * uq.re, s * xp.im + c * uq.im};
        }
      }
      __syncthreads();
      // rows of A: row_p <- c row_p - s u row_q ; row_q <- s row_p + c u row_q
      for (int e = tid; e < (m / 2) * n; e += 64) {
        const int pr = e / n, col = e % n;
        const int p = rp[pr], q = rq[pr];
        if (q >= n) continue;
        const double c = rc[pr], s = rs[pr];
        const zc u = ru[pr];
        const zc xp = A[p * kJacobiMaxN + col], xq = A[q * kJacobiMaxN + col];
        const zc uq = cmul(u, xq);
        A[p * kJacobiMaxN + col] = {c * xp.re - s * uq.re, c * xp.im - s * uq.im};
        A[q * kJacobiMaxN + col] = {s * xp.re + c * uq.re, s * xp.im + c * uq.im};
      }
      __syncthreads();
      // keep A exactly Hermitian: lower triangle from the upper one, real diagonal
      for (int e = tid; e < n * n; e += 64) {
        const int r = e / n, col = e % n;
        if (r > col) {
          const zc u = A[col * kJacobiMaxN + r];
          A[r * kJacobiMaxN + col] = {u.re, -u.im};
        } else if (r == col) {
          A[r * kJacobiMaxN + r].im = 0.0;
        }
      }
      __syncthreads();
    }
  }
  // ascending order by rank (ties broken by index), eigenvector s contiguous
  for (int s = tid; s < n; s += 64) {
    const double ls = A[s * kJacobiMaxN + s].re;
    int rank = 0;
    for (int t = 0; t < n; ++t) {
      const double lt = A[t * kJacobiMaxN + t].re;
      rank += (lt < ls) || (lt == ls && t < s);
    }
    lambda[(size_t)k * n + rank] = ls;
    for (int a = 0; a < n; ++a) Dk[(size_t)rank * n + a] = V[a * kJacobiMaxN + s];
  }
  if (tid == 0) info[k] = done ? 0 : 1;
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
    if (n <= kJacobiMaxN) {
      if (n <= 8)
        hipLaunchKernelGGL(k_jacobi_hermitian<8>, dim3(nk), dim3(64), 0, st, D, ctx->d_lambda.as<double>(), info, n);
      else if (n <= 16)
        hipLaunchKernelGGL(k_jacobi_hermitian<16>, dim3(nk), dim3(64), 0, st, D, ctx->d_lambda.as<double>(), info, n);
      else
        hipLaunchKernelGGL(k_jacobi_hermitian<32>, dim3(nk), dim3(64), 0, st, D, ctx->d_lambda.as<double>(), info, n);
      KALDO_HIP(ctx, hipGetLastError());
    } else {
      rocblas_status rs = rocsolver_zheev_strided_batched(
          ctx->blas, rocblas_evect_original, rocblas_fill_upper, n, reinterpret_cast<rocblas_double_complex*>(D), n,
          (rocblas_stride)nn, ctx->d_lambda.as<double>(), (rocblas_stride)n, ctx->d_dyn.as<double>(),
          (rocblas_stride)n, info, nk);
      if (rs != rocblas_status_success) return fail(ctx, KALDO_EDEVICE, "rocsolver_zheev_strided_batched failed");
    }
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
