// Conductivities from the linewidths.
//   RTA  (paper eq. RTA):   kappa_ab = 1/(N_k V) sum_mu c_mu tau_mu v_mu,a v_mu,b, tau = 1/(2 gamma)
//   QHGK (Sec. II.C):       kappa_ab = 1/V sum_{mu mu'} c_{mu mu'} v_{mu mu' a} v_{mu mu' b} tau_{mu mu'}
// All accumulation is FP64 with fixed-order (deterministic) reductions.
#include <mutex>

#include "common.h"
#include "gemm.h"
#include "internal.h"
#include "mfma.h"

namespace kaldo {

__device__ __forceinline__ double heat_capacity(double w, double T, int classical) {
  if (classical) return kBoltzmann;
  const double x = kHbar * w / (kBoltzmann * T);
  if (x == 0.0) return kBoltzmann;
  const double h = 0.5 * x / sinh(0.5 * x);
  return kBoltzmann * h * h;
}

__device__ __forceinline__ double occupation(double w, double T, int classical) {
  if (classical) return kBoltzmann * T / (kHbar * w);
  if (T <= 0.0) return 0.0;
  return 1.0 / expm1(kHbar * w / (kBoltzmann * T));
}

template <int B>
__device__ void block_sum9(double (&v)[9], double* out) {
  __shared__ double red[B / 64][9];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    double x = v[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[wave][c] = x;
  }
  __syncthreads();
  if (threadIdx.x < 9) {
    double x = 0.0;
    for (int w = 0; w < B / 64; ++w) x += red[w][threadIdx.x];
    out[threadIdx.x] = x;
  }
}

// one block per (temperature, slice of modes); partial[t][slice][9].  Modes
// m0 <= m < m1 (the first-mode points the linewidths cover) enter the sum.
__global__ void __launch_bounds__(256) k_kappa_rta(double* __restrict__ partial, const double* __restrict__ gamma,
                                                   const double* __restrict__ omega, const double* __restrict__ vv,
                                                   int nmode, int m0, int m1, double4 T03, double4 T47,
                                                   int classical) {
  const int t = blockIdx.y;
  const double Ts[8] = {T03.x, T03.y, T03.z, T03.w, T47.x, T47.y, T47.z, T47.w};
  const double T = Ts[t];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int m = m0 + blockIdx.x * blockDim.x + threadIdx.x; m < m1; m += gridDim.x * blockDim.x) {
    const double w = omega[m];
    if (w / kTwoPi < kNuMinThz) continue;
    const double ct = heat_capacity(w, T, classical) / (2.0 * gamma[(size_t)t * nmode + m]);
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] += ct * vv[(size_t)m * 9 + c];
  }
  block_sum9<256>(acc, partial + ((size_t)t * gridDim.x + blockIdx.x) * 9);
}

__global__ void k_reduce_slices(double* __restrict__ out, const double* __restrict__ partial, int nslice, int nT,
                                double scale) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nT * 9) return;
  const int t = idx / 9, c = idx % 9;
  double s = 0.0;
  for (int b = 0; b < nslice; ++b) s += partial[((size_t)t * nslice + b) * 9 + c];
  out[idx] = s * scale;
}

static double cell_volume(const double* c) {
  const double det = c[0] * (c[4] * c[8] - c[5] * c[7]) - c[1] * (c[3] * c[8] - c[5] * c[6]) +
                     c[2] * (c[3] * c[7] - c[4] * c[6]);
  return det < 0 ? -det : det;
}

kaldo_status run_kappa_rta(kaldo_ctx ctx) {
  const int nmode = ctx->nk * ctx->nm;
  const int nT = ctx->nT;
  const int nslice = 64;
  hipStream_t st = ctx->stream;
  KALDO_HIP(ctx, ctx->d_kappa.ensure((size_t)nT * 9 * sizeof(double)));
  KALDO_HIP(ctx, ctx->d_partial.ensure((size_t)nT * nslice * 9 * sizeof(double)));
  double4 T03 = make_double4(ctx->T[0], ctx->T[1], ctx->T[2], ctx->T[3]);
  double4 T47 = make_double4(ctx->T[4], ctx->T[5], ctx->T[6], ctx->T[7]);
  prof_begin(ctx);
  hipLaunchKernelGGL(k_kappa_rta, dim3(nslice, nT), dim3(256), 0, st, ctx->d_partial.as<double>(),
                     ctx->d_gamma.as<double>(), ctx->d_omega.as<double>(), ctx->d_vv.as<double>(), nmode,
                     ctx->g_lo * ctx->nm, ctx->g_hi * ctx->nm, T03, T47, ctx->stats == KALDO_CLASSICAL ? 1 : 0);
  KALDO_HIP(ctx, hipGetLastError());
  prof_end(ctx, "kappa_rta");
  const double scale = kKappaSI / (ctx->nk * cell_volume(ctx->cell));
  hipLaunchKernelGGL(k_reduce_slices, dim3(1), dim3(256), 0, st, ctx->d_kappa.as<double>(),
                     ctx->d_partial.as<double>(), nslice, nT, scale);
  KALDO_HIP(ctx, hipGetLastError());
  return KALDO_OK;
}

// ---- RTA without allocation ----------------------------------------------------------
// kaldo_kappa_rta_noalloc keeps its slice partials and the reduced kappa in
// this file-scope device array instead of context buffers.  Each device the
// library runs on holds its own copy for the life of the process.  In host
// code `scratch` names a host-side stand-in, never the device memory: the
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current (noalloc_setup, called by kaldo_create) and kept below.
constexpr int kNoAllocSlices = 64;
constexpr size_t kNoAllocDoubles = (size_t)KALDO_MAX_T * (kNoAllocSlices + 1) * 9;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
    g_scratch_done[device] = true;
  }
  return g_scratch_err[device];
}

kaldo_status run_kappa_rta_noalloc(kaldo_ctx ctx, double* kappa_out) {
  const int nT = ctx->nT;
  const size_t need = (size_t)nT * (kNoAllocSlices + 1) * 9;
  if (need > kNoAllocDoubles)
    return fail(ctx, KALDO_EINVAL,
                "kaldo_kappa_rta_noalloc: " + std::to_string(need) + " doubles of scratch needed, at most " +
                    std::to_string(kNoAllocDoubles));
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices && g_scratch_done[ctx->device])
      base = static_cast<double*>(g_scratch_ptr[ctx->device]);
  }
  if (!base) return fail(ctx, KALDO_EDEVICE, "kaldo_kappa_rta_noalloc: no device address of the scratch array");
  double* partial = base;                                       // [nT][slices][9]
  double* kappa = base + (size_t)KALDO_MAX_T * kNoAllocSlices * 9;  // [nT][9]
  const int nmode = ctx->nk * ctx->nm;
  hipStream_t st = ctx->stream;
  double4 T03 = make_double4(ctx->T[0], ctx->T[1], ctx->T[2], ctx->T[3]);
  double4 T47 = make_double4(ctx->T[4], ctx->T[5], ctx->T[6], ctx->T[7]);
  // every slice of every temperature is written by the first kernel, every
  // kappa entry by the second: nothing left from an earlier call is read
  hipLaunchKernelGGL(k_kappa_rta, dim3(kNoAllocSlices, nT), dim3(256), 0, st, partial, ctx->d_gamma.as<double>(),
                     ctx->d_omega.as<double>(), ctx->d_vv.as<double>(), nmode, ctx->g_lo * ctx->nm,
                     ctx->g_hi * ctx->nm, T03, T47, ctx->stats == KALDO_CLASSICAL ? 1 : 0);
  KALDO_HIP(ctx, hipGetLastError());
  const double scale = kKappaSI / (ctx->nk * cell_volume(ctx->cell));
  hipLaunchKernelGGL(k_reduce_slices, dim3(1), dim3(256), 0, st, kappa, partial, kNoAllocSlices, nT, scale);
  KALDO_HIP(ctx, hipGetLastError());
  return copy_out(ctx, kappa_out, kappa, (size_t)nT * 9 * sizeof(double));
}

// ---- QHGK ---------------------------------------------------------------------------
// most (first-mode block, u slice) partial sums per temperature of k_qhgk_pairs
constexpr int kQhgkMaxSlices = 2048;

// The second modes u that a block of first modes s0 <= s < s1 pairs with
// under an energy threshold: frequencies ascend at Gamma, so every u with
// |w_s - w_u| <= thr lies in [lo, hi), found by bisection with the bounds
// widened by a relative 1e-9 (the exact test decides each pair).  Without a
// threshold, every u.
__device__ __forceinline__ void qhgk_band(const double* __restrict__ omega, int n, int s0, int s1, double thr,
                                          int* lo, int* hi) {
  if (!(thr > 0.0)) {
    *lo = 0;
    *hi = n;
    return;
  }
  const double slack = 1e-9 * (fabs(omega[0]) + fabs(omega[n - 1]) + thr);
  const double wlo = omega[s0] - thr - slack, whi = omega[s1 - 1] + thr + slack;
  int a = 0, b = n;  // first u with omega[u] >= wlo
  while (a < b) {
    const int m = (a + b) >> 1;
    if (omega[m] < wlo) a = m + 1; else b = m;
  }
  *lo = a;
  b = n;  // first u with omega[u] > whi
  while (a < b) {
    const int m = (a + b) >> 1;
    if (omega[m] <= whi) a = m + 1; else b = m;
  }
  *hi = a;
}

// Lorentzian lifetime of a pair (Sec. II.C, eq. lorentzian_amorphous) with the
// options of Appendix A: gs is the pair width (the two linewidths, or twice
// the bandwidth); 0 beyond the threshold.
__device__ __forceinline__ double qhgk_tau(double ws, double wu, double gs, double thr) {
  const double dw = ws - wu;
  if (thr > 0.0 && fabs(dw) > thr) return 0.0;
  return gs / (dw * dw + gs * gs);
}

// QHGK pair sum over (s, u) of c tau v_a v_b.  V_d column major: V_d[u * n + s]
// = (E^T M_d E)[s][u].  One thread per first mode s (lanes over consecutive s
// read V_d coalesced) and slice z of the second modes; each block writes its
// 9 sums to partial[t][z * gridDim.x + blockIdx.x].  With a threshold only the
// band of u a block can pair with is read.
__global__ void __launch_bounds__(256) k_qhgk_pairs(double* __restrict__ partial, const double* __restrict__ Vm,
                                                    const double* __restrict__ omega, const double* __restrict__ gamma,
                                                    int n, int ul, double4 T03, double4 T47, int classical,
                                                    double bandwidth, double thr) {
  const int t = blockIdx.y, z = blockIdx.z;
  const double Ts[8] = {T03.x, T03.y, T03.z, T03.w, T47.x, T47.y, T47.z, T47.w};
  const double T = Ts[t];
  const double* g = gamma + (size_t)t * n;
  const size_t nn = (size_t)n * n;
  const int s0 = blockIdx.x * blockDim.x, s1 = min(n, s0 + (int)blockDim.x);
  const int s = s0 + threadIdx.x;
  __shared__ int band[2];
  if (threadIdx.x == 0) qhgk_band(omega, n, s0, s1, thr, &band[0], &band[1]);
  __syncthreads();
  const int u0 = max(z * ul, band[0]), u1 = min(min(n, (z + 1) * ul), band[1]);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const double ws = s < n ? omega[s] : 0.0;
  if (s < n && ws / kTwoPi >= kNuMinThz) {
    const double gss = bandwidth > 0.0 ? bandwidth : g[s];
    for (int u = u0; u < u1; ++u) {
      const double wu = omega[u];
      if (wu / kTwoPi < kNuMinThz) continue;
      const double tau = qhgk_tau(ws, wu, gss + (bandwidth > 0.0 ? bandwidth : g[u]), thr);
      if (tau == 0.0) continue;
      double c;
      if (classical) {
        c = kBoltzmann;
      } else if (fabs(ws - wu) < 1e-9 * fmax(fabs(ws), fabs(wu))) {
        c = heat_capacity(0.5 * (ws + wu), T, 0);
      } else {
        c = kHbar * ws * wu / T * (occupation(wu, T, 0) - occupation(ws, T, 0)) / (ws - wu);
      }
      const double inv = 1.0 / (2.0 * sqrt(ws * wu));
      const size_t m = (size_t)u * n + s;
      const double v0 = Vm[m] * inv, v1 = Vm[nn + m] * inv, v2 = Vm[2 * nn + m] * inv;
      const double w = c * tau;
      acc[0] += w * v0 * v0;
      acc[1] += w * v0 * v1;
      acc[2] += w * v0 * v2;
      acc[3] += w * v1 * v1;
      acc[4] += w * v1 * v2;
      acc[5] += w * v2 * v2;
    }
  }
  double full[9] = {acc[0], acc[1], acc[2], acc[1], acc[3], acc[4], acc[2], acc[4], acc[5]};
  block_sum9<256>(full, partial + ((size_t)t * gridDim.z * gridDim.x + (size_t)z * gridDim.x + blockIdx.x) * 9);
}

// Mode diffusivity (Sec. II.C, eq. diffusivity_per_mode) per direction a:
// D[t][s][a] = sum_u v_{s u a}^2 tau_{s u} in mm^2/s (the printed 1/(N_k V) is
// not applied: it would not leave a diffusivity).  One thread per (s, t, u
// slice): the lanes read consecutive s of V_d (coalesced) and slice z of the
// grid sums u in [z * ul, (z + 1) * ul) (within the block's band under a
// threshold) into partial[z][t][s][a].
__global__ void __launch_bounds__(256) k_qhgk_diffusivity(double* __restrict__ partial, const double* __restrict__ Vm,
                                                          const double* __restrict__ omega,
                                                          const double* __restrict__ gamma, int n, int nT, int ul,
                                                          double bandwidth, double thr) {
  const int t = blockIdx.y, z = blockIdx.z;
  const int s0 = blockIdx.x * blockDim.x, s1 = min(n, s0 + (int)blockDim.x);
  const int s = s0 + threadIdx.x;
  __shared__ int band[2];
  if (threadIdx.x == 0) qhgk_band(omega, n, s0, s1, thr, &band[0], &band[1]);
  __syncthreads();
  if (s >= n) return;
  const size_t nn = (size_t)n * n;
  const double* g = gamma + (size_t)t * n;
  const double ws = omega[s];
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  if (ws / kTwoPi >= kNuMinThz) {
    const double gss = bandwidth > 0.0 ? bandwidth : g[s];
    const int u0 = max(z * ul, band[0]), u1 = min(min(n, (z + 1) * ul), band[1]);
    for (int u = u0; u < u1; ++u) {
      const double wu = omega[u];
      if (wu / kTwoPi < kNuMinThz) continue;
      const double tau = qhgk_tau(ws, wu, gss + (bandwidth > 0.0 ? bandwidth : g[u]), thr);
      const double inv = 1.0 / (4.0 * ws * wu);  // 1 / (2 sqrt(w w'))^2
      const size_t m = (size_t)u * n + s;
      const double v0 = Vm[m], v1 = Vm[nn + m], v2 = Vm[2 * nn + m];
      d0 += tau * inv * v0 * v0;
      d1 += tau * inv * v1 * v1;
      d2 += tau * inv * v2 * v2;
    }
  }
  double* o = partial + (((size_t)z * nT + t) * n + s) * 3;
  o[0] = d0;
  o[1] = d1;
  o[2] = d2;
}

// D[t][s][a] = 1e-2 (A^2/ps -> mm^2/s) times the sum over the nz slices of
// partial[z][t][s][a], averaged over the degenerate set of s (a run of equal
// set ids): within a set only the sum is independent of the eigenvector basis.
__global__ void k_diffusivity_reduce(double* __restrict__ D, const double* __restrict__ partial,
                                     const int* __restrict__ setid, int n, int nz, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int a = (int)(i % 3);
  const int s = (int)((i / 3) % n);
  const long long base = i - 3LL * s - a;  // element (t, 0, 0)
  int lo = s, hi = s + 1;
  while (lo > 0 && setid[lo - 1] == setid[s]) --lo;
  while (hi < n && setid[hi] == setid[s]) ++hi;
  double v = 0.0;
  for (int u = lo; u < hi; ++u)
    for (int z = 0; z < nz; ++z) v += partial[(size_t)z * count + base + 3 * u + a];
  D[i] = 1e-2 * v / (hi - lo);
}

// ---- generalised velocity V_d = E^T M_d E at Gamma ----------------------------------
// M_d[a][b] = sum over the fc2 blocks of the pair (i, j) of
// (x_i - x_j - R.cell)_d fc2[alpha][beta] / sqrt(m_i m_j) (a = 3 i + alpha,
// b = 3 j + beta) has one 3 x 3 block per coupled atom pair: it is applied as
// a sparse product (k_vel_spmm), and the dense E^T (M_d E) runs on the FP64
// matrix cores (the GEMM core of the projection with a plain store).

// C[p][d][alpha][beta]: the three displacement-weighted blocks of coupled pair p
__global__ void k_vel_coeffs(double* __restrict__ C, const int4* __restrict__ plist, const int* __restrict__ R,
                             const double* __restrict__ val, const double* __restrict__ mass,
                             const double* __restrict__ pos, const double* __restrict__ cell, int npairs) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 9LL * npairs) return;
  const int p = (int)(idx / 9), ab = (int)(idx % 9);
  const int4 pr = plist[p];
  const int i = pr.x, j = pr.y;
  double acc[3] = {0, 0, 0};
  for (int q = pr.z; q < pr.w; ++q) {
    const double v = val[9 * q + ab];
    for (int d = 0; d < 3; ++d) {
      const double Rc = R[3 * q] * cell[d] + R[3 * q + 1] * cell[3 + d] + R[3 * q + 2] * cell[6 + d];
      acc[d] += (pos[3 * i + d] - pos[3 * j + d] - Rc) * v;
    }
  }
  const double scale = kEvUnit / sqrt(mass[i] * mass[j]);
  for (int d = 0; d < 3; ++d) C[(size_t)p * 27 + d * 9 + ab] = acc[d] * scale;
}

// XT_d[u][a] = (M_d E)[a][u] for d = 0..2, rows of length ld (zeros for a >= n):
// one block per eigenvector u, staged in LDS when it fits, one thread per row a.
template <bool LDS>
__global__ void __launch_bounds__(256) k_vel_spmm(double* __restrict__ XT, const double* __restrict__ E,
                                                  const double* __restrict__ C, const int* __restrict__ rows,
                                                  const int4* __restrict__ plist, int n, int ld) {
  extern __shared__ double ecol[];
  const int u = blockIdx.x;
  const double* eu = E + (size_t)u * n;
  if constexpr (LDS) {
    for (int b = threadIdx.x; b < n; b += blockDim.x) ecol[b] = eu[b];
    __syncthreads();
  }
  const double* ev = LDS ? ecol : eu;
  const size_t plane = (size_t)n * ld;
  for (int a = threadIdx.x; a < ld; a += blockDim.x) {
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    if (a < n) {
      const int i = a / 3, al = a % 3;
      for (int p = rows[i]; p < rows[i + 1]; ++p) {
        const int j = plist[p].y;
        const double* c = C + (size_t)p * 27 + 3 * al;
#pragma unroll
        for (int be = 0; be < 3; ++be) {
          const double e = ev[3 * j + be];
          x0 += c[be] * e;
          x1 += c[9 + be] * e;
          x2 += c[18 + be] * e;
        }
      }
    }
    const size_t o = (size_t)u * ld + a;
    XT[o] = x0;
    XT[plane + o] = x1;
    XT[2 * plane + o] = x2;
  }
}

// E rows of length ld (zeros for a >= n): the B operand of the velocity GEMM
__global__ void k_vel_pad(double* __restrict__ Ep, const double* __restrict__ E, int n, int ld) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * ld) return;
  const int s = (int)(idx / ld), a = (int)(idx % ld);
  Ep[idx] = a < n ? E[(size_t)s * n + a] : 0.0;
}

// GEMM epilogue: the FP64 tile stored as out[row * ldc + col] (row < m, col < c)
struct EpiStoreV {
  double* out;
  long long ldc;
  int m, c;
  template <int P, int FM, int FN>
  __device__ __forceinline__ void apply(typename Operand<P>::Acc (&acc)[FM][FN], const TileAt& at, char*) const {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int q = 0; q < FN; ++q) {
        const int col = (int)at.c0 + 16 * q + (at.lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = at.m0 + 16 * a + acc_row<P>(at.lane, r);
          if (row < m && col < c) out[(size_t)row * ldc + col] = acc[a][q][r];
        }
      }
  }
};

// V_d = E^T M_d E for d = 0..2, column major (V_d[u * n + s] = (E^T M_d E)[s][u]),
// in d_scratch2, computed as V_d^T[u][s] = sum_a XT_d[u][a] E[s][a]
static kaldo_status qhgk_velocity(kaldo_ctx ctx, double** Vout, double** part_out) {
  const int n = ctx->nm, np = (n + 15) & ~15, npairs = ctx->n_fc2_pairs;
  const size_t nn = (size_t)n * n, xn = (size_t)n * np;
  hipStream_t st = ctx->stream;
  // real eigenvectors: column s of d_dyn (Gamma path keeps them real)
  const double* E = ctx->d_dyn.as<double>();
  KALDO_HIP(ctx, ctx->d_scratch2.ensure((3 * nn + 4 * xn + (size_t)npairs * 27 +
                                         (size_t)kQhgkMaxSlices * 9 * KALDO_MAX_T) * sizeof(double)));
  double* V = ctx->d_scratch2.as<double>();
  double* XT = V + 3 * nn;
  double* Ep = XT + 3 * xn;
  double* Cp = Ep + xn;
  double* part = Cp + (size_t)npairs * 27;
  KALDO_HIP(ctx, ctx->d_tabs.ensure(9 * sizeof(double)));
  KALDO_HIP(ctx, hipMemcpyAsync(ctx->d_tabs.p, ctx->cell, 9 * sizeof(double), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_vel_coeffs, dim3(blocks_for(9LL * npairs, 256)), dim3(256), 0, st, Cp,
                     ctx->d_fc2_plist.as<int4>(), ctx->d_fc2_R.as<int>(), ctx->d_fc2_val.as<double>(),
                     ctx->d_masses.as<double>(), ctx->d_positions.as<double>(), ctx->d_tabs.as<double>(), npairs);
  KALDO_HIP(ctx, hipGetLastError());
  const size_t lds = (size_t)n * sizeof(double);
  if (lds <= 64 * 1024)
    hipLaunchKernelGGL(k_vel_spmm<true>, dim3(n), dim3(256), lds, st, XT, E, Cp, ctx->d_fc2_rows.as<int>(),
                       ctx->d_fc2_plist.as<int4>(), n, np);
  else
    hipLaunchKernelGGL(k_vel_spmm<false>, dim3(n), dim3(256), 0, st, XT, E, Cp, ctx->d_fc2_rows.as<int>(),
                       ctx->d_fc2_plist.as<int4>(), n, np);
  KALDO_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL(k_vel_pad, dim3(blocks_for((long long)xn, 256)), dim3(256), 0, st, Ep, E, n, np);
  KALDO_HIP(ctx, hipGetLastError());
  for (int d = 0; d < 3; ++d) {
    GemmOps g{};
    g.a_hi = XT + d * xn;
    g.b_hi = Ep;
    g.lda = g.ldb = np;
    g.K = np;
    g.nz = 1;
    g.m_valid = n;
    g.c_valid = n;
    const EpiStoreV e{V + d * nn, n, n, n};
    gemm_launch_tile<KALDO_FP64, 2, 4>(g, e, st);
    KALDO_HIP(ctx, hipGetLastError());
  }
  *Vout = V;
  *part_out = part;
  return KALDO_OK;
}

// u slices per block of 256 first modes, so that the grid holds about 1024
// blocks (each slice at least 32 u): more slices make the reductions
// latency-bound
static int qhgk_slices(int n, int nT, int* ul) {
  const int bs = (int)blocks_for(n, 256);
  int nz = std::max(1, std::min(1024 / std::max(1, bs * nT), (n + 31) / 32));
  *ul = (n + nz - 1) / nz;
  return (n + *ul - 1) / *ul;
}

kaldo_status run_kappa_qhgk(kaldo_ctx ctx) {
  const int n = ctx->nm, nT = ctx->nT;
  hipStream_t st = ctx->stream;
  double *M = nullptr, *part = nullptr;
  const kaldo_status vs = qhgk_velocity(ctx, &M, &part);
  if (vs != KALDO_OK) return vs;
  const int bs = (int)blocks_for(n, 256);
  int ul = 0;
  const int nz = qhgk_slices(n, nT, &ul);
  if (bs * nz > kQhgkMaxSlices) return fail(ctx, KALDO_EINVAL, "kaldo_kappa_qhgk: too many modes");
  double4 T03 = make_double4(ctx->T[0], ctx->T[1], ctx->T[2], ctx->T[3]);
  double4 T47 = make_double4(ctx->T[4], ctx->T[5], ctx->T[6], ctx->T[7]);
  prof_begin(ctx);
  hipLaunchKernelGGL(k_qhgk_pairs, dim3(bs, nT, nz), dim3(256), 0, st, part, M, ctx->d_omega.as<double>(),
                     ctx->d_gamma.as<double>(), n, ul, T03, T47, ctx->stats == KALDO_CLASSICAL ? 1 : 0,
                     ctx->qhgk_bandwidth, ctx->qhgk_threshold);
  KALDO_HIP(ctx, hipGetLastError());
  prof_end(ctx, "kappa_qhgk");
  KALDO_HIP(ctx, ctx->d_kappa.ensure((size_t)nT * 9 * sizeof(double)));
  hipLaunchKernelGGL(k_reduce_slices, dim3(1), dim3(256), 0, st, ctx->d_kappa.as<double>(), part, bs * nz, nT,
                     kKappaSI / cell_volume(ctx->cell));
  KALDO_HIP(ctx, hipGetLastError());
  return KALDO_OK;
}

kaldo_status run_mode_diffusivity(kaldo_ctx ctx) {
  const int n = ctx->nm, nT = ctx->nT;
  hipStream_t st = ctx->stream;
  double *M = nullptr, *part = nullptr;
  const kaldo_status vs = qhgk_velocity(ctx, &M, &part);
  if (vs != KALDO_OK) return vs;
  const int bs = (int)blocks_for(n, 256);
  int ul = 0;
  const int nz = qhgk_slices(n, nT, &ul);
  const long long count = (long long)nT * n * 3;
  KALDO_HIP(ctx, ctx->d_diff.ensure((size_t)(nz + 1) * count * sizeof(double)));
  double* D = ctx->d_diff.as<double>();
  prof_begin(ctx);
  hipLaunchKernelGGL(k_qhgk_diffusivity, dim3(bs, nT, nz), dim3(256), 0, st, D + count, M, ctx->d_omega.as<double>(),
                     ctx->d_gamma.as<double>(), n, nT, ul, ctx->qhgk_bandwidth, ctx->qhgk_threshold);
  KALDO_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL(k_diffusivity_reduce, dim3(blocks_for(count, 256)), dim3(256), 0, st, D, D + count,
                     ctx->d_setid.as<int>(), n, nz, count);
  KALDO_HIP(ctx, hipGetLastError());
  prof_end(ctx, "diffusivity");
  return KALDO_OK;
}

}  // namespace kaldo
