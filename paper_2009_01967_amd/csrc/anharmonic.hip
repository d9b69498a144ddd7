// Three-phonon projection and scattering-rate sum (paper Sec. II.B) for
// crystals with few branches.
//
// With k'' = k + p on the grid, the phases of eq. projection_plus factor as
//   exp(-2 pi i p.R1) exp(2 pi i (k+p).R2) = exp(2 pi i k.R2) exp(2 pi i p.Delta),
// Delta = R2 - R1, so the work splits into
//   step A  A_k[s][Delta][a'][a''] = sum_{blocks with Delta} sum_a eta_ks[a] phi[a,a',a''] / sqrt(m m' m'') e^{2 pi i k.R2}
//   step B  Phi_ks(p)[a'][a''] = sum_Delta e^{2 pi i p.Delta} A_k[s][Delta][a'][a'']
//   step C  V[s][s'][s''] = sum_{a' a''} eta_p[a'][s'] conj(eta_{k+p}[a''][s'']) Phi_ks(p)[a'][a'']
// V is phi+ of (k,s),(p,s'),(k+p,s'').  Because D(-p) = conj(D(p)), the span of
// conj(eta_{-p}) inside each degenerate set equals that of eta_p, so the same V
// also gives phi- of (k,s),(-p,s'),(k+p,s'') after the sums over s', s'':
// one V feeds both the annihilation (+) and creation (-) weights.
//
// Epilogue (fused, V never leaves registers):
//   w = (n' - n'') G(w + w' - w'') + 1/2 (1 + n' + n'') G(w - w' - w''),
//   gamma_ks += |V|^2 w / (w w' w'') for every temperature,
// with G the unnormalised Gaussian; the constant hbar pi / 8, the Gaussian
// normalisation, 1 / N_k and 1 / w are applied by the finalising kernel.
#include <algorithm>

#include "common.h"
#include "internal.h"
#include "mfma.h"

namespace kaldo {

struct ProjArgs {
  int G0, G1, G2;
  int nk, nd, nT;
  int k0;
  int ppt;       // p points per thread
  int k_local;   // XCD-aware order: the p tiles of one k on one XCD
  double rc;     // 1 / (scale of the delta): frequencies are scaled by it
  int kind;      // kaldo_delta (selects the kernel instance)
  int npair;     // leading slot pairs (2m, 2m + 1) of A_k in sum/difference form
  const int* klist;  // first-mode point of block row kl: klist[k0 + kl] (null: k0 + kl)
  const double* UT;  // adaptive widths: scaled velocity projections [n][3][nk] (kDeltaGaussAdaptive)
};

// ---- adaptive widths -------------------------------------------------------------
// UT[s][a][k] = (c / sigma_min) vbar_ks . b_a / G_a with c = scale / sqrt(12):
// the degenerate-set mean velocity of mode (k, s) (a single mode's velocity
// depends on the basis inside its set, the mean does not) projected on the
// reciprocal vectors over the grid divisions (Bg[a][x] = b_a[x] / G_a).  The
// Gaussian of a process with partner modes 1 and 2 then has standard
// deviation sigma_min rho, rho = max(1, |UT_1 -+ UT_2|) (minus for
// absorption, plus for decay, where the partner at -p has velocity -v).
__global__ void k_adapt_table(double* __restrict__ UT, const double* __restrict__ vel, const int* __restrict__ setid,
                              int nk, int n, double3 B0, double3 B1, double3 B2, double scale) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nk * n) return;
  const int k = (int)(idx / n), s = (int)(idx % n);
  const int* sid = setid + (size_t)k * n;
  const int first = sid[s];
  int last = first;
  while (last + 1 < n && sid[last + 1] == first) ++last;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int u = first; u <= last; ++u) {
    const double* v = vel + ((size_t)k * n + u) * 3;
    v0 += v[0];
    v1 += v[1];
    v2 += v[2];
  }
  const double m = scale / (last - first + 1);
  v0 *= m;
  v1 *= m;
  v2 *= m;
  UT[((size_t)s * 3 + 0) * nk + k] = v0 * B0.x + v1 * B0.y + v2 * B0.z;
  UT[((size_t)s * 3 + 1) * nk + k] = v0 * B1.x + v1 * B1.y + v2 * B1.z;
  UT[((size_t)s * 3 + 2) * nk + k] = v0 * B2.x + v1 * B2.y + v2 * B2.z;
}

kaldo_status adaptive_table(kaldo_ctx ctx, double sigma_omega, const double** UT) {
  const int nk = ctx->nk, n = ctx->nm;
  // reciprocal vectors b_a = 2 pi (cell^-1)^T rows, over the grid divisions
  const double* c = ctx->cell;
  const double det = c[0] * (c[4] * c[8] - c[5] * c[7]) - c[1] * (c[3] * c[8] - c[5] * c[6]) +
                     c[2] * (c[3] * c[7] - c[4] * c[6]);
  // inverse of the cell matrix (rows = lattice vectors): inv[x][a]
  double inv[9];
  inv[0] = (c[4] * c[8] - c[5] * c[7]) / det;
  inv[1] = (c[2] * c[7] - c[1] * c[8]) / det;
  inv[2] = (c[1] * c[5] - c[2] * c[4]) / det;
  inv[3] = (c[5] * c[6] - c[3] * c[8]) / det;
  inv[4] = (c[0] * c[8] - c[2] * c[6]) / det;
  inv[5] = (c[2] * c[3] - c[0] * c[5]) / det;
  inv[6] = (c[3] * c[7] - c[4] * c[6]) / det;
  inv[7] = (c[1] * c[6] - c[0] * c[7]) / det;
  inv[8] = (c[0] * c[4] - c[1] * c[3]) / det;
  // b_a[x] = 2 pi inv[x][a]
  double3 B[3];
  for (int a = 0; a < 3; ++a) {
    const double f = kTwoPi / ctx->grid[a];
    B[a] = make_double3(f * inv[0 * 3 + a], f * inv[1 * 3 + a], f * inv[2 * 3 + a]);
  }
  KALDO_HIP(ctx, ctx->d_adapt.ensure((size_t)nk * n * 3 * sizeof(double)));
  const double scale = ctx->adaptive_scale / sqrt(12.0) / sigma_omega;
  hipLaunchKernelGGL(k_adapt_table, dim3(blocks_for((long long)nk * n, 256)), dim3(256), 0, ctx->stream,
                     ctx->d_adapt.as<double>(), ctx->d_vel.as<double>(), ctx->d_setid.as<int>(), nk, n, B[0], B[1],
                     B[2], scale);
  KALDO_HIP(ctx, hipGetLastError());
  *UT = ctx->d_adapt.as<double>();
  return KALDO_OK;
}

// ---- zero fill (a kernel, so that it can sit in a captured graph) ----------------
__global__ void k_fill_zero(uint4* __restrict__ p16, unsigned char* __restrict__ tail, size_t n16, size_t ntail) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) p16[i] = make_uint4(0u, 0u, 0u, 0u);
  if (i < ntail) tail[i] = 0;
}

kaldo_status fill_zero(kaldo_ctx ctx, void* p, size_t bytes) {
  if (bytes == 0) return KALDO_OK;
  // device allocations are 256-byte aligned; sub-buffers passed here are 16-byte aligned
  const size_t n16 = bytes / 16, ntail = bytes % 16;
  const size_t work = std::max(n16, ntail);
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, ctx->stream,
                     static_cast<uint4*>(p), static_cast<unsigned char*>(p) + n16 * 16, n16, ntail);
  KALDO_HIP(ctx, hipGetLastError());
  return KALDO_OK;
}

// ---- mode tables ---------------------------------------------------------------
// OM[s][k], IW[s][k] (1/omega or 0 if masked), OCC[t][s][k]
__global__ void k_tables(double* __restrict__ OM, double* __restrict__ IW, double* __restrict__ OCC,
                         const double* __restrict__ omega, int nk, int n, int nT, double4 T03, double4 T47,
                         int classical) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nk * n) return;
  const int s = (int)(idx % n);
  const int k = (int)(idx / n);
  const double w = omega[idx];
  const bool on = w / kTwoPi >= kNuMinThz;
  const size_t o = (size_t)s * nk + k;
  OM[o] = w;
  IW[o] = on ? 1.0 / w : 0.0;
  const double Ts[8] = {T03.x, T03.y, T03.z, T03.w, T47.x, T47.y, T47.z, T47.w};
  for (int t = 0; t < nT; ++t) {
    double occ = 0.0;
    if (on) {
      if (classical) occ = kBoltzmann * Ts[t] / (kHbar * w);
      else if (Ts[t] > 0.0) occ = 1.0 / expm1(kHbar * w / (kBoltzmann * Ts[t]));
    }
    OCC[((size_t)t * n + s) * nk + k] = occ;
  }
}

// PH[d][p] = exp(2 pi i q_p . Delta_d)
template <typename R>
__global__ void k_delta_phase(cplx<R>* __restrict__ PH, const int* __restrict__ delta, int nd, int G0, int G1,
                              int G2) {
  const int nk = G0 * G1 * G2;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nk * nd) return;
  const int p = (int)(idx % nk);
  const int d = (int)(idx / nk);
  const int m0 = p / (G1 * G2), m1 = (p / G2) % G1, m2 = p % G2;
  const long long num = (long long)m0 * delta[3 * d] * (G1 * G2) + (long long)m1 * delta[3 * d + 1] * (G0 * G2) +
                        (long long)m2 * delta[3 * d + 2] * (G0 * G1);
  double c, s;
  unit_phase(num, (long long)nk, c, s);
  PH[idx] = {(R)c, (R)s};
}

// ET[s][a][k] = eta_ks[a]
template <typename R>
__global__ void k_evec_transpose(cplx<R>* __restrict__ ET, const cplx<double>* __restrict__ E, int nk, int n) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nk * n * n) return;
  const int k = (int)(idx % nk);
  const int a = (int)((idx / nk) % n);
  const int s = (int)(idx / ((long long)nk * n));
  const cplx<double> v = E[((size_t)k * n + s) * n + a];
  ET[idx] = {(R)v.re, (R)v.im};
}

// ---- step A ---------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) k_step_a(cplx<R>* __restrict__ A, const cplx<double>* __restrict__ E, const int2* __restrict__ group,
                         const int* __restrict__ bi, const int* __restrict__ bR2, const double* __restrict__ bval,
                         int N, int nd, int G0, int G1, int G2, const int* __restrict__ klist, int k0, int kcount) {
  // one thread per (k, s, Delta, j, l): all 9 (beta, gamma) elements of the
  // 3 x 3 block share the eigenvector loads and the phase of every fc3 block
  const int n = 3 * N;
  const long long per_k = (long long)n * nd * N * N;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= per_k * kcount) return;
  const int kl = (int)(idx / per_k);
  int r = (int)(idx - kl * per_k);
  const int l = r % N;
  r /= N;
  const int j = r % N;
  r /= N;
  const int d = r % nd;
  const int s = r / nd;
  const int k = klist ? klist[k0 + kl] : k0 + kl;
  const int m0 = k / (G1 * G2), m1 = (k / G2) % G1, m2 = k % G2;
  const long long Gt = (long long)G0 * G1 * G2;
  const int2 g = group[((size_t)d * N + j) * N + l];
  const cplx<double>* e = E + ((size_t)k * n + s) * n;
  double re[9], im[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) re[q] = im[q] = 0.0;
  for (int b = g.x; b < g.y; ++b) {
    const int i = bi[b];
    const cplx<double> e0 = e[3 * i], e1 = e[3 * i + 1], e2 = e[3 * i + 2];
    const long long num = (long long)m0 * bR2[3 * b] * (G1 * G2) + (long long)m1 * bR2[3 * b + 1] * (G0 * G2) +
                          (long long)m2 * bR2[3 * b + 2] * (G0 * G1);
    double c, sn;
    unit_phase(num, Gt, c, sn);  // exp(+2 pi i k.R2)
    const double* v = bval + 27 * (size_t)b;
#pragma unroll
    for (int q = 0; q < 9; ++q) {  // q = 3 beta + gamma
      const double f0 = v[q], f1 = v[9 + q], f2 = v[18 + q];
      const double sr = e0.re * f0 + e1.re * f1 + e2.re * f2;
      const double si = e0.im * f0 + e1.im * f1 + e2.im * f2;
      re[q] += sr * c - si * sn;
      im[q] += sr * sn + si * c;
    }
  }
  cplx<R>* out = A + (((size_t)kl * n + s) * nd + d) * n * n;
#pragma unroll
  for (int be = 0; be < 3; ++be)
#pragma unroll
    for (int ga = 0; ga < 3; ++ga)
      out[(size_t)(3 * j + be) * n + 3 * l + ga] = {(R)re[3 * be + ga], (R)im[3 * be + ga]};
}

// ---- step B in pairs ------------------------------------------------------------
// Slots 2m and 2m + 1 of A_k hold Delta and -Delta, whose phases are conjugate:
// with a = A_k[Delta], b = A_k[-Delta] and ph = e^{2 pi i p.Delta},
//   ph a + conj(ph) b = Re(ph) (a + b) + Im(ph) i (a - b).
// Rewriting the slots as a + b and i (a - b) lets step B spend two real
// multiplies per element of the pair instead of two complex ones.
template <typename R>
__global__ void k_pair_delta(cplx<R>* __restrict__ A, int n, int nd, int npair, long long count) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;  // count = kc * n * npair * n * n
  const long long nn = (long long)n * n;
  const long long e = idx % nn;
  const long long r = idx / nn;
  const long long m = r % npair, ks = r / npair;  // ks = kl * n + s
  cplx<R>* a = A + ((size_t)ks * nd + 2 * m) * nn + e;
  cplx<R>* b = a + nn;
  const cplx<R> x = *a, y = *b;
  *a = {x.re + y.re, x.im + y.im};
  *b = {y.im - x.im, x.re - y.re};
}

// ---- fused step B + step C + epilogue ----------------------------------------------
// Opaque zero: keeps loads inside a loop (bounds register pressure).
__device__ __forceinline__ int opaque_zero() {
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return z;
}

// LDS_A: the block's A_k (all s and Delta) is staged in LDS once and read as
// wave-wide broadcasts; otherwise it is read from global memory through the
// scalar cache (cells whose A_k does not fit).
template <typename R, int NM, int NT, bool LDS_A, int DK>
__global__ void __launch_bounds__(256)
    k_project_small(const cplx<R>* __restrict__ A, const cplx<R>* __restrict__ PH, const cplx<R>* __restrict__ ET,
                    const double* __restrict__ OM, const double* __restrict__ IW, const double* __restrict__ OCC,
                    ProjArgs P, double* __restrict__ partial) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  // XCD-aware order.  Workgroups are dealt round-robin to the 8 XCDs, so in
  // launch order each XCD sees a fixed subset of p tiles for every k: its L2
  // holds 1/8 of the p-side tables but every XCD fetches every A_k.  When the
  // p-side tables fit one L2 (P.k_local), the flat id is remapped instead so
  // that the p tiles of one k run on one XCD and A_k is fetched once.
  int pchunk = (int)blockIdx.x, kl = (int)blockIdx.y;
  if (P.k_local) {
    const int nb = (int)(gridDim.x * gridDim.y), b = (int)(blockIdx.x + gridDim.x * blockIdx.y);
    const int q8 = nb >> 3, r8 = nb & 7, x8 = b & 7;
    const int tile = x8 * q8 + (x8 < r8 ? x8 : r8) + (b >> 3);
    pchunk = tile % (int)gridDim.x;
    kl = tile / (int)gridDim.x;
  }
  const int k = P.klist ? P.klist[P.k0 + kl] : P.k0 + kl;
  const int nk = P.nk;
  const int km0 = k / (P.G1 * P.G2), km1 = (k / P.G2) % P.G1, km2 = k % P.G2;
  // per-wave partial sums [wave][s][t]
  __shared__ double red[4][NM * NT];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < 4 * NM * NT) (&red[0][0])[threadIdx.x] = 0.0;
  const size_t a_per_k = (size_t)NM * P.nd * NM * NM;  // complex elements of A_k
  const cplx<R>* Ablk = A + (size_t)kl * a_per_k;
  if constexpr (LDS_A) {
    cplx<R>* As = reinterpret_cast<cplx<R>*>(smem);
    for (size_t i = threadIdx.x; i < a_per_k; i += blockDim.x) As[i] = Ablk[i];
    Ablk = As;
  }
  __syncthreads();

  for (int it = 0; it < P.ppt; ++it) {
    const int p = (pchunk * P.ppt + it) * blockDim.x + threadIdx.x;
    if (p < nk) {
      const int pm0 = p / (P.G1 * P.G2), pm1 = (p / P.G2) % P.G1, pm2 = p % P.G2;
      int q0 = km0 + pm0, q1 = km1 + pm1, q2 = km2 + pm2;
      q0 -= q0 >= P.G0 ? P.G0 : 0;
      q1 -= q1 >= P.G1 ? P.G1 : 0;
      q2 -= q2 >= P.G2 ? P.G2 : 0;
      const int kk = (q0 * P.G1 + q1) * P.G2 + q2;
      // p-side mode data stays in registers for all first modes s
      cplx<R> Ep[NM][NM];
      double wp[NM];
      R np_[NT][NM], iwp[NM];
      constexpr bool ADAPT = DK == kDeltaGaussAdaptive;
      R up[ADAPT ? NM : 1][3];  // adaptive widths: scaled velocity projections of (p, s')
#pragma unroll
      for (int s1 = 0; s1 < NM; ++s1) {
#pragma unroll
        for (int a = 0; a < NM; ++a) Ep[a][s1] = ET[((size_t)s1 * NM + a) * nk + p];
        if constexpr (ADAPT) {
#pragma unroll
          for (int a = 0; a < 3; ++a) up[s1][a] = (R)P.UT[((size_t)s1 * 3 + a) * nk + p];
        }
        wp[s1] = OM[(size_t)s1 * nk + p] * P.rc;  // frequencies in units of the delta's scale
        iwp[s1] = (R)IW[(size_t)s1 * nk + p];
#pragma unroll
        for (int t = 0; t < NT; ++t) np_[t][s1] = t < P.nT ? (R)OCC[((size_t)t * NM + s1) * nk + p] : (R)0;
      }
#pragma unroll 1
      for (int s = 0; s < NM; ++s) {
        const double iws = IW[(size_t)s * nk + k];
        if (iws == 0.0) continue;  // masked first mode: uniform across the block
        const double ws = OM[(size_t)s * nk + k] * P.rc;
        R acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = (R)0;
        // step B: Phi = sum_Delta e^{2 pi i p.Delta} A_k[s][Delta]
        cplx<R> F[NM][NM];
#pragma unroll
        for (int a = 0; a < NM; ++a)
#pragma unroll
          for (int b = 0; b < NM; ++b) F[a][b] = {(R)0, (R)0};
        const cplx<R>* As = Ablk + (size_t)s * P.nd * NM * NM;
        // the phase of the next Delta is in flight while this one is applied
        cplx<R> ph = PH[p];
        int d = 0;
        // pairs: slots a + b, i (a - b) (FP32 only; FP64 keeps every slot
        // as written by step A)
        if constexpr (sizeof(R) == 4) {
          for (; d < 2 * P.npair; d += 2) {
            const cplx<R> cur = ph;
            if (d + 2 < P.nd) ph = PH[(size_t)(d + 2) * nk + p];
            const cplx<R>* Sd = As + (size_t)d * NM * NM;
            const cplx<R>* Dd = Sd + NM * NM;
#pragma unroll
            for (int a = 0; a < NM; ++a)
#pragma unroll
              for (int b = 0; b < NM; ++b) {
                const cplx<R> sv = Sd[a * NM + b], dv = Dd[a * NM + b];
                F[a][b].re += cur.re * sv.re + cur.im * dv.re;
                F[a][b].im += cur.re * sv.im + cur.im * dv.im;
              }
          }
        }
        for (; d < P.nd; ++d) {
          const cplx<R> cur = ph;
          if (d + 1 < P.nd) ph = PH[(size_t)(d + 1) * nk + p];
          const cplx<R>* Ad = As + (size_t)d * NM * NM;
#pragma unroll
          for (int a = 0; a < NM; ++a)
#pragma unroll
            for (int b = 0; b < NM; ++b) cfma(F[a][b], cur, Ad[a * NM + b]);
        }
        // step C + epilogue, one column s'' at a time; k''-side data is
        // re-read per column instead of being held for all s.
        const int z = opaque_zero();
#pragma unroll 1
        for (int s2 = 0; s2 < NM; ++s2) {
          const size_t col = (size_t)s2 * NM * nk + kk + z;
          const double d2 = ws - OM[(size_t)s2 * nk + kk + z] * P.rc;  // (w - w'') / scale
          if constexpr ((DK == KALDO_DELTA_GAUSS || DK == KALDO_DELTA_TRIANGLE) && std::is_same<R, float>::value) {
            // a column whose every element, over the wave's partners and all
            // s', lies beyond the delta's cut adds nothing: skip its step C
            // (FP32 only: FP64 keeps more of the tail and runs one wave per
            // SIMD, where the test costs more than it saves)
            constexpr double cut = delta_cut<KALDO_FP32>(DK);
            bool need = false;
#pragma unroll
            for (int s1 = 0; s1 < NM; ++s1) {
              const double xp = d2 + wp[s1], xm = d2 - wp[s1];
              need = need || fmin(xp * xp, xm * xm) < cut;
            }
            if (__ballot(need) == 0) continue;
          }
          cplx<R> Tc[NM];
#pragma unroll
          for (int a = 0; a < NM; ++a) {
            Tc[a] = {(R)0, (R)0};
#pragma unroll
            for (int b = 0; b < NM; ++b) cfma_conj(Tc[a], F[a][b], ET[col + (size_t)b * nk]);
          }
          const R iw2 = (R)IW[(size_t)s2 * nk + kk + z];
          R uq[3];  // adaptive widths: (k + p, s'')
          if constexpr (ADAPT) {
#pragma unroll
            for (int a = 0; a < 3; ++a) uq[a] = (R)P.UT[((size_t)s2 * 3 + a) * nk + kk + z];
          }
          R n2[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) n2[t] = t < P.nT ? (R)OCC[((size_t)t * NM + s2) * nk + kk + z] : (R)0;
#pragma unroll
          for (int s1 = 0; s1 < NM; ++s1) {
            cplx<R> V = {(R)0, (R)0};
#pragma unroll
            for (int a = 0; a < NM; ++a) cfma(V, Ep[a][s1], Tc[a]);
            const R v2 = (V.re * V.re + V.im * V.im) * (iwp[s1] * iw2);
            R gp, gm;
            if constexpr (ADAPT) {
              // widths sigma_min rho: rho = max(1, |u' - u''|) (absorption), max(1, |u' + u''|) (decay)
              R dp = 0, dm = 0;
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                const R x = up[s1][a] - uq[a], y = up[s1][a] + uq[a];
                dp += x * x;
                dm += y * y;
              }
              const R ip = (R)1 / sqrt(dp > (R)1 ? dp : (R)1), im = (R)1 / sqrt(dm > (R)1 ? dm : (R)1);
              gp = delta_shape<R, KALDO_DELTA_GAUSS>((d2 + wp[s1]) * (double)ip) * (ip * v2);
              gm = (R)0.5 * delta_shape<R, KALDO_DELTA_GAUSS>((d2 - wp[s1]) * (double)im) * (im * v2);
            } else {
              gp = delta_shape<R, DK>(d2 + wp[s1]) * v2;
              gm = (R)0.5 * delta_shape<R, DK>(d2 - wp[s1]) * v2;
            }
            // gp (n' - n'') + gm (1 + n' + n'') = gm + n' (gp + gm) + n'' (gm - gp)
            const R sp = gp + gm, sm = gm - gp;
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] += gm + np_[t][s1] * sp + n2[t] * sm;
          }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          double v = (double)acc[t];
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
          if (lane == 0) red[wave][s * NT + t] += v;
        }
      }
    }
  }
  // block reduction -> partial[kl][pchunk][t][s]
  __syncthreads();
  if (threadIdx.x < NM * NT) {
    const int s = threadIdx.x / NT, t = threadIdx.x % NT;
    const double v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
    if (t < P.nT) partial[(((size_t)kl * gridDim.x + pchunk) * P.nT + t) * NM + s] = v;
  }
}

// gamma[t][k][s] = C / w_ks * sum_chunks partial, then the mean over each
// degenerate set, stored at k and at -k (time reversal) where these lie in the
// k range [klo, khi).
__global__ void k_finalize(double* __restrict__ gamma, const double* __restrict__ partial, const double* __restrict__ IW,
                           const int* __restrict__ setid, int nk, int n, int nT, int nchunk, const int* __restrict__ klist,
                           int k0, int kcount, double C, int klo, int khi, int G0, int G1, int G2) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)kcount * nT) return;
  const int kl = (int)(idx % kcount);
  const int t = (int)(idx / kcount);
  const int k = klist[k0 + kl];
  const int km = k_mirror(k, G0, G1, G2);
  const bool in_k = k >= klo && k < khi, in_km = km >= klo && km < khi;
  double g[64];
  for (int s = 0; s < n; ++s) {
    double v = 0.0;
    for (int c = 0; c < nchunk; ++c) v += partial[(((size_t)kl * nchunk + c) * nT + t) * n + s];
    g[s] = C * IW[(size_t)s * nk + k] * v;
  }
  const int* sid = setid + (size_t)k * n;
  for (int s = 0; s < n;) {
    int e = s + 1;
    while (e < n && sid[e] == sid[s]) ++e;
    double m = 0.0;
    for (int u = s; u < e; ++u) m += g[u];
    m /= (e - s);
    for (int u = s; u < e; ++u) {
      if (in_k) gamma[((size_t)t * nk + k) * n + u] = m;
      if (in_km) gamma[((size_t)t * nk + km) * n + u] = m;
    }
    s = e;
  }
}

template <typename R, int NM, bool LDS_A, int DK>
static void launch_project_t(dim3 grid, size_t lds, hipStream_t st, const cplx<R>* A, const cplx<R>* PH,
                             const cplx<R>* ET, const double* OM, const double* IW, const double* OCC,
                             const ProjArgs& P, double* partial) {
#define KALDO_LAUNCH(NTV)                                                                                    \
  {                                                                                                           \
    if (lds > 64 * 1024)                                                                                      \
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_project_small<R, NM, NTV, LDS_A, DK>),          \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                        \
    hipLaunchKernelGGL((k_project_small<R, NM, NTV, LDS_A, DK>), grid, dim3(256), lds, st, A, PH, ET, OM, IW, OCC, \
                       P, partial);                                                                           \
  }
  if (P.nT <= 1) KALDO_LAUNCH(1)
  else if (P.nT <= 2) KALDO_LAUNCH(2)
  else if (P.nT <= 3) KALDO_LAUNCH(3)
  else if (P.nT <= 4) KALDO_LAUNCH(4)
  else KALDO_LAUNCH(8)
#undef KALDO_LAUNCH
}

// A_k goes to LDS when it fits: beside a second resident block for FP32 (two
// waves per SIMD), alone for FP64 (whose registers allow one)
template <typename R, int NM>
static void launch_project(dim3 grid, hipStream_t st, const cplx<R>* A, const cplx<R>* PH, const cplx<R>* ET,
                           const double* OM, const double* IW, const double* OCC, const ProjArgs& P,
                           double* partial) {
  const size_t lds = (size_t)NM * P.nd * NM * NM * sizeof(cplx<R>);
  const bool in_lds = lds <= (sizeof(R) == 4 ? 76 : 150) * 1024;
#define KALDO_KIND(DKV)                                                                  \
  {                                                                                      \
    if (in_lds)                                                                          \
      launch_project_t<R, NM, true, DKV>(grid, lds, st, A, PH, ET, OM, IW, OCC, P, partial); \
    else                                                                                 \
      launch_project_t<R, NM, false, DKV>(grid, 0, st, A, PH, ET, OM, IW, OCC, P, partial);  \
  }
  if (P.kind == KALDO_DELTA_GAUSS) KALDO_KIND(KALDO_DELTA_GAUSS)
  else if (P.kind == KALDO_DELTA_LORENTZ) KALDO_KIND(KALDO_DELTA_LORENTZ)
  else if (P.kind == kDeltaGaussAdaptive) KALDO_KIND(kDeltaGaussAdaptive)
  else KALDO_KIND(KALDO_DELTA_TRIANGLE)
#undef KALDO_KIND
}

template <typename R>
static kaldo_status linewidths_small(kaldo_ctx ctx, double sigma_thz) {
  const int N = ctx->n_atoms, n = ctx->nm, nk = ctx->nk, nT = ctx->nT;
  const int nd = ctx->fc3.n_delta;
  hipStream_t st = ctx->stream;
  const int TB = 256;
  // tables: OM, IW [n][nk], OCC [nT][n][nk], PH [nd][nk], ET [n][n][nk]
  const size_t nmode = (size_t)nk * n;
  const size_t tab_bytes = (2 + (size_t)nT) * nmode * sizeof(double);
  const size_t ph_bytes = (size_t)nd * nk * sizeof(cplx<R>);
  const size_t et_bytes = (size_t)n * n * nk * sizeof(cplx<R>);
  KALDO_HIP(ctx, ctx->d_tabs.ensure(tab_bytes + ph_bytes + et_bytes + 256));
  double* OM = ctx->d_tabs.as<double>();
  double* IW = OM + nmode;
  double* OCC = IW + nmode;
  cplx<R>* PH = reinterpret_cast<cplx<R>*>(OCC + (size_t)nT * nmode);
  cplx<R>* ET = PH + (size_t)nd * nk;
  double4 T03 = make_double4(ctx->T[0], ctx->T[1], ctx->T[2], ctx->T[3]);
  double4 T47 = make_double4(ctx->T[4], ctx->T[5], ctx->T[6], ctx->T[7]);
  hipLaunchKernelGGL(k_tables, dim3(blocks_for((long long)nmode, TB)), dim3(TB), 0, st, OM, IW, OCC,
                     ctx->d_omega.as<double>(), nk, n, nT, T03, T47, ctx->stats == KALDO_CLASSICAL ? 1 : 0);
  KALDO_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL((k_delta_phase<R>), dim3(blocks_for((long long)nd * nk, TB)), dim3(TB), 0, st, PH,
                     ctx->fc3.d_delta.as<int>(), nd, ctx->grid[0], ctx->grid[1], ctx->grid[2]);
  KALDO_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL((k_evec_transpose<R>), dim3(blocks_for((long long)n * n * nk, TB)), dim3(TB), 0, st, ET,
                     ctx->d_evec.as<cplx<double>>(), nk, n);
  KALDO_HIP(ctx, hipGetLastError());

  // k chunks bounded by the size of the step-A intermediate
  const size_t a_per_k = (size_t)n * nd * n * n * sizeof(cplx<R>);
  const size_t a_budget = (size_t)1 << 30;
  int kchunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)nk, a_budget / a_per_k));
  const int ppt = 1;
  const int nchunk = (int)blocks_for(nk, TB * ppt);
  kchunk = std::min(kchunk, 65535);
  KALDO_HIP(ctx, ctx->d_A.ensure(a_per_k * kchunk));
  KALDO_HIP(ctx, ctx->d_partial.ensure((size_t)kchunk * nchunk * nT * n * sizeof(double)));
  KALDO_HIP(ctx, ctx->d_gamma.ensure((size_t)nT * nmode * sizeof(double)));
  const double sig = kTwoPi * sigma_thz;
  ProjArgs P;
  P.G0 = ctx->grid[0];
  P.G1 = ctx->grid[1];
  P.G2 = ctx->grid[2];
  P.nk = nk;
  P.nd = nd;
  P.nT = nT;
  P.ppt = ppt;
  // p-side tables read by every block: eigenvectors, phases, mode tables
  const size_t p_side = et_bytes + ph_bytes + tab_bytes;
  P.k_local = p_side <= ((size_t)7 << 19) ? 1 : 0;  // 3.5 MB of a 4 MB L2
  double dscale, dnorm;
  delta_scale(ctx->delta, sig, dscale, dnorm);
  P.rc = 1.0 / dscale;
  P.kind = ctx->delta;
  P.UT = nullptr;
  if (ctx->adaptive_scale > 0.0) {
    // Gaussian widths per process, sig the smallest (the scale and norm above are sig's)
    P.kind = kDeltaGaussAdaptive;
    const kaldo_status as = adaptive_table(ctx, sig, &P.UT);
    if (as != KALDO_OK) return as;
  }
  // FP64 runs step B over single slots: at one wave per SIMD the paired
  // loop was slower there
  P.npair = sizeof(R) == 4 ? ctx->fc3.n_dpair : 0;
  const double C = kPi / 8.0 * kHbar * kEvUnit * kEvUnit * kEvUnit / nk * dnorm;
  cplx<R>* A = ctx->d_A.as<cplx<R>>();
  double* partial = ctx->d_partial.as<double>();
  // the first-mode points to compute (one of each pair k, -k on the whole grid)
  int npts = 0;
  kaldo_status ks = upload_linewidth_points(ctx, &npts);
  if (ks != KALDO_OK) return ks;
  P.klist = ctx->d_klist.as<int>();
  if (k_partial(ctx) && !planning(ctx)) {
    const kaldo_status fs = fill_zero(ctx, ctx->d_gamma.p, (size_t)nT * nmode * sizeof(double));
    if (fs != KALDO_OK) return fs;
  }
  for (int k0 = 0; k0 < npts && !planning(ctx); k0 += kchunk) {
    const int kc = std::min(kchunk, npts - k0);
    P.k0 = k0;
    prof_begin(ctx);
    hipLaunchKernelGGL((k_step_a<R>), dim3(blocks_for((long long)n * nd * N * N * kc, TB)), dim3(TB), 0,
                       st, A, ctx->d_evec.as<cplx<double>>(), ctx->fc3.d_group.as<int2>(), ctx->fc3.d_blk_i.as<int>(),
                       ctx->fc3.d_blk_R2.as<int>(), ctx->fc3.d_blk_val.as<double>(), N, nd, P.G0, P.G1, P.G2, P.klist,
                       k0, kc);
    KALDO_HIP(ctx, hipGetLastError());
    if (P.npair > 0) {
      const long long cnt = (long long)kc * n * P.npair * n * n;
      hipLaunchKernelGGL((k_pair_delta<R>), dim3(blocks_for(cnt, TB)), dim3(TB), 0, st, A, n, nd, P.npair, cnt);
      KALDO_HIP(ctx, hipGetLastError());
    }
    prof_end(ctx, "step_a");
    dim3 grid(nchunk, kc);
    prof_begin(ctx);
    if (n == 6)
      launch_project<R, 6>(grid, st, A, PH, ET, OM, IW, OCC, P, partial);
    else
      launch_project<R, 3>(grid, st, A, PH, ET, OM, IW, OCC, P, partial);
    KALDO_HIP(ctx, hipGetLastError());
    prof_end(ctx, "project");
    prof_begin(ctx);
    hipLaunchKernelGGL(k_finalize, dim3(blocks_for((long long)kc * nT, TB)), dim3(TB), 0, st,
                       ctx->d_gamma.as<double>(), partial, IW, ctx->d_setid.as<int>(), nk, n, nT, nchunk, P.klist, k0,
                       kc, C, k_lo(ctx), k_hi(ctx), P.G0, P.G1, P.G2);
    KALDO_HIP(ctx, hipGetLastError());
    prof_end(ctx, "finalize");
  }
  return KALDO_OK;
}

// FP64 tables of the few-branch path (the same layout as linewidths_small),
// for the scattering operator of the full BTE.
kaldo_status small_tables_fp64(kaldo_ctx ctx, SmallTables* t) {
  const int n = ctx->nm, nk = ctx->nk, nT = ctx->nT, nd = ctx->fc3.n_delta;
  hipStream_t st = ctx->stream;
  const int TB = 256;
  const size_t nmode = (size_t)nk * n;
  const size_t tab_bytes = (2 + (size_t)nT) * nmode * sizeof(double);
  const size_t ph_bytes = (size_t)nd * nk * sizeof(cplx<double>);
  const size_t et_bytes = (size_t)n * n * nk * sizeof(cplx<double>);
  KALDO_HIP(ctx, ctx->d_tabs.ensure(tab_bytes + ph_bytes + et_bytes + 256));
  t->OM = ctx->d_tabs.as<double>();
  t->IW = t->OM + nmode;
  t->OCC = t->IW + nmode;
  t->PH = reinterpret_cast<cplx<double>*>(t->OCC + (size_t)nT * nmode);
  t->ET = t->PH + (size_t)nd * nk;
  double4 T03 = make_double4(ctx->T[0], ctx->T[1], ctx->T[2], ctx->T[3]);
  double4 T47 = make_double4(ctx->T[4], ctx->T[5], ctx->T[6], ctx->T[7]);
  hipLaunchKernelGGL(k_tables, dim3(blocks_for((long long)nmode, TB)), dim3(TB), 0, st, t->OM, t->IW, t->OCC,
                     ctx->d_omega.as<double>(), nk, n, nT, T03, T47, ctx->stats == KALDO_CLASSICAL ? 1 : 0);
  KALDO_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL((k_delta_phase<double>), dim3(blocks_for((long long)nd * nk, TB)), dim3(TB), 0, st, t->PH,
                     ctx->fc3.d_delta.as<int>(), nd, ctx->grid[0], ctx->grid[1], ctx->grid[2]);
  KALDO_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL((k_evec_transpose<double>), dim3(blocks_for((long long)n * n * nk, TB)), dim3(TB), 0, st,
                     t->ET, ctx->d_evec.as<cplx<double>>(), nk, n);
  KALDO_HIP(ctx, hipGetLastError());
  return KALDO_OK;
}

// Step A (FP64, single Delta slots) of first-mode points [k0, k0 + kc) into A.
kaldo_status small_step_a_fp64(kaldo_ctx ctx, cplx<double>* A, int k0, int kc) {
  const int N = ctx->n_atoms, n = ctx->nm, nd = ctx->fc3.n_delta;
  hipLaunchKernelGGL((k_step_a<double>), dim3(blocks_for((long long)n * nd * N * N * kc, 256)), dim3(256), 0,
                     ctx->stream, A, ctx->d_evec.as<cplx<double>>(), ctx->fc3.d_group.as<int2>(),
                     ctx->fc3.d_blk_i.as<int>(), ctx->fc3.d_blk_R2.as<int>(), ctx->fc3.d_blk_val.as<double>(), N, nd,
                     ctx->grid[0], ctx->grid[1], ctx->grid[2], nullptr, k0, kc);
  KALDO_HIP(ctx, hipGetLastError());
  return KALDO_OK;
}

// Mode tables and the Delta phase table (FP64) for the many-branch crystal path.
kaldo_status run_crystal_tables(kaldo_ctx ctx, double** OM, double** IW, double** OCC, cplx<double>** PH) {
  const int n = ctx->nm, nk = ctx->nk, nT = ctx->nT, nd = ctx->fc3.n_delta;
  hipStream_t st = ctx->stream;
  const int TB = 256;
  const size_t nmode = (size_t)nk * n;
  KALDO_HIP(ctx, ctx->d_tabs.ensure((2 + (size_t)nT) * nmode * sizeof(double) +
                                    (size_t)nd * nk * sizeof(cplx<double>)));
  *OM = ctx->d_tabs.as<double>();
  *IW = *OM + nmode;
  *OCC = *IW + nmode;
  *PH = reinterpret_cast<cplx<double>*>(*OCC + (size_t)nT * nmode);
  double4 T03 = make_double4(ctx->T[0], ctx->T[1], ctx->T[2], ctx->T[3]);
  double4 T47 = make_double4(ctx->T[4], ctx->T[5], ctx->T[6], ctx->T[7]);
  hipLaunchKernelGGL(k_tables, dim3(blocks_for((long long)nmode, TB)), dim3(TB), 0, st, *OM, *IW, *OCC,
                     ctx->d_omega.as<double>(), nk, n, nT, T03, T47, ctx->stats == KALDO_CLASSICAL ? 1 : 0);
  KALDO_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL((k_delta_phase<double>), dim3(blocks_for((long long)nd * nk, TB)), dim3(TB), 0, st, *PH,
                     ctx->fc3.d_delta.as<int>(), nd, ctx->grid[0], ctx->grid[1], ctx->grid[2]);
  KALDO_HIP(ctx, hipGetLastError());
  return KALDO_OK;
}

kaldo_status run_linewidths(kaldo_ctx ctx, double sigma_thz, int precision) {
  const int n = ctx->nm;
  if (ctx->nk == 1) return run_linewidths_gamma(ctx, sigma_thz, precision);
  if (n > 6 || precision == KALDO_BF16X3) return run_linewidths_crystal(ctx, sigma_thz, precision);
  if (n == 3 || n == 6) {
    if (precision == KALDO_FP64) return linewidths_small<double>(ctx, sigma_thz);
    if (precision == KALDO_FP32) return linewidths_small<float>(ctx, sigma_thz);
    return fail(ctx, KALDO_EINVAL, "unknown projection precision");
  }
  return fail(ctx, KALDO_EINVAL, "no linewidth kernel for " + std::to_string(n) + " modes per grid point");
}

}  // namespace kaldo
