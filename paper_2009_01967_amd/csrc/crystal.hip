// Three-phonon projection and scattering-rate sum (paper Sec. II.B,
// eq. projection_plus .. delta_deconstructed) for crystals with many branches,
// as two chained complex GEMMs on MFMA per (first mode (k,s), partner p):
//
//   Z_k[s][g]    = sum_{blocks b in group g} e^{2 pi i k.R2_b} sum_a eta_ks[a] phi_b / sqrt(m m' m'')
//                  (group g = one (Delta, j, l), Delta = R2 - R1)
//   X_ks(p)      = sum_g e^{2 pi i p.Delta_g} Z_k[s][g] placed at the (j, l) block     (dense n x n)
//   Y^T[s''][a'] = sum_a'' conj(eta_{k+p}[a''][s'']) X[a'][a'']                       (GEMM 1)
//   V[s'][s'']   = sum_a' eta_p[a'][s'] Y^T[s''][a']                                   (GEMM 2)
//
// V is phi+ of (k,s),(p,s'),(k+p,s''); as in the few-branch path the same V
// also serves the creation process of (k,s),(-p,s'),(k+p,s'').  GEMM 2 carries
// the fused epilogue (|V|^2, occupations, Gaussian delta, every temperature,
// tile reduction), so V never reaches memory.  Complex products use four real
// MFMA products (no three-multiplication trick); BF16X3 splits each operand
// into bf16 hi + lo and keeps hi*hi + hi*lo + lo*hi with FP32 accumulation.
#include <algorithm>

#include "common.h"
#include "internal.h"
#include "mfma.h"

namespace kaldo {

constexpr int kCTile = 64;

// Z[s][g][e9] for one first-mode k
__global__ void k_cr_zg(cplx<double>* __restrict__ Z, const cplx<double>* __restrict__ E,
                        const int2* __restrict__ cgb, const int* __restrict__ bi, const int* __restrict__ bR2,
                        const double* __restrict__ bval, int n, int ng, int G0, int G1, int G2, int k) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * ng * 9) return;
  const int e9 = (int)(idx % 9);
  const int g = (int)((idx / 9) % ng);
  const int s = (int)(idx / (9LL * ng));
  const int m0 = k / (G1 * G2), m1 = (k / G2) % G1, m2 = k % G2;
  const long long Gt = (long long)G0 * G1 * G2;
  const cplx<double>* e = E + ((size_t)k * n + s) * n;
  const int2 r = cgb[g];
  double re = 0.0, im = 0.0;
  for (int b = r.x; b < r.y; ++b) {
    const int i3 = 3 * bi[b];
    const double* v = bval + 27 * (size_t)b + e9;
    const cplx<double> e0 = e[i3], e1 = e[i3 + 1], e2 = e[i3 + 2];
    const double sr = e0.re * v[0] + e1.re * v[9] + e2.re * v[18];
    const double si = e0.im * v[0] + e1.im * v[9] + e2.im * v[18];
    const long long num = (long long)m0 * bR2[3 * b] * (G1 * G2) + (long long)m1 * bR2[3 * b + 1] * (G0 * G2) +
                          (long long)m2 * bR2[3 * b + 2] * (G0 * G1);
    double c, sn;
    unit_phase(num, Gt, c, sn);  // e^{+2 pi i k.R2}
    re += sr * c - si * sn;
    im += sr * sn + si * c;
  }
  Z[idx] = {re, im};
}

// eigenvector planes for every k: [k][c][npad][npad] with row s, column a;
// c = 0: Re eta, 1: Im eta, 2: -Im eta (zero padded)
template <int P>
__global__ void k_cr_eplanes(typename Operand<P>::T* __restrict__ Ehi, typename Operand<P>::T* __restrict__ Elo,
                             const cplx<double>* __restrict__ E, int nk, int n, int npad) {
  const size_t nn = (size_t)npad * npad;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nk * nn) return;
  const int a = (int)(idx % npad);
  const int s = (int)((idx / npad) % npad);
  const int k = (int)(idx / nn);
  cplx<double> v = {0.0, 0.0};
  if (s < n && a < n) v = E[((size_t)k * n + s) * n + a];
  const size_t o = (size_t)k * 3 * nn + (size_t)s * npad + a;
  store_operand<P>(Ehi, Elo, o, v.re);
  store_operand<P>(Ehi, Elo, o + nn, v.im);
  store_operand<P>(Ehi, Elo, o + 2 * nn, -v.im);
}

// dense X planes for items it0 .. it0+count-1, item = p * n + s: [it][c][a'][a'']
template <int P>
__global__ void k_cr_xs(typename Operand<P>::T* __restrict__ Xhi, typename Operand<P>::T* __restrict__ Xlo,
                        const cplx<double>* __restrict__ Z, const cplx<double>* __restrict__ PH,
                        const int* __restrict__ cg_delta, const int* __restrict__ cg_order,
                        const int4* __restrict__ cpair, int n, int nk, int ng, int ncp, int npad, int it0,
                        int count) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)count * ncp * 9) return;
  const int e9 = (int)(idx % 9);
  const int cp = (int)((idx / 9) % ncp);
  const int it = (int)(idx / (9LL * ncp));
  const int item = it0 + it;
  const int p = item / n, s = item % n;
  const int4 pr = cpair[cp];
  double re = 0.0, im = 0.0;
  for (int q = pr.z; q < pr.w; ++q) {
    const int g = cg_order[q];
    const cplx<double> ph = PH[(size_t)cg_delta[g] * nk + p];
    const cplx<double> z = Z[((size_t)s * ng + g) * 9 + e9];
    re += ph.re * z.re - ph.im * z.im;
    im += ph.re * z.im + ph.im * z.re;
  }
  const size_t nn = (size_t)npad * npad;
  const size_t o = (size_t)it * 2 * nn + (size_t)(3 * pr.x + e9 / 3) * npad + 3 * pr.y + e9 % 3;
  store_operand<P>(Xhi, Xlo, o, re);
  store_operand<P>(Xhi, Xlo, o + nn, im);
}

struct CrArgs {
  int n, npad, nk, G0, G1, G2, k, it0, nT;
  double c;  // 1 / (2 sigma^2)
};

template <int P>
struct CrKc;
template <>
struct CrKc<KALDO_FP64> {
  static constexpr int v = 16;
};
template <>
struct CrKc<KALDO_FP32> {
  static constexpr int v = 16;
};
template <>
struct CrKc<KALDO_BF16X3> {
  static constexpr int v = 32;
};

// One complex 64x64 output tile of GEMM 1 (MODE 0, stores Y^T planes) or
// GEMM 2 (MODE 1, fused linewidth epilogue) for batch item blockIdx.y.
template <int P, int MODE, int NT>
__global__ void __launch_bounds__(256)
    k_cr_gemm(const typename Operand<P>::T* __restrict__ Ehi, const typename Operand<P>::T* __restrict__ Elo,
              const typename Operand<P>::T* __restrict__ Bhi, const typename Operand<P>::T* __restrict__ Blo,
              typename Operand<P>::T* __restrict__ Yhi, typename Operand<P>::T* __restrict__ Ylo,
              const double* __restrict__ OM, const double* __restrict__ IW, const double* __restrict__ OCC,
              CrArgs A, double* __restrict__ partial) {
  using T = typename Operand<P>::T;
  using Acc = typename Operand<P>::Acc;
  constexpr int S = Operand<P>::split;
  constexpr int KC = CrKc<P>::v;
  constexpr int LD = KC + (sizeof(T) == 8 ? 2 : (sizeof(T) == 4 ? 4 : 8));
  // A planes: 0 = Re, 1 = Im (of the operand), 2 = -Im; B planes: 0 = Re, 1 = Im
  __shared__ __attribute__((aligned(16))) T As[3 * S][kCTile * LD];
  __shared__ __attribute__((aligned(16))) T Bs[2 * S][kCTile * LD];
  __shared__ double red[4][NT];

  const int npad = A.npad, n = A.n, nk = A.nk;
  const size_t nn = (size_t)npad * npad;
  const int ntile = npad / kCTile;
  const int ti = blockIdx.x / ntile, tj = blockIdx.x % ntile;
  const int it = blockIdx.y;
  const int item = A.it0 + it;
  const int p = item / n, s = item % n;
  const int km0 = A.k / (A.G1 * A.G2), km1 = (A.k / A.G2) % A.G1, km2 = A.k % A.G2;
  const int pm0 = p / (A.G1 * A.G2), pm1 = (p / A.G2) % A.G1, pm2 = p % A.G2;
  const int kk = ((km0 + pm0) % A.G0 * A.G1 + (km1 + pm1) % A.G1) * A.G2 + (km2 + pm2) % A.G2;
  const int ka = MODE == 0 ? kk : p;
  // GEMM 1 multiplies by conj(eta_{k''}): its "Im" is plane 2 and its "-Im" plane 1
  const int pl[3] = {0, MODE == 0 ? 2 : 1, MODE == 0 ? 1 : 2};
  const T* Ab[3 * S];
  const T* Bb[2 * S];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    Ab[c] = Ehi + ((size_t)ka * 3 + pl[c]) * nn + (size_t)ti * kCTile * npad;
    if constexpr (S == 2) Ab[3 + c] = Elo + ((size_t)ka * 3 + pl[c]) * nn + (size_t)ti * kCTile * npad;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    Bb[c] = Bhi + ((size_t)it * 2 + c) * nn + (size_t)tj * kCTile * npad;
    if constexpr (S == 2) Bb[2 + c] = Blo + ((size_t)it * 2 + c) * nn + (size_t)tj * kCTile * npad;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  Acc accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) accR[a][b][r] = accI[a][b][r] = 0;

  constexpr int kPer = kCTile * KC / 256;
  for (int k0 = 0; k0 < npad; k0 += KC) {
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int q = threadIdx.x * kPer + e;
      const int row = q / KC, col = q % KC;
#pragma unroll
      for (int c = 0; c < 3 * S; ++c) As[c][row * LD + col] = Ab[c][(size_t)row * npad + k0 + col];
#pragma unroll
      for (int c = 0; c < 2 * S; ++c) Bs[c][row * LD + col] = Bb[c][(size_t)row * npad + k0 + col];
    }
    __syncthreads();
    if constexpr (P == KALDO_BF16X3) {
#pragma unroll
      for (int k8 = 0; k8 < KC; k8 += 32) {
        bf16x8 av[2][3][2], bv[2][2][2];  // [sub-tile][plane][hi/lo]
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int r = wi * 32 + a * 16 + (lane & 15);
          const int cc = wj * 32 + a * 16 + (lane & 15);
          const int kq = k8 + 8 * (lane >> 4);
#pragma unroll
          for (int e = 0; e < 8; ++e) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              av[a][c][0][e] = As[c][r * LD + kq + e];
              av[a][c][1][e] = As[3 + c][r * LD + kq + e];
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              bv[a][c][0][e] = Bs[c][cc * LD + kq + e];
              bv[a][c][1][e] = Bs[2 + c][cc * LD + kq + e];
            }
          }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            // R += Ar Br + (-Ai) Bi ; I += Ar Bi + Ai Br, each product as hi*hi + hi*lo + lo*hi
#define KALDO_X3(ACC, X, Y)                                                                \
  ACC = __builtin_amdgcn_mfma_f32_16x16x32_bf16(X[0], Y[0], ACC, 0, 0, 0);                \
  ACC = __builtin_amdgcn_mfma_f32_16x16x32_bf16(X[0], Y[1], ACC, 0, 0, 0);                \
  ACC = __builtin_amdgcn_mfma_f32_16x16x32_bf16(X[1], Y[0], ACC, 0, 0, 0);
            KALDO_X3(accR[a][b], av[a][0], bv[b][0])
            KALDO_X3(accR[a][b], av[a][2], bv[b][1])
            KALDO_X3(accI[a][b], av[a][0], bv[b][1])
            KALDO_X3(accI[a][b], av[a][1], bv[b][0])
#undef KALDO_X3
          }
      }
    } else {
#pragma unroll
      for (int k4 = 0; k4 < KC; k4 += 4) {
        T av[2][3], bv[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int r = wi * 32 + a * 16 + (lane & 15);
          const int cc = wj * 32 + a * 16 + (lane & 15);
          const int kq = k4 + (lane >> 4);
#pragma unroll
          for (int c = 0; c < 3; ++c) av[a][c] = As[c][r * LD + kq];
#pragma unroll
          for (int c = 0; c < 2; ++c) bv[a][c] = Bs[c][cc * LD + kq];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            if constexpr (P == KALDO_FP64) {
              accR[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][0], bv[b][0], accR[a][b], 0, 0, 0);
              accR[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][2], bv[b][1], accR[a][b], 0, 0, 0);
              accI[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][0], bv[b][1], accI[a][b], 0, 0, 0);
              accI[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][1], bv[b][0], accI[a][b], 0, 0, 0);
            } else {
              accR[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][0], bv[b][0], accR[a][b], 0, 0, 0);
              accR[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][2], bv[b][1], accR[a][b], 0, 0, 0);
              accI[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][0], bv[b][1], accI[a][b], 0, 0, 0);
              accI[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][1], bv[b][0], accI[a][b], 0, 0, 0);
            }
          }
      }
    }
    __syncthreads();
  }

  if constexpr (MODE == 0) {
    // store Y^T planes (row s'' = A row, column a' = B row)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = ti * kCTile + wi * 32 + a * 16 + acc_row<P>(lane, r);
          const int j = tj * kCTile + wj * 32 + b * 16 + (lane & 15);
          const size_t o = (size_t)it * 2 * nn + (size_t)i * npad + j;
          store_operand<P>(Yhi, Ylo, o, (double)accR[a][b][r]);
          store_operand<P>(Yhi, Ylo, o + nn, (double)accI[a][b][r]);
        }
  } else {
    double out[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) out[t] = 0.0;
    const double ws = OM[(size_t)s * nk + A.k];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = ti * kCTile + wi * 32 + a * 16 + acc_row<P>(lane, r);  // s' (mode of p)
          const int j = tj * kCTile + wj * 32 + b * 16 + (lane & 15);        // s'' (mode of k+p)
          if (i < n && j < n) {
            const double vr = (double)accR[a][b][r], vi = (double)accI[a][b][r];
            const double v2 = (vr * vr + vi * vi) * IW[(size_t)i * nk + p] * IW[(size_t)j * nk + kk];
            if (v2 != 0.0) {
              const double w1 = OM[(size_t)i * nk + p], w2 = OM[(size_t)j * nk + kk];
              const double xp = ws + w1 - w2, xm = ws - w1 - w2;
              double gp, gm;
              if constexpr (P == KALDO_FP64) {
                gp = exp(-xp * xp * A.c);
                gm = exp(-xm * xm * A.c);
              } else {
                gp = (double)__expf((float)(-xp * xp * A.c));
                gm = (double)__expf((float)(-xm * xm * A.c));
              }
#pragma unroll
              for (int t = 0; t < NT; ++t) {
                if (t < A.nT) {
                  const double n1 = OCC[((size_t)t * n + i) * nk + p];
                  const double n2 = OCC[((size_t)t * n + j) * nk + kk];
                  out[t] += v2 * (gp * (n1 - n2) + 0.5 * gm * (1.0 + n1 + n2));
                }
              }
            }
          }
        }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      double v = out[t];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) red[wave][t] = v;
    }
    __syncthreads();
    if (threadIdx.x < A.nT) {
      const int t = threadIdx.x;
      partial[((size_t)item * gridDim.x + blockIdx.x) * A.nT + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
    }
  }
}

// graw[t][k][s] = C / w_ks * sum over partners and tiles
__global__ void k_cr_collect(double* __restrict__ graw, const double* __restrict__ partial,
                             const double* __restrict__ IW, int n, int nk, int nT, int ntiles, int k, double C) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * nT) return;
  const int s = idx % n, t = idx / n;
  double v = 0.0;
  for (int p = 0; p < nk; ++p) {
    const size_t item = (size_t)p * n + s;
    for (int b = 0; b < ntiles; ++b) v += partial[(item * ntiles + b) * nT + t];
  }
  graw[((size_t)t * nk + k) * n + s] = C * IW[(size_t)s * nk + k] * v;
}

__global__ void k_cr_set_average(double* __restrict__ gamma, const double* __restrict__ graw,
                                 const int* __restrict__ setid, int n, int nk, int nT) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * nk * nT) return;
  const int s = (int)(idx % n);
  const int k = (int)((idx / n) % nk);
  const int t = (int)(idx / ((long long)n * nk));
  const int* sid = setid + (size_t)k * n;
  const int first = sid[s];
  int last = first;
  while (last + 1 < n && sid[last + 1] == first) ++last;
  double m = 0.0;
  const double* g = graw + ((size_t)t * nk + k) * n;
  for (int u = first; u <= last; ++u) m += g[u];
  gamma[idx] = m / (last - first + 1);
}

template <int P, int MODE>
static void launch_cr(int nT, dim3 grid, hipStream_t st, const void* Eh, const void* El, const void* Bh,
                      const void* Bl, void* Yh, void* Yl, const double* OM, const double* IW, const double* OCC,
                      const CrArgs& A, double* partial) {
  using T = typename Operand<P>::T;
#define KALDO_LAUNCH(NTV)                                                                                      \
  hipLaunchKernelGGL((k_cr_gemm<P, MODE, NTV>), grid, dim3(256), 0, st, (const T*)Eh, (const T*)El, (const T*)Bh, \
                     (const T*)Bl, (T*)Yh, (T*)Yl, OM, IW, OCC, A, partial)
  if (MODE == 0 || nT <= 1) KALDO_LAUNCH(1);
  else if (nT <= 2) KALDO_LAUNCH(2);
  else if (nT <= 4) KALDO_LAUNCH(4);
  else KALDO_LAUNCH(8);
#undef KALDO_LAUNCH
}

kaldo_status run_crystal_tables(kaldo_ctx ctx, double** OM, double** IW, double** OCC, cplx<double>** PH);

template <int P>
static kaldo_status crystal_impl(kaldo_ctx ctx, double sigma_thz) {
  using T = typename Operand<P>::T;
  constexpr int S = Operand<P>::split;
  const int n = ctx->nm, nk = ctx->nk, nT = ctx->nT;
  const int npad = (n + kCTile - 1) / kCTile * kCTile;
  const int ntile = npad / kCTile;
  const size_t nn = (size_t)npad * npad;
  const Fc3Layout& L = ctx->fc3;
  const int ng = std::max(L.n_cgroups, 1), ncp = L.n_cpairs, nd = L.n_delta;
  hipStream_t st = ctx->stream;
  const int TB = 256;
  double *OM, *IW, *OCC;
  cplx<double>* PH;
  kaldo_status rs = run_crystal_tables(ctx, &OM, &IW, &OCC, &PH);
  if (rs != KALDO_OK) return rs;
  // items per batch (p, s pairs), bounded by the X and Y plane memory
  const size_t item_bytes = 4 * S * nn * sizeof(T);
  int batch = (int)std::max<size_t>(1, std::min<size_t>((size_t)nk * n, ((size_t)512 << 20) / item_bytes));
  batch = std::min(batch, 65535);
  const size_t items = (size_t)nk * n;
  // device buffers: d_A = [E planes | X planes | Y planes]; d_scratch2 = [Z | partial | graw]
  const size_t e_elems = (size_t)nk * 3 * nn;
  const size_t xy_elems = (size_t)batch * 2 * nn;
  KALDO_HIP(ctx, ctx->d_A.ensure((e_elems + 2 * xy_elems) * S * sizeof(T)));
  T* Eh = ctx->d_A.as<T>();
  T* El = S == 2 ? Eh + e_elems : nullptr;
  T* Xh = Eh + e_elems * S;
  T* Xl = S == 2 ? Xh + xy_elems : nullptr;
  T* Yh = Xh + xy_elems * S;
  T* Yl = S == 2 ? Yh + xy_elems : nullptr;
  const size_t z_elems = (size_t)n * ng * 9;
  const size_t part = items * ntile * ntile * nT;
  const size_t graw = (size_t)nT * nk * n;
  KALDO_HIP(ctx, ctx->d_scratch2.ensure(z_elems * sizeof(cplx<double>) + (part + graw) * sizeof(double)));
  cplx<double>* Z = ctx->d_scratch2.as<cplx<double>>();
  double* partial = reinterpret_cast<double*>(Z + z_elems);
  double* gr = partial + part;
  KALDO_HIP(ctx, ctx->d_gamma.ensure((size_t)nT * nk * n * sizeof(double)));
  hipLaunchKernelGGL((k_cr_eplanes<P>), dim3(blocks_for((long long)nk * nn, TB)), dim3(TB), 0, st, Eh, El,
                     ctx->d_evec.as<cplx<double>>(), nk, n, npad);
  KALDO_HIP(ctx, hipGetLastError());
  const double sig = kTwoPi * sigma_thz;
  CrArgs A;
  A.n = n;
  A.npad = npad;
  A.nk = nk;
  A.G0 = ctx->grid[0];
  A.G1 = ctx->grid[1];
  A.G2 = ctx->grid[2];
  A.nT = nT;
  A.c = 1.0 / (2.0 * sig * sig);
  const double C = kPi / 8.0 * kHbar * kEvUnit * kEvUnit * kEvUnit / nk / (sqrt(kTwoPi) * sig);
  for (int k = 0; k < nk; ++k) {
    A.k = k;
    prof_begin(ctx);
    hipLaunchKernelGGL(k_cr_zg, dim3(blocks_for((long long)z_elems, TB)), dim3(TB), 0, st, Z,
                       ctx->d_evec.as<cplx<double>>(), L.d_cg_block.as<int2>(), L.d_blk_i.as<int>(),
                       L.d_blk_R2.as<int>(), L.d_blk_val.as<double>(), n, ng, A.G0, A.G1, A.G2, k);
    KALDO_HIP(ctx, hipGetLastError());
    prof_end(ctx, "step_a");
    for (size_t it0 = 0; it0 < items; it0 += batch) {
      const int cnt = (int)std::min<size_t>(batch, items - it0);
      A.it0 = (int)it0;
      prof_begin(ctx);
      KALDO_HIP(ctx, hipMemsetAsync(Xh, 0, (size_t)cnt * 2 * nn * sizeof(T), st));
      if (S == 2) KALDO_HIP(ctx, hipMemsetAsync(Xl, 0, (size_t)cnt * 2 * nn * sizeof(T), st));
      if (ncp > 0)
        hipLaunchKernelGGL((k_cr_xs<P>), dim3(blocks_for((long long)cnt * ncp * 9, TB)), dim3(TB), 0, st, Xh, Xl, Z,
                           PH, L.d_cg_delta.as<int>(), L.d_cg_order.as<int>(), L.d_cpair.as<int4>(), n, nk, ng, ncp,
                           npad, (int)it0, cnt);
      KALDO_HIP(ctx, hipGetLastError());
      prof_end(ctx, "step_b");
      prof_begin(ctx);
      launch_cr<P, 0>(nT, dim3(ntile * ntile, cnt), st, Eh, El, Xh, Xl, Yh, Yl, OM, IW, OCC, A, partial);
      KALDO_HIP(ctx, hipGetLastError());
      launch_cr<P, 1>(nT, dim3(ntile * ntile, cnt), st, Eh, El, Yh, Yl, nullptr, nullptr, OM, IW, OCC, A, partial);
      KALDO_HIP(ctx, hipGetLastError());
      prof_end(ctx, "project");
    }
    hipLaunchKernelGGL(k_cr_collect, dim3(blocks_for(n * nT, TB)), dim3(TB), 0, st, gr, partial, IW, n, nk, nT,
                       ntile * ntile, k, C);
    KALDO_HIP(ctx, hipGetLastError());
  }
  hipLaunchKernelGGL(k_cr_set_average, dim3(blocks_for((long long)n * nk * nT, TB)), dim3(TB), 0, st,
                     ctx->d_gamma.as<double>(), gr, ctx->d_setid.as<int>(), n, nk, nT);
  KALDO_HIP(ctx, hipGetLastError());
  return KALDO_OK;
}

kaldo_status run_linewidths_crystal(kaldo_ctx ctx, double sigma_thz, int precision) {
  if (precision == KALDO_FP64) return crystal_impl<KALDO_FP64>(ctx, sigma_thz);
  if (precision == KALDO_FP32) return crystal_impl<KALDO_FP32>(ctx, sigma_thz);
  return crystal_impl<KALDO_BF16X3>(ctx, sigma_thz);
}

}  // namespace kaldo
