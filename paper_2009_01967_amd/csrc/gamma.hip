// Gamma-point linewidths (grid {1,1,1}) for cells with many branches: the
// disordered-solid path that feeds QHGK (paper Sec. II.C), where the paper
// notes the whole calculation can be done in real space at Gamma.
//
// With N_k = 1 every phase of eq. projection_plus is 1 and the eigenvectors
// are real, so phi+ = phi- = V and, for each first mode s,
//   X_s[a'][a''] = sum_a eta_s[a] phi[a,a',a''] / sqrt(m m' m'')     (sparse, symmetric)
//   Y_s = X_s E                                                    (sparse x dense)
//   V_s = E^T Y_s                                                  (dense GEMM, MFMA)
// and the epilogue of the crystal path is fused into the GEMM: V never leaves
// registers; each tile is reduced to one partial linewidth per temperature.
//
// Precisions of the GEMM: FP64 (f64 MFMA), FP32 (f32 MFMA), BF16X3 (each
// operand split into bf16 hi + lo, three bf16 MFMAs hi*hi + hi*lo + lo*hi with
// FP32 accumulation).  Mode tables, occupations and all sums stay FP64.
#include <algorithm>

#include "common.h"
#include "internal.h"
#include "mfma.h"

namespace kaldo {

constexpr int kTile = 64;  // output tile (rows s', columns s'') per block

// ---- X_s: contract fc3 with eta_s over the home atom ---------------------------------
// Xs[sl][pair][beta][gamma]; pairs are the distinct (j, l) atom pairs.
__global__ void k_gamma_xs(double* __restrict__ Xs, const double* __restrict__ E, const int* __restrict__ pstart,
                           const int* __restrict__ gi, const double* __restrict__ gval, int n, int npairs, int s0,
                           int sb) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)sb * npairs * 9) return;
  const int e9 = (int)(idx % 9);
  const int pr = (int)((idx / 9) % npairs);
  const int sl = (int)(idx / (9LL * npairs));
  const int s = s0 + sl;
  double v = 0.0;
  if (s < n) {
    const double* es = E + (size_t)s * n;
    for (int b = pstart[pr]; b < pstart[pr + 1]; ++b) {
      const double* f = gval + 27 * (size_t)b + e9;
      const int i3 = 3 * gi[b];
      v += es[i3] * f[0] + es[i3 + 1] * f[9] + es[i3 + 2] * f[18];
    }
  }
  Xs[idx] = v;
}

// ---- Y_s^T[s''][a'] = sum_a'' X_s[a'][a''] E[a''][s''] in the GEMM operand format ---------
template <int P>
__global__ void k_gamma_y(typename Operand<P>::T* __restrict__ Yhi, typename Operand<P>::T* __restrict__ Ylo,
                          const double* __restrict__ Xs, const double* __restrict__ E,
                          const int* __restrict__ rstart, const int* __restrict__ pl, int n, int N, int npairs,
                          int npad, int s0, int sb) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)sb * n * N) return;
  const int j = (int)(idx % N);
  const int s2 = (int)((idx / N) % n);
  const int sl = (int)(idx / ((long long)N * n));
  double y0 = 0.0, y1 = 0.0, y2 = 0.0;
  if (s0 + sl < n) {
    const double* e = E + (size_t)s2 * n;
    const double* xs = Xs + (size_t)sl * npairs * 9;
    for (int p = rstart[j]; p < rstart[j + 1]; ++p) {
      const double* x = xs + 9 * (size_t)p;
      const int l3 = 3 * pl[p];
      const double e0 = e[l3], e1 = e[l3 + 1], e2 = e[l3 + 2];
      y0 += x[0] * e0 + x[1] * e1 + x[2] * e2;
      y1 += x[3] * e0 + x[4] * e1 + x[5] * e2;
      y2 += x[6] * e0 + x[7] * e1 + x[8] * e2;
    }
  }
  const size_t o = ((size_t)sl * npad + s2) * npad + 3 * j;
  store_operand<P>(Yhi, Ylo, o, y0);
  store_operand<P>(Yhi, Ylo, o + 1, y1);
  store_operand<P>(Yhi, Ylo, o + 2, y2);
}

// Et[s'][a] = E[a][s'] (the solver's column-major output), zero padded to npad x npad.
template <int P>
__global__ void k_gamma_et(typename Operand<P>::T* __restrict__ Ehi, typename Operand<P>::T* __restrict__ Elo,
                           const double* __restrict__ E, int n, int npad) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)npad * npad) return;
  const int a = (int)(idx % npad), s = (int)(idx / npad);
  const double v = (a < n && s < n) ? E[(size_t)s * n + a] : 0.0;
  store_operand<P>(Ehi, Elo, idx, v);
}

// ---- GEMM V_s = E^T Y_s with the fused epilogue ----------------------------------------
struct GammaArgs {
  int n, npad, nT, s0;
  double c;  // 1 / (2 sigma^2)
};

template <int P>
struct Kc;
template <>
struct Kc<KALDO_FP64> {
  static constexpr int v = 16;
};
template <>
struct Kc<KALDO_FP32> {
  static constexpr int v = 32;
};
template <>
struct Kc<KALDO_BF16X3> {
  static constexpr int v = 64;
};

template <int P, int NT>
__global__ void __launch_bounds__(256)
    k_gamma_gemm(const typename Operand<P>::T* __restrict__ Ehi, const typename Operand<P>::T* __restrict__ Elo,
                 const typename Operand<P>::T* __restrict__ Yhi, const typename Operand<P>::T* __restrict__ Ylo,
                 const double* __restrict__ OM, const double* __restrict__ IW, const double* __restrict__ OCC,
                 GammaArgs G, double* __restrict__ partial) {
  using T = typename Operand<P>::T;
  constexpr int KC = Kc<P>::v;
  constexpr bool kSplit = P == KALDO_BF16X3;
  // row stride in elements: keeps the per-lane MFMA operand reads on distinct banks
  constexpr int LD = KC + (sizeof(T) == 8 ? 2 : (sizeof(T) == 4 ? 4 : 8));
  __shared__ __attribute__((aligned(16))) T As[kSplit ? 2 : 1][kTile * LD];
  __shared__ __attribute__((aligned(16))) T Bs[kSplit ? 2 : 1][kTile * LD];
  __shared__ double red[4][NT];

  const int ntile = G.npad / kTile;
  const int ti = blockIdx.x / ntile, tj = blockIdx.x % ntile;
  const int sl = blockIdx.y;
  const int s = G.s0 + sl;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const size_t nn = (size_t)G.npad * G.npad;
  const T* Ah = Ehi + (size_t)ti * kTile * G.npad;
  const T* Al = kSplit ? Elo + (size_t)ti * kTile * G.npad : nullptr;
  const T* Bh = Yhi + (size_t)sl * nn + (size_t)tj * kTile * G.npad;
  const T* Bl = kSplit ? Ylo + (size_t)sl * nn + (size_t)tj * kTile * G.npad : nullptr;

  using Acc = typename std::conditional<P == KALDO_FP64, f64x4, f32x4>::type;
  Acc acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][b][r] = 0;

  // cooperative tile loads: 64 rows x KC elements per operand
  constexpr int kElemsPerThread = kTile * KC / 256;
  for (int k0 = 0; k0 < G.npad; k0 += KC) {
#pragma unroll
    for (int e = 0; e < kElemsPerThread; ++e) {
      const int q = threadIdx.x * kElemsPerThread + e;
      const int row = q / KC, col = q % KC;
      As[0][row * LD + col] = Ah[(size_t)row * G.npad + k0 + col];
      Bs[0][row * LD + col] = Bh[(size_t)row * G.npad + k0 + col];
      if constexpr (kSplit) {
        As[1][row * LD + col] = Al[(size_t)row * G.npad + k0 + col];
        Bs[1][row * LD + col] = Bl[(size_t)row * G.npad + k0 + col];
      }
    }
    __syncthreads();
    if constexpr (P == KALDO_BF16X3) {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 32) {
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int r = wi * 32 + a * 16 + (lane & 15);
          const int c = wj * 32 + a * 16 + (lane & 15);
          const int k = kk + 8 * (lane >> 4);
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            ah[a][e] = As[0][r * LD + k + e];
            al[a][e] = As[1][r * LD + k + e];
            bh[a][e] = Bs[0][c * LD + k + e];
            bl[a][e] = Bs[1][c * LD + k + e];
          }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
          }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        T av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          av[a] = As[0][(wi * 32 + a * 16 + (lane & 15)) * LD + kk + (lane >> 4)];
          bv[a] = Bs[0][(wj * 32 + a * 16 + (lane & 15)) * LD + kk + (lane >> 4)];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            if constexpr (P == KALDO_FP64)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
            else
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
          }
      }
    }
    __syncthreads();
  }

  // epilogue: weights of both processes at every temperature, reduced over the tile
  double out[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) out[t] = 0.0;
  const double ws = OM[s < G.n ? s : 0];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // accumulator rows: f32 MFMA lane l holds rows 4(l/16)+r, f64 MFMA rows l/16+4r
        const int i = ti * kTile + wi * 32 + a * 16 + (P == KALDO_FP64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
        const int j = tj * kTile + wj * 32 + b * 16 + (lane & 15);         // s''
        if (i < G.n && j < G.n) {
          const double v = (double)acc[a][b][r];
          const double v2 = v * v * IW[i] * IW[j];
          if (v2 != 0.0) {
            const double w1 = OM[i], w2 = OM[j];
            const double xp = ws + w1 - w2, xm = ws - w1 - w2;
            double gp, gm;
            if constexpr (P == KALDO_FP64) {
              gp = exp(-xp * xp * G.c);
              gm = exp(-xm * xm * G.c);
            } else {
              gp = (double)__expf((float)(-xp * xp * G.c));
              gm = (double)__expf((float)(-xm * xm * G.c));
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
              if (t < G.nT) {
                const double n1 = OCC[(size_t)t * G.n + i], n2 = OCC[(size_t)t * G.n + j];
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
  if (threadIdx.x < G.nT) {
    const int t = threadIdx.x;
    partial[((size_t)sl * gridDim.x + blockIdx.x) * G.nT + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
  }
}

// g[t][s] = C / w_s * sum over tiles (before set averaging)
__global__ void k_gamma_collect(double* __restrict__ graw, const double* __restrict__ partial,
                                const double* __restrict__ IW, int n, int nT, int ntiles, int s0, int sb, double C) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= sb * nT) return;
  const int sl = idx % sb, t = idx / sb;
  const int s = s0 + sl;
  if (s >= n) return;
  double v = 0.0;
  for (int b = 0; b < ntiles; ++b) v += partial[((size_t)sl * ntiles + b) * nT + t];
  graw[(size_t)t * n + s] = C * IW[s] * v;
}

__global__ void k_set_average_gamma(double* __restrict__ gamma, const double* __restrict__ graw,
                                    const int* __restrict__ setid, int n, int nT) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * nT) return;
  const int s = idx % n, t = idx / n;
  const int first = setid[s];
  int last = first;
  while (last + 1 < n && setid[last + 1] == first) ++last;
  double m = 0.0;
  for (int u = first; u <= last; ++u) m += graw[(size_t)t * n + u];
  gamma[(size_t)t * n + s] = m / (last - first + 1);
}

__global__ void k_tables_gamma(double* __restrict__ OM, double* __restrict__ IW, double* __restrict__ OCC,
                               const double* __restrict__ omega, int n, int nT, double4 T03, double4 T47,
                               int classical) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double w = omega[s];
  const bool on = w / kTwoPi >= kNuMinThz;
  OM[s] = w;
  IW[s] = on ? 1.0 / w : 0.0;
  const double Ts[8] = {T03.x, T03.y, T03.z, T03.w, T47.x, T47.y, T47.z, T47.w};
  for (int t = 0; t < nT; ++t) {
    double occ = 0.0;
    if (on) {
      if (classical) occ = kBoltzmann * Ts[t] / (kHbar * w);
      else if (Ts[t] > 0.0) occ = 1.0 / expm1(kHbar * w / (kBoltzmann * Ts[t]));
    }
    OCC[(size_t)t * n + s] = occ;
  }
}

template <int P, int NT>
static void launch_gemm(dim3 grid, hipStream_t st, const void* Eh, const void* El, const void* Yh, const void* Yl,
                        const double* OM, const double* IW, const double* OCC, const GammaArgs& A,
                        double* partial) {
  using T = typename Operand<P>::T;
  hipLaunchKernelGGL((k_gamma_gemm<P, NT>), grid, dim3(256), 0, st, (const T*)Eh, (const T*)El, (const T*)Yh,
                     (const T*)Yl, OM, IW, OCC, A, partial);
}

template <int P>
static void launch_gemm_nt(int nT, dim3 grid, hipStream_t st, const void* Eh, const void* El, const void* Yh,
                           const void* Yl, const double* OM, const double* IW, const double* OCC, const GammaArgs& A,
                           double* partial) {
  if (nT <= 1) launch_gemm<P, 1>(grid, st, Eh, El, Yh, Yl, OM, IW, OCC, A, partial);
  else if (nT <= 2) launch_gemm<P, 2>(grid, st, Eh, El, Yh, Yl, OM, IW, OCC, A, partial);
  else if (nT <= 4) launch_gemm<P, 4>(grid, st, Eh, El, Yh, Yl, OM, IW, OCC, A, partial);
  else launch_gemm<P, 8>(grid, st, Eh, El, Yh, Yl, OM, IW, OCC, A, partial);
}

template <int P>
static kaldo_status gamma_point_impl(kaldo_ctx ctx, double sigma_thz) {
  using T = typename Operand<P>::T;
  const int N = ctx->n_atoms, n = ctx->nm, nT = ctx->nT;
  const int npad = (n + kTile - 1) / kTile * kTile;
  const int ntile = npad / kTile;
  const Fc3Layout& L = ctx->fc3;
  const int npairs = L.n_pairs;
  hipStream_t st = ctx->stream;
  const double* E = ctx->d_dyn.as<double>();  // real eigenvectors, column s contiguous
  const int nsplit = P == KALDO_BF16X3 ? 2 : 1;
  const size_t op_bytes = (size_t)npad * npad * sizeof(T);
  // first-mode batch bounded by the Y buffer size
  int sb = (int)std::max<size_t>(1, std::min<size_t>((size_t)n, ((size_t)768 << 20) / (op_bytes * nsplit)));
  sb = std::min(sb, 64);
  const int nbatch = (n + sb - 1) / sb;
  // buffers: tables | graw | partial | Xs ; operands in d_A
  const size_t tab = (2 + (size_t)nT) * n;
  const size_t graw = (size_t)nT * n;
  const size_t part = (size_t)sb * ntile * ntile * nT;
  const size_t xs = (size_t)sb * std::max(npairs, 1) * 9;
  KALDO_HIP(ctx, ctx->d_tabs.ensure((tab + graw + part + xs) * sizeof(double)));
  double* OM = ctx->d_tabs.as<double>();
  double* IW = OM + n;
  double* OCC = IW + n;
  double* gr = OCC + (size_t)nT * n;
  double* partial = gr + graw;
  double* Xs = partial + part;
  KALDO_HIP(ctx, ctx->d_A.ensure(op_bytes * nsplit * (1 + (size_t)sb)));
  T* Eh = ctx->d_A.as<T>();
  T* El = P == KALDO_BF16X3 ? Eh + (size_t)npad * npad : nullptr;
  T* Yh = Eh + (size_t)nsplit * npad * npad;
  T* Yl = P == KALDO_BF16X3 ? Yh + (size_t)sb * npad * npad : nullptr;
  KALDO_HIP(ctx, ctx->d_gamma.ensure((size_t)nT * n * sizeof(double)));
  // Y pads (rows >= n, columns >= n) stay zero
  KALDO_HIP(ctx, hipMemsetAsync(Yh, 0, op_bytes * nsplit * sb, st));
  double4 T03 = make_double4(ctx->T[0], ctx->T[1], ctx->T[2], ctx->T[3]);
  double4 T47 = make_double4(ctx->T[4], ctx->T[5], ctx->T[6], ctx->T[7]);
  const int TB = 256;
  hipLaunchKernelGGL(k_tables_gamma, dim3(blocks_for(n, TB)), dim3(TB), 0, st, OM, IW, OCC,
                     ctx->d_omega.as<double>(), n, nT, T03, T47, ctx->stats == KALDO_CLASSICAL ? 1 : 0);
  hipLaunchKernelGGL((k_gamma_et<P>), dim3(blocks_for((long long)npad * npad, TB)), dim3(TB), 0, st, Eh, El, E, n,
                     npad);
  KALDO_HIP(ctx, hipGetLastError());
  const double sig = kTwoPi * sigma_thz;
  GammaArgs A;
  A.n = n;
  A.npad = npad;
  A.nT = nT;
  A.c = 1.0 / (2.0 * sig * sig);
  const double C = kPi / 8.0 * kHbar * kEvUnit * kEvUnit * kEvUnit / (sqrt(kTwoPi) * sig);
  for (int b = 0; b < nbatch; ++b) {
    const int s0 = b * sb;
    const int cnt = std::min(sb, n - s0);
    A.s0 = s0;
    prof_begin(ctx);
    hipLaunchKernelGGL(k_gamma_xs, dim3(blocks_for((long long)cnt * npairs * 9, TB)), dim3(TB), 0, st, Xs, E,
                       L.d_gpair_start.as<int>(), L.d_gblk_i.as<int>(), L.d_gblk_val.as<double>(), n, npairs, s0,
                       cnt);
    KALDO_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL((k_gamma_y<P>), dim3(blocks_for((long long)cnt * n * N, TB)), dim3(TB), 0, st, Yh, Yl, Xs,
                       E, L.d_grow_start.as<int>(), L.d_gpair_l.as<int>(), n, N, npairs, npad, s0, cnt);
    KALDO_HIP(ctx, hipGetLastError());
    prof_end(ctx, "gamma_sparse");
    prof_begin(ctx);
    launch_gemm_nt<P>(nT, dim3(ntile * ntile, cnt), st, Eh, El, Yh, Yl, OM, IW, OCC, A, partial);
    KALDO_HIP(ctx, hipGetLastError());
    prof_end(ctx, "project");
    hipLaunchKernelGGL(k_gamma_collect, dim3(blocks_for(cnt * nT, TB)), dim3(TB), 0, st, gr, partial, IW, n, nT,
                       ntile * ntile, s0, cnt, C);
    KALDO_HIP(ctx, hipGetLastError());
  }
  hipLaunchKernelGGL(k_set_average_gamma, dim3(blocks_for(n * nT, TB)), dim3(TB), 0, st, ctx->d_gamma.as<double>(),
                     gr, ctx->d_setid.as<int>(), n, nT);
  KALDO_HIP(ctx, hipGetLastError());
  return KALDO_OK;
}

kaldo_status run_linewidths_gamma(kaldo_ctx ctx, double sigma_thz, int precision) {
  if (precision == KALDO_FP64) return gamma_point_impl<KALDO_FP64>(ctx, sigma_thz);
  if (precision == KALDO_FP32) return gamma_point_impl<KALDO_FP32>(ctx, sigma_thz);
  return gamma_point_impl<KALDO_BF16X3>(ctx, sigma_thz);
}

}  // namespace kaldo
