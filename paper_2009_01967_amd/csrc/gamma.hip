// Gamma-point linewidths (grid {1,1,1}) for cells with many branches: the
// disordered-solid path that feeds QHGK (paper Sec. II.C), where the paper
// notes the whole calculation can be done in real space at Gamma.
//
// With N_k = 1 every phase of eq. projection_plus is 1 and the eigenvectors
// are real, so phi+ = phi- = V and, for each first mode s,
//   X_s[a'][a''] = sum_a eta_s[a] phi[a,a',a''] / sqrt(m m' m'')     (sparse, symmetric)
//   Y_s = X_s E                                                    (sparse x dense)
//   V_s = E^T Y_s                                                  (dense GEMM, MFMA)
// The GEMM runs on the shared MFMA core with the linewidth epilogue fused in:
// V never leaves registers; each block tile is reduced to one partial sum per
// output column and temperature.
//
// Precisions of the GEMM: FP64 (f64 MFMA), FP32 (f32 MFMA), BF16X3 (each
// operand split into bf16 hi + lo, three bf16 MFMAs hi*hi + hi*lo + lo*hi with
// FP32 accumulation).  X_s and Y_s are formed in FP64; mode tables,
// occupations and every sum past the tile stay FP64.
#include <algorithm>
#include <string>

#include "common.h"
#include "gemm.h"
#include "internal.h"
#include "mfma.h"
#include "tune.h"

namespace kaldo {

// Bytes per K block of the Y operand (see GemmOps::b_kb): one 16-byte slot.
constexpr int kYBlock = 32;

// ---- X_s: contract fc3 with eta_s over the home atom ---------------------------------
// X_s[j beta][l gamma] for the first modes s0 + sl, sl < sbp (zero where
// s0 + sl >= n), in the layout the sparse step stages into LDS as it is:
// Xs[sl / 16][pair][gamma][beta][sl % 16] (R values), pairs being the distinct
// (j, l) atom pairs, so that the values of one atom's pairs for a group of 16
// modes are contiguous.  Et64[a][s] = eta_s[a] (FP64).
template <typename R>
__global__ void k_gamma_xs(R* __restrict__ Xs, const double* __restrict__ Et64, const int* __restrict__ pstart,
                           const int* __restrict__ gi, const double* __restrict__ gval, int n, int npairs, int s0,
                           int sbp) {
  // one thread per (pair, sl): all 9 (beta, gamma) values share the
  // eigenvector loads of every fc3 block of the pair
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)sbp * npairs) return;
  const int sl = (int)(idx % sbp);
  const int pr = (int)(idx / sbp);
  const int s = s0 + sl;
  double v[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) v[q] = 0.0;
  if (s < n) {
    // Et64[a][s] = eta_s[a]: the lanes (consecutive s) read neighbouring values
    for (int b = pstart[pr]; b < pstart[pr + 1]; ++b) {
      const double* f = gval + 27 * (size_t)b;
      const double* e = Et64 + (size_t)(3 * gi[b]) * n + s;
      const double e0 = e[0], e1 = e[n], e2 = e[2 * (size_t)n];
#pragma unroll
      for (int q = 0; q < 9; ++q) v[q] += e0 * f[q] + e1 * f[9 + q] + e2 * f[18 + q];
    }
  }
  R* out = Xs + ((size_t)(sl >> 4) * npairs + pr) * 144 + (sl & 15);
#pragma unroll
  for (int q = 0; q < 9; ++q) {  // q = 3 beta + gamma, stored at [gamma][beta]
    const int beta = q / 3, gamma = q % 3;
    out[(gamma * 3 + beta) * 16] = (R)v[q];
  }
}

// Et[a][s] = eta_s[a]: 32 x 32 tiles through LDS, both sides coalesced.
template <typename R>
__global__ void k_transpose(R* __restrict__ Et, const double* __restrict__ E, int n) {
  __shared__ double t[32][33];
  const int s0 = blockIdx.x * 32, a0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows per pass
  for (int r = ty; r < 32; r += 8) {
    const int s = s0 + r, a = a0 + tx;
    t[r][tx] = (s < n && a < n) ? E[(size_t)s * n + a] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int a = a0 + r, s = s0 + tx;
    if (a < n && s < n) Et[(size_t)a * n + s] = (R)t[tx][r];
  }
}

// ---- Y_s^T[s''][a'] = sum_a'' X_s[a'][a''] E[a''][s''] as the GEMM's B operand ---------
// For one atom j and 16 first modes u this is a small dense product on the
// matrix cores: C_alpha[u][s''] = sum_k A_alpha[u][k] B[k][s''] with k = (pair
// (j, l), gamma) running over the 3 P_j components of the atoms l paired with j,
// A_alpha[u][(l, gamma)] = X_s(u)[j alpha][l gamma] and B[(l, gamma)][s''] =
// E[l gamma][s''] (rows of Et, read straight from global memory into the B
// fragments: each lane one value, 16 consecutive s'' per k).  The block stages
// A of the atom in LDS as [k][alpha][u] (zero past the last k), with the Et row
// offset of every k; each of its W waves covers 16 columns s''.  R is FP64
// (f64 16x16x4) for the FP64 path and FP32 (f32 16x16x4) for the mixed ones
// (Y then enters FP32 or BF16 hi + lo operands).
// Y rows (sl, s''), columns a', K-blocked (GemmOps::b_kb): element (row, a') at
// (a' / E) * bkb + row * E + a' % E with E the elements of kYBlock bytes.  A
// block takes a run of E atoms: its lanes hold all 3 E elements a' of their
// rows, three whole K blocks, and store each with full 16-byte writes (the 16
// lanes of a row group cover 16 neighbouring blocks).  With FP32 values the
// staging is double buffered: the next atom's values are loaded into registers
// while this one's MFMAs run.  LDS: NBUF kmax * (48 * sizeof(R) + 4) bytes,
// NBUF = 2 for FP32 and 1 for FP64, kmax = 3 * (most pairs of one atom)
// rounded up to 4.
template <int P, typename R, int W>
__global__ void __launch_bounds__(64 * W)
    k_gamma_y(typename Operand<P>::T* __restrict__ Yhi, typename Operand<P>::T* __restrict__ Ylo,
              const R* __restrict__ Xs, const R* __restrict__ Et, const int* __restrict__ rstart,
              const int* __restrict__ pl, int n, int N, int npairs, long long bkb, int cnt, int kmax) {
  using T = typename Operand<P>::T;
  using Acc = typename std::conditional<std::is_same<R, double>::value, f64x4, f32x4>::type;
  constexpr int E = kYBlock / (int)sizeof(T);  // atoms per block: 3 E elements = 3 K blocks
  constexpr int V = 16 / (int)sizeof(T);        // elements per 16-byte store
  constexpr int KS = sizeof(R) == 8 ? 8 : 16;   // k steps whose B loads are in flight together
  constexpr int AR = (W >= 8 ? 2 : 16 / W) * (int)sizeof(R) / 4;  // 16-byte staging registers per thread
  extern __shared__ __attribute__((aligned(16))) char ylds[];
  // double-buffered staging for FP32 values; FP64 keeps one buffer (its
  // registers would drop a wave per SIMD)
  constexpr bool DB = sizeof(R) == 4;
  constexpr int NBUF = DB ? 2 : 1;
  R* As = reinterpret_cast<R*>(ylds);                                             // [NBUF][kmax][3][16]
  int* Ko = reinterpret_cast<int*>(ylds + (size_t)NBUF * kmax * 48 * sizeof(R));  // [NBUF][kmax]
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int s2 = ((int)blockIdx.x * W + wave) * 16 + li;
  const bool active = ((int)blockIdx.x * W + wave) * 16 < n;  // waves past the last column only stage
  const int s2c = min(s2, n - 1);
  const int slb = (int)blockIdx.y * 16;
  const int jb = (int)blockIdx.z * E;
  const int jend = min(N, jb + E);
  Acc acc[E][3];
#pragma unroll
  for (int jj = 0; jj < E; ++jj)
#pragma unroll
    for (int al = 0; al < 3; ++al) acc[jj][al] = Acc{};
  if constexpr (DB) {
    // Double-buffered staging: buffer b holds atom jb + jj while the loads of the
    // next atom are in flight in registers; one barrier per atom.
    const int bufR = kmax * 48;  // R values of one A buffer
    auto stage_direct = [&](int j, int b) __attribute__((always_inline)) {
      const int p0 = rstart[j], np = rstart[j + 1] - p0;
      const int kj = 3 * np, kjp = (kj + 3) & ~3;
      const u32x4* src = reinterpret_cast<const u32x4*>(Xs + ((size_t)blockIdx.y * npairs + p0) * 144);
      u32x4* dst = reinterpret_cast<u32x4*>(As + b * bufR);
      for (int i = tid; i < np * 144 * (int)sizeof(R) / 16; i += 64 * W) dst[i] = src[i];
      for (int i = kj * 48 + tid; i < kjp * 48; i += 64 * W) As[b * bufR + i] = (R)0;
      for (int k = tid; k < kjp; k += 64 * W) Ko[b * kmax + k] = k < kj ? (3 * pl[p0 + k / 3] + k % 3) * n : 0;
    };
    stage_direct(jb, 0);
    __syncthreads();
    // atoms of the run as compile-time indices (the accumulators stay in registers)
    static_for<E>([&](auto jc) __attribute__((always_inline)) {
      constexpr int jj = decltype(jc)::value;
      constexpr int b = jj & 1;
      const int j = jb + jj;
      if (j >= jend) return;  // uniform across the block; so are the later atoms
      const int kjp = (3 * (rstart[j + 1] - rstart[j]) + 3) & ~3;
      // next atom: X_s values (16-byte pieces) and Et row offsets into registers
      const bool more = j + 1 < jend;
      int np1 = 0, p01 = 0, n16 = 0;
      u32x4 areg[AR];
      int ko = 0;
      bool inreg = false;
      if (more) {
        p01 = rstart[j + 1];
        np1 = rstart[j + 2] - p01;
        n16 = np1 * 144 * (int)sizeof(R) / 16;
        inreg = n16 <= AR * 64 * W && 3 * np1 <= 64 * W;
        if (inreg) {
          const u32x4* src = reinterpret_cast<const u32x4*>(Xs + ((size_t)blockIdx.y * npairs + p01) * 144);
#pragma unroll
          for (int r = 0; r < AR; ++r) {
            const int i = tid + r * 64 * W;
            if (i < n16) areg[r] = src[i];
          }
          if (tid < 3 * np1) ko = (3 * pl[p01 + tid / 3] + tid % 3) * n;
        }
      }
      if (active) {
        const R* Ab = As + b * bufR;
        const int* Kb = Ko + b * kmax;
        // KS k steps at a time: all their Et loads are issued before the first MFMA
        for (int k0 = 0; k0 < kjp; k0 += 4 * KS) {
          R bv[KS];
#pragma unroll
          for (int q = 0; q < KS; ++q)
            bv[q] = k0 + 4 * q < kjp ? Et[Kb[k0 + 4 * q + lk] + s2c] : (R)0;  // padded k: row 0, A = 0
#pragma unroll
          for (int q = 0; q < KS; ++q) {
            if (k0 + 4 * q >= kjp) break;
            const int k = k0 + 4 * q + lk;
            const R a0 = Ab[(k * 3 + 0) * 16 + li], a1 = Ab[(k * 3 + 1) * 16 + li], a2 = Ab[(k * 3 + 2) * 16 + li];
            if constexpr (std::is_same<R, double>::value) {
              acc[jj][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv[q], acc[jj][0], 0, 0, 0);
              acc[jj][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv[q], acc[jj][1], 0, 0, 0);
              acc[jj][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, bv[q], acc[jj][2], 0, 0, 0);
            } else {
              acc[jj][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, bv[q], acc[jj][0], 0, 0, 0);
              acc[jj][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, bv[q], acc[jj][1], 0, 0, 0);
              acc[jj][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, bv[q], acc[jj][2], 0, 0, 0);
            }
          }
        }
      }
      if (more) {
        // the other buffer was last read before the previous barrier
        if (inreg) {
          const int kj1 = 3 * np1, kjp1 = (kj1 + 3) & ~3;
          u32x4* dst = reinterpret_cast<u32x4*>(As + (b ^ 1) * bufR);
#pragma unroll
          for (int r = 0; r < AR; ++r) {
            const int i = tid + r * 64 * W;
            if (i < n16) dst[i] = areg[r];
          }
          for (int i = kj1 * 48 + tid; i < kjp1 * 48; i += 64 * W) As[(b ^ 1) * bufR + i] = (R)0;
          if (tid < kjp1) Ko[(b ^ 1) * kmax + tid] = tid < kj1 ? ko : 0;
        } else {
          stage_direct(j + 1, b ^ 1);
        }
        __syncthreads();
      }
    });
  } else {
#pragma unroll
    for (int jj = 0; jj < E; ++jj) {
      const int j = jb + jj;
      if (j >= jend) break;  // uniform across the block
      const int p0 = rstart[j];
      const int np = rstart[j + 1] - p0;
      const int kj = 3 * np, kjp = (kj + 3) & ~3;
      __syncthreads();  // the previous atom is done with the staged values
      // the X_s values of the atom's pairs for this group of 16 modes, stored by
      // k_gamma_xs as [pair][gamma][alpha][u]: As[k][alpha][u] with k = 3 q + gamma
      {
        const uint4* src = reinterpret_cast<const uint4*>(Xs + ((size_t)blockIdx.y * npairs + p0) * 144);
        uint4* dst = reinterpret_cast<uint4*>(As);
        for (int i = tid; i < np * 144 * (int)sizeof(R) / 16; i += 64 * W) dst[i] = src[i];
      }
      for (int i = kj * 48 + tid; i < kjp * 48; i += 64 * W) As[i] = (R)0;
      for (int k = tid; k < kjp; k += 64 * W) Ko[k] = k < kj ? (3 * pl[p0 + k / 3] + k % 3) * n : 0;
      __syncthreads();
      if (active) {
        // KS k steps at a time: all their Et loads are issued before the first MFMA
        for (int k0 = 0; k0 < kjp; k0 += 4 * KS) {
          R bv[KS];
#pragma unroll
          for (int q = 0; q < KS; ++q)
            bv[q] = k0 + 4 * q < kjp ? Et[Ko[k0 + 4 * q + lk] + s2c] : (R)0;  // padded k: row 0, A = 0
#pragma unroll
          for (int q = 0; q < KS; ++q) {
            if (k0 + 4 * q >= kjp) break;
            const int k = k0 + 4 * q + lk;
            const R a0 = As[(k * 3 + 0) * 16 + li], a1 = As[(k * 3 + 1) * 16 + li], a2 = As[(k * 3 + 2) * 16 + li];
            if constexpr (std::is_same<R, double>::value) {
              acc[jj][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv[q], acc[jj][0], 0, 0, 0);
              acc[jj][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv[q], acc[jj][1], 0, 0, 0);
              acc[jj][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, bv[q], acc[jj][2], 0, 0, 0);
            } else {
              acc[jj][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, bv[q], acc[jj][0], 0, 0, 0);
              acc[jj][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, bv[q], acc[jj][1], 0, 0, 0);
              acc[jj][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, bv[q], acc[jj][2], 0, 0, 0);
            }
          }
        }
      }
    }
  }
  if (!active || s2 >= n) return;
  // lane: column s2, rows u = acc_row(lane, r); local element e = 3 jj + alpha
  // of a' = 3 jb + e (3 jb is a multiple of E: the three K blocks of the run)
  const int ne = 3 * (jend - jb);
  const size_t kb0 = (size_t)(3 * jb / E);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int u = acc_row<P == KALDO_FP64 ? KALDO_FP64 : KALDO_FP32>(lane, r);
    if (slb + u >= cnt) continue;
    const size_t row = (size_t)(slb + u) * n + s2;
    if (ne == 3 * E) {
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int h = 0; h < E; h += V) {
          double v[V];
#pragma unroll
          for (int q = 0; q < V; ++q) {
            const int e = m * E + h + q;
            v[q] = (double)acc[e / 3][e % 3][r];
          }
          store_operand_vec<P>(Yhi, Ylo, (kb0 + m) * bkb + row * E + h, v);
        }
    } else {
#pragma unroll
      for (int e = 0; e < 3 * E; ++e)
        if (e < ne)
          store_operand<P>(Yhi, Ylo, (kb0 + e / E) * bkb + row * E + e % E, (double)acc[e / 3][e % 3][r]);
    }
  }
}

// A operand: row s' = eta_{s'} (K = a' contiguous), zero in the K padding.
template <int P>
__global__ void k_gamma_a(typename Operand<P>::T* __restrict__ Ahi, typename Operand<P>::T* __restrict__ Alo,
                          const double* __restrict__ E, int n, int ld) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * ld) return;
  const int a = (int)(idx % ld), s = (int)(idx / ld);
  store_operand<P>(Ahi, Alo, idx, a < n ? E[(size_t)s * n + a] : 0.0);
}

// ---- fused linewidth epilogue of V_s = E^T Y_s ---------------------------------------
// Output row i = s' and column c = sl * n + s''.  For every element, both
// processes at every temperature:
//   |V|^2 / (w' w'') * [ g+ (n' - n'') + 1/2 g- (1 + n' + n'') ]
// with g+- the delta shape at (w +- w' - w''); the 1/w of the first mode, the
// delta normalisation and the prefactor are applied when collecting.  DK is
// the delta kind.
template <int NT, int DK>
struct EpiGamma {
  const double *OM, *IW, *OCC;
  double* partial;     // [m_tiles][ncol][nT]
  long long ncol;      // cnt * n
  int n, nT, s0;
  double rs;           // 1 / (scale of the delta)
  static constexpr bool kAllShapes = DK == KALDO_DELTA_GAUSS;
  static constexpr int kBlockBytes = kYBlock;  // B = Y is K-blocked
  static constexpr bool kSkipEmpty = DK != KALDO_DELTA_LORENTZ;  // the Lorentzian has no cut

  // Every element of block tile (mt, nt) beyond the delta's cut: frequencies
  // ascend with the mode index, so the mismatches w -+ w' - w'' over the tile
  // span intervals given by its corner modes (widened by a rounding margin).
  template <int P, int FM, int FN>
  __device__ bool tile_empty(int, int nt, int, int r0) const {
    constexpr int BM = 32 * FM, BN = 32 * FN;
    if (r0 >= n) return true;  // padding rows only
    const double a = OM[r0] * rs, b = OM[min(n, r0 + BM) - 1] * rs;  // w' range
    const double W = sqrt(delta_cut<P>(DK)) * (1.0 + 1e-9) + 1e-9;
    const long long c1 = min(ncol, (long long)nt * BN + BN) - 1;
    for (long long c = (long long)nt * BN; c <= c1;) {
      const int sl = (int)(c / n);
      const long long ce = min(c1, (long long)(sl + 1) * n - 1);
      const double ws = OM[s0 + sl] * rs;
      const double lo = OM[(int)(c - (long long)sl * n)] * rs, hi = OM[(int)(ce - (long long)sl * n)] * rs;
      if (ws - hi + a < W && ws - lo + b > -W) return false;  // w + w' - w''
      if (ws - hi - b < W && ws - lo - a > -W) return false;  // w - w' - w''
      c = ce + 1;
    }
    return true;
  }
  template <int P, int FM, int FN>
  __device__ void clear_tile(int mt, int nt, int) const {
    const long long first = (long long)nt * 32 * FN;
    for (int i = threadIdx.x; i < 32 * FN * nT; i += blockDim.x) {
      const int col = i / nT, t = i % nT;
      if (first + col < ncol) partial[((size_t)mt * ncol + first + col) * nT + t] = 0.0;
    }
  }

  template <int P, int FM, int FN>
  __device__ __forceinline__ void apply(typename Operand<P>::Acc (&acc)[FM][FN], const TileAt& at,
                                        char* lds) const {
    using R = typename std::conditional<P == KALDO_FP64, double, float>::type;
    constexpr double cut = delta_cut<P>(DK);
    // column data: (w - w'') / scale (first mode minus s''), 1/w'', n''
    double dcol[FN];
    R iw2[FN], n2[FN][NT], o[FN][NT];
#pragma unroll
    for (int q = 0; q < FN; ++q) {
      const long long col = at.c0 + 16 * q + (at.lane & 15);
      const bool cv = col < ncol;
      const int sl = cv ? (int)(col / n) : 0;
      const int s2 = cv ? (int)(col - (long long)sl * n) : 0;
      dcol[q] = (OM[s0 + sl] - OM[s2]) * rs;
      iw2[q] = cv ? (R)IW[s2] : (R)0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        n2[q][t] = t < nT ? (R)OCC[(size_t)t * n + s2] : (R)0;
        o[q][t] = 0;
      }
    }
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      // row data of the lane's four rows s': w', 1/w', n'
      double w1[4];
      R iw1[4], n1[4][NT];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = at.m0 + 16 * a + acc_row<P>(at.lane, r);
        const int ic = i < n ? i : n - 1;
        w1[r] = OM[ic] * rs;
        iw1[r] = i < n ? (R)IW[ic] : (R)0;
#pragma unroll
        for (int t = 0; t < NT; ++t) n1[r][t] = t < nT ? (R)OCC[(size_t)t * n + ic] : (R)0;
      }
#pragma unroll
      for (int q = 0; q < FN; ++q) {
        // a 16 x 16 sub-tile with every element outside the delta's cutoff adds nothing
        bool need = false;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double xp = dcol[q] + w1[r], xm = dcol[q] - w1[r];
          need = need || fmin(xp * xp, xm * xm) < cut;
        }
        if (__ballot(need) == 0) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const R v = (R)acc[a][q][r];
          const R v2 = v * v * iw1[r] * iw2[q];
          const R gp = delta_shape<R, DK>(dcol[q] + w1[r]);
          const R gm = delta_shape<R, DK>(dcol[q] - w1[r]);
          const R h = (R)0.5 * gm, a1 = gp + h, a2 = h - gp;
#pragma unroll
          for (int t = 0; t < NT; ++t) o[q][t] += v2 * (h + n1[r][t] * a1 + n2[q][t] * a2);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < FN; ++q) {
      double od[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) od[t] = (double)o[q][t];
      column_put<FN, NT>(od, q, at, lds);
    }
    const long long first = (long long)at.nt * 32 * FN;
    column_flush<FN, NT>(lds, partial + ((size_t)at.mt * ncol + first) * nT, ncol - first, nT);
  }
};

// g[t][s] = C / w_s * sum over row tiles and the n columns of s (one block per (sl, t))
__global__ void __launch_bounds__(1024)
    k_gamma_collect(double* __restrict__ graw, const double* __restrict__ partial, const double* __restrict__ IW,
                    int n, int nT, int m_tiles, long long ncol, int s0, double C) {
  // one block of 1024 threads per (first mode, temperature): the (row tile,
  // s'') partial sums are walked flat, so that many loads are in flight
  __shared__ double red[1024];
  const int sl = blockIdx.x, t = blockIdx.y;
  double v = 0.0;
  const int total = m_tiles * n;
  for (int i = threadIdx.x; i < total; i += 1024) {
    const int mt = i / n, s2 = i - mt * n;
    v += partial[((size_t)mt * ncol + (size_t)sl * n + s2) * nT + t];
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) graw[(size_t)t * n + s0 + sl] = C * IW[s0 + sl] * red[0];
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

template <int P, class Epi>
static int gemm_lw(kaldo_ctx ctx, const std::string& key, const GemmOps& g, const Epi& e) {
  hipStream_t st = ctx->stream;
  const int v = autotune(ctx, key, gemm_variants<P, Epi>(), 0, [&](int w) { gemm_launch<P>(w, g, e, st); });
  if (!planning(ctx)) {
    GemmOps gt = g;
    prof_tally(ctx, gt);
    gemm_launch<P>(v, gt, e, st);
  }
  return v;
}

template <int P>
static kaldo_status gamma_point_impl(kaldo_ctx ctx, double sigma_thz) {
  using T = typename Operand<P>::T;
  constexpr int S = Operand<P>::split;
  // sparse step: FP64 for the FP64 path, FP32 otherwise; 16 first modes per block
  using RY = typename std::conditional<P == KALDO_FP64, double, float>::type;
  constexpr int SB = 16;
  const int N = ctx->n_atoms, n = ctx->nm, nT = ctx->nT;
  const int KC = GemmChunk<P>::KC;
  const int ld = (n + KC - 1) / KC * KC;  // K padded to whole chunks
  const Fc3Layout& L = ctx->fc3;
  const int npairs = std::max(L.n_pairs, 1);
  hipStream_t st = ctx->stream;
  const double* E = ctx->d_dyn.as<double>();  // real eigenvectors, column s contiguous
  const size_t y_item = (size_t)n * ld * sizeof(T) * S;
  // first-mode batch bounded by the Y buffer size
  int sb = (int)std::max<size_t>(1, std::min<size_t>((size_t)n, ((size_t)2 << 30) / y_item));
  sb = std::min(sb, 256);
  const int sbp = (sb + SB - 1) / SB * SB;
  const int nbatch = (n + sb - 1) / sb;
  const long long ncol_max = (long long)sb * n;
  const int mt_max = (n + 63) / 64;  // the smallest candidate block tile has 64 rows
  // d_tabs: tables | graw | partial | Xs | Et | Et64 (FP32 Et only)
  const size_t tab = (2 + (size_t)nT) * n;
  const size_t graw = (size_t)nT * n;
  const size_t part = (size_t)mt_max * ncol_max * nT;
  const size_t xs = (size_t)sbp * npairs * 9;
  const size_t et = (size_t)n * n;
  const size_t xs_at = (tab + graw + part + 1) & ~(size_t)1;  // Xs 16-byte aligned (read as uint4)
  // an FP64 transposed copy of E for k_gamma_xs when Et holds FP32 values
  const size_t et64 = std::is_same<RY, double>::value ? 0 : (size_t)n * n;
  KALDO_HIP(ctx, ctx->d_tabs.ensure((xs_at + xs + et + et64) * sizeof(double)));
  double* OM = ctx->d_tabs.as<double>();
  double* IW = OM + n;
  double* OCC = IW + n;
  double* gr = OCC + (size_t)nT * n;
  double* partial = gr + graw;
  double* Xs = ctx->d_tabs.as<double>() + xs_at;
  RY* Et = reinterpret_cast<RY*>(Xs + xs);
  double* Et64 = std::is_same<RY, double>::value ? reinterpret_cast<double*>(Et) : Xs + xs + et;
  // operands: A [n][ld] planes, Y [sb * n][ld] planes
  const size_t a_elems = (size_t)n * ld, y_elems = (size_t)sb * n * ld;
  // Y is K-blocked: blocks of kYBlock bytes of elements, each block column
  // holding all sb * n rows
  constexpr int EY = kYBlock / (int)sizeof(T);
  const long long y_kb = (long long)sb * n * EY;
  KALDO_HIP(ctx, ctx->d_A.ensure((a_elems + y_elems) * S * sizeof(T)));
  T* Ah = ctx->d_A.as<T>();
  T* Al = S == 2 ? Ah + a_elems : nullptr;
  T* Yh = Ah + a_elems * S;
  T* Yl = S == 2 ? Yh + y_elems : nullptr;
  KALDO_HIP(ctx, ctx->d_gamma.ensure((size_t)nT * n * sizeof(double)));
  // the K padding of Y (columns a' >= n) stays zero; the rest is rewritten per batch
  kaldo_status fs;
  if (ld > n && (fs = fill_zero(ctx, Yh, y_elems * S * sizeof(T))) != KALDO_OK) return fs;
  double4 T03 = make_double4(ctx->T[0], ctx->T[1], ctx->T[2], ctx->T[3]);
  double4 T47 = make_double4(ctx->T[4], ctx->T[5], ctx->T[6], ctx->T[7]);
  const int TB = 256;
  hipLaunchKernelGGL(k_tables_gamma, dim3(blocks_for(n, TB)), dim3(TB), 0, st, OM, IW, OCC,
                     ctx->d_omega.as<double>(), n, nT, T03, T47, ctx->stats == KALDO_CLASSICAL ? 1 : 0);
  hipLaunchKernelGGL((k_gamma_a<P>), dim3(blocks_for((long long)n * ld, TB)), dim3(TB), 0, st, Ah, Al, E, n, ld);
  hipLaunchKernelGGL((k_transpose<RY>), dim3((n + 31) / 32, (n + 31) / 32), dim3(256), 0, st, Et, E, n);
  if constexpr (!std::is_same<RY, double>::value)
    hipLaunchKernelGGL((k_transpose<double>), dim3((n + 31) / 32, (n + 31) / 32), dim3(256), 0, st, Et64, E, n);
  KALDO_HIP(ctx, hipGetLastError());
  const double sig = kTwoPi * sigma_thz;
  double dscale, dnorm;
  delta_scale(ctx->delta, sig, dscale, dnorm);
  const double C = kPi / 8.0 * kHbar * kEvUnit * kEvUnit * kEvUnit * dnorm;
  int max_pairs = 1;
  if ((int)L.grow_start.size() == N + 1)
    for (int j = 0; j < N; ++j) max_pairs = std::max(max_pairs, L.grow_start[j + 1] - L.grow_start[j]);
  const int kmax = (3 * max_pairs + 3) & ~3;
  const size_t y_lds = (size_t)(sizeof(RY) == 4 ? 2 : 1) * kmax * (48 * sizeof(RY) + sizeof(int));
  if (y_lds > 160 * 1024) return fail(ctx, KALDO_EINVAL, "Gamma path: too many fc3 atom pairs per atom");
  for (int b = 0; b < nbatch; ++b) {
    // planning visits the batches whose GEMM shapes differ: the first and the last
    if (planning(ctx) && b != 0 && b != nbatch - 1) continue;
    const int s0 = b * sb;
    const int cnt = std::min(sb, n - s0);
    const int cntp = (cnt + SB - 1) / SB * SB;
    prof_begin(ctx);
    if (planning(ctx)) {
    } else if (L.n_pairs > 0) {
      hipLaunchKernelGGL(k_gamma_xs<RY>, dim3(blocks_for((long long)cntp * npairs, TB)), dim3(TB), 0, st,
                         reinterpret_cast<RY*>(Xs), Et64, L.d_gpair_start.as<int>(), L.d_gblk_i.as<int>(),
                         L.d_gblk_val.as<double>(), n, npairs, s0, cntp);
      KALDO_HIP(ctx, hipGetLastError());
      // waves per block (16 columns s'' each, sharing the staged X_s values):
      // 8, 4 or 2, tuned per problem; smaller blocks overlap one block's staging
      // with another's MFMAs on the same CU, larger ones stage less
      auto ylaunch = [&](int w) {
        const dim3 grid_yz(0, cntp / SB, (N + EY - 1) / EY);
        auto go = [&](auto wc) {
          constexpr int W = decltype(wc)::value;
          if (y_lds > 64 * 1024)  // beyond the default dynamic LDS limit (gfx950 has 160 KB)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gamma_y<P, RY, W>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)y_lds);
          hipLaunchKernelGGL((k_gamma_y<P, RY, W>), dim3((n + 16 * W - 1) / (16 * W), grid_yz.y, grid_yz.z),
                             dim3(64 * W), y_lds, st, Yh, Yl, reinterpret_cast<const RY*>(Xs), Et,
                             L.d_grow_start.as<int>(), L.d_gpair_l.as<int>(), n, N, npairs, y_kb, cnt, kmax);
        };
        if (w == 0) go(std::integral_constant<int, 8>{});
        else if (w == 1) go(std::integral_constant<int, 4>{});
        else go(std::integral_constant<int, 2>{});
      };
      const std::string ykey = "gy/" + std::to_string(P) + "/" + std::to_string(n) + "/" + std::to_string(cnt);
      ylaunch(autotune(ctx, ykey, 3, 0, ylaunch));
    } else if ((fs = fill_zero(ctx, Yh, y_elems * S * sizeof(T))) != KALDO_OK) {
      return fs;
    }
    KALDO_HIP(ctx, hipGetLastError());
    prof_end(ctx, "gamma_sparse");
    GemmOps g{};
    g.a_hi = Ah;
    g.a_lo = Al;
    g.b_hi = Yh;
    g.b_lo = Yl;
    g.lda = ld;
    g.ldb = EY;
    g.b_kb = y_kb;
    g.K = ld;
    g.nz = 1;
    g.m_valid = n;
    g.c_valid = (long long)cnt * n;
    // With a cut delta most tiles are skipped and the rest form two bands
    // across the tile grid.  The tiles go in chunks of 16 column panels, and
    // inside a chunk in groups of 2 row tiles: each XCD's run then holds whole
    // chunks (the skipped work is spread evenly), and the tiles that run at the
    // same time share A and B panels in L2 (measured against all row tiles of
    // a column together: 88 -> 85 ms on the 1000-atom SiGe cell, BF16X3).
    // (FP64 keeps all row tiles of a column together: its smaller tiles did
    // not gain from the chunks)
    const bool cut = ctx->delta != KALDO_DELTA_LORENTZ;
    g.group_m = !cut ? 8 : (P == KALDO_FP64 ? 1 << 20 : 2);
    g.group_n = !cut || P == KALDO_FP64 ? 0 : 16;
    const std::string key = "gamma/" + std::to_string(P) + "/" + std::to_string(n) + "/" + std::to_string(cnt) +
                            "/" + std::to_string(nT) + "/" + std::to_string(ctx->delta);
    int v = 0;
    prof_begin(ctx);
#define KALDO_EPI(NTV, DKV)                                                                   \
  {                                                                                           \
    EpiGamma<NTV, DKV> e{OM, IW, OCC, partial, (long long)cnt * n, n, nT, s0, 1.0 / dscale}; \
    v = gemm_lw<P>(ctx, key, g, e);                                                           \
  }
#define KALDO_EPI_NT(DKV)              \
  {                                    \
    if (nT <= 1) KALDO_EPI(1, DKV)     \
    else if (nT <= 4) KALDO_EPI(4, DKV) \
    else KALDO_EPI(8, DKV)             \
  }
    if (ctx->delta == KALDO_DELTA_GAUSS) KALDO_EPI_NT(KALDO_DELTA_GAUSS)
    else if (ctx->delta == KALDO_DELTA_LORENTZ) KALDO_EPI_NT(KALDO_DELTA_LORENTZ)
    else KALDO_EPI_NT(KALDO_DELTA_TRIANGLE)
#undef KALDO_EPI_NT
#undef KALDO_EPI
    KALDO_HIP(ctx, hipGetLastError());
    prof_end(ctx, "project");
    if (planning(ctx)) continue;
    hipLaunchKernelGGL(k_gamma_collect, dim3(cnt, nT), dim3(1024), 0, st, gr, partial, IW, n, nT, gemm_m_tiles<P>(v, n),
                       (long long)cnt * n, s0, C);
    KALDO_HIP(ctx, hipGetLastError());
  }
  if (planning(ctx)) return KALDO_OK;
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
