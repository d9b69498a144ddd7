// Three-phonon projection and scattering-rate sum (paper Sec. II.B,
// eq. projection_plus .. delta_deconstructed) for crystals with many branches,
// as two chained complex GEMMs on the shared MFMA core per (first-mode point k,
// partner p), batched over the first-mode branch s:
//
//   Z_k[s][g]    = sum_{blocks b in group g} e^{2 pi i k.R2_b} sum_a eta_ks[a] phi_b / sqrt(m m' m'')
//                  (group g = one (Delta, j, l), Delta = R2 - R1)                      (step A)
//   X_ks(p)      = sum_g e^{2 pi i p.Delta_g} Z_k[s][g] placed at the (j, l) block     (step B, dense n x n)
//   Y^T[s''][a'] = sum_a'' conj(eta_{k+p}[a''][s'']) X[a'][a'']                       (GEMM 1)
//   V[s'][s'']   = sum_a' eta_p[a'][s'] Y^T[s''][a']                                   (GEMM 2)
//
// V is phi+ of (k,s),(p,s'),(k+p,s''); as in the few-branch path the same V
// also serves the creation process of (k,s),(-p,s'),(k+p,s'').  GEMM 2 carries
// the fused epilogue (|V|^2, occupations, Gaussian delta, every temperature,
// per-column reduction), so V never reaches memory.
//
// Complex products run as real GEMMs on "realified" operands: a complex A
// (M x K) becomes the real 2M x 2K matrix whose row pair for output i is
// [Re A_i | -Im A_i] and [Im A_i | Re A_i] with the K index interleaved
// (k' = 2a + d, d = 0 meets Re B, d = 1 meets Im B).  The two rows of a pair
// are placed so that one lane's accumulator holds both Re V and Im V of the
// same element: rows 2i, 2i+1 for the FP32/BF16 MFMA layouts, rows
// 8(i/4) + 4c + i%4 for the FP64 one.  The GEMM columns run over (s, a') or
// (s, s'') contiguously, so no per-item padding is multiplied.
#include <algorithm>
#include <string>

#include "common.h"
#include "gemm.h"
#include "internal.h"
#include "mfma.h"
#include "tune.h"

namespace kaldo {

// a complex value from a device buffer through the global-memory view
template <typename R>
__device__ __forceinline__ cplx<R> gload(const cplx<R>* p) {
  const R* q = reinterpret_cast<const R*>(p);
  return {gmem(q)[0], gmem(q)[1]};
}

// output row of the realified pair (i, c)
template <int P>
__host__ __device__ __forceinline__ int cr_row(int i, int c) {
  return P == KALDO_FP64 ? 8 * (i >> 2) + 4 * c + (i & 3) : 2 * i + c;
}
template <int P>
__host__ __device__ __forceinline__ int cr_rows(int n) {
  return P == KALDO_FP64 ? 8 * ((n + 3) / 4) : 2 * n;
}

// Z[s][g][e9] for one first-mode k (formed in FP64, stored as RZ: FP64 for the
// FP64 path, FP32 for the mixed ones)
template <typename RZ>
__device__ __forceinline__ void cr_zg_elem(cplx<RZ>* __restrict__ Z, const cplx<double>* __restrict__ E,
                                           const int2* __restrict__ cgb, const int* __restrict__ bi,
                                           const int* __restrict__ bR2, const double* __restrict__ bval, int n, int ng,
                                           int G0, int G1, int G2, int k, long long idx) {
  // idx = (s ng + g) 9 + e9 < n ng 9, well inside 32 bits
  const int ii = (int)idx;
  const int e9 = ii % 9;
  const int g = (ii / 9) % ng;
  const int s = ii / (9 * ng);
  const int m0 = k / (G1 * G2), m1 = (k / G2) % G1, m2 = k % G2;
  const long long Gt = (long long)G0 * G1 * G2;
  const cplx<double>* e = E + ((size_t)k * n + s) * n;
  const int* rg = reinterpret_cast<const int*>(cgb) + 2 * (size_t)g;  // (first, end) blocks of group g
  const int b0 = gmem(rg)[0], b1 = gmem(rg)[1];
  double re = 0.0, im = 0.0;
  for (int b = b0; b < b1; ++b) {
    const int i3 = 3 * gmem(bi)[b];
    const double* v = bval + 27 * (size_t)b + e9;
    const cplx<double> e0 = gload(e + i3), e1 = gload(e + i3 + 1), e2 = gload(e + i3 + 2);
    const double v0 = gmem(v)[0], v9 = gmem(v)[9], v18 = gmem(v)[18];
    const double sr = e0.re * v0 + e1.re * v9 + e2.re * v18;
    const double si = e0.im * v0 + e1.im * v9 + e2.im * v18;
    const long long num = (long long)m0 * gmem(bR2)[3 * b] * (G1 * G2) +
                          (long long)m1 * gmem(bR2)[3 * b + 1] * (G0 * G2) +
                          (long long)m2 * gmem(bR2)[3 * b + 2] * (G0 * G1);
    double c, sn;
    unit_phase(num, Gt, c, sn);  // e^{+2 pi i k.R2}
    re += sr * c - si * sn;
    im += sr * sn + si * c;
  }
  RZ* zp = reinterpret_cast<RZ*>(Z + idx);
  gmem(zp)[0] = (RZ)re;
  gmem(zp)[1] = (RZ)im;
}

template <typename RZ>
__global__ void k_cr_zg(cplx<RZ>* __restrict__ Z, const cplx<double>* __restrict__ E,
                        const int2* __restrict__ cgb, const int* __restrict__ bi, const int* __restrict__ bR2,
                        const double* __restrict__ bval, int n, int ng, int G0, int G1, int G2, int k) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * ng * 9) return;
  cr_zg_elem<RZ>(Z, E, cgb, bi, bR2, bval, n, ng, G0, G1, G2, k, idx);
}

// Realified eigenvector operands for every grid point, rows cr_row(i, c), K = ldk:
//   Ac[k]: A[i][a] = conj(eta_ki[a])  (GEMM 1, i = s'')
//   Ap[k]: A[i][a] = eta_ki[a]        (GEMM 2, i = s')
template <int P>
__global__ void k_cr_realify(typename Operand<P>::T* __restrict__ Ach, typename Operand<P>::T* __restrict__ Acl,
                             typename Operand<P>::T* __restrict__ Aph, typename Operand<P>::T* __restrict__ Apl,
                             const cplx<double>* __restrict__ E, int nk, int n, int mrows, int ldk) {
  const int half = ldk / 2;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nk * mrows * half) return;
  const int a = (int)(idx % half);
  const int R = (int)((idx / half) % mrows);
  const int k = (int)(idx / ((long long)half * mrows));
  int i, c;
  if (P == KALDO_FP64) {
    i = 4 * (R >> 3) + (R & 3);
    c = (R >> 2) & 1;
  } else {
    i = R >> 1;
    c = R & 1;
  }
  cplx<double> e = {0.0, 0.0};
  if (i < n && a < n) e = E[((size_t)k * n + i) * n + a];
  // rows: c = 0 -> [Re, -Im], c = 1 -> [Im, Re] of A; conj flips the sign of Im
  const double pr0 = c == 0 ? e.re : e.im, pr1 = c == 0 ? -e.im : e.re;
  const double cr0 = c == 0 ? e.re : -e.im, cr1 = c == 0 ? e.im : e.re;
  const size_t o = ((size_t)k * mrows + R) * ldk + 2 * (size_t)a;
  store_operand<P>(Aph, Apl, o, pr0);
  store_operand<P>(Aph, Apl, o + 1, pr1);
  store_operand<P>(Ach, Acl, o, cr0);
  store_operand<P>(Ach, Acl, o + 1, cr1);
}

// idx = (s n + a') half + a'' split into its parts, with 32-bit divisions
// when idx fits (64-bit integer division is a long instruction sequence)
__device__ __forceinline__ void idx_split(long long idx, int half, int n, int& a2, long long& row, int& a1, int& s) {
  if (idx < 0x7fffffffLL) {
    const int ii = (int)idx;
    const int r = ii / half;
    a2 = ii - r * half;
    s = r / n;
    a1 = r - s * n;
    row = r;
  } else {
    row = idx / half;
    a2 = (int)(idx - row * half);
    s = (int)(row / n);
    a1 = (int)(row - (long long)s * n);
  }
}

// Step B into the realified B operand of GEMM 1, every element written (zeros
// outside the fc3 pairs and in the K padding): X[z][(s, a')][2 a'' + d] for
// partners p = p0 + z.  One thread serves up to ZT partners of the same
// element, so each Z value is read once per ZT partners.
template <int P, int ZT, typename RZ>
__device__ __forceinline__ void cr_x_elem(typename Operand<P>::T* __restrict__ Xh, typename Operand<P>::T* __restrict__ Xl,
                                          const cplx<RZ>* __restrict__ Z, const cplx<double>* __restrict__ PH,
                                          const int* __restrict__ cg_delta, const int* __restrict__ cg_order,
                                          const int4* __restrict__ cpair, const int* __restrict__ pairmap, int n,
                                          int N, int nk, int ng, int ldk, int p0, int zb, long long idx) {
  const int half = ldk / 2;
  const long long nn = (long long)n * n;
  int a2, a1, s;
  long long row;  // s * n + a'
  idx_split(idx, half, n, a2, row, a1, s);
  int cp = -1;
  if (a2 < n) cp = pairmap[(size_t)(a1 / 3) * N + a2 / 3];
  const int e9 = 3 * (a1 % 3) + a2 % 3;
  for (int z0 = 0; z0 < zb; z0 += ZT) {
    RZ re[ZT], im[ZT];
#pragma unroll
    for (int u = 0; u < ZT; ++u) re[u] = im[u] = (RZ)0;
    if (cp >= 0) {
      const int4 pr = cpair[cp];
      for (int q = pr.z; q < pr.w; ++q) {
        const int g = cg_order[q];
        const cplx<RZ> zz = Z[((size_t)s * ng + g) * 9 + e9];
        const cplx<double>* ph = PH + (size_t)cg_delta[g] * nk + p0 + z0;
#pragma unroll
        for (int u = 0; u < ZT; ++u) {
          if (z0 + u < zb) {
            const RZ fr = (RZ)ph[u].re, fi = (RZ)ph[u].im;
            re[u] += fr * zz.re - fi * zz.im;
            im[u] += fr * zz.im + fi * zz.re;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < ZT; ++u)
      if (z0 + u < zb)
        store_operand2<P>(Xh, Xl, ((size_t)(z0 + u) * nn + row) * ldk + 2 * (size_t)a2, (double)re[u], (double)im[u]);
  }
}

template <int P, int ZT, typename RZ>
__global__ void k_cr_x(typename Operand<P>::T* __restrict__ Xh, typename Operand<P>::T* __restrict__ Xl,
                       const cplx<RZ>* __restrict__ Z, const cplx<double>* __restrict__ PH,
                       const int* __restrict__ cg_delta, const int* __restrict__ cg_order,
                       const int4* __restrict__ cpair, const int* __restrict__ pairmap, int n, int N, int nk, int ng,
                       int ldk, int p0, int zb) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * n * (ldk / 2)) return;
  cr_x_elem<P, ZT, RZ>(Xh, Xl, Z, PH, cg_delta, cg_order, cpair, pairmap, n, N, nk, ng, ldk, p0, zb, idx);
}

// Step B as cr_x_elem, for the partners zc .. zc + zn of the batch with their
// phases staged in LDS: phs[d * ZC + u] = e^{2 pi i p.Delta_d} for p = p0 +
// zc + u (written by the caller).
template <int P, int ZT, typename RZ>
__device__ __forceinline__ void cr_x_elem_lds(typename Operand<P>::T* __restrict__ Xh,
                                              typename Operand<P>::T* __restrict__ Xl,
                                              const cplx<RZ>* __restrict__ Z, const cplx<RZ>* __restrict__ phs,
                                              int ZC, const int* __restrict__ cg_delta,
                                              const int* __restrict__ cg_order, const int4* __restrict__ cpair,
                                              const int* __restrict__ pairmap, int n, int N, int ng, int ldk, int zc,
                                              int zn, long long idx) {
  const int half = ldk / 2;
  const long long nn = (long long)n * n;
  int a2, a1, s;
  long long row;  // s * n + a'
  idx_split(idx, half, n, a2, row, a1, s);
  int cp = -1;
  if (a2 < n) cp = gmem(pairmap)[(size_t)(a1 / 3) * N + a2 / 3];
  const int e9 = 3 * (a1 % 3) + a2 % 3;
  for (int z0 = 0; z0 < zn; z0 += ZT) {
    RZ re[ZT], im[ZT];
#pragma unroll
    for (int u = 0; u < ZT; ++u) re[u] = im[u] = (RZ)0;
    if (cp >= 0) {
      // (z, w) of cpair[cp]: the range of this block pair's groups in cg_order
      const int* prw = reinterpret_cast<const int*>(cpair) + 4 * (size_t)cp;
      const int q0 = gmem(prw)[2], q1 = gmem(prw)[3];
      for (int q = q0; q < q1; ++q) {
        const int g = gmem(cg_order)[q];
        const cplx<RZ> zz = gload(Z + ((size_t)s * ng + g) * 9 + e9);
        const cplx<RZ>* ph = phs + (size_t)gmem(cg_delta)[g] * ZC + z0;
#pragma unroll
        for (int u = 0; u < ZT; ++u) {
          const RZ fr = ph[u].re, fi = ph[u].im;
          re[u] += fr * zz.re - fi * zz.im;
          im[u] += fr * zz.im + fi * zz.re;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < ZT; ++u)
      if (z0 + u < zn)
        store_operand2<P>(Xh, Xl, ((size_t)(zc + z0 + u) * nn + row) * ldk + 2 * (size_t)a2, (double)re[u],
                          (double)im[u]);
  }
}

// the realified pair h (0, 1) of a lane's 4 accumulator rows inside a 16-row tile at row m
template <int P>
__device__ __forceinline__ int cr_pair_mode(int m, int lane, int h) {
  return P == KALDO_FP64 ? (m >> 1) + (lane >> 4) + 4 * h : (m >> 1) + 2 * (lane >> 4) + h;
}

// GEMM 1 epilogue: store Y^T as the realified B operand of GEMM 2,
// Y[z][(s, s'')][2 a' + c] from output row pair s'' and column (s, a').
template <int P>
struct EpiStoreY {
  typename Operand<P>::T* yh;
  typename Operand<P>::T* yl;
  long long yz;  // elements per batch item
  long long ncol;
  int n, ldk;

  template <int Q, int FM, int FN>
  __device__ __forceinline__ void apply(typename Operand<Q>::Acc (&acc)[FM][FN], const TileAt& at, char*) const {
#pragma unroll
    for (int q = 0; q < FN; ++q) {
      const long long col = at.c0 + 16 * q + (at.lane & 15);
      if (col >= ncol) continue;
      // col < n^2 fits in 32 bits: 32-bit division
      const int ci = (int)col;
      const int s = ci / n, a1 = ci - s * n;
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = cr_pair_mode<Q>(at.m0 + 16 * a, at.lane, h);
          if (i < n) {
            const size_t o = (size_t)at.z * yz + ((size_t)s * n + i) * ldk + 2 * (size_t)a1;
            store_operand2<Q>(yh, yl, o, (double)acc[a][q][2 * h], (double)acc[a][q][2 * h + 1]);
          }
        }
    }
  }
};

// GEMM 2 epilogue: linewidth weights of V[s'][s''] for first mode (k, s), per
// column (s, s'') summed over the rows s':
//   |V|^2 / (w' w'') * [ g+ (n' - n'') + 1/2 g- (1 + n' + n'') ]
// with g+- the shape of the delta of kind DK.
template <int NT, int DK>
struct EpiCrystal {
  const double *OM, *IW, *OCC;  // [s][k], [s][k], [t][s][k]
  const int* kmap;              // index of k + p for p = p0 + z
  double* partial;              // [z][m_tiles][ncol][nT]
  long long ncol;               // n * n
  int n, nk, nT, k, p0, m_tiles;
  double rs;                    // 1 / (scale of the delta)
  const double* UT = nullptr;   // adaptive widths: scaled velocity projections [s][3][k] (kDeltaGaussAdaptive)
  static constexpr bool kAllShapes = DK == KALDO_DELTA_GAUSS;
  static constexpr bool kAdapt = DK == kDeltaGaussAdaptive;
  // the Lorentzian has no cut; adaptive widths have no common one
  static constexpr bool kSkipEmpty = DK == KALDO_DELTA_GAUSS || DK == KALDO_DELTA_TRIANGLE;

  // Every element of block tile (mt, nt) of partner z beyond the delta's cut:
  // frequencies ascend with the mode index at every grid point, rows hold the
  // (Re, Im) pairs of modes s' in [mt BM / 2, (mt + 1) BM / 2), columns (s, s'').
  template <int P, int FM, int FN>
  __device__ bool tile_empty(int, int nt, int z, int r0) const {
    constexpr int BM = 32 * FM, BN = 32 * FN;
    const int m0 = r0 / 2;
    if (m0 >= n) return true;
    const int p = p0 + z, kk = gmem(kmap)[z];
    const double a = gmem(OM)[(size_t)m0 * nk + p] * rs, b = gmem(OM)[(size_t)(min(n, m0 + BM / 2) - 1) * nk + p] * rs;
    const double W = sqrt(delta_cut<P>(DK)) * (1.0 + 1e-9) + 1e-9;
    const long long c1 = min(ncol, (long long)nt * BN + BN) - 1;
    for (long long c = (long long)nt * BN; c <= c1;) {
      const int s = (int)c / n;  // c < n^2
      const long long ce = min(c1, (long long)(s + 1) * n - 1);
      const double ws = gmem(OM)[(size_t)s * nk + k] * rs;
      const double lo = gmem(OM)[(size_t)(c - (long long)s * n) * nk + kk] * rs;
      const double hi = gmem(OM)[(size_t)(ce - (long long)s * n) * nk + kk] * rs;
      if (ws - hi + a < W && ws - lo + b > -W) return false;  // w + w' - w''
      if (ws - hi - b < W && ws - lo - a > -W) return false;  // w - w' - w''
      c = ce + 1;
    }
    return true;
  }
  template <int P, int FM, int FN>
  __device__ void clear_tile(int mt, int nt, int z) const {
    const long long first = (long long)nt * 32 * FN;
    for (int i = threadIdx.x; i < 32 * FN * nT; i += blockDim.x) {
      const int col = i / nT, t = i % nT;
      if (first + col < ncol) gmem(partial)[(((size_t)z * m_tiles + mt) * ncol + first + col) * nT + t] = 0.0;
    }
  }

  template <int P, int FM, int FN>
  __device__ __forceinline__ void apply(typename Operand<P>::Acc (&acc)[FM][FN], const TileAt& at,
                                        char* lds) const {
    using R = typename std::conditional<P == KALDO_FP64, double, float>::type;
    constexpr double cut = delta_cut<P>(DK);
    const int p = p0 + at.z;
    const int kk = gmem(kmap)[at.z];
    // column data: w - w'' (first mode minus k+p mode), 1/w'', n''
    double dcol[FN];
    R iw2[FN], n2[FN][NT], o[FN][NT];
    R uq[kAdapt ? FN : 1][3];  // adaptive widths: (k + p, s'')
#pragma unroll
    for (int q = 0; q < FN; ++q) {
      const long long col = at.c0 + 16 * q + (at.lane & 15);
      const bool cv = col < ncol;
      const int ci = cv ? (int)col : 0;  // < n^2: 32-bit division
      const int s = ci / n;
      const int s2 = ci - s * n;
      // unconditional loads of valid addresses, then selects: no branches
      // (and no wait for each load at their joins)
      dcol[q] = (gmem(OM)[(size_t)s * nk + k] - gmem(OM)[(size_t)s2 * nk + kk]) * rs;
      const R iwv = (R)gmem(IW)[(size_t)s2 * nk + kk];
      iw2[q] = cv ? iwv : (R)0;
      if constexpr (kAdapt) {
#pragma unroll
        for (int a = 0; a < 3; ++a) uq[q][a] = (R)gmem(UT)[((size_t)s2 * 3 + a) * nk + kk];
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        // (one temperature: nT = 1, the load needs no guard)
        n2[q][t] = NT == 1 || t < nT ? (R)gmem(OCC)[((size_t)t * n + s2) * nk + kk] : (R)0;
        o[q][t] = 0;
      }
    }
    // row data of the lane's two (Re, Im) pairs in every row fragment: w',
    // 1/w', n'; with one temperature all of it is loaded before any use, so
    // that the loads are in flight together instead of one fragment at a time
    constexpr int FA = NT == 1 && !kAdapt ? FM : 1;
    double w1a[FA][2];
    R iw1a[FA][2], n1a[FA][2][NT];
    const auto rows = [&](int a, double (&w1)[2], R (&iw1)[2], R (&n1)[2][NT], R (&up)[kAdapt ? 2 : 1][3]) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = cr_pair_mode<P>(at.m0 + 16 * a, at.lane, h);
        const int ic = i < n ? i : n - 1;
        w1[h] = gmem(OM)[(size_t)ic * nk + p] * rs;
        const R iwv = (R)gmem(IW)[(size_t)ic * nk + p];
        iw1[h] = i < n ? iwv : (R)0;
        if constexpr (kAdapt) {
#pragma unroll
          for (int c = 0; c < 3; ++c) up[h][c] = (R)gmem(UT)[((size_t)ic * 3 + c) * nk + p];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
          n1[h][t] = NT == 1 || t < nT ? (R)gmem(OCC)[((size_t)t * n + ic) * nk + p] : (R)0;
      }
    };
    if constexpr (FA > 1) {
      R up0[1][3];
#pragma unroll
      for (int a = 0; a < FM; ++a) rows(a, w1a[a], iw1a[a], n1a[a], up0);
    }
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      double w1[2];
      R iw1[2], n1[2][NT];
      R up[kAdapt ? 2 : 1][3];  // adaptive widths: (p, s')
      if constexpr (FA > 1) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          w1[h] = w1a[a][h];
          iw1[h] = iw1a[a][h];
#pragma unroll
          for (int t = 0; t < NT; ++t) n1[h][t] = n1a[a][h][t];
        }
      } else {
        rows(a, w1, iw1, n1, up);
      }
#pragma unroll
      for (int q = 0; q < FN; ++q) {
        // a 16 x 16 sub-tile with every element outside the delta's cutoff adds nothing
        if constexpr (!kAdapt) {
          bool need = false;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const double xp = dcol[q] + w1[h], xm = dcol[q] - w1[h];
            need = need || fmin(xp * xp, xm * xm) < cut;
          }
          if (__ballot(need) == 0) continue;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const R vr = (R)acc[a][q][2 * h], vi = (R)acc[a][q][2 * h + 1];
          const R v2 = (vr * vr + vi * vi) * iw1[h] * iw2[q];
          R gp, gm;
          if constexpr (kAdapt) {
            // widths sigma_min rho: rho = max(1, |u' - u''|) (absorption), max(1, |u' + u''|) (decay)
            R dp = 0, dm = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const R x = up[h][c] - uq[q][c], y = up[h][c] + uq[q][c];
              dp += x * x;
              dm += y * y;
            }
            const R ip = (R)1 / sqrt(dp > (R)1 ? dp : (R)1), im = (R)1 / sqrt(dm > (R)1 ? dm : (R)1);
            gp = delta_shape<R, KALDO_DELTA_GAUSS>((dcol[q] + w1[h]) * (double)ip) * ip;
            gm = delta_shape<R, KALDO_DELTA_GAUSS>((dcol[q] - w1[h]) * (double)im) * im;
          } else {
            gp = delta_shape<R, DK>(dcol[q] + w1[h]);
            gm = delta_shape<R, DK>(dcol[q] - w1[h]);
          }
          const R hh = (R)0.5 * gm, a1 = gp + hh, a2 = hh - gp;
#pragma unroll
          for (int t = 0; t < NT; ++t) o[q][t] += v2 * (hh + n1[h][t] * a1 + n2[q][t] * a2);
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
    column_flush<FN, NT>(lds, partial + (((size_t)at.z * m_tiles + at.mt) * ncol + first) * nT, ncol - first, nT);
  }
};

// Sum of partial over batch items, row tiles and s'' for one (s, t), by a
// 256-thread block (fixed order); the result is valid in thread 0.
__device__ __forceinline__ double cr_collect_sum(const double* __restrict__ partial, int n, int nT, int m_tiles,
                                                 int zb, int s, int t, double* red) {
  const long long nn = (long long)n * n;
  double v = 0.0;
  for (int z = 0; z < zb; ++z)
    for (int mt = 0; mt < m_tiles; ++mt)
      for (int s2 = threadIdx.x; s2 < n; s2 += 256)
        v += gmem(partial)[(((size_t)z * m_tiles + mt) * nn + (size_t)s * n + s2) * nT + t];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// gacc[t][s] (+)= sum over batch items, row tiles and s'' (one block per (s, t))
__global__ void k_cr_collect(double* __restrict__ gacc, const double* __restrict__ partial, int n, int nT,
                             int m_tiles, int zb, int first) {
  __shared__ double red[256];
  const int s = blockIdx.x, t = blockIdx.y;
  const double v = cr_collect_sum(partial, n, nT, m_tiles, zb, s, t, red);
  if (threadIdx.x == 0) gacc[(size_t)t * n + s] = (first ? 0.0 : gacc[(size_t)t * n + s]) + v;
}

// graw[t][k][s] = C / w_ks * gacc[t][s], stored at k and at km = -k (time
// reversal) where these lie in the k range [klo, khi)
__global__ void k_cr_finish(double* __restrict__ graw, const double* __restrict__ gacc,
                            const double* __restrict__ IW, int n, int nk, int nT, int k, int km, int klo, int khi,
                            double C) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * nT) return;
  const int s = idx % n, t = idx / n;
  const double v = C * IW[(size_t)s * nk + k] * gacc[(size_t)t * n + s];
  if (k >= klo && k < khi) graw[((size_t)t * nk + k) * n + s] = v;
  if (km >= klo && km < khi) graw[((size_t)t * nk + km) * n + s] = v;
}

// kmap[k][p] = index of k + p on the grid
__global__ void k_cr_kmap(int* __restrict__ kmap, int nk, int G0, int G1, int G2) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nk * nk) return;
  const int k = (int)(idx / nk), p = (int)(idx % nk);
  const int km0 = k / (G1 * G2), km1 = (k / G2) % G1, km2 = k % G2;
  const int pm0 = p / (G1 * G2), pm1 = (p / G2) % G1, pm2 = p % G2;
  kmap[idx] = ((km0 + pm0) % G0 * G1 + (km1 + pm1) % G1) * G2 + (km2 + pm2) % G2;
}

__device__ __forceinline__ void cr_set_average_elem(double* __restrict__ gamma, const double* __restrict__ graw,
                                                    const int* __restrict__ setid, int n, int nk, long long idx) {
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

__global__ void k_cr_set_average(double* __restrict__ gamma, const double* __restrict__ graw,
                                 const int* __restrict__ setid, int n, int nk, int nT) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * nk * nT) return;
  cr_set_average_elem(gamma, graw, setid, n, nk, idx);
}

kaldo_status launch_set_average(kaldo_ctx ctx, double* gamma, const double* graw, int nT) {
  const int n = ctx->nm, nk = ctx->nk;
  hipLaunchKernelGGL(k_cr_set_average, dim3(blocks_for((long long)n * nk * nT, 256)), dim3(256), 0, ctx->stream,
                     gamma, graw, ctx->d_setid.as<int>(), n, nk, nT);
  KALDO_HIP(ctx, hipGetLastError());
  return KALDO_OK;
}

kaldo_status run_crystal_tables(kaldo_ctx ctx, double** OM, double** IW, double** OCC, cplx<double>** PH);

// lo plane of an operand at an offset (BF16X3 only; null otherwise)
template <int P>
__device__ __forceinline__ const void* S_lo(const void* lo, size_t off) {
  if constexpr (Operand<P>::split == 2) return static_cast<const typename Operand<P>::T*>(lo) + off;
  else return nullptr;
}

template <int P, class Epi>
static int cr_gemm(kaldo_ctx ctx, const std::string& key, const GemmOps& g, const Epi& e) {
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
static kaldo_status crystal_impl(kaldo_ctx ctx, double sigma_thz) {
  using T = typename Operand<P>::T;
  constexpr int S = Operand<P>::split;
  const int N = ctx->n_atoms, n = ctx->nm, nk = ctx->nk, nT = ctx->nT;
  const int KC = GemmChunk<P>::KC;
  const int ldk = (2 * n + KC - 1) / KC * KC;
  const int mrows = cr_rows<P>(n);
  const long long nn = (long long)n * n;
  const Fc3Layout& L = ctx->fc3;
  const int ng = std::max(L.n_cgroups, 1);
  hipStream_t st = ctx->stream;
  const int TB = 256;
  double *OM, *IW, *OCC;
  cplx<double>* PH;
  kaldo_status rs = run_crystal_tables(ctx, &OM, &IW, &OCC, &PH);
  if (rs != KALDO_OK) return rs;
  // partners per batch: X and Y of a batch sized to stay in the last-level cache
  const size_t per_z = 2 * (size_t)nn * ldk * S * sizeof(T);
  const int zb = (int)std::max<size_t>(1, std::min<size_t>((size_t)nk, ctx->xy_budget / per_z));
  const int mt_max = (mrows + 63) / 64;  // the smallest candidate block tile has 64 rows
  // d_A: [Ac | Ap | X | Y], planes hi then lo of each
  const size_t a_elems = (size_t)nk * mrows * ldk;
  const size_t xy_elems = (size_t)zb * nn * ldk;
  // a batch plan leaves X and Y out: the persistent kernel runs every crystal
  // in one shared pool (batch_persistent_prepare)
  const bool shared_xy = planning(ctx) && ctx->xy_shared;
  KALDO_HIP(ctx, ctx->d_A.ensure((2 * a_elems + (shared_xy ? 0 : 2 * xy_elems)) * S * sizeof(T)));
  T* Ach = ctx->d_A.as<T>();
  T* Acl = S == 2 ? Ach + a_elems : nullptr;
  T* Aph = Ach + a_elems * S;
  T* Apl = S == 2 ? Aph + a_elems : nullptr;
  T* Xh = Aph + a_elems * S;
  T* Xl = S == 2 ? Xh + xy_elems : nullptr;
  T* Yh = Xh + xy_elems * S;
  T* Yl = S == 2 ? Yh + xy_elems : nullptr;
  // d_scratch2: [Z | partial | gacc | graw | kmap]
  const size_t z_elems = (size_t)n * ng * 9;
  // step A indexes Z in 32 bits
  if (z_elems >= ((size_t)1 << 31))
    return fail(ctx, KALDO_EINVAL, "crystal path: too many fc3 cell-offset groups for the step-A tensor");
  const size_t part = (size_t)zb * mt_max * nn * nT;
  const size_t gacc_n = (size_t)nT * n;
  const size_t graw_n = (size_t)nT * nk * n;
  KALDO_HIP(ctx, ctx->d_scratch2.ensure(z_elems * sizeof(cplx<double>) + (part + gacc_n + graw_n) * sizeof(double) +
                                        (size_t)nk * nk * sizeof(int)));
  // Z is stored in RZ (FP64 for the FP64 path, FP32 otherwise) in a slot sized for FP64
  using RZ = typename std::conditional<P == KALDO_FP64, double, float>::type;
  cplx<RZ>* Z = ctx->d_scratch2.as<cplx<RZ>>();
  double* partial = reinterpret_cast<double*>(ctx->d_scratch2.as<cplx<double>>() + z_elems);
  double* gacc = partial + part;
  double* gr = gacc + gacc_n;
  int* kmap = reinterpret_cast<int*>(gr + graw_n);
  KALDO_HIP(ctx, ctx->d_gamma.ensure((size_t)nT * nk * n * sizeof(double)));
  // the K padding of Y (columns >= 2n) is never written by GEMM 1: clear once
  if (ldk > 2 * n && !shared_xy) {
    const kaldo_status fs = fill_zero(ctx, Yh, xy_elems * S * sizeof(T));
    if (fs != KALDO_OK) return fs;
  }
  hipLaunchKernelGGL((k_cr_realify<P>), dim3(blocks_for((long long)nk * mrows * (ldk / 2), TB)), dim3(TB), 0, st,
                     Ach, Acl, Aph, Apl, ctx->d_evec.as<cplx<double>>(), nk, n, mrows, ldk);
  hipLaunchKernelGGL(k_cr_kmap, dim3(blocks_for((long long)nk * nk, TB)), dim3(TB), 0, st, kmap, nk, ctx->grid[0],
                     ctx->grid[1], ctx->grid[2]);
  KALDO_HIP(ctx, hipGetLastError());
  const double sig = kTwoPi * sigma_thz;
  double dscale, dnorm;
  delta_scale(ctx->delta, sig, dscale, dnorm);
  const double C = kPi / 8.0 * kHbar * kEvUnit * kEvUnit * kEvUnit / nk * dnorm;
  const std::string shape = std::to_string(P) + "/" + std::to_string(n) + "/";
  // adaptive widths: Gaussian per process, sig the smallest (dscale and dnorm are sig's)
  const double* UT = nullptr;
  if (ctx->adaptive_scale > 0.0) {
    const kaldo_status as = adaptive_table(ctx, sig, &UT);
    if (as != KALDO_OK) return as;
  }
  if (planning(ctx)) {
    // everything the persistent batch kernel needs to run this crystal
    CrystalPlan& cp = ctx->cplan;
    cp = CrystalPlan{};
    cp.valid = 1;
    cp.precision = P;
    cp.n = n;
    cp.N = N;
    cp.nk = nk;
    cp.ng = ng;
    cp.nd = ctx->fc3.n_delta;
    cp.nT = nT;
    cp.ldk = ldk;
    cp.mrows = mrows;
    cp.zb = zb;
    cp.G0 = ctx->grid[0];
    cp.G1 = ctx->grid[1];
    cp.G2 = ctx->grid[2];
    cp.klo = k_lo(ctx);
    cp.khi = k_hi(ctx);
    cp.m_tiles2 = gemm_m_tiles<P>(0, mrows);
    cp.xy_elems = (long long)xy_elems;
    cp.C = C;
    cp.rs = 1.0 / dscale;
    cp.Z = Z;
    cp.Xh = shared_xy ? nullptr : Xh;
    cp.Xl = shared_xy ? nullptr : Xl;
    cp.Yh = shared_xy ? nullptr : Yh;
    cp.Yl = shared_xy ? nullptr : Yl;
    cp.Ach = Ach;
    cp.Acl = Acl;
    cp.Aph = Aph;
    cp.Apl = Apl;
    cp.E = ctx->d_evec.p;
    cp.cgb = L.d_cg_block.p;
    cp.bi = L.d_blk_i.p;
    cp.bR2 = L.d_blk_R2.p;
    cp.bval = L.d_blk_val.p;
    cp.PH = PH;
    cp.cg_delta = L.d_cg_delta.p;
    cp.cg_order = L.d_cg_order.p;
    cp.cpair = L.d_cpair.p;
    cp.pairmap = L.d_cpairmap.p;
    cp.kmap = kmap;
    cp.OM = OM;
    cp.IW = IW;
    cp.OCC = OCC;
    cp.partial = partial;
    cp.gacc = gacc;
    cp.graw = gr;
    cp.gamma = ctx->d_gamma.as<double>();
    cp.setid = ctx->d_setid.as<int>();
    // X and Y do not exist in this context (they come from the shared pool):
    // nothing below may launch on them, the autotuner's trial GEMMs included
    // (the persistent kernel uses fixed tile shapes); the first-mode points
    // are recorded for its rounds
    if (shared_xy) {
      int npts = 0;
      return upload_linewidth_points(ctx, &npts);
    }
  }
  // planning visits one first-mode point and the batches whose GEMM shapes differ
  const bool plan = planning(ctx);
  // the first-mode points to compute (one of each pair k, -k on the whole grid)
  int npts = 0;
  kaldo_status ks = upload_linewidth_points(ctx, &npts);
  if (ks != KALDO_OK) return ks;
  const std::vector<int> pts = ctx->klist_host;
  if (k_partial(ctx) && !plan) {
    const kaldo_status fs = fill_zero(ctx, gr, graw_n * sizeof(double));
    if (fs != KALDO_OK) return fs;
  }
  for (int ik = 0; ik < (plan ? 1 : npts); ++ik) {
    const int k = pts[ik];
    const int km = k_mirror(k, ctx->grid[0], ctx->grid[1], ctx->grid[2]);
    prof_begin(ctx);
    if (!plan)
      hipLaunchKernelGGL((k_cr_zg<RZ>), dim3(blocks_for((long long)z_elems, TB)), dim3(TB), 0, st, Z,
                       ctx->d_evec.as<cplx<double>>(), L.d_cg_block.as<int2>(), L.d_blk_i.as<int>(),
                       L.d_blk_R2.as<int>(), L.d_blk_val.as<double>(), n, ng, ctx->grid[0], ctx->grid[1],
                       ctx->grid[2], k);
    KALDO_HIP(ctx, hipGetLastError());
    prof_end(ctx, "step_a");
    for (int p0 = 0; p0 < nk; p0 += zb) {
      const int cnt = std::min(zb, nk - p0);
      if (plan && p0 != 0 && p0 + zb < nk) continue;
      prof_begin(ctx);
      if (!plan)
        hipLaunchKernelGGL((k_cr_x<P, 8, RZ>), dim3(blocks_for(nn * (ldk / 2), TB)), dim3(TB), 0, st, Xh, Xl,
                         Z, PH, L.d_cg_delta.as<int>(), L.d_cg_order.as<int>(), L.d_cpair.as<int4>(),
                         L.d_cpairmap.as<int>(), n, N, nk, ng, ldk, p0, cnt);
      KALDO_HIP(ctx, hipGetLastError());
      prof_end(ctx, "step_b");
      prof_begin(ctx);
      // GEMM 1: Y = conj(E_{k+p})^T X
      GemmOps g1{};
      g1.a_hi = Ach;
      g1.a_lo = Acl;
      g1.b_hi = Xh;
      g1.b_lo = Xl;
      g1.lda = g1.ldb = ldk;
      g1.a_z = (long long)mrows * ldk;
      g1.b_z = nn * ldk;
      g1.a_map = kmap + (size_t)k * nk + p0;
      g1.K = ldk;
      g1.kv = 2 * n;  // realified contraction over the n atoms' coordinates
      g1.nz = cnt;
      g1.m_valid = mrows;
      g1.c_valid = nn;
      EpiStoreY<P> e1{Yh, Yl, nn * ldk, nn, n, ldk};
      cr_gemm<P>(ctx, "cr1/" + shape + std::to_string(cnt), g1, e1);
      KALDO_HIP(ctx, hipGetLastError());
      // GEMM 2: V = E_p^T Y with the linewidth epilogue
      GemmOps g2 = g1;
      g2.a_hi = Aph + (size_t)p0 * mrows * ldk;
      g2.a_lo = S == 2 ? Apl + (size_t)p0 * mrows * ldk : nullptr;
      g2.b_hi = Yh;
      g2.b_lo = Yl;
      g2.a_map = nullptr;
      int v = 0;
      const std::string key2 = "cr2/" + shape + std::to_string(cnt) + "/" + std::to_string(nT) + "/" +
                               std::to_string(UT ? kDeltaGaussAdaptive : ctx->delta);
#define KALDO_EPI(NTV, DKV)                                                                                          \
  {                                                                                                             \
    EpiCrystal<NTV, DKV> e2{OM, IW, OCC, kmap + (size_t)k * nk + p0, partial, nn, n, nk, nT, k, p0, 0, 1.0 / dscale, UT}; \
    /* the partial layout depends on the row tiling of the variant that runs */                               \
    const int vt = autotune(ctx, key2, gemm_variants<P, decltype(e2)>(), 0, [&](int w) {                                           \
      e2.m_tiles = gemm_m_tiles<P>(w, mrows);                                                                   \
      gemm_launch<P>(w, g2, e2, st);                                                                            \
    });                                                                                                         \
    e2.m_tiles = gemm_m_tiles<P>(vt, mrows);                                                                    \
    prof_tally(ctx, g2);                                                                                        \
    if (!plan) gemm_launch<P>(vt, g2, e2, st);                                                                  \
    v = vt;                                                                                                     \
  }
#define KALDO_EPI_NT(DKV)               \
  {                                     \
    if (nT <= 1) KALDO_EPI(1, DKV)      \
    else if (nT <= 4) KALDO_EPI(4, DKV) \
    else KALDO_EPI(8, DKV)              \
  }
      if (UT) KALDO_EPI_NT(kDeltaGaussAdaptive)
      else if (ctx->delta == KALDO_DELTA_GAUSS) KALDO_EPI_NT(KALDO_DELTA_GAUSS)
      else if (ctx->delta == KALDO_DELTA_LORENTZ) KALDO_EPI_NT(KALDO_DELTA_LORENTZ)
      else KALDO_EPI_NT(KALDO_DELTA_TRIANGLE)
#undef KALDO_EPI_NT
#undef KALDO_EPI
      KALDO_HIP(ctx, hipGetLastError());
      prof_end(ctx, "project");
      if (plan) continue;
      hipLaunchKernelGGL(k_cr_collect, dim3(n, nT), dim3(256), 0, st, gacc, partial, n, nT,
                         gemm_m_tiles<P>(v, mrows), cnt, p0 == 0 ? 1 : 0);
      KALDO_HIP(ctx, hipGetLastError());
    }
    if (plan) continue;
    hipLaunchKernelGGL(k_cr_finish, dim3(blocks_for(n * nT, TB)), dim3(TB), 0, st, gr, gacc, IW, n, nk, nT, k, km,
                       k_lo(ctx), k_hi(ctx), C);
    KALDO_HIP(ctx, hipGetLastError());
  }
  if (plan) return KALDO_OK;
  hipLaunchKernelGGL(k_cr_set_average, dim3(blocks_for((long long)n * nk * nT, TB)), dim3(TB), 0, st,
                     ctx->d_gamma.as<double>(), gr, ctx->d_setid.as<int>(), n, nk, nT);
  KALDO_HIP(ctx, hipGetLastError());
  return KALDO_OK;
}

// ---- persistent batch kernel ----------------------------------------------------------
// One launch runs the linewidths of every planned many-branch crystal of a
// batch.  Its work queue is a table of rounds (crystal, first-mode point k,
// partners p0 .. p0 + cnt), the crystals in order of decreasing cost (points x
// N_k x n^4); each round takes the stages of the per-launch path (step A for a
// new k, step B, GEMM 1, GEMM 2 with the linewidth epilogue, the collection)
// as phases over all workgroups, separated by grid barriers.  The grid holds
// exactly the workgroups that fit on the device at once.  A barrier that waits
// longer than about two seconds (a workgroup that never became resident) sets
// an abort flag; every workgroup then leaves, and the host reports the error.
struct BatchRound {
  int c, k, km, p0, cnt, first, last, first_crystal;
};
struct GridSync {
  unsigned count, gen, abort, pad;
  unsigned long long flops;     // MFMA flops of the GEMM block tiles that ran (not skipped)
  unsigned long long phase[7];  // block 0's constant-rate clock ticks: step A with the collection
                                // and Y padding, step B, GEMM 1, GEMM 2, waits at the grid barrier
                                // after the GEMM 1 phase, set average, waits after the GEMM 2 phase
  unsigned long long t_begin;   // block 0's clock before the first round
  unsigned long long claims[5]; // chunks claimed so far by step B, step A, the collection, GEMM 1, GEMM 2
};

// Stage work handed out in chunks: workgroups claim chunk indices from the
// stage's counter until a claim comes back past the stage's nch chunks, so a
// workgroup that left the phase's GEMM tiles early takes more of the stage.
// Every workgroup makes exactly one claim past the end per stage, so after a
// stage the counter stands at base + nch + G in every workgroup's view, and
// the grid barriers between phases keep two uses of one counter apart.
// Elements per chunk: about four chunks per workgroup, between one and 16
// elements per thread (small stages keep every workgroup busy, large ones
// claim seldom).
__device__ __forceinline__ long long stage_chunk(long long cnt, int G) {
  long long ch = cnt / (4LL * G);
  ch = ch < 256 ? 256 : (ch > 4096 ? 4096 : ch);
  return (ch + 255) & ~255LL;
}

template <class F>
__device__ __forceinline__ void claimed(unsigned long long* ctr, unsigned long long& base, long long nch, int G,
                                        F&& f) {
  __shared__ long long s_chunk;
  for (;;) {
    if (threadIdx.x == 0) s_chunk = (long long)(atomicAdd(ctr, 1ull) - base);
    __syncthreads();
    const long long c = s_chunk;
    __syncthreads();
    if (c >= nch) break;
    f(c);
  }
  base += (unsigned long long)nch + (unsigned long long)G;
}

// block 0 adds the ticks since *t0 to phase p and restarts the clock
__device__ __forceinline__ void phase_mark(GridSync* gs, int b, unsigned long long& t0, int p) {
  if (b == 0 && threadIdx.x == 0) {
    const unsigned long long t = wall_clock64();
    gs->phase[p] += t - t0;
    t0 = t;
  }
}

// Returns true when the kernel is to be abandoned.
__device__ __forceinline__ bool grid_barrier(GridSync* gs, unsigned nblocks) {
  __shared__ unsigned s_abort;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned ab = __hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!ab) {
      const unsigned g = __hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();  // this block's writes (all its waves passed the block barrier) reach memory
      if (__hip_atomic_fetch_add(&gs->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == nblocks - 1) {
        __hip_atomic_store(&gs->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&gs->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        unsigned it = 0;
        while (__hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
          __builtin_amdgcn_s_sleep(4);
          if ((++it & 1023u) == 0) {
            if (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
              ab = 1;
              break;
            }
            if (it >= (1u << 23)) {  // ~2^23 x 256 cycles
              __hip_atomic_store(&gs->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              ab = 1;
              break;
            }
          }
        }
      }
      __threadfence();  // the other blocks' writes are visible from here on
    }
    s_abort = ab;
  }
  __syncthreads();
  return s_abort != 0;
}

// The tiles of one GEMM phase over the persistent grid, in chunks of up to 8
// consecutive logical tiles (a chunk of 8 holds the row tiles of two or three
// column panels, which share their operand panels in L2; phases with fewer
// than 4 G tiles get smaller chunks, and the last 2 G tiles go singly) that
// the workgroups claim one at a time (claimed(): a workgroup that finished
// early takes more).  Row tile mt has 32 rt_fm[mt] rows from row 32 rt_u0[mt] (tiles of
// several heights cover the 2n realified rows with little padding).
// FP32 tiles take 128-byte K chunks (gemm_tile's WD): the operands stream
// from HBM, and a 64-byte chunk's MFMAs were too short to cover the next
// chunk's loads.
template <int P>
struct BatchWide : std::integral_constant<bool, P == KALDO_FP32> {};

template <int P, int FN, class Epi>
__device__ __forceinline__ void gemm_persistent(GemmOps& g, const Epi& e, char* lds, int G, const CrystalPlan& C,
                                                unsigned long long* ctr, unsigned long long& base) {
  constexpr bool WD = BatchWide<P>::value;
  constexpr unsigned long long mult = P == KALDO_BF16X3 ? 3 : 1;
  g.m_tiles = C.m_tiles2;
  g.n_tiles = (int)((g.c_valid + 32 * FN - 1) / (32 * FN));
  g.group_m = g.m_tiles < 8 ? g.m_tiles : 8;
  g.group_n = g.n_tiles;
  const int total = g.m_tiles * g.n_tiles * g.nz;
  // fewer tiles per chunk when the phase has few: every workgroup gets some;
  // the last 2 G tiles (at most) go one at a time, so that the phase ends
  // within about one tile of its last workgroup
  int CH = total / (4 * G);
  CH = CH < 1 ? 1 : (CH > 8 ? 8 : CH);
  const int nbig = (total - (total < 2 * G ? total : 2 * G)) / CH;
  const int single0 = nbig * CH;
  claimed(ctr, base, nbig + (total - single0), G, [&](long long c) {
    const int t0 = c < nbig ? (int)c * CH : single0 + (int)(c - nbig);
    const int t1 = c < nbig ? t0 + CH : t0 + 1;
    for (int t = t0; t < t1; ++t) {
      int mt, nt, z;
      gemm_tile_coords(g, t, mt, nt, z);
      const int fm = C.rt_fm[mt], r0 = 32 * C.rt_u0[mt];
      g.tile_flops = 2ull * (32 * fm) * (32 * FN) * (unsigned long long)gemm_k_exec<P>(g) * mult;
      if constexpr (P == KALDO_FP64) {
        gemm_tile<P, 2, FN, Epi>(g, e, mt, nt, z, lds, r0);
      } else {
        if (fm == 4) gemm_tile<P, 4, FN, Epi, false, false, WD>(g, e, mt, nt, z, lds, r0);
        else if (fm == 3) gemm_tile<P, 3, FN, Epi, false, false, WD>(g, e, mt, nt, z, lds, r0);
        else gemm_tile<P, 2, FN, Epi, false, false, WD>(g, e, mt, nt, z, lds, r0);
      }
      __syncthreads();
    }
  });
}

// Columns of the persistent kernel's GEMM tiles: 32 FN = 128.
template <int P>
struct BatchShape {
  static constexpr int FN = 4;
};

// Row tiles covering the realified rows of a crystal: u units of 32 rows in
// tiles of 4 units (128 rows), the remainder in tiles of 3 or 2 units (FP32
// and BF16X3).  With 64-byte K chunks (BF16X3) a tile of 3 units did about
// 0.75-0.8 of the work per second of a tile of 4 on the 32-crystal batch, so
// there the remainder tiles pay only where the contraction is long (2n >= 256
// rows) or tiles of 4 alone would pad the rows by more than a quarter; with
// the 128-byte chunks of FP32 they always pay (216 rows: 128 + 96 instead of
// 2 x 128 took the 36-atom cells from 0.48 to 0.52 of the peak).  FP64 (tiles
// of 2 units: its accumulators are twice as wide) keeps equal tiles.
// KALDO_TUNE_FIXED keeps the eager calls' tile (4 units, FP64 2) for bitwise
// agreement with them.
static std::vector<int> batch_row_tiles(int precision, int mrows, bool fixed) {
  const int u = (mrows + 31) / 32;
  std::vector<int> f;
  const bool mixed = precision == KALDO_FP32 || mrows >= 256 || 4 * (128 * ((u + 3) / 4)) > 5 * mrows;
  if (precision == KALDO_FP64 || fixed || !mixed) {
    const int fm = precision == KALDO_FP64 ? 2 : 4;
    f.assign((u + fm - 1) / fm, fm);
    return f;
  }
  const int q4 = u / 4, rem = u % 4;
  if (rem == 0) {
    f.assign(q4, 4);
  } else if (rem == 3) {
    f.assign(q4, 4);
    f.push_back(3);
  } else if (rem == 2) {
    if (q4 >= 1) {
      f.assign(q4 - 1, 4);
      f.push_back(3);
      f.push_back(3);
    } else {
      f.push_back(2);
    }
  } else if (q4 >= 2) {
    f.assign(q4 - 2, 4);
    f.insert(f.end(), {3, 3, 3});
  } else if (q4 == 1) {
    f = {3, 2};
  } else {
    f = {2};
  }
  return f;
}

// The stages of one round, each over every workgroup of the grid (grid-stride
// elements or the XCD-aware tile runs of the GEMMs).
template <int P, int NT>
struct BatchStages {
  using T = typename Operand<P>::T;
  using RZ = typename std::conditional<P == KALDO_FP64, double, float>::type;
  using E1 = EpiStoreY<P>;
  using E2 = EpiCrystal<NT, KALDO_DELTA_GAUSS>;
  static constexpr int FN = BatchShape<P>::FN;
  const CrystalPlan* plans;
  const BatchRound* rounds;
  GridSync* gs;
  char* lds;
  int b, G;
  long long gtid, gthreads;
  int lds_bytes;

  // K padding of the crystal's Y layout in the shared pool (never written by
  // GEMM 1, read as zeros by GEMM 2)
  __device__ void zero_pad(const BatchRound& R) const {
    const CrystalPlan& C = plans[R.c];
    const int n = C.n, ldk = C.ldk;
    if (ldk <= 2 * n) return;
    const int pad = ldk - 2 * n;
    const long long rows = (long long)C.zb * n * n;
    for (long long i = gtid; i < rows * pad; i += gthreads) {
      const size_t o = (size_t)(i / pad) * ldk + 2 * n + (size_t)(i % pad);
      static_cast<T*>(C.Yh)[o] = T{};
      if constexpr (Operand<P>::split == 2) static_cast<T*>(C.Yl)[o] = T{};
    }
  }
  // step A of a new first-mode point, in claimed chunks
  __device__ void step_a(const BatchRound& R, unsigned long long& base) const {
    const CrystalPlan& C = plans[R.c];
    const long long cnt = (long long)C.n * C.ng * 9;
    const long long CH = stage_chunk(cnt, G);
    claimed(&gs->claims[1], base, (cnt + CH - 1) / CH, G, [&](long long c) {
      const long long e = c * CH + CH < cnt ? c * CH + CH : cnt;
      for (long long i = c * CH + threadIdx.x; i < e; i += blockDim.x)
        cr_zg_elem<RZ>(static_cast<cplx<RZ>*>(C.Z), static_cast<const cplx<double>*>(C.E),
                       static_cast<const int2*>(C.cgb), static_cast<const int*>(C.bi),
                       static_cast<const int*>(C.bR2), static_cast<const double*>(C.bval), C.n, C.ng, C.G0, C.G1,
                       C.G2, R.k, i);
    });
  }
  // step B of a round, in claimed chunks; the phases of as many partners as
  // fit (a multiple of 8) are staged in LDS per pass, in the compute precision
  __device__ void step_b(const BatchRound& R, unsigned long long& base) const {
    const CrystalPlan& C = plans[R.c];
    const long long cnt = (long long)C.n * C.n * (C.ldk / 2);
    const long long CH = stage_chunk(cnt, G);
    const int nd = C.nd;
    // partners per thread at a time (16 where the registers allow it: FP32 with
    // one temperature), and per LDS pass a multiple of that
    constexpr int ZT = P == KALDO_FP32 && NT == 1 ? 16 : 8;
    int ZC = (int)(lds_bytes / ((long long)nd * sizeof(cplx<RZ>))) & ~(ZT - 1);
    ZC = ZC < ((R.cnt + ZT - 1) & ~(ZT - 1)) ? ZC : ((R.cnt + ZT - 1) & ~(ZT - 1));
    cplx<RZ>* phs = reinterpret_cast<cplx<RZ>*>(lds);
    const cplx<double>* PH = static_cast<const cplx<double>*>(C.PH);
    claimed(&gs->claims[0], base, (cnt + CH - 1) / CH, G, [&](long long c) {
      const long long e = c * CH + CH < cnt ? c * CH + CH : cnt;
      for (int zc = 0; zc < R.cnt; zc += ZC) {
        const int zn = R.cnt - zc < ZC ? R.cnt - zc : ZC;
        for (int i = threadIdx.x; i < nd * zn; i += blockDim.x) {
          const int d = i / zn, u = i - d * zn;
          const cplx<double> v = PH[(size_t)d * C.nk + R.p0 + zc + u];
          phs[d * ZC + u] = {(RZ)v.re, (RZ)v.im};
        }
        __syncthreads();
        for (long long i = c * CH + threadIdx.x; i < e; i += blockDim.x)
          cr_x_elem_lds<P, ZT, RZ>(static_cast<T*>(C.Xh), static_cast<T*>(C.Xl), static_cast<const cplx<RZ>*>(C.Z),
                                  phs, ZC, static_cast<const int*>(C.cg_delta), static_cast<const int*>(C.cg_order),
                                  static_cast<const int4*>(C.cpair), static_cast<const int*>(C.pairmap), C.n, C.N,
                                  C.ng, C.ldk, zc, zn, i);
        __syncthreads();
      }
    });
  }
  __device__ GemmOps gemm1_ops(const BatchRound& R) const {
    const CrystalPlan& C = plans[R.c];
    const long long nn = (long long)C.n * C.n;
    GemmOps g{};
    g.a_hi = C.Ach;
    g.a_lo = C.Acl;
    g.b_hi = C.Xh;
    g.b_lo = C.Xl;
    g.lda = g.ldb = C.ldk;
    g.a_z = (long long)C.mrows * C.ldk;
    g.b_z = nn * C.ldk;
    g.a_map = C.kmap + (size_t)R.k * C.nk + R.p0;
    g.K = C.ldk;
    g.kv = 2 * C.n;
    g.nz = R.cnt;
    g.m_valid = C.mrows;
    g.c_valid = nn;
    g.tally = &gs->flops;
    return g;
  }
  __device__ void gemm1(const BatchRound& R, unsigned long long& base) const {
    const CrystalPlan& C = plans[R.c];
    const long long nn = (long long)C.n * C.n;
    GemmOps g = gemm1_ops(R);
    const E1 e{static_cast<T*>(C.Yh), static_cast<T*>(C.Yl), nn * C.ldk, nn, C.n, C.ldk};
    gemm_persistent<P, FN>(g, e, lds, G, C, &gs->claims[3], base);
  }
  __device__ void gemm2(const BatchRound& R, unsigned long long& base) const {
    const CrystalPlan& C = plans[R.c];
    const long long nn = (long long)C.n * C.n;
    GemmOps g = gemm1_ops(R);
    g.a_hi = static_cast<const T*>(C.Aph) + (size_t)R.p0 * C.mrows * C.ldk;
    g.a_lo = S_lo<P>(C.Apl, (size_t)R.p0 * C.mrows * C.ldk);
    g.b_hi = C.Yh;
    g.b_lo = C.Yl;
    g.a_map = nullptr;
    const E2 e{C.OM, C.IW, C.OCC, C.kmap + (size_t)R.k * C.nk + R.p0, C.partial, nn, C.n, C.nk, C.nT, R.k, R.p0,
               C.m_tiles2, C.rs};
    gemm_persistent<P, FN>(g, e, lds, G, C, &gs->claims[4], base);
  }
  // the partial sums of the round into gacc (first round of k: overwrite),
  // after the last round of k the raw linewidths of k and -k
  __device__ void collect(const BatchRound& R, unsigned long long& base) const {
    const CrystalPlan& C = plans[R.c];
    const int n = C.n, nk = C.nk;
    claimed(&gs->claims[2], base, (long long)n * C.nT, G, [&](long long st) {
      const int s = (int)st % n, t = (int)st / n;  // st < n nT
      const double v = cr_collect_sum(C.partial, n, C.nT, C.m_tiles2, R.cnt, s, t, reinterpret_cast<double*>(lds));
      if (threadIdx.x == 0) {
        double* ga = C.gacc + (size_t)t * n + s;
        const double acc = (R.first ? 0.0 : *ga) + v;
        *ga = acc;
        if (R.last) {
          const double w = C.C * C.IW[(size_t)s * nk + R.k] * acc;
          if (R.k >= C.klo && R.k < C.khi) C.graw[((size_t)t * nk + R.k) * n + s] = w;
          if (R.km >= C.klo && R.km < C.khi) C.graw[((size_t)t * nk + R.km) * n + s] = w;
        }
      }
      __syncthreads();
    });
  }
};

// The rounds run as a two-phase pipeline: phase X of round r holds GEMM 1 of
// r with step A of r + 1 (a new point), the collection of r - 1 and, at a new
// crystal, the zeroing of its Y padding; phase Y holds GEMM 2 of r with step
// B of r + 1.  Every pair of stages in one phase touches disjoint buffers
// (GEMM 1 reads X and writes Y; step A writes Z, read by step B one phase
// later; the collection reads the partial sums that GEMM 2 writes one phase
// later; step B writes X, read by GEMM 1 one phase later), so two grid
// barriers per round suffice.
// LDS bytes of the persistent kernel: the larger GEMM stage (row tiles of up
// to 128 rows), at least 2 KB for the collection's reduction
template <int P, int NT>
struct BatchLds {
  using S = BatchStages<P, NT>;
  static constexpr int FN = BatchShape<P>::FN;
  static constexpr bool WD = BatchWide<P>::value;
  static constexpr int L1 = GemmLds<P, 4, FN, typename S::E1, false, false, WD>::bytes,
                       L2 = GemmLds<P, 4, FN, typename S::E2, false, false, WD>::bytes;
  static constexpr int LM = L1 > L2 ? L1 : L2;
  static constexpr int bytes = LM > 2048 ? LM : 2048;
};

// Two waves per SIMD (the occupancy the grid is sized for) up to four
// temperatures: told so, the compiler schedules the FP64 kernel in fewer
// registers (228 -> 212 VGPRs, its launch 8 % faster); with eight
// temperatures the accumulators need more registers than that allows.
template <int P, int NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT <= 4 ? 2 : 1)))
    k_batch_persistent(const CrystalPlan* __restrict__ plans, int nplans, const BatchRound* __restrict__ rounds,
                       int nrounds, GridSync* __restrict__ gs, unsigned long long* __restrict__ rtimes) {
  using S = BatchStages<P, NT>;
  constexpr int FN = BatchShape<P>::FN;
  constexpr int LB = BatchLds<P, NT>::bytes;
  __shared__ __attribute__((aligned(16))) char lds[LB];
  const int G = (int)gridDim.x, b = (int)blockIdx.x;
  const S st{plans, rounds, gs, lds, b, G, (long long)b * 256 + threadIdx.x, (long long)G * 256, LB};
  // points outside a crystal's k range keep gamma = 0
  for (int c = 0; c < nplans; ++c) {
    const CrystalPlan& C = plans[c];
    if (C.klo > 0 || C.khi < C.nk) {
      const long long cnt = (long long)C.nT * C.nk * C.n;
      for (long long i = st.gtid; i < cnt; i += st.gthreads) C.graw[i] = 0.0;
    }
  }
  unsigned long long t0 = wall_clock64();
  if (b == 0 && threadIdx.x == 0) gs->t_begin = t0;
  // claim counters' bases: step B, step A, the collection, GEMM 1, GEMM 2
  unsigned long long base_b = 0, base_a = 0, base_c = 0, base_g1 = 0, base_g2 = 0;
  if (nrounds > 0) {
    st.step_a(rounds[0], base_a);
    if (grid_barrier(gs, G)) return;
    phase_mark(gs, b, t0, 0);
    st.step_b(rounds[0], base_b);
    if (grid_barrier(gs, G)) return;
    phase_mark(gs, b, t0, 1);
  }
  for (int r = 0; r < nrounds; ++r) {
    const BatchRound R = rounds[r];
    // phase X
    st.gemm1(R, base_g1);
    phase_mark(gs, b, t0, 2);
    if (R.first_crystal) st.zero_pad(R);
    if (r + 1 < nrounds && rounds[r + 1].first) st.step_a(rounds[r + 1], base_a);
    if (r > 0) st.collect(rounds[r - 1], base_c);
    phase_mark(gs, b, t0, 0);
    if (grid_barrier(gs, G)) return;
    phase_mark(gs, b, t0, 4);
    // phase Y
    st.gemm2(R, base_g2);
    phase_mark(gs, b, t0, 3);
    if (r + 1 < nrounds) st.step_b(rounds[r + 1], base_b);
    phase_mark(gs, b, t0, 1);
    if (grid_barrier(gs, G)) return;
    phase_mark(gs, b, t0, 6);
    // block 0's clock at the end of each round (per-crystal times for the profile)
    if (b == 0 && threadIdx.x == 0) rtimes[r] = t0;
  }
  if (nrounds > 0) {
    st.collect(rounds[nrounds - 1], base_c);
    if (grid_barrier(gs, G)) return;
  }
  // degenerate-set averages of every crystal
  for (int c = 0; c < nplans; ++c) {
    const CrystalPlan& C = plans[c];
    const long long cnt = (long long)C.n * C.nk * C.nT;
    for (long long i = st.gtid; i < cnt; i += st.gthreads) cr_set_average_elem(C.gamma, C.graw, C.setid, C.n, C.nk, i);
  }
  phase_mark(gs, b, t0, 5);
}

// MFMA flops of every GEMM block tile of the rounds (run or skipped), for the tally.
template <int P>
static double batch_dense_flops(const std::vector<CrystalPlan>& plans, const std::vector<BatchRound>& rounds) {
  constexpr int FN = BatchShape<P>::FN;
  double total = 0.0;
  for (const BatchRound& r : rounds) {
    const CrystalPlan& C = plans[r.c];
    double rows = 0.0;
    for (int i = 0; i < C.m_tiles2; ++i) rows += 32.0 * C.rt_fm[i];
    const double ntiles = (double)(((long long)C.n * C.n + 32 * FN - 1) / (32 * FN)) * r.cnt;
    GemmOps g{};
    g.K = C.ldk;
    g.kv = 2 * C.n;
    total += 2.0 * 2.0 * rows * (32 * FN) * ntiles * gemm_k_exec<P>(g) * (P == KALDO_BF16X3 ? 3.0 : 1.0);
  }
  return total;
}

template <int P, int NT>
static const void* batch_kernel() {
  return reinterpret_cast<const void*>(&k_batch_persistent<P, NT>);
}

static const void* batch_kernel_for(int precision, int nt) {
  if (precision == KALDO_FP64) return nt == 1 ? batch_kernel<KALDO_FP64, 1>() : nt == 4 ? batch_kernel<KALDO_FP64, 4>() : batch_kernel<KALDO_FP64, 8>();
  if (precision == KALDO_FP32) return nt == 1 ? batch_kernel<KALDO_FP32, 1>() : nt == 4 ? batch_kernel<KALDO_FP32, 4>() : batch_kernel<KALDO_FP32, 8>();
  return nt == 1 ? batch_kernel<KALDO_BF16X3, 1>() : nt == 4 ? batch_kernel<KALDO_BF16X3, 4>() : batch_kernel<KALDO_BF16X3, 8>();
}

kaldo_status batch_persistent_prepare(kaldo_ctx parent, const std::vector<kaldo_ctx>& subs, int precision) {
  parent->batch_nplans = parent->batch_nrounds = 0;
  std::vector<CrystalPlan> plans;
  std::vector<std::vector<int>> points;
  std::vector<double> cost;
  for (kaldo_ctx sub : subs) {
    plans.push_back(sub->cplan);
    points.push_back(sub->klist_host);
    const double n = sub->cplan.n;
    cost.push_back((double)sub->klist_host.size() * sub->cplan.nk * n * n * n * n);
  }
  if (plans.empty()) return KALDO_OK;
  std::vector<int> order(plans.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<CrystalPlan> sorted;
  std::vector<BatchRound> rounds;
  std::vector<int> round_handle;
  size_t pool = 0;  // elements of X (and of Y) of the largest crystal's partner batch
  for (int idx : order) {
    const CrystalPlan& cp = plans[idx];
    const int c = (int)sorted.size();
    sorted.push_back(cp);
    pool = std::max(pool, (size_t)cp.xy_elems);
    const int handle = (int)(std::find(parent->batch.begin(), parent->batch.end(), subs[idx]) - parent->batch.begin());
    bool fc = true;
    for (int k : points[idx]) {
      const int km = k_mirror(k, cp.G0, cp.G1, cp.G2);
      for (int p0 = 0; p0 < cp.nk; p0 += cp.zb) {
        const int cnt = std::min(cp.zb, cp.nk - p0);
        rounds.push_back(BatchRound{c, k, km, p0, cnt, p0 == 0 ? 1 : 0, p0 + cnt >= cp.nk ? 1 : 0, fc ? 1 : 0});
        round_handle.push_back(handle);
        fc = false;
      }
    }
  }
  // the shared X and Y pool: planes hi then lo of X, then of Y
  const int split = precision == KALDO_BF16X3 ? 2 : 1;
  const size_t esz = precision == KALDO_FP64 ? 8 : (precision == KALDO_FP32 ? 4 : 2);
  const size_t plane = (pool * esz + 255) & ~(size_t)255;
  KALDO_HIP(parent, parent->d_batch_xy.ensure(2 * split * plane));
  char* xy = parent->d_batch_xy.as<char>();
  // KALDO_TUNE_FIXED keeps the fixed tile shape of eager calls (variant 0), so
  // that batch and eager results agree bit for bit
  const bool fixed = parent->tuning == KALDO_TUNE_FIXED;
  // step B stages the phases of 16 partners for every cell offset Delta in LDS
  const int lds_bytes = precision == KALDO_FP64 ? BatchLds<KALDO_FP64, 1>::bytes
                        : precision == KALDO_FP32 ? BatchLds<KALDO_FP32, 1>::bytes
                                                  : BatchLds<KALDO_BF16X3, 1>::bytes;
  const size_t ph_bytes = precision == KALDO_FP64 ? 16 : 8;
  for (CrystalPlan& cp : sorted) {
    if ((size_t)cp.nd * 16 * ph_bytes > (size_t)lds_bytes)
      return fail(parent, KALDO_EINVAL, "persistent batch kernel: too many fc3 cell offsets for its LDS");
    const std::vector<int> fms = batch_row_tiles(precision, cp.mrows, fixed);
    // the partial sums were sized for tiles of 64 rows
    if ((int)fms.size() > 32 || (int)fms.size() > (cp.mrows + 63) / 64)
      return fail(parent, KALDO_EINVAL, "persistent batch kernel: too many row tiles for a crystal");
    cp.m_tiles2 = (int)fms.size();
    int u0 = 0;
    for (size_t i = 0; i < fms.size(); ++i) {
      cp.rt_fm[i] = (unsigned char)fms[i];
      cp.rt_u0[i] = (unsigned char)u0;
      u0 += fms[i];
    }
    cp.Xh = xy;
    cp.Xl = split == 2 ? xy + plane : nullptr;
    cp.Yh = xy + split * plane;
    cp.Yl = split == 2 ? xy + 3 * plane : nullptr;
  }
  const size_t pb = (sorted.size() * sizeof(CrystalPlan) + 255) & ~(size_t)255;
  const size_t rb = (rounds.size() * sizeof(BatchRound) + 255) & ~(size_t)255;
  const size_t tb = (rounds.size() * sizeof(unsigned long long) + 255) & ~(size_t)255;
  KALDO_HIP(parent, parent->d_batch.ensure(pb + rb + 256 + tb));
  char* base = parent->d_batch.as<char>();
  KALDO_HIP(parent, hipMemcpy(base, sorted.data(), sorted.size() * sizeof(CrystalPlan), hipMemcpyHostToDevice));
  KALDO_HIP(parent, hipMemcpy(base + pb, rounds.data(), rounds.size() * sizeof(BatchRound), hipMemcpyHostToDevice));
  int nT = sorted[0].nT;
  const int nt = nT <= 1 ? 1 : (nT <= 4 ? 4 : 8);
  // the grid: every workgroup that fits on the device at once, a multiple of 8 (one run per XCD)
  int per_cu = 0, cus = 0;
  KALDO_HIP(parent, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel_for(precision, nt), 256, 0));
  KALDO_HIP(parent, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, parent->device));
  const int grid = (per_cu * cus) & ~7;
  if (grid < 8) return fail(parent, KALDO_EDEVICE, "persistent batch kernel: no resident workgroups");
  parent->batch_grid = grid;
  parent->batch_nplans = (int)sorted.size();
  parent->batch_nrounds = (int)rounds.size();
  parent->batch_precision = precision;
  parent->batch_nt = nt;
  parent->batch_rounds_off = pb;
  parent->batch_sync_off = pb + rb;
  parent->batch_times_off = pb + rb + 256;
  parent->batch_round_handle = round_handle;
  parent->batch_dense = precision == KALDO_FP64    ? batch_dense_flops<KALDO_FP64>(sorted, rounds)
                        : precision == KALDO_FP32 ? batch_dense_flops<KALDO_FP32>(sorted, rounds)
                                                  : batch_dense_flops<KALDO_BF16X3>(sorted, rounds);
  return KALDO_OK;
}

kaldo_status batch_persistent_launch(kaldo_ctx parent) {
  if (parent->batch_nplans == 0) return KALDO_OK;
  char* base = parent->d_batch.as<char>();
  const CrystalPlan* plans = reinterpret_cast<const CrystalPlan*>(base);
  const BatchRound* rounds = reinterpret_cast<const BatchRound*>(base + parent->batch_rounds_off);
  GridSync* gs = reinterpret_cast<GridSync*>(base + parent->batch_sync_off);
  kaldo_status st = fill_zero(parent, gs, sizeof(GridSync));
  if (st != KALDO_OK) return st;
  const dim3 grid(parent->batch_grid), block(256);
  const int np = parent->batch_nplans, nr = parent->batch_nrounds;
  hipStream_t s = parent->stream;
  unsigned long long* rtimes = reinterpret_cast<unsigned long long*>(base + parent->batch_times_off);
#define KALDO_BP(PV, NTV) \
  hipLaunchKernelGGL((k_batch_persistent<PV, NTV>), grid, block, 0, s, plans, np, rounds, nr, gs, rtimes)
  const int nt = parent->batch_nt;
  if (parent->batch_precision == KALDO_FP64) {
    if (nt == 1) KALDO_BP(KALDO_FP64, 1); else if (nt == 4) KALDO_BP(KALDO_FP64, 4); else KALDO_BP(KALDO_FP64, 8);
  } else if (parent->batch_precision == KALDO_FP32) {
    if (nt == 1) KALDO_BP(KALDO_FP32, 1); else if (nt == 4) KALDO_BP(KALDO_FP32, 4); else KALDO_BP(KALDO_FP32, 8);
  } else {
    if (nt == 1) KALDO_BP(KALDO_BF16X3, 1); else if (nt == 4) KALDO_BP(KALDO_BF16X3, 4); else KALDO_BP(KALDO_BF16X3, 8);
  }
#undef KALDO_BP
  KALDO_HIP(parent, hipGetLastError());
  return KALDO_OK;
}

kaldo_status batch_persistent_check(kaldo_ctx parent) {
  if (parent->batch_nplans == 0) return KALDO_OK;
  GridSync h{};
  KALDO_HIP(parent, hipMemcpyAsync(&h, parent->d_batch.as<char>() + parent->batch_sync_off, sizeof(h),
                                   hipMemcpyDeviceToHost, parent->stream));
  KALDO_HIP(parent, hipStreamSynchronize(parent->stream));
  if (h.abort)
    return fail(parent, KALDO_EDEVICE,
                "persistent batch kernel: a grid barrier timed out (not every workgroup became resident); "
                "results are incomplete");
  if (parent->prof) {
    parent->prof_batch_executed += (double)h.flops;
    parent->prof_dense += parent->batch_dense;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, parent->device) == hipSuccess && khz > 0) {
      static const char* names[7] = {"batch_a_collect", "batch_step_b", "batch_gemm1", "batch_gemm2",
                                     "batch_wait_gemm1_phase", "batch_set_average", "batch_wait_gemm2_phase"};
      for (int p = 0; p < 7; ++p) {
        auto& e = parent->prof_tab[names[p]];
        e.total_ms += (double)h.phase[p] / (double)khz;
        e.launches += 1;
      }
      auto& w = parent->prof_tab["batch_barrier_wait"];
      w.total_ms += (double)(h.phase[4] + h.phase[6]) / (double)khz;
      w.launches += 1;
      // per crystal: the clock between the ends of consecutive rounds, summed
      // over the crystal's rounds ("batch_crystal_<handle>")
      const size_t nr = parent->batch_round_handle.size();
      std::vector<unsigned long long> t(nr);
      KALDO_HIP(parent, hipMemcpy(t.data(), parent->d_batch.as<char>() + parent->batch_times_off,
                                  nr * sizeof(unsigned long long), hipMemcpyDeviceToHost));
      std::map<int, double> per;
      unsigned long long prev = h.t_begin;
      for (size_t r = 0; r < nr; ++r) {
        per[parent->batch_round_handle[r]] += (double)(t[r] - prev) / (double)khz;
        prev = t[r];
      }
      for (const auto& kv : per) {
        auto& e = parent->prof_tab["batch_crystal_" + std::to_string(kv.first)];
        e.total_ms += kv.second;
        e.launches += 1;
      }
    }
  }
  return KALDO_OK;
}

kaldo_status run_linewidths_crystal(kaldo_ctx ctx, double sigma_thz, int precision) {
  if (precision == KALDO_FP64) return crystal_impl<KALDO_FP64>(ctx, sigma_thz);
  if (precision == KALDO_FP32) return crystal_impl<KALDO_FP32>(ctx, sigma_thz);
  return crystal_impl<KALDO_BF16X3>(ctx, sigma_thz);
}

}  // namespace kaldo
