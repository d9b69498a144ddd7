// A real MFMA GEMM core shared by the projection paths:
//
//   C[m][c] = sum_k A[m][k] * B[c][k]          (both operands K-contiguous rows)
//
// with a caller-supplied epilogue that consumes the accumulator tile in
// registers (so C never reaches memory unless the epilogue stores it).
//
// Tiling for gfx950: 256 threads = 4 wavefronts in a 2 x 2 grid; a wavefront
// owns (16 FM) x (16 FN) outputs as FM x FN 16x16 MFMA tiles; the block tile
// is (32 FM) x (32 FN).  K is consumed in chunks of CB bytes per row (64 for
// BF16 and FP32: 32 bf16 or 16 fp32; 128 for FP64: 16 fp64), staged through a
// double-buffered LDS tile by 16-byte vector loads (one global_load_dwordx4 +
// one ds_write_b128 per slot); the next chunk is in flight in registers while
// the current one feeds the matrix cores.  The short chunk keeps the staging
// registers and the LDS tile small enough for two blocks per CU, so one
// block's loads and epilogue overlap the other's matrix work, and it keeps the
// K padding of short contractions small.  The LDS layout (see lds_off) keeps
// fragment reads and staging stores free of bank conflicts.
//
// Fragment reads: the MFMA sums over k, so any bijection between (lane group
// g = lane / 16, step j) and the k index of a chunk gives the same result as
// long as A and B use the same one.  FP32 and FP64 take k = 4 g + j within each
// 16-wide group, so a lane fetches the four k it needs for four consecutive
// 16x16x4 steps with one contiguous read; BF16 16x16x32 reads 8 consecutive k
// per lane as the instruction defines.
//
// Block order: workgroups are dealt round-robin to the 8 XCDs, each with its
// own L2.  The flat block id is remapped so that every XCD receives a
// contiguous run of logical tiles, ordered in groups of 8 row tiles with M
// fastest inside a group: the blocks resident on one XCD at a time cover a
// roughly square patch of tiles and read both operand panels from that XCD's L2.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "internal.h"
#include "mfma.h"

namespace kaldo {

struct GemmOps {
  const void* a_hi;
  const void* a_lo;   // lo planes: BF16X3 only
  const void* b_hi;
  const void* b_lo;
  long long lda, ldb; // row strides in elements
  long long a_z, b_z; // element offsets between batch items (blockIdx -> z)
  long long b_kb;     // K-blocked B (epilogues with kBlockBytes > 0): element (c, k)
                      // at (k / L) * b_kb + c * L + k % L, L = kBlockBytes of
                      // elements (ldb = L); otherwise B rows are K-contiguous
  const int* a_map;   // if set, batch item z takes A item a_map[z] (else z)
  int K;              // multiple of 16 elements (FP64 and the BF16X3 wide chunks: of the chunk)
  int kv;             // FP32: the contraction's own length, K - 16 < kv <= K, beyond which
                      // one operand is zero: the MFMA steps of the last 16 k stop at kv
                      // (rounded up to 4); 0 = K
  int m_tiles, n_tiles, nz; // filled in by the launcher from the tile shape
  int m_valid;        // rows of A (= output rows); loads beyond are clamped
  long long c_valid;  // rows of B (= output columns) per batch item
  // Flop tally of timed runs (null otherwise): each block tile that runs adds
  // tile_flops (its MFMA flops, filled in by the launcher) to *tally; the
  // launcher adds the flops of every tile it launches, run or skipped, to the
  // host value *tally_dense.
  unsigned long long* tally;
  double* tally_dense;
  unsigned long long tile_flops;
  int group_m;        // row tiles per group of the tile order (0: 8; clamped to m_tiles)
  int group_n;        // column panels per chunk of the tile order (0: all)
};

// The contraction length the MFMAs run over (FP32 stops at kv, rounded up to 4).
template <int P>
__host__ __device__ inline int gemm_k_exec(const GemmOps& g) {
  if (P != KALDO_FP32 || g.kv <= g.K - 16 || g.kv >= g.K) return g.K;
  return g.K - 16 + ((g.kv - (g.K - 16) + 3) / 4) * 4;
}

// Bytes of one row per K chunk, and the chunk in elements.
template <int P>
struct GemmChunk {
  static constexpr int CB = P == KALDO_FP64 ? 128 : 64;
  static constexpr int KC = CB / (int)sizeof(typename Operand<P>::T);
};

// An epilogue with kBlockBytes > 0 reads B in the K-blocked layout of GemmOps::b_kb.
template <class Epi, class = void>
struct BlockBytes : std::integral_constant<int, 0> {};
template <class Epi>
struct BlockBytes<Epi, std::void_t<decltype(Epi::kBlockBytes)>> : std::integral_constant<int, Epi::kBlockBytes> {};

// An epilogue with kSkipEmpty = true provides tile_empty<P, FM, FN>(mt, nt, z, r0),
// true when it would discard every output of block tile (mt, nt, z) whose first
// row is r0, and
// clear_tile<P, FM, FN>(mt, nt, z), which writes what it would have written for
// such a tile; the core then skips the tile's loads and MFMAs.
template <class Epi, class = void>
struct SkipEmpty : std::false_type {};
template <class Epi>
struct SkipEmpty<Epi, std::void_t<decltype(Epi::kSkipEmpty)>> : std::integral_constant<bool, Epi::kSkipEmpty> {};

// Coordinates of one block tile, handed to the epilogue.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// f(std::integral_constant<int, I>) for I = 0 .. N-1, unrolled at compile time
// (array indices are constants from the start, so staging arrays stay in registers)
template <class F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

struct TileAt {
  int mt, nt, z;      // tile indices and batch item
  int m0;             // first row of this wavefront's 16 FM rows
  long long c0;       // first column of this wavefront's 16 FN columns
  int lane, wm, wn;   // lane and wavefront position in the 2 x 2 grid
};

__device__ __forceinline__ uint4 lds_read16(const char* p) { return *reinterpret_cast<const uint4*>(p); }

// LDS byte offset of 16-byte slot `slot` of tile row `row`.  64-byte rows
// (the BF16 and FP32 chunks) are unpadded and XOR-swizzled: the physical slot
// is slot ^ f(row mod 16) with f = (0,0,1,1,3,3,2,2,1,1,0,0,2,2,3,3).  Of the
// layouts measured (16-byte row padding, this swizzle, slot-major groups with
// either staging order) it gave the fastest GEMMs: slot-major groups remove
// every bank conflict of the fragment reads but move them to the staging
// stores or cost coalescing of the staging loads.  128-byte rows (FP64) are
// padded by 16 bytes.
template <int CB>
__device__ __forceinline__ int lds_off(int row, int slot) {
  if constexpr (CB == 64) return row * 64 + ((slot ^ (int)((0xfa05af50u >> (2 * (row & 15))) & 3u)) << 4);
  else return row * (CB + 16) + slot * 16;
}

// LDS bytes of one block tile of k_gemm<P, FM, FN, Epi, BD, WC> (and of
// gemm_tile with wide double-buffered chunks, WD).
template <int P, int FM, int FN, class Epi, bool BD = false, bool WC = false, bool WD = false>
struct GemmLds {
  using T = typename Operand<P>::T;
  static constexpr int S = Operand<P>::split;
  static constexpr int BM = 32 * FM, BN = 32 * FN;
  static constexpr int CB = WC || WD ? 128 : GemmChunk<P>::CB;
  static constexpr int NBUF = WC ? 1 : 2;
  static constexpr int RB = CB == 64 ? 64 : CB + 16;
  static constexpr int ROWS = BM + (BD ? 0 : BN);
  static constexpr int BUF = S * ROWS * RB;
  static constexpr int bytes = NBUF * BUF;
};

// Block tile (mt, nt) of batch item z for the logical tile index `tile`:
// within an item, tiles go in groups of GM row tiles (group_m, 8 by default),
// M fastest inside a group: the blocks that run at the same time on one XCD
// then cover about GM x (64 / GM) tiles and share both operand panels in L2
// (with M fastest over all row tiles, every N tile streams the whole A panel
// again from beyond L2).  Optionally the column panels first go in chunks of
// GN (group_n); the ordering above then applies inside each chunk.
__device__ __forceinline__ void gemm_tile_coords(const GemmOps& g, int tile, int& mt, int& nt, int& z) {
  const int GM = g.group_m;
  const int per_z = g.m_tiles * g.n_tiles;
  z = tile / per_z;
  int tz = tile - z * per_z;
  const int GN = g.group_n;
  const int chunk = tz / (g.m_tiles * GN);
  tz -= chunk * g.m_tiles * GN;
  const int width = min(GN, g.n_tiles - chunk * GN);
  const int per_group = GM * width;
  const int first_m = (tz / per_group) * GM;
  const int gm = min(g.m_tiles - first_m, GM);
  const int tg = tz - (tz / per_group) * per_group;
  mt = first_m + tg % gm;
  nt = chunk * GN + tg / gm;
}

// One block tile (mt, nt, z): skip test, staged K loop and epilogue.  `lds`
// holds at least GemmLds<...>::bytes; the caller synchronises the block
// before reusing it for another tile.
// BD (BF16X3 only): B fragments go from global memory (L1/L2) straight to the
// wavefront's registers one chunk ahead, and LDS stages A alone.  The split
// operands make BF16X3 LDS-bound; this halves its LDS traffic.
// WC (BF16X3 only, K a multiple of 64): 128-byte chunks in a single LDS
// buffer, refilled between two barriers from registers loaded during the
// chunk's MFMAs.  Twice the MFMA work per barrier in the same LDS space as the
// double-buffered 64-byte chunks; faster on long contractions.
// WD (FP32 only, K a multiple of 16): 128-byte chunks (32 k) in two LDS
// buffers, so that the next chunk's loads have twice the MFMA time of a
// 64-byte chunk to arrive; a last chunk of 16 k runs its first half alone.
// The MFMAs run in the same order as with 64-byte chunks (bitwise the same
// result).
template <int P, int FM, int FN, class Epi, bool BD = false, bool WC = false, bool WD = false>
__device__ __forceinline__ void gemm_tile(const GemmOps& g, const Epi& epi, int mt, int nt, int z, char* lds,
                                          int rbase = -1) {
  using T = typename Operand<P>::T;
  using Acc = typename Operand<P>::Acc;
  constexpr int S = Operand<P>::split;
  static_assert(!BD || P == KALDO_BF16X3, "direct B fragments are a BF16X3 variant");
  static_assert(!WC || (P == KALDO_BF16X3 && !BD), "wide chunks are a BF16X3 variant with B in LDS");
  static_assert(!WD || P == KALDO_FP32, "wide double-buffered chunks are an FP32 variant");
  constexpr int BM = 32 * FM, BN = 32 * FN;
  constexpr int CB = WC || WD ? 128 : GemmChunk<P>::CB;
  constexpr int KCH = CB / (int)sizeof(T);    // elements per row chunk
  constexpr int RB = CB == 64 ? 64 : CB + 16; // LDS bytes per tile row (see lds_off)
  constexpr int SLOTS = CB / 16;              // 16-byte slots per row chunk
  constexpr int RPP = 256 / SLOTS;            // rows loaded per pass of the block
  constexpr int NA = (BM + RPP - 1) / RPP;    // passes for A (the last one partial unless RPP divides BM)
  constexpr int NB = BD ? 0 : BN / RPP;       // passes for B (none when B is direct)
  static_assert(BD || NB * RPP == BN, "B tile rows must be whole load passes");
  constexpr int ROWS = BM + (BD ? 0 : BN);
  constexpr int BUF = S * ROWS * RB;          // one buffer: all planes, A rows then B rows
  constexpr int EPT = 16 / (int)sizeof(T);    // elements per 16-byte slot
  // first row of the tile: row tile mt of equal tiles, unless the caller
  // places tiles of several heights (rbase)
  const int rb = rbase >= 0 ? rbase : mt * BM;
  if constexpr (SkipEmpty<Epi>::value) {
    // uniform across the block (block indices and operand-independent data only)
    if (epi.template tile_empty<P, FM, FN>(mt, nt, z, rb)) {
      epi.template clear_tile<P, FM, FN>(mt, nt, z);
      return;
    }
  }
  if (g.tally && threadIdx.x == 0) atomicAdd(g.tally, g.tile_flops);

  const int tid = (int)threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // 16-byte slot of the row chunk and first row of this thread's slots: each
  // quad of lanes loads one contiguous row chunk (coalesced global reads)
  const int slot = tid % SLOTS;
  const int row0 = tid / SLOTS;

  // global element offsets of this thread's load slots (rows clamped to existing ones)
  // element offset of B's k within a row (see GemmOps::b_kb); L divides the
  // chunk, so a chunk start and a slot offset inside the chunk add without carry
  constexpr int BKL = BlockBytes<Epi>::value / (int)sizeof(T);
  static_assert(BKL == 0 || (KCH % BKL == 0 && BKL % EPT == 0), "B blocks must tile the chunk");
  static_assert(!WD || BKL == 0, "wide double-buffered chunks read K-contiguous B rows");
  // WD: a half last chunk (K = 16 mod 32) loads its second half's slots from
  // the first half again (inside the row; those LDS slots are never read)
  const int kshift = WD ? (slot * EPT >= 16 ? 16 : 0) : 0;
  const auto kin = [&](int k0) -> int {
    if constexpr (WD) return k0 + slot * EPT < g.K ? k0 : k0 - kshift;
    else return k0;
  };
  const auto bk = [&](int k0) -> long long {
    if constexpr (BKL > 0) return (long long)(k0 / BKL) * g.b_kb + k0 % BKL;
    else return (long long)k0;
  };
  long long aoff[NA], boff[NB > 0 ? NB : 1];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    int row = rb + row0 + RPP * u;
    row = row < g.m_valid ? row : g.m_valid - 1;
    aoff[u] = (long long)(g.a_map ? g.a_map[z] : z) * g.a_z + (long long)row * g.lda + slot * EPT;
  }
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    long long row = (long long)nt * BN + row0 + RPP * u;
    row = row < g.c_valid ? row : g.c_valid - 1;
    boff[u] = (long long)z * g.b_z + row * g.ldb + bk(slot * EPT);
  }
  const T* ap[S];
  const T* bp[S];
  ap[0] = static_cast<const T*>(g.a_hi);
  bp[0] = static_cast<const T*>(g.b_hi);
  if constexpr (S == 2) {
    ap[S - 1] = static_cast<const T*>(g.a_lo);
    bp[S - 1] = static_cast<const T*>(g.b_lo);
  }

  // staging registers of the next chunk (declared per use, below; native
  // vectors, so that the copies stay register moves): rg[s][u],
  // u < NA for A rows, then NB for B rows
#define KALDO_GLOAD(K0)                                                                \
  static_for<S>([&](auto sc) __attribute__((always_inline)) {                                                         \
    constexpr int s_ = decltype(sc)::value;                                            \
    static_for<NA + NB>([&](auto uc) __attribute__((always_inline)) {                                                 \
      constexpr int u_ = decltype(uc)::value;                                          \
      if constexpr (u_ < NA)                                                           \
        rg[s_][u_] = *gmem(reinterpret_cast<const u32x4*>(ap[s_] + aoff[u_] + kin(K0))); \
      else                                                                             \
        rg[s_][u_] = *gmem(reinterpret_cast<const u32x4*>(bp[s_] + boff[u_ - NA] + bk(kin(K0)))); \
    });                                                                                \
  });
#define KALDO_SSTORE(BUFI)                                                             \
  static_for<S>([&](auto sc) __attribute__((always_inline)) {                                                         \
    constexpr int s_ = decltype(sc)::value;                                            \
    static_for<NA + NB>([&](auto uc) __attribute__((always_inline)) {                                                 \
      constexpr int u_ = decltype(uc)::value;                                          \
      const int row = (u_ < NA ? 0 : BM - RPP * NA) + row0 + RPP * u_;                 \
      if (u_ + 1 != NA || BM % RPP == 0 || row < BM)  /* rows of a partial last A pass */ \
        *reinterpret_cast<u32x4*>(lds + (BUFI) * BUF + lds_off<CB>(s_ * ROWS + row, slot)) = rg[s_][u_]; \
    });                                                                                \
  });

  Acc acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int c = 0; c < FN; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][c][r] = 0;

  const int arow = wm * 16 * FM + (lane & 15);
  const int brow = BM + wn * 16 * FN + (lane & 15);
  const int grp = lane >> 4;

  // direct B fragments: this lane's element offsets of its FN fragment rows
  long long bfo[BD ? FN : 1];
  bf16x8 bcur[BD ? FN : 1][2], bnx[BD ? FN : 1][2];
  if constexpr (BD) {
#pragma unroll
    for (int c = 0; c < FN; ++c) {
      long long row = (long long)nt * BN + wn * 16 * FN + 16 * c + (lane & 15);
      row = row < g.c_valid ? row : g.c_valid - 1;
      bfo[c] = (long long)z * g.b_z + row * g.ldb + bk(8 * grp);
    }
  }
#define KALDO_BLOAD(K0, DST)                                                                              \
  _Pragma("unroll") for (int c = 0; c < FN; ++c) {                                                      \
    _Pragma("unroll") for (int s = 0; s < 2; ++s) DST[c][s] =                                           \
        *gmem(reinterpret_cast<const bf16x8*>(bp[s] + bfo[c] + bk(K0)));                                 \
  }

  // WD: chunks of 32 k, the last one of 16 k when K = 16 mod 32
  const int nchunk = WD ? (g.K + KCH - 1) / KCH : g.K / KCH;
  const bool half_last = WD && (g.K % KCH) != 0;
  // FP32: MFMA steps of 4 k in the last 16 k (4: all of them)
  const int kvalid = g.kv > g.K - 16 && g.kv < g.K ? g.kv : g.K;
  const int tail_q = P == KALDO_FP32 ? (kvalid - (g.K - 16) + 3) / 4 : 4;
  {
    u32x4 rg[S][NA + NB];
    KALDO_GLOAD(0)
    KALDO_SSTORE(0)
  }
  if constexpr (BD) {
    KALDO_BLOAD(0, bcur)
  }
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    // the next chunk (the last one again on the final pass: a harmless reload
    // into the buffer nobody reads any more keeps the loop free of branches)
    const int nxt = (ch + 1 < nchunk ? ch + 1 : ch) * KCH;
    u32x4 rg[S][NA + NB];
    KALDO_GLOAD(nxt)
    if constexpr (BD) {
      KALDO_BLOAD(nxt, bnx)
    }
    // BF16X3: keep the next chunk's global loads ahead of this chunk's MFMAs.
    // Left to itself the scheduler sinks them behind most of the MFMAs (to
    // reuse fragment registers) and the wait before the LDS stores then
    // exposes their latency.  (Measured: 2 % faster BF16X3 GEMMs, 3-5 %
    // slower FP64 ones, whose chunks carry half as many MFMAs.)
    if constexpr (P == KALDO_BF16X3) __builtin_amdgcn_sched_barrier(0);
    const char* base = lds + (WC ? 0 : (ch & 1) * BUF);
    if constexpr (P == KALDO_BF16X3) {
#pragma unroll
      for (int j = 0; j < CB / 64; ++j) {
        bf16x8 af[FM][2], bf[FN][2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
#pragma unroll
          for (int a = 0; a < FM; ++a) {
            const uint4 v = lds_read16(base + lds_off<CB>(s * ROWS + arow + 16 * a, 4 * j + grp));
            af[a][s] = __builtin_bit_cast(bf16x8, v);
          }
#pragma unroll
          for (int c = 0; c < FN; ++c) {
            if constexpr (BD) {
              bf[c][s] = bcur[c][s];
            } else {
              const uint4 v = lds_read16(base + lds_off<CB>(s * ROWS + brow + 16 * c, 4 * j + grp));
              bf[c][s] = __builtin_bit_cast(bf16x8, v);
            }
          }
        }
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int c = 0; c < FN; ++c) {
            acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a][0], bf[c][0], acc[a][c], 0, 0, 0);
            acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a][0], bf[c][1], acc[a][c], 0, 0, 0);
            acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a][1], bf[c][0], acc[a][c], 0, 0, 0);
          }
      }
    } else if constexpr (P == KALDO_FP32) {
      const bool lastc = ch + 1 == nchunk;
      const int hn = half_last && lastc ? 1 : CB / 64;
#pragma unroll
      for (int h = 0; h < CB / 64; ++h) {
        if (h >= hn) break;
        // a partial last 16 k goes after the loop (fewer registers live here)
        if (lastc && h + 1 == hn && tail_q < 4) break;
        f32x4 af[FM], bf[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a)
          af[a] = __builtin_bit_cast(f32x4, lds_read16(base + lds_off<CB>(arow + 16 * a, 4 * h + grp)));
#pragma unroll
        for (int c = 0; c < FN; ++c)
          bf[c] = __builtin_bit_cast(f32x4, lds_read16(base + lds_off<CB>(brow + 16 * c, 4 * h + grp)));
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int c = 0; c < FN; ++c)
              acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a][j], bf[c][j], acc[a][c], 0, 0, 0);
      }
    } else {
      static_assert(P != KALDO_FP64 || CB == 128, "FP64 reads 32 bytes per lane group");
      double af[FM][4], bf[FN][4];
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        const char* p = base + lds_off<CB>(arow + 16 * a, 2 * grp);
        const uint4 v0 = lds_read16(p), v1 = lds_read16(p + 16);
        const double2 d0 = __builtin_bit_cast(double2, v0), d1 = __builtin_bit_cast(double2, v1);
        af[a][0] = d0.x;
        af[a][1] = d0.y;
        af[a][2] = d1.x;
        af[a][3] = d1.y;
      }
#pragma unroll
      for (int c = 0; c < FN; ++c) {
        const char* p = base + lds_off<CB>(brow + 16 * c, 2 * grp);
        const uint4 v0 = lds_read16(p), v1 = lds_read16(p + 16);
        const double2 d0 = __builtin_bit_cast(double2, v0), d1 = __builtin_bit_cast(double2, v1);
        bf[c][0] = d0.x;
        bf[c][1] = d0.y;
        bf[c][2] = d1.x;
        bf[c][3] = d1.y;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int c = 0; c < FN; ++c)
            acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a][j], bf[c][j], acc[a][c], 0, 0, 0);
    }
    if constexpr (WC) {
      __syncthreads();  // every wavefront is done reading the buffer
      KALDO_SSTORE(0)
    } else {
      KALDO_SSTORE((ch + 1) & 1)
    }
    if constexpr (BD) {
#pragma unroll
      for (int c = 0; c < FN; ++c) {
        bcur[c][0] = bnx[c][0];
        bcur[c][1] = bnx[c][1];
      }
    }
    __syncthreads();
  }
#undef KALDO_GLOAD
#undef KALDO_SSTORE
#undef KALDO_BLOAD
  if constexpr (P == KALDO_FP32) {
    if (tail_q < 4) {
      // the last 16 k hold 4 tail_q that are not padding (their chunk is still
      // in its buffer): step j takes k = 4 j + (lane group), one float per lane
      // from slot j of the group
      const char* base = lds + (WC ? 0 : ((nchunk - 1) & 1) * BUF);
      const int h = half_last ? 0 : CB / 64 - 1;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (j >= tail_q) break;
        float a1[FM], b1[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a)
          a1[a] = *reinterpret_cast<const float*>(base + lds_off<CB>(arow + 16 * a, 4 * h + j) + 4 * grp);
#pragma unroll
        for (int c = 0; c < FN; ++c)
          b1[c] = *reinterpret_cast<const float*>(base + lds_off<CB>(brow + 16 * c, 4 * h + j) + 4 * grp);
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int c = 0; c < FN; ++c)
            acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[a], b1[c], acc[a][c], 0, 0, 0);
      }
      __syncthreads();  // the epilogue may reuse the operand buffers
    }
  }

  TileAt at;
  at.mt = mt;
  at.nt = nt;
  at.z = z;
  at.m0 = rb + wm * 16 * FM;
  at.c0 = (long long)nt * BN + wn * 16 * FN;
  at.lane = lane;
  at.wm = wm;
  at.wn = wn;
  // the operand buffers are free after the last barrier: the epilogue may use them
  epi.template apply<P, FM, FN>(acc, at, lds);
}

template <int P, int FM, int FN, class Epi, bool BD = false, bool WC = false>
__global__ void __launch_bounds__(256) k_gemm(GemmOps g, Epi epi) {
  __shared__ __attribute__((aligned(16))) char lds[GemmLds<P, FM, FN, Epi, BD, WC>::bytes];
  // XCD-aware order: logical tile = start of this XCD's run + position in it
  const int nb = (int)gridDim.x, b = (int)blockIdx.x;
  const int q = nb >> 3, r8 = nb & 7, x = b & 7;
  const int tile = x * q + (x < r8 ? x : r8) + (b >> 3);
  int mt, nt, z;
  gemm_tile_coords(g, tile, mt, nt, z);
  gemm_tile<P, FM, FN, Epi, BD, WC>(g, epi, mt, nt, z, lds);
}

// Per-column partial sums of a linewidth epilogue, in two steps.  column_put
// reduces o[t] (this lane's sum over its rows of column 16 q + lane % 16 of the
// wavefront tile) over the 4 lane groups and parks it in LDS; column_flush
// adds the 2 wavefront rows and writes dst[col * nT + t] for the block's valid
// columns (dst already offset to the block's first column).
template <int FN, int NT>
__device__ __forceinline__ void column_put(double (&o)[NT], int q, const TileAt& at, char* lds) {
  double* red = reinterpret_cast<double*>(lds);  // [2 wm][32 FN columns][NT]
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double v = o[t];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    o[t] = v;
  }
  if (at.lane < 16) {
#pragma unroll
    for (int t = 0; t < NT; ++t) red[(at.wm * 32 * FN + at.wn * 16 * FN + 16 * q + at.lane) * NT + t] = o[t];
  }
}

template <int FN, int NT>
__device__ __forceinline__ void column_flush(char* lds, double* dst, long long ncols_left, int nT) {
  const double* red = reinterpret_cast<const double*>(lds);
  __syncthreads();
  for (int i = (int)threadIdx.x; i < 32 * FN * NT; i += 256) {
    const int col = i / NT, t = i % NT;
    if (t < nT && col < ncols_left) gmem(dst)[(long long)col * nT + t] = red[i] + red[32 * FN * NT + i];
  }
}

// ---- tile variants and launch ----------------------------------------------------------
// Candidate (FM, FN) shapes, block tile 32 FM x 32 FN.  FP64 accumulators take
// twice the registers of FP32 ones, so its candidates are one size smaller;
// the 64-byte chunks of BF16 and FP32 load 64 rows per pass (FM, FN even).
// BF16X3 adds candidates 4 and 5, whose B fragments bypass LDS, 6, a
// 128 x 256 block tile (64 x 128 per wavefront: twice the MFMA work per LDS
// fragment read and half the A-panel re-reads), and 7 and 8, the tiles of 0
// and 1 with wide chunks (WC; they fall back to 0 and 1 when K is not a
// multiple of 64).  BF16X3 9 and FP32 4 are 96 x 128 block tiles, whose 96
// rows fit M = 276 (a 46-atom cell, realified) in three tiles with 4 % padding.
constexpr int kGemmVariantsMax = 10;

template <int P>
inline int gemm_variants() {
  return P == KALDO_BF16X3 ? 10 : (P == KALDO_FP32 ? 5 : 4);
}

// An epilogue with kAllShapes = false is instantiated with the first tile shape
// only (variant 0): fewer kernel instances for its less used cases.
template <class Epi, class = void>
struct AllShapes : std::true_type {};
template <class Epi>
struct AllShapes<Epi, std::void_t<decltype(Epi::kAllShapes)>> : std::integral_constant<bool, Epi::kAllShapes> {};

template <int P, class Epi>
inline int gemm_variants() {
  return AllShapes<Epi>::value ? gemm_variants<P>() : 1;
}

template <int P>
inline int gemm_fm(int v) {
  if (P == KALDO_FP64) return v == 1 ? 4 : (v == 3 ? 3 : 2);
  if (P == KALDO_FP32 && v == 4) return 3;
  if (P == KALDO_BF16X3 && v == 9) return 3;
  return v == 1 || v == 3 || v == 5 || v == 8 ? 2 : 4;
}

template <int P>
inline int gemm_m_tiles(int v, int m) {
  const int bm = 32 * gemm_fm<P>(v);
  return (m + bm - 1) / bm;
}

template <int P, int FM, int FN, class Epi, bool BD = false, bool WC = false>
inline void gemm_launch_tile(GemmOps g, const Epi& e, hipStream_t st) {
  g.m_tiles = (g.m_valid + 32 * FM - 1) / (32 * FM);
  g.n_tiles = (int)((g.c_valid + 32 * FN - 1) / (32 * FN));
  g.group_m = g.group_m <= 0 ? 8 : (g.group_m < g.m_tiles ? g.group_m : g.m_tiles);
  g.group_n = g.group_n <= 0 ? g.n_tiles : (g.group_n < g.n_tiles ? g.group_n : g.n_tiles);
  const long long blocks = (long long)g.m_tiles * g.n_tiles * g.nz;
  // BF16X3 issues three bf16 products per element product
  g.tile_flops = 2ull * (32 * FM) * (32 * FN) * (unsigned long long)gemm_k_exec<P>(g) * (P == KALDO_BF16X3 ? 3 : 1);
  if (g.tally_dense) *g.tally_dense += (double)g.tile_flops * (double)blocks;
  hipLaunchKernelGGL((k_gemm<P, FM, FN, Epi, BD, WC>), dim3((unsigned)blocks), dim3(256), 0, st, g, e);
}

template <int P, class Epi>
inline void gemm_launch(int v, const GemmOps& g, const Epi& e, hipStream_t st) {
  if constexpr (!AllShapes<Epi>::value) {
    (void)v;
    if constexpr (P == KALDO_FP64) gemm_launch_tile<P, 2, 4>(g, e, st);
    else gemm_launch_tile<P, 4, 4>(g, e, st);
  } else if constexpr (P == KALDO_FP64) {
    if (v == 0) gemm_launch_tile<P, 2, 4>(g, e, st);
    else if (v == 1) gemm_launch_tile<P, 4, 2>(g, e, st);
    else if (v == 2) gemm_launch_tile<P, 2, 2>(g, e, st);
    else gemm_launch_tile<P, 3, 2>(g, e, st);
  } else if constexpr (P == KALDO_FP32) {
    if (v == 0) gemm_launch_tile<P, 4, 4>(g, e, st);
    else if (v == 1) gemm_launch_tile<P, 2, 4>(g, e, st);
    else if (v == 2) gemm_launch_tile<P, 4, 2>(g, e, st);
    else if (v == 3) gemm_launch_tile<P, 2, 2>(g, e, st);
    else gemm_launch_tile<P, 3, 4>(g, e, st);
  } else {
    if (v == 0) gemm_launch_tile<P, 4, 4>(g, e, st);
    else if (v == 1) gemm_launch_tile<P, 2, 4>(g, e, st);
    else if (v == 2) gemm_launch_tile<P, 4, 2>(g, e, st);
    else if (v == 3) gemm_launch_tile<P, 2, 2>(g, e, st);
    else if (v == 4) gemm_launch_tile<P, 4, 4, Epi, true>(g, e, st);
    else if (v == 5) gemm_launch_tile<P, 2, 4, Epi, true>(g, e, st);
    else if (v == 7 && g.K % 64 == 0) gemm_launch_tile<P, 4, 4, Epi, false, true>(g, e, st);
    else if (v == 7) gemm_launch_tile<P, 4, 4>(g, e, st);
    else if (v == 8 && g.K % 64 == 0) gemm_launch_tile<P, 2, 4, Epi, false, true>(g, e, st);
    else if (v == 8) gemm_launch_tile<P, 2, 4>(g, e, st);
    else if (v == 9) gemm_launch_tile<P, 3, 4>(g, e, st);
    else gemm_launch_tile<P, 4, 8>(g, e, st);
  }
}

// Attach the context's flop tally to the operands of a projection GEMM launch
// when kernel timing is on (kaldo_profile_enable) and the launch is not captured.
inline void prof_tally(kaldo_ctx ctx, GemmOps& g) {
  if (!ctx->prof || ctx->mode != kRun || !ctx->d_prof_flops.p) return;
  g.tally = ctx->d_prof_flops.as<unsigned long long>();
  g.tally_dense = &ctx->prof_dense;
}

}  // namespace kaldo
