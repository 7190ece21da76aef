// MFMA GEMM family for gfx950 (CDNA4) used by every contraction of the ladder
// term and its adjoint.
//
//   C[m][n] (+)= sum_k A(m,k) B(k,n)
//
// Operands are addressed through a pointer and a leading dimension in one of
// two layouts:
//   KC: the contracted index is contiguous   A(m,k) = A[m*lda + k], B(k,n) = B[n*ldb + k]
//   RC: the row / column index is contiguous A(m,k) = A[k*lda + m], B(k,n) = B[k*ldb + n]
// which covers every product of the path without operand copies: the integral
// build reads the Cholesky vectors [x][(p,q)] directly (RC, K = x), the
// amplitude contraction reads t and the integral block with K = (c,d)
// contiguous (KC), and so on.
//
// Epilogues:
//   EPI_ACC : C[m*ldc + n] += alpha * acc                 (float64 accumulation)
//   EPI_PERM: m = (a, x), n = (y, d) with x, d < v and y < N/v:
//             C[a*N*v + y*v^2 + x*v + d] = acc            (stores, in the operand type, an
//                                                          integral-shaped block with its
//                                                          middle indices swapped; N = v^2
//                                                          for the virtual-virtual build,
//                                                          o*v for occupied columns)
//   EPI_PACK: the build restricted to b >= a: m = (a - a0, c), n = (b - a0, d);
//             C[(pair(a,b) - pair(a0,a0))*v^2 + c*v + d] = acc for b >= a, where
//             pair(a,b) = prefix(a) + b - a numbers the rows a <= b (tiles wholly
//             below the diagonal exit at once)
//   EPI_PAIR: the contraction over packed rows: m = (i,j), n = pair(a,b) - pair(a0,a0);
//             C[m*ldc + a*v + b] += acc and, for a != b, C[(j,i)*ldc + b*v + a] += acc
//   EPI_PM:   the symmetric (pm = 1) or antisymmetric (pm = 2) combination over rows
//             m = pair (i,j), i <= j (i < j for pm = 2), and columns n = pair (a,b) from
//             a0, a <= b (a < b for pm = 2): val = alpha * acc is added to the set
//             {R[i,j,a,b], R[j,i,b,a]} and, as +val (pm = 1) or -val (pm = 2), to
//             {R[i,j,b,a], R[j,i,a,b]}, each distinct element once
//   EPI_PART: split K: workgroup s of a tile sums K-steps [s*split_steps, (s+1)*split_steps)
//             and stores C[s*part_stride + m*ldc + n] = acc (float64 partials, summed
//             in order of s by a separate pass)
//   EPI_SYM:  a symmetric product (A = B): only the tiles on or above the diagonal run
//             (the compact grid of EPI_PACK with v = 1), and each stores C[m*ldc + n] = acc
//             and its mirror C[n*ldc + m] = acc (the same value: the products commute)
//   EPI_UNPACK: rows are packed pairs: m = pair(a,b) - pair(a0,a0) (a <= b), n = (c, d);
//             C[(a - a0)*v^3 + c*v^2 + b*v + d] = acc for m < m_keep (the integral-shaped
//             block of EPI_PERM with only its b >= a half written)
//
// K bands (kband, any epilogue): a product whose B operand is such a half-written
// block skips the K-steps that only meet its zero half.  kband 1: columns
// n = (a - a0, c), K = (b, d) over every b, non-zero for b >= a: a tile's K range
// starts at its smallest a.  kband 2: columns n = (b - a0, d), K rows (a - a0, c),
// non-zero for a <= b: a tile's range ends after its largest b.  The ranges are
// whole K-steps, so B must hold zeros in the few (b, a) rows next to the diagonal
// that a rounded range still covers.
//
// Tiling: 256 threads = 4 wave64s in a 2x2 grid, 128x128 workgroup tile, each
// wave owns a 64x64 sub-tile = 4x4 MFMA 16x16 blocks.  Global tiles are read
// 16 bytes per lane into registers one K-step ahead and written into a
// double-buffered LDS tile, so one barrier per K-step separates the two halves.
//
// MFMA operand layout (v_mfma_*_16x16x4): lane l supplies A[l%16][slot l/16]
// and B[slot l/16][l%16]; the 16x16 result sits as 4 values per lane in
// column l%16: value r is row 4*(l/16)+r for the float32 instruction and row
// (l/16)+4*r for the float64 one (measured on gfx950).  A "k-group" of CH*4 consecutive k is read with one
// 16-byte LDS access per lane and consumed by CH MFMA steps: in step e, slot j
// carries k = group_base + CH*j + e, for both operands alike.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccl {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
enum { KC = 0, RC = 1 };
enum { EPI_ACC = 0, EPI_PERM = 1, EPI_PACK = 2, EPI_PAIR = 3, EPI_PART = 4, EPI_PM = 5,
       EPI_UNPACK = 6, EPI_SYM = 7 };

// float64 operands on v_mfma_f64_16x16x4_f64.
struct TrF64 {
  using T = double;
  using Chunk = f64x2;   // 16 bytes
  using Acc = f64x4;
  static constexpr int CH = 2;     // elements per 16-byte chunk = MFMA steps per k-group
  static constexpr int BK = 16;    // K per LDS stage
  static constexpr bool kDrain = false;
  static constexpr int kWaves = 2;  // waves per SIMD the register budget is sized for
  static constexpr bool kDirectKC = true;  // KC x KC products use the direct-to-LDS kernel
  // RC x RC integral builds stay on the register-staged kernel: two workgroups per
  // CU hide its short-K prologue/epilogue better (measured 290 vs 295 ms at o=40 v=360 P=1200)
  static constexpr bool kDirectRC = false;
  static constexpr bool kDirectKR = true;  // KC x RC products: mixed direct-to-LDS kernel
  __device__ static inline Acc mfma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of result value r held by `lane`
  __device__ static inline int row_of(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// float32 operands on v_mfma_f32_16x16x4_f32; partial sums drained to float64.
struct TrF32 {
  using T = float;
  using Chunk = f32x4;
  using Acc = f32x4;
  static constexpr int CH = 4;
  static constexpr int BK = 32;
  static constexpr bool kDrain = true;
  static constexpr int kWaves = 1;  // float64 drain registers double the accumulator footprint
  static constexpr bool kDirectKC = true;
  static constexpr bool kDirectRC = true;  // builds: 442 -> 317 ms at o=40 v=360 P=1200
  static constexpr bool kDirectKR = true;
  __device__ static inline Acc mfma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row_of(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <class T>
struct GemmArgs {
  const T* A;
  long long lda;
  const T* B;
  long long ldb;
  void* C;          // EPI_ACC: double; EPI_PERM: T
  long long ldc;
  int M, N, K;
  int v;             // EPI_PERM/PACK/PAIR index split
  int o;             // EPI_PAIR: occupied count (rows are (i,j))
  int a0;            // EPI_PACK/PAIR: first virtual of the integral block
  int tiles_m, tiles_n;
  int group_m;       // tile-order swizzle: rows of tiles walked together
  int drain_steps;   // K-steps between float32 -> float64 drains (TrF32)
  const int* row_tiles;  // EPI_PACK compact grid: first linear tile of each tile row
  int split_steps;       // EPI_PART: K-steps per split
  long long part_stride; // EPI_PART: elements between consecutive splits' partials
  double alpha;          // EPI_ACC: C += alpha * acc (1, or 2 for a term counted twice)
  int m_off = 0;         // EPI_PAIR/PM: global row of this launch's row 0 (a remainder launch)
  int pm = 0;            // EPI_PM: 1 = symmetric pairs (i <= j, a <= b), 2 = antisymmetric (<)
  int kband = 0;         // K bands of a half-written B operand (0 = the whole K range)
  int m_keep = 0;        // EPI_UNPACK: rows stored (M may be padded to whole 16-byte chunks)
};

// K-steps [ks0, ks1) of the tile whose columns start at n0 (bn wide), steps of bk.
template <class T>
__device__ __forceinline__ void k_band(const GemmArgs<T>& g, int n0, int bn, int bk, int& ks0,
                                       int& ks1) {
  ks0 = 0;
  ks1 = (g.K + bk - 1) / bk;
  if (g.kband == 1) {
    const long long k = (long long)(g.a0 + n0 / g.v) * g.v;  // first (b, d) with b = smallest a
    ks0 = static_cast<int>(k / bk);
  } else if (g.kband == 2) {
    const int nl = (n0 + bn < g.N ? n0 + bn : g.N) - 1;
    long long k = (long long)(nl / g.v + 1) * g.v;  // past the rows a - a0 <= largest b - a0
    if (k > g.K) k = g.K;
    const int e = static_cast<int>((k + bk - 1) / bk);
    ks1 = e < ks1 ? e : ks1;
  }
}

// First needed tile column of tile row tm in the packed build: columns whose
// largest b is at least the row's smallest a.
__host__ __device__ inline int pack_first_tile(int tm, int bm, int bn, int v) {
  const long long amin = (long long)tm * bm / v;  // smallest (a - a0) of the tile row
  return static_cast<int>(amin * v / bn);
}

constexpr int kBM = 128, kBN = 128;

// Number of packed rows (a', b) with a' < a, i.e. sum_{a' < a} (v - a').
__device__ __forceinline__ long long pair_prefix_d(long long a, long long v) {
  return a * v - a * (a - 1) / 2;
}

// Largest a with pair_prefix(a) <= q (q < v(v+1)/2): the smaller root of
// a^2 - (2v+1) a + 2q = 0, floored.  In float64 (exact squares for v < 2^26) the
// computed root is within far less than 1 of the true one, so one correction
// step each way gives the floor; no loops (they keep epilogues unrolled).
__device__ __forceinline__ int pair_row(long long q, int v) {
  const double b = 2.0 * v + 1.0;
  int a = static_cast<int>((b - sqrt(b * b - 8.0 * static_cast<double>(q))) * 0.5);
  a = a < 0 ? 0 : (a >= v ? v - 1 : a);
  if (a + 1 < v && pair_prefix_d(a + 1, v) <= q) ++a;
  if (a > 0 && pair_prefix_d(a, v) > q) --a;
  return a;
}

// Column-dependent part of an epilogue address, computed once per column.
struct EpiCol {
  long long off;  // PERM: y*v^2 + d; PACK: d; PAIR: a*v + b
  int x;          // PACK: b - a0; PAIR: a
  int y;          // PAIR: b
};

template <class T, int EPI>
__device__ __forceinline__ EpiCol epi_col(const GemmArgs<T>& g, int n) {
  EpiCol c{n, 0, 0};
  const long long v = g.v;
  if (EPI == EPI_PERM || EPI == EPI_UNPACK) {
    const int y = n / g.v, d = n - y * g.v;
    c.off = (long long)y * v * v + d;
  } else if (EPI == EPI_PACK) {
    const int bl = n / g.v;
    c.x = bl;
    c.off = n - bl * g.v;
  } else if (EPI == EPI_PAIR) {
    const long long q = pair_prefix_d(g.a0, v) + n;
    const int a = pair_row(q, g.v);
    const int b = a + static_cast<int>(q - pair_prefix_d(a, v));
    c.x = a;
    c.y = b;
    c.off = (long long)a * v + b;
  } else if (EPI == EPI_PM) {
    // pairs a < b of v are the pairs a <= b' = b - 1 of v - 1
    const int s = g.pm == 2 ? 1 : 0;
    const long long q = pair_prefix_d(g.a0, v - s) + n;
    const int a = pair_row(q, g.v - s);
    const int b = a + s + static_cast<int>(q - pair_prefix_d(a, v - s));
    c.x = a;
    c.y = b;
    c.off = (long long)a * v + b;
  }
  return c;
}

// Stores result element (m, n) of a product according to the epilogue mode.
template <class T, int EPI>
__device__ __forceinline__ void epi_store(const GemmArgs<T>& g, int m, int n, const EpiCol& c,
                                          double val) {
  const long long v = g.v;
  if (EPI == EPI_ACC) {
    static_cast<double*>(g.C)[(long long)m * g.ldc + n] += g.alpha * val;
  } else if (EPI == EPI_PART) {
    static_cast<double*>(g.C)[(long long)m * g.ldc + n] = val;
  } else if (EPI == EPI_PERM) {
    const int a = m / g.v, x = m - a * g.v;
    static_cast<T*>(g.C)[(long long)a * g.N * v + c.off + (long long)x * v] = static_cast<T>(val);
  } else if (EPI == EPI_SYM) {
    T* C = static_cast<T*>(g.C);
    C[(long long)m * g.ldc + n] = static_cast<T>(val);
    C[(long long)n * g.ldc + m] = static_cast<T>(val);
  } else if (EPI == EPI_UNPACK) {
    if (m >= g.m_keep) return;
    const long long q = pair_prefix_d(g.a0, v) + m;
    const int a = pair_row(q, g.v);
    const int b = a + static_cast<int>(q - pair_prefix_d(a, v));
    static_cast<T*>(g.C)[(long long)(a - g.a0) * v * v * v + c.off + (long long)b * v] =
        static_cast<T>(val);
  } else if (EPI == EPI_PACK) {
    const int al = m / g.v, cc = m - al * g.v;
    if (c.x < al) return;
    const long long row = pair_prefix_d(g.a0 + al, v) - pair_prefix_d(g.a0, v) + (c.x - al);
    static_cast<T*>(g.C)[row * v * v + (long long)cc * v + c.off] = static_cast<T>(val);
  } else if (EPI == EPI_PM) {
    double* C = static_cast<double*>(g.C);
    const int s = g.pm == 2 ? 1 : 0;
    const int mg = m + g.m_off;
    const int i = pair_row(mg, g.o - s);
    const int j = i + s + static_cast<int>(mg - pair_prefix_d(i, g.o - s));
    const double w = g.alpha * val;
    const double x = s ? -w : w;  // weight of the a <-> b exchanged elements
    const long long rij = (long long)(i * g.o + j) * g.ldc, rji = (long long)(j * g.o + i) * g.ldc;
    const long long ab = c.off, ba = (long long)c.y * v + c.x;
    C[rij + ab] += w;
    if (c.x != c.y) C[rij + ba] += x;
    if (i != j) {
      C[rji + ba] += w;
      if (c.x != c.y) C[rji + ab] += x;
    }
  } else {  // EPI_PAIR
    double* C = static_cast<double*>(g.C);
    const int mg = m + g.m_off;
    C[(long long)mg * g.ldc + c.off] += val;
    if (c.x != c.y) {
      const int i = mg / g.o, j = mg - i * g.o;
      C[(long long)(j * g.o + i) * g.ldc + (long long)c.y * v + c.x] += val;
    }
  }
}

template <class Tr, int LAY, int ROWS>
struct TileIO {
  using T = typename Tr::T;
  using Chunk = typename Tr::Chunk;
  static constexpr int CH = Tr::CH;
  static constexpr int BK = Tr::BK;
  static constexpr int PADK = CH;              // KC row pad: 16 bytes
  static constexpr int PADR = 64 / sizeof(T);  // RC row pad: 64 bytes
  static constexpr int LD = (LAY == KC) ? (BK + PADK) : (ROWS + PADR);
  static constexpr int ELEMS = (LAY == KC) ? ROWS * LD : BK * LD;  // one LDS stage
  static constexpr int NCH = ROWS * BK / CH / kThreads;            // chunks per thread
  static_assert(NCH * CH * kThreads == ROWS * BK, "tile must split evenly into 16-byte chunks");

  // Chunk c of this thread: its (row, k) origin inside the tile.
  __device__ static inline void coord(int c, int tid, int& row, int& kk) {
    const int q = c * kThreads + tid;
    if (LAY == KC) {
      row = q / (BK / CH);
      kk = (q % (BK / CH)) * CH;
    } else {
      kk = q / (ROWS / CH);
      row = (q % (ROWS / CH)) * CH;
    }
  }

  // Chunk c of a thread sits a fixed, thread-independent distance from its chunk 0:
  // KC: rows advance by kThreads*CH/BK per chunk; RC: k advances by kThreads*CH/ROWS.
  static constexpr int kChunkRows = (LAY == KC) ? kThreads * CH / BK : kThreads * CH / ROWS;
  static_assert((LAY == KC ? BK / CH : ROWS / CH) <= kThreads, "chunk layout");

  // Thread's chunk-0 address at the current K-step; chunks and K-steps are uniform strides.
  struct Cursor {
    const T* p;
    long long cstride;  // elements from chunk c to chunk c+1
    long long kstep;    // elements between consecutive K-steps
  };

  __device__ static inline void init(Cursor& cu, const T* __restrict__ base, long long ld, int row0,
                                     int tid) {
    int row, kk;
    coord(0, tid, row, kk);
    cu.p = base + ((LAY == KC) ? (long long)(row0 + row) * ld + kk
                               : (long long)kk * ld + (row0 + row));
    cu.cstride = (long long)kChunkRows * ld;
    cu.kstep = (LAY == KC) ? BK : (long long)BK * ld;
  }

  __device__ static inline void advance(Cursor& cu) { cu.p += cu.kstep; }

  // Whole tile in bounds and 16-byte aligned: one vector load per chunk.
  __device__ static inline void load_full(Chunk (&r)[NCH], const Cursor& cu) {
#pragma unroll
    for (int c = 0; c < NCH; ++c)
      r[c] = *reinterpret_cast<const Chunk*>(cu.p + c * cu.cstride);
  }

  // Any tile: element loads, zero outside [0, nrows) x [0, K).
  __device__ static inline void load_masked(Chunk (&r)[NCH], const Cursor& cu, int row0, int nrows,
                                            int k0, int K, int tid) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      int row, kk;
      coord(c, tid, row, kk);
      const T* src = cu.p + c * cu.cstride;
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        const bool ok = (LAY == KC) ? (row0 + row < nrows && k0 + kk + e < K)
                                    : (k0 + kk < K && row0 + row + e < nrows);
        r[c][e] = ok ? src[e] : T(0);
      }
    }
  }

  __device__ static inline void store(T* s, const Chunk (&r)[NCH], int tid) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      int row, kk;
      coord(c, tid, row, kk);
      T* dst = (LAY == KC) ? s + row * LD + kk : s + kk * LD + row;
      *reinterpret_cast<Chunk*>(dst) = r[c];
    }
  }

  // Operand values of k-group g for the 16 rows starting at rb: element e feeds MFMA step e.
  __device__ static inline Chunk frag(const T* s, int rb, int g, int lane) {
    const int kb = g * (CH * 4) + CH * (lane >> 4);
    if (LAY == KC) {
      return *reinterpret_cast<const Chunk*>(s + (rb + (lane & 15)) * LD + kb);
    } else {
      Chunk f;
#pragma unroll
      for (int e = 0; e < CH; ++e) f[e] = s[(kb + e) * LD + rb + (lane & 15)];
      return f;
    }
  }
};

// Maps the linear workgroup id to a tile.  Workgroups are handed to the 8 XCDs
// round-robin; the remap gives each XCD a contiguous range of logical tiles so
// that co-resident tiles share operand panels in that XCD's L2.  Logical tiles
// are walked in bands of group_m tile rows.
// Dispatch order -> linear work index: workgroups are handed to the 8 XCDs
// round-robin, so consecutive indices of one XCD get consecutive ids.
__device__ inline int xcd_linear(int bid, int nwg) {
  const int per = nwg / 8, extra = nwg % 8;
  const int xcd = bid % 8, local = bid / 8;
  return xcd * per + (xcd < extra ? xcd : extra) + local;
}

// Linear tile id -> (tile row, tile column), walking bands of group_m tile rows
// column by column so that co-resident tiles share row and column panels.
__device__ inline void tile_from_linear(int id, int ntiles, int tiles_m, int group_m, int& tm,
                                        int& tn) {
  const int band = group_m * (ntiles / tiles_m);  // tiles in one band (tiles_n tiles per row)
  const int b = id / band;
  const int first = b * group_m;
  const int rows = (tiles_m - first) < group_m ? (tiles_m - first) : group_m;
  const int in = id - b * band;
  tm = first + in % rows;
  tn = in / rows;
}

__device__ inline void tile_of(int bid, int nwg, int tiles_m, int group_m, int& tm, int& tn) {
  tile_from_linear(xcd_linear(bid, nwg), nwg, tiles_m, group_m, tm, tn);
}

// Tile of a K-banded product, whose tiles' K ranges shrink (kband 1) or grow
// (kband 2) along the tile columns: the dispatch order itself, so that the
// round-robin hands every XCD long and short tiles alike (contiguous runs per
// XCD would give one XCD all the long ones), longest first.
__device__ inline void tile_of_banded(int kband, int bid, int nwg, int tiles_m, int group_m,
                                      int& tm, int& tn) {
  tile_from_linear(kband == 2 ? nwg - 1 - bid : bid, nwg, tiles_m, group_m, tm, tn);
}

// K loop of one tile.  FAST: the tile lies inside M x N and its operands are
// 16-byte aligned, so every full K-step is one vector load per chunk with no
// test; only a ragged last K-step is masked.  Otherwise every load is masked.
template <class Tr, int LA, int LB, bool FAST>
__device__ __forceinline__ void tile_mainloop(const GemmArgs<typename Tr::T>& g, int m0, int n0,
                                              int ks0, int ks1,
                                              typename Tr::T* sA0, typename Tr::T* sA1,
                                              typename Tr::T* sB0, typename Tr::T* sB1,
                                              typename Tr::Acc (&acc)[4][4],
                                              f64x4 (&acc64)[4][4]) {
  using IA = TileIO<Tr, LA, kBM>;
  using IB = TileIO<Tr, LB, kBN>;
  constexpr int BK = Tr::BK;
  constexpr int CH = Tr::CH;
  constexpr int NG = BK / (CH * 4);  // k-groups per stage
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;
  const int nk = ks1;                   // one past the tile's last K-step
  const int nkf = FAST ? g.K / BK : 0;  // K-steps loaded without masks

  typename IA::Cursor ca;
  typename IB::Cursor cb;
  IA::init(ca, g.A, g.lda, m0, tid);
  IB::init(cb, g.B, g.ldb, n0, tid);
  ca.p += ks0 * ca.kstep;
  cb.p += ks0 * cb.kstep;
  typename IA::Chunk ra[IA::NCH];
  typename IB::Chunk rb[IB::NCH];

  auto fetch = [&](int kt) {
    if (kt < nkf) {
      IA::load_full(ra, ca);
      IB::load_full(rb, cb);
    } else {
      IA::load_masked(ra, ca, m0, g.M, kt * BK, g.K, tid);
      IB::load_masked(rb, cb, n0, g.N, kt * BK, g.K, tid);
    }
    IA::advance(ca);
    IB::advance(cb);
  };
  auto compute = [&](const typename Tr::T* sa, const typename Tr::T* sb) {
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      typename Tr::Chunk fa[4], fb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) fa[i] = IA::frag(sa, wm + 16 * i, gi, lane);
#pragma unroll
      for (int j = 0; j < 4; ++j) fb[j] = IB::frag(sb, wn + 16 * j, gi, lane);
#pragma unroll
      for (int e = 0; e < CH; ++e)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = Tr::mfma(fa[i][e], fb[j][e], acc[i][j]);
    }
  };
  // float32 forms: partial sums of one chunk of drain_steps K-steps stay in the
  // MFMA accumulators and are drained into float64 once per chunk.
  auto drain = [&]() {
    if (!Tr::kDrain) return;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc64[i][j][r] += static_cast<double>(acc[i][j][r]);
          acc[i][j][r] = 0;
        }
  };

  fetch(ks0);
  IA::store(sA0, ra, tid);
  IB::store(sB0, rb, tid);
  __syncthreads();
  int kt = ks0;
  for (;;) {
    const int kend = (Tr::kDrain && kt + g.drain_steps < nk) ? kt + g.drain_steps : nk;
    // Steady state, two K-steps per trip so the LDS stages stay compile-time
    // (chunks hold an even number of steps, so kt - ks0 is even here).
    for (; kt + 2 <= kend && kt + 2 < nkf; kt += 2) {
      fetch(kt + 1);
      compute(sA0, sB0);
      IA::store(sA1, ra, tid);
      IB::store(sB1, rb, tid);
      __syncthreads();
      fetch(kt + 2);
      compute(sA1, sB1);
      IA::store(sA0, ra, tid);
      IB::store(sB0, rb, tid);
      __syncthreads();
    }
    // Remaining steps of the chunk (masked loads where needed); stage parity follows kt.
    for (; kt < kend; ++kt) {
      const int odd = (kt - ks0) & 1;
      typename Tr::T* sa = odd ? sA1 : sA0;
      typename Tr::T* sb = odd ? sB1 : sB0;
      const bool more = kt + 1 < nk;
      if (more) fetch(kt + 1);
      compute(sa, sb);
      if (more) {
        IA::store(odd ? sA0 : sA1, ra, tid);
        IB::store(odd ? sB0 : sB1, rb, tid);
      }
      __syncthreads();
    }
    drain();
    if (kt >= nk) break;
  }
}

template <class Tr, int LA, int LB, int EPI, bool VEC>
__global__ __launch_bounds__(kThreads, Tr::kWaves) void gemm_kernel(GemmArgs<typename Tr::T> g) {
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  using IA = TileIO<Tr, LA, kBM>;
  using IB = TileIO<Tr, LB, kBN>;

  __shared__ __attribute__((aligned(16))) T sA[2][IA::ELEMS];
  __shared__ __attribute__((aligned(16))) T sB[2][IB::ELEMS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;

  int tm, tn;
  if (EPI == EPI_PACK || EPI == EPI_SYM) {
    // compact grid over the tiles on or above the a = b diagonal: tile row by
    // binary search over the row offsets, then columns from the row's first
    const int id = blockIdx.x;
    int lo = 0, hi = g.tiles_m - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (g.row_tiles[mid] <= id) lo = mid; else hi = mid - 1;
    }
    tm = lo;
    tn = pack_first_tile(tm, kBM, kBN, g.v) + (id - g.row_tiles[tm]);
  } else if (g.kband) {
    tile_of_banded(g.kband, blockIdx.x, gridDim.x, g.tiles_m, g.group_m, tm, tn);
  } else {
    tile_of(blockIdx.x, gridDim.x, g.tiles_m, g.group_m, tm, tn);
  }
  const int m0 = tm * kBM;
  const int n0 = tn * kBN;
  if (EPI == EPI_PACK || EPI == EPI_SYM) {
    // every column's b below every row's a: nothing of this tile is kept
    const int nlast = ((n0 + kBN < g.N) ? n0 + kBN : g.N) - 1;
    if (nlast / g.v < m0 / g.v) return;
  }

  Acc acc[4][4];
  f64x4 acc64[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = Acc{0, 0, 0, 0};
      acc64[i][j] = f64x4{0, 0, 0, 0};
    }

  int ks0, ks1;
  k_band(g, n0, kBN, Tr::BK, ks0, ks1);
  const bool interior = (m0 + kBM <= g.M) && (n0 + kBN <= g.N);
  if (VEC && interior)
    tile_mainloop<Tr, LA, LB, true>(g, m0, n0, ks0, ks1, sA[0], sA[1], sB[0], sB[1], acc, acc64);
  else
    tile_mainloop<Tr, LA, LB, false>(g, m0, n0, ks0, ks1, sA[0], sA[1], sB[0], sB[1], acc, acc64);

  // Epilogue: lane holds column lane%16 of each 16x16 block, rows Tr::row_of(lane, r).
  const int col = lane & 15;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + wn + 16 * j + col;
    if (n >= g.N) continue;
    const EpiCol ec = epi_col<T, EPI>(g, n);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + Tr::row_of(lane, r);
        if (m >= g.M) continue;
        const double val = Tr::kDrain ? acc64[i][j][r] : static_cast<double>(acc[i][j][r]);
        epi_store<T, EPI>(g, m, n, ec, val);
      }
    }
  }
}

}  // namespace ccl
