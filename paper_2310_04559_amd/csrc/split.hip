// Split-bf16 form of the ladder forward.
//
// Three or four slices: every operand row (a row of the matrix along its
// contracted index) gets an exponent e with max|x| < 2^e -- one per row for the
// integral build, one per (row, chunk of contracted indices) for the amplitude
// contraction -- and each value is cut into S balanced base-256 digits:
//   x = 2^e * sum_{p=1..S} d_p 2^(-8p) + r,   d_1 in [-256, 256], d_p in [-128, 128] (p > 1),
// |r| <= 2^(e - 8S - 1).  Digits are integers, exact in bf16.  A product of two
// such matrices is, per K-chunk c,
//   C[m][n] += 2^(eA[m,c] + eB[n,c]) sum_{g} 2^(-8g) sum_{p+q=g} sum_{k in c} dA_p[m][k] dB_q[n][k],
// keeping the anti-diagonals g = p + q <= S + D (D = 1: the S(S+1)/2-product
// triangle; D = 2 adds the next anti-diagonal).  Each inner sum is a sum of
// integer products.  A chunk is 256 indices with four slices: the products of
// the two leading anti-diagonals are at most 2^16 each and 2^24 over the
// chunk, so those float32 sums are exact (the anti-diagonals g >= 2 share one
// rounded sum); with three slices, whose third anti-diagonal has three
// products, it is 128 indices and every group is exact.  Each chunk is drained
// into float64 with its own scale.  Exponents per chunk follow the operands'
// magnitude along the contracted index and cut the contraction's error at the
// same digit count (1.0e-9 with one exponent per row, 4.0e-10 per 128 and
// 4.4e-10 per 256 indices at o=20 v=180 P=600 in the exact NumPy model of the
// scheme); for the build, whose rows (Cholesky vectors along x) are evenly
// scaled, they change nothing.  Chunks of 256 halve the drains against 128.
//
// Two slices are the per-element hi/lo split instead: hi = bf16(x) and
// lo = bf16(x - hi), both rounded to nearest even, so each operand carries about
// 16 significant bits of its own magnitude (no shared exponent).  The products
// hi*hi, hi*lo and lo*hi (D = 1; D = 2 adds lo*lo) are summed in float32 over
// each 256-index chunk (rounded, not exact) and drained to float64.  The same
// kernels serve it with every exponent fixed at 8, which makes every scale 1.
//
// The two contractions then run as:
//   build    V_A = L-slices x L-slices (K = x), float64 block, permuted store
//   re-slice V_A rows (a,b) along (c,d)
//   contract R += t-slices x V_A-slices (K = (c,d)), float64 accumulation
#include "split.hpp"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "gemm.hpp"

namespace ccl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kSBN = 128;   // workgroup tile columns (N)
constexpr int kSBK = 32;    // K per stage = one bf16 MFMA depth
// K-steps per float32 chunk (one exponent per chunk of the contraction's rows)
template <int S>
constexpr int chunk_steps() { return exp_chunk_len(S) / kSBK; }

// Balanced base-256 digits of y in (-1, 1): y = 2^-8 sum_p q_p 2^(-8p) with
// integers |q_0| <= 256, |q_p| <= 128.  Slice p holds q_p 2^(-8p) (exact in
// bf16), so the product of slices p and q carries its own scale 2^(-8(p+q)).
template <int S>
__device__ __forceinline__ void digits(double y, __bf16 (&d)[S]) {
  static_assert(S <= 4, "slice scales 2^(-8p) as float constants");
#pragma unroll
  for (int p = 0; p < S; ++p) {
    y *= 256.0;
    const double q = rint(y);
    y -= q;
    // |q| <= 256 is exact as an int and as a float, and so is q 2^(-8p); going
    // through int keeps the bf16 conversion a plain exact one
    const float scale = 1.0f / static_cast<float>(1u << (8 * p));
    d[p] = static_cast<__bf16>(static_cast<float>(static_cast<int>(q)) * scale);
  }
}

// Per-element split for two slices: x = hi + lo + r with hi = bf16(x),
// lo = bf16(x - hi) (x - hi is exact in float64), |r| <= 2^-16 |x|.
__device__ __forceinline__ void hi_lo(double x, __bf16 (&d)[2]) {
  const __bf16 h = static_cast<__bf16>(x);  // round to nearest even
  d[0] = h;
  d[1] = static_cast<__bf16>(x - static_cast<double>(h));
}

// Cuts x (scaled by 2^-e in the digit forms) into the S slices of the form.
template <int S>
__device__ __forceinline__ void cut(double x, int e, __bf16 (&d)[S]) {
  if constexpr (S == 2)
    hi_lo(x, d);
  else
    digits<S>(ldexp(x, -e), d);
}

// The exponent every row gets in the hi/lo form: 2^(eA + eB - 16) = 1.
constexpr int kHiLoExp = 8;

// Digit buffers are [rows][k_pad / 32][S][32]: for each 32-deep K-step the S
// slices of one row are adjacent, so the loads of a K-step read whole 128-byte
// lines (two slices per line).  Offset of slice 0 of indices k .. k+7 of row r
// (k a multiple of 8); slice p is kSBK elements further.
template <int S>
__device__ __forceinline__ long long digit_offset(long long r, int k, int Kp) {
  return r * Kp * S + (long long)(k / kSBK) * (S * kSBK) + (k % kSBK);
}

// ---------------------------------------------------------------------------
// slicing
// ---------------------------------------------------------------------------

// Rows with the contracted index contiguous: X[r][k] = X[r*ld + k], r < R, k < K.
// One workgroup per output row (R_pad rows, the padding rows get zero digits).
// Exponents per (row, chunk of exp_chunk_len(S)): ex[c * ex_stride + r].  The
// 32 (16 for three slices) threads that cut one chunk (8 values each) are
// adjacent lanes of one wave and agree on its maximum through shuffles.  A wave's 512 indices are 16 K-steps,
// whose digits are S KB of contiguous memory: the wave lays them out in a
// private LDS block and stores them as whole 1 KB rows (a lane's own digits
// would cover only 64 bytes of a line per store).
template <int S>
__global__ __launch_bounds__(256) void slice_kc_kernel(const double* __restrict__ X, long long ld,
                                                       int R, int K, int Kp,
                                                       __bf16* __restrict__ out, int* __restrict__ ex,
                                                       int ex_stride) {
  constexpr int TPC = exp_chunk_len(S) / 8;  // threads per chunk
  static_assert(TPC == 16 || TPC == 32, "a chunk is cut by 16 or 32 threads of 8 values");
  constexpr int STEP_BYTES = S * kSBK * 2;  // one K-step of one row, all slices
  __shared__ __attribute__((aligned(16))) unsigned char stage[4][16 * STEP_BYTES];
  const int r = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  unsigned char* wl = stage[wave];
  const double* row = X + (long long)r * ld;
  unsigned char* orow = reinterpret_cast<unsigned char*>(out + (long long)r * Kp * S);
  // rows starting on 16 bytes load 8 values as four 16-byte vectors
  const bool vec = r < R && (reinterpret_cast<unsigned long long>(row) & 15) == 0;
  // every thread runs every iteration (indices past Kp are cut as zeros and not
  // stored), so the wave-level exchange below always has the whole wave
  for (int base = 0; base < Kp; base += 256 * 8) {
    const int k0 = base + tid * 8;
    const int cstart = base + (tid & ~(TPC - 1)) * 8;  // first index of this lane's chunk
    double x[8];
    if (vec && k0 + 8 <= K) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double2 y = *reinterpret_cast<const double2*>(row + k0 + 2 * j);
        x[2 * j] = y.x;
        x[2 * j + 1] = y.y;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + j;
        x[j] = (r < R && k < K) ? row[k] : 0.0;
      }
    }
    int e = kHiLoExp;
    if constexpr (S != 2) {
      double m = 0.0;
#pragma unroll
      for (int j = 0; j < 8; ++j) m = fmax(m, fabs(x[j]));
#pragma unroll
      for (int w = TPC / 2; w >= 1; w >>= 1) m = fmax(m, __shfl_xor(m, w, TPC));
      e = 0;
      if (m > 0.0) (void)frexp(m, &e);  // max|x| < 2^e over the chunk
    }
    if ((tid & (TPC - 1)) == 0 && cstart < Kp)
      ex[(cstart / exp_chunk_len(S)) * (long long)ex_stride + r] = e;
    __bf16 d[8][S];
#pragma unroll
    for (int j = 0; j < 8; ++j) cut<S>(x[j], e, d[j]);
    // memory image of the wave's 16 K-steps: step lane/4, slice p, piece lane%4
#pragma unroll
    for (int p = 0; p < S; ++p) {
      bf16x8 v;
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = d[j][p];
      *reinterpret_cast<bf16x8*>(wl + (lane >> 2) * STEP_BYTES + p * kSBK * 2 + (lane & 3) * 16) = v;
    }
    __builtin_amdgcn_wave_barrier();
    const int step0 = (base + wave * 512) / kSBK;  // first K-step of the wave's block
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const int byte = i * 1024 + lane * 16;
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(wl + byte);
      if ((step0 + byte / STEP_BYTES) * kSBK < Kp)
        *reinterpret_cast<bf16x8*>(orow + (long long)step0 * STEP_BYTES + byte) = v;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Rows with the row index contiguous: X[r][k] = X[k*ld + r] (the Cholesky
// vectors seen as rows (p,q) along x).  Exponents first, one thread per row.
__global__ __launch_bounds__(256) void rc_rowmax_kernel(const double* __restrict__ X, long long ld,
                                                        int R, int Rp, int K, int* __restrict__ ex) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= Rp) return;
  double m = 0.0;
  if (r < R)
    for (int k = 0; k < K; ++k) m = fmax(m, fabs(X[(long long)k * ld + r]));
  int e = 0;
  if (m > 0.0) (void)frexp(m, &e);
  ex[r] = e;
}

// Digits: thread per (row, 8 consecutive k); consecutive threads take consecutive rows.
template <int S>
__global__ __launch_bounds__(256) void slice_rc_kernel(const double* __restrict__ X, long long ld,
                                                       int R, int Rp, int K, int Kp,
                                                       int* __restrict__ ex,
                                                       __bf16* __restrict__ out) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long total = (long long)Rp * (Kp / 8);
  if (idx >= total) return;
  const int r = static_cast<int>(idx % Rp);
  const int k0 = static_cast<int>(idx / Rp) * 8;
  int e = kHiLoExp;
  if constexpr (S == 2) {
    if (k0 == 0) ex[r] = e;  // the hi/lo form needs no row maximum
  } else {
    e = ex[r];
  }
  __bf16 d[8][S];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = k0 + j;
    const double x = (r < R && k < K) ? X[(long long)k * ld + r] : 0.0;
    cut<S>(x, e, d[j]);
  }
#pragma unroll
  for (int p = 0; p < S; ++p) {
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = d[j][p];
    *reinterpret_cast<bf16x8*>(out + digit_offset<S>(r, k0, Kp) + p * kSBK) = v;
  }
}

// ---------------------------------------------------------------------------
// slice-pair GEMM
// ---------------------------------------------------------------------------

struct SplitArgs {
  const __bf16* A;   // [rows][Kp/32][S][32] digits, row 0 = this product's first row
  const int* ea;     // exponents of A's rows (same row origin); with chunk exponents
                     // ea[c * ea_stride + m] for K-chunk c
  const __bf16* B;
  const int* eb;
  int ea_stride, eb_stride;
  int M, N, Kp;
  void* C;           // EPI_ACC: float64 C[m*ldc + n] +=; EPI_PERM: float64 integral block;
                     // EPI_PACK: packed rows a <= b of the block; EPI_PAIR: R (both mirrors);
                     // EPI_SYM: float64 symmetric product C[m*ldc + n] of one operand with itself
  long long ldc;
  int v;
  int o;             // EPI_PAIR: occupied count (rows are (i,j))
  int a0;            // EPI_PACK/PAIR: first virtual of the integral block
  const int* row_tiles;  // EPI_PACK/EPI_SYM compact grid: first linear tile of each tile row
  int tiles_m, tiles_n, group_m;
  int m_off;             // EPI_ACC/PAIR: output row of this product's row 0 (a remainder launch)
};

// Workgroup tile BM x 128 (M x N), K-steps of 32 (one bf16 MFMA depth).  Slice
// products (p, q) (0-based) are kept when p + q < S + D - 1: D = 1 is the
// triangle p'+q' <= S+1 of 1-based slices, D = 2 adds its next anti-diagonal.
//
// Operand tiles go from global memory straight into LDS (global_load_lds_dwordx4:
// lane l of a wave writes 16 bytes at the wave's LDS base + 16*l), STAGES - 1
// K-steps loading ahead in a ring of LDS stages, one barrier per K-step.  A 16-row slab of a
// slice is one load instruction: lane l takes row l/4 and physical 16-byte slot
// l%4, which holds the logical k-chunk (l%4) ^ ((row/2)%4); fragment reads undo the
// XOR.  Keying on row/2 (pairs of 64-byte rows share a key) makes the 16-byte
// fragment reads free of bank conflicts on gfx950; keying on row/4, or no
// swizzle, costs one extra LDS cycle per read (measured with the hardware's
// bank-conflict counter on a read-pattern probe).
constexpr int kRowBytes = kSBK * 2;  // 64 bytes: one 32-deep row of bf16 digits

typedef __attribute__((address_space(3))) void lds_void_t;

__device__ __forceinline__ void wait_vm(int n) {
  // s_waitcnt with vmcnt = n (0..63); lgkmcnt and expcnt left unconstrained
  switch (n) {
#define CCL_VM(N) \
  case N:         \
    __builtin_amdgcn_s_waitcnt(((N)&15) | (7 << 4) | (15 << 8) | (((N) >> 4) << 14)); \
    break;
    CCL_VM(0) CCL_VM(3) CCL_VM(4) CCL_VM(6) CCL_VM(8) CCL_VM(9) CCL_VM(12)
#undef CCL_VM
    default:
      __builtin_amdgcn_s_waitcnt(7 << 4 | 15 << 8);
  }
}

// Slice-pair GEMM.  Every wave owns a sub-tile of MI x NJ 16 x 16 blocks and
// NACC anti-diagonal accumulators of it (shapes per slice count in SplitShape).
// Per K-step a wave reads the S slices of its column blocks once and streams the
// S slices of its row blocks; the float32 sums of a chunk (exact for the first
// NACC - 1 anti-diagonals, and for the last when it holds one) are drained into
// float64, and the epilogue applies 2^(eA + eB).
// Measured at o=40 v=360 P=1200 (S = 4): the MFMA units busy 62% of the time.
// 128 x 128 tiles (two stages) against 64 x 128 (three stages): 15% faster
// build, 4% faster contraction (whose 1600 rows waste 4% in 128-row tiles).
// A third stage for B only (all 160 KB of LDS) measured 2% slower; splitting the
// products of a sub-tile over two waves, or one wave per SIMD, the same or
// slower.  Raising the wave priority over the product loop gains 2-3%; the same
// in the float64 and float32 contraction loses 2%.
template <int S, int D, int EPI, int WAVES, int BM, int STAGES, int NACC, int NJ = 2>
__global__ __launch_bounds__(64 * WAVES, 1) void split_gemm_kernel(SplitArgs g) {
  // the contraction's operands carry chunk exponents
  constexpr bool CE = EPI == EPI_ACC || EPI == EPI_PAIR;
  constexpr int NG = S + D - 1;            // anti-diagonals kept
  constexpr int WCOLS = kSBN / (16 * NJ);  // waves along N (NJ column blocks per wave)
  constexpr int MI = BM / (16 * (WAVES / WCOLS));  // row blocks per wave
  constexpr int A_BYTES = S * BM * kRowBytes;
  constexpr int B_BYTES = S * kSBN * kRowBytes;
  constexpr int ASLABS = S * BM / 16, BSLABS = S * kSBN / 16;  // 16-row slabs per stage
  constexpr int LOADS = (ASLABS + BSLABS) / WAVES;              // per wave and stage
  constexpr int NLA = ASLABS / WAVES, NLB = BSLABS / WAVES;     // loads per wave and stage
  constexpr int AHEAD = STAGES - 1;                              // K-steps loading ahead
  constexpr int LDS_BYTES = STAGES * (A_BYTES + B_BYTES);
  static_assert((ASLABS % WAVES) == 0 && (BSLABS % WAVES) == 0, "slab split");
  static_assert(WCOLS * (WAVES / WCOLS) == WAVES && (WAVES / WCOLS) * MI * 16 == BM, "wave grid");
  static_assert(LDS_BYTES <= 160 * 1024, "LDS");
  static_assert(NACC >= 1 && NACC <= NG && (NACC == NG || NACC >= 3), "accumulator groups");
  static_assert(AHEAD >= 1 && LOADS * (AHEAD - 1) <= 12, "vmcnt of the loads left in flight");
  __shared__ __attribute__((aligned(1024))) unsigned char lds[LDS_BYTES];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave / WCOLS) * (16 * MI);
  const int wn = (wave % WCOLS) * (16 * NJ);
  // Tiles of linear ids it * G + xcd_linear(b) for workgroup b of G, so each
  // XCD walks contiguous runs of the tile order.  With two stages the kernel is
  // launched persistent (one workgroup per compute unit) and loads the first
  // K-step of its next tile while the current tile drains; otherwise G covers
  // every tile once.
  const int G = gridDim.x;
  constexpr bool kCompact = EPI == EPI_PACK || EPI == EPI_SYM;
  const int ntiles = kCompact ? g.row_tiles[g.tiles_m] : g.tiles_m * g.tiles_n;
  const int lin0 = xcd_linear(blockIdx.x, G);
  auto coords = [&](int lin, int& m0, int& n0) {
    int tm, tn;
    if (kCompact) {
      // compact grid over the tiles on or above the a = b diagonal (EPI_SYM:
      // v = 1, the tiles on or above the matrix diagonal)
      int lo = 0, hi = g.tiles_m - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.row_tiles[mid] <= lin) lo = mid; else hi = mid - 1;
      }
      tm = lo;
      tn = pack_first_tile(tm, BM, kSBN, g.v) + (lin - g.row_tiles[tm]);
    } else {
      tile_from_linear(lin, ntiles, g.tiles_m, g.group_m, tm, tn);
    }
    // uniform over the workgroup: kept in scalar registers
    m0 = __builtin_amdgcn_readfirstlane(tm * BM);
    n0 = __builtin_amdgcn_readfirstlane(tn * kSBN);
  };
  if (lin0 >= ntiles) return;

  const int lrow = lane >> 2;
  const int lchunk = (lane & 3) ^ ((lane >> 3) & 3);  // key (row >> 1) & 3
  const long long row_len = (long long)g.Kp * S;  // digits of one row, all slices
  const long long loff = (long long)lrow * row_len + lchunk * 8;
  // a wave loads slab after slab of the same 16 rows (consecutive slices), so
  // its instructions of a K-step cover whole lines
  // stage rings: A's STAGES stages, then B's
  // stages by global step gs (steps counted over all tiles of this workgroup)
  auto a_stage = [&](int gs) { return lds + (gs % STAGES) * A_BYTES; };
  auto b_stage = [&](int gs) { return lds + STAGES * A_BYTES + (gs % STAGES) * B_BYTES; };
  auto issue_a = [&](int m0, int kt, int gs) {
    unsigned char* st = a_stage(gs);
    const long long ko = (long long)kt * (S * kSBK);
#pragma unroll
    for (int j = 0; j < NLA; ++j) {
      const int ai = wave * NLA + j, r = ai / S, s = ai % S;
      __builtin_amdgcn_global_load_lds(
          (const void*)(g.A + (long long)(m0 + 16 * r) * row_len + loff + ko + s * kSBK),
          (lds_void_t*)(st + (s * BM + 16 * r) * kRowBytes), 16, 0, 0);
    }
  };
  auto issue_b = [&](int n0, int kt, int gs) {
    unsigned char* st = b_stage(gs);
    const long long ko = (long long)kt * (S * kSBK);
#pragma unroll
    for (int j = 0; j < NLB; ++j) {
      const int bi = wave * NLB + j, r = bi / S, s = bi % S;
      __builtin_amdgcn_global_load_lds(
          (const void*)(g.B + (long long)(n0 + 16 * r) * row_len + loff + ko + s * kSBK),
          (lds_void_t*)(st + (s * kSBN + 16 * r) * kRowBytes), 16, 0, 0);
    }
  };

  const int frag_off = (lane & 15) * kRowBytes + (((lane >> 4) ^ ((lane >> 1) & 3)) * 16);
  const int nk = g.Kp / kSBK;
  if (nk <= 0) return;
  const long long v = g.v;

  int lin = lin0, m0, n0;
  coords(lin, m0, n0);
  int gbase = 0;  // global step of this tile's first K-step
  // issue order: per K-step A then B; the wait counts below follow from it
#pragma unroll
  for (int k = 0; k < AHEAD; ++k) {
    if (k < nk) issue_a(m0, k, k);
    if (k < nk) issue_b(n0, k, k);
  }
  for (;;) {
  const int lin_next = lin + G;
  const bool more = lin_next < ntiles;  // only in a persistent (two-stage) launch
  int m0n = 0, n0n = 0;
  if (more) coords(lin_next, m0n, n0n);
  f64x4 acc64[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc64[i][j] = f64x4{0, 0, 0, 0};
  constexpr int kChunkSteps = chunk_steps<S>();
  for (int k0 = 0; k0 < nk; k0 += kChunkSteps) {
    // one chunk: float32 sums per anti-diagonal g = p + q (the last accumulator
    // takes every g >= NACC - 1)
    f32x4 acc[NACC][MI][NJ];
#pragma unroll
    for (int q = 0; q < NACC; ++q)
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[q][i][j] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < kChunkSteps; ++u) {
      const int kt = k0 + u;
      if (kt < nk) {
        // this K-step's loads are done when at most the later K-steps' remain
        const int later = (nk - 1 - kt) < (AHEAD - 1) ? (nk - 1 - kt) : (AHEAD - 1);
        wait_vm(later * LOADS);
        __builtin_amdgcn_s_barrier();
        {
          // this tile's step kt + AHEAD, or with two stages the next tile's
          // first step, into the stage this tile is done with
          const bool same = kt + AHEAD < nk;
          if (same || (STAGES == 2 && more)) {
            issue_a(same ? m0 : m0n, same ? kt + AHEAD : 0, gbase + kt + AHEAD);
            issue_b(same ? n0 : n0n, same ? kt + AHEAD : 0, gbase + kt + AHEAD);
          }
        }
        const unsigned char* sta = a_stage(gbase + kt);
        const unsigned char* stb = b_stage(gbase + kt);
        bf16x8 fb[S][NJ];
#pragma unroll
        for (int q = 0; q < S; ++q)
#pragma unroll
          for (int j = 0; j < NJ; ++j)
            fb[q][j] = *reinterpret_cast<const bf16x8*>(
                stb + (q * kSBN + wn + 16 * j) * kRowBytes + frag_off);
        // raised priority while this wave issues its products: the other wave
        // on the SIMD then takes its LDS reads and drains between them
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int p = 0; p < S; ++p) {
          if (p >= NG) continue;
          bf16x8 fa[MI];
#pragma unroll
          for (int i = 0; i < MI; ++i)
            fa[i] = *reinterpret_cast<const bf16x8*>(sta + (p * BM + wm + 16 * i) * kRowBytes +
                                                     frag_off);
#pragma unroll
          for (int q = 0; q < S; ++q) {
            if (p + q >= NG) continue;
            const int gq = (p + q) < NACC - 1 ? (p + q) : NACC - 1;
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
              for (int j = 0; j < NJ; ++j)
                acc[gq][i][j] =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[q][j], acc[gq][i][j], 0, 0, 0);
          }
        }
        __builtin_amdgcn_s_setprio(0);
      }
    }
    if constexpr (CE) {
      // this chunk's row and column scales 2^eA, 2^eB; the groups (each with
      // its own scale already) are first combined, then scaled once per element
      const int c = k0 / kChunkSteps;
      double sa[MI][4], sb[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          sa[i][r] = S == 2 ? 256.0  // hi/lo: every exponent is kHiLoExp
                            : ldexp(1.0, g.ea[(long long)c * g.ea_stride + m0 + wm + 16 * i +
                                               4 * (lane >> 4) + r]);
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        sb[j] = S == 2 ? 256.0
                       : ldexp(1.0, g.eb[(long long)c * g.eb_stride + n0 + wn + 16 * j + (lane & 15)]);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double u = 0.0;
#pragma unroll
            for (int q = 0; q < NACC; ++q) u += static_cast<double>(acc[q][i][j][r]);
            acc64[i][j][r] = fma(u, sa[i][r] * sb[j] * (1.0 / 65536.0), acc64[i][j][r]);
          }
    } else {
#pragma unroll
      for (int q = 0; q < NACC; ++q)
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              acc64[i][j][r] =
                  fma(static_cast<double>(acc[q][i][j][r]), 1.0 / 65536.0, acc64[i][j][r]);
    }
  }

  // this lane's first row, opaque to the optimiser (the row arithmetic of the
  // stores stays here instead of registers held across the K loop); the builds'
  // per-row exponents of its 16 rows and NJ columns are loaded together first,
  // rows past M and columns past N reading the exponent tables' padding
  int mb = m0 + wm + 4 * (lane >> 4);
  asm volatile("" : "+v"(mb));
  int erow[MI][4] = {}, ecol[NJ] = {};
  if constexpr (!CE && S != 2) {
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) erow[i][r] = g.ea[mb + 16 * i + r];
#pragma unroll
    for (int j = 0; j < NJ; ++j) ecol[j] = g.eb[n0 + wn + 16 * j + (lane & 15)];
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int n = n0 + wn + 16 * j + (lane & 15);
    if (n >= g.N) continue;
    const int en = CE ? 0 : (S == 2 ? kHiLoExp : ecol[j]);
    long long ncol = n;
    int pa = 0, pb = 0;  // EPI_PACK: b - a0 and d; EPI_PAIR: a and b
    if (EPI == EPI_PERM) {
      const int y = n / g.v, d = n - y * g.v;
      ncol = (long long)y * v * v + d;
    } else if (EPI == EPI_PACK) {
      pa = n / g.v;
      pb = n - pa * g.v;
    } else if (EPI == EPI_PAIR) {
      const long long q = pair_prefix_d(g.a0, v) + n;
      pa = pair_row(q, g.v);
      pb = pa + static_cast<int>(q - pair_prefix_d(pa, v));
    }
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mb + 16 * i + r;
        if (m >= g.M) continue;
        const double val =
            CE ? acc64[i][j][r] : ldexp(acc64[i][j][r], (S == 2 ? kHiLoExp : erow[i][r]) + en);
        double* C = static_cast<double*>(g.C);
        const int mo = m + g.m_off;  // output row
        if (EPI == EPI_ACC) {
          C[(long long)mo * g.ldc + n] += val;
        } else if (EPI == EPI_PERM) {
          const int a = m / g.v, x = m - a * g.v;
          C[(long long)a * v * v * v + ncol + (long long)x * v] = val;
        } else if (EPI == EPI_PACK) {
          // rows (a, c) of the block, columns (b, d) from b = a0; keep b >= a
          const int al = m / g.v, c = m - al * g.v;
          if (pa < al) continue;
          const long long row = pair_prefix_d(g.a0 + al, v) - pair_prefix_d(g.a0, v) + (pa - al);
          C[row * v * v + (long long)c * v + pb] = val;
        } else if (EPI == EPI_SYM) {
          // C[m][n] and its mirror C[n][m], from the element on or above the
          // diagonal (A and B are one operand: the element below it in a
          // diagonal tile holds the same value)
          if (m > n) continue;
          C[(long long)m * g.ldc + n] = val;
          if (m < n) C[(long long)n * g.ldc + m] = val;
        } else {  // EPI_PAIR: R[i][j][a][b] and, for a != b, R[j][i][b][a]
          C[(long long)mo * g.ldc + (long long)pa * v + pb] += val;
          if (pa != pb) {
            const int ii = mo / g.o, jj = mo - ii * g.o;
            C[(long long)(jj * g.o + ii) * g.ldc + (long long)pb * v + pa] += val;
          }
        }
      }
  }
  if (!more) break;
  lin = lin_next;
  m0 = m0n;
  n0 = n0n;
  gbase += nk;
  }
}

// Tile-row offsets of the packed build's compact grid (one thread; a few
// thousand tile rows at most).
__global__ void split_pack_rows_kernel(int* row_tiles, int tiles_m, int tiles_n, int v, int bm) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int acc = 0;
  for (int tm = 0; tm < tiles_m; ++tm) {
    row_tiles[tm] = acc;
    const int first = pack_first_tile(tm, bm, kSBN, v);
    acc += first < tiles_n ? tiles_n - first : 0;
  }
  row_tiles[tiles_m] = acc;
}

// Kernel shape per slice count.  S = 4: 128 x 128 tiles in two 64 KB stages,
// 8 waves of 64 x 32 sub-tiles, anti-diagonals g >= 2 (scales <= 2^-16 of the
// leading one) in one rounded float32 accumulator so that the sub-tile fits 256
// registers; S = 2 (hi/lo): 128 x 128 tiles in four 32 KB stages, one float32
// sum per anti-diagonal; S = 3: 64 x 128 tiles in three stages and 4 waves (its
// stage does not split 8 ways) of 64 x 32 sub-tiles, exact.
template <int S, int D>
struct SplitShape {
  static constexpr int NG = S + D - 1;
  static constexpr int NJ = 2;  // column blocks per wave
  static constexpr int W = S == 3 ? 4 : 8;
  static constexpr int BM = S == 3 ? 64 : 128;
  static constexpr int STAGES = S == 4 ? 2 : (S == 2 ? 4 : 3);
  static constexpr int NACC = S == 4 && NG > 3 ? 3 : NG;
};

// Compute units of the current device (queried once per device).
int split_compute_units() {
  static int cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

// Rows of a 128-row-tile product that a launch of 64-row tiles takes over (0 =
// none): the remainder, when the last tile row would be at most half full and
// the two launches finish first by (rounds of the grid over the 256 CUs) x
// (tile height).
long long split_remainder_rows(long long M, long long N) {
  constexpr long long kCUs = 256;
  const long long tn = (N + kSBN - 1) / kSBN;
  auto span = [&](long long rows, long long bm) {
    return ((rows + bm - 1) / bm * tn + kCUs - 1) / kCUs * bm;
  };
  const long long rem = M % 128;
  if (M <= 128 || rem == 0 || rem > 64) return 0;
  return span(M - rem, 128) + span(rem, 64) < span(M, 128) ? rem : 0;
}

template <int S, int D, int EPI>
int launch_split_gemm(const SplitArgs& a0, hipStream_t s) {
  using Sh = SplitShape<S, D>;
  SplitArgs a = a0;
  if (a.M <= 0 || a.N <= 0) return CC_LADDER_OK;
  if constexpr ((EPI == EPI_ACC || EPI == EPI_PAIR) && Sh::BM == 128) {
    // the remainder rows of the amplitude contraction in a launch of 64-row
    // tiles (8 waves of 32 x 32, three stages, or four with two slices)
    const long long rem = split_remainder_rows(a.M, a.N);
    if (rem > 0) {
      SplitArgs r = a;
      a.M -= static_cast<int>(rem);
      r.M = static_cast<int>(rem);
      r.A += (long long)a.M * a.Kp * S;
      r.ea += a.M;
      r.m_off = a.m_off + a.M;
      r.tiles_m = 1;
      r.tiles_n = (r.N + kSBN - 1) / kSBN;
      r.group_m = 1;
      constexpr int RST = S == 2 ? 4 : 3;
      hipLaunchKernelGGL((split_gemm_kernel<S, D, EPI, 8, 64, RST, Sh::NACC>),
                         dim3(static_cast<unsigned>(r.tiles_n)), dim3(512), 0, s, r);
      if (hipGetLastError() != hipSuccess) return CC_LADDER_EHIP;
    }
  }
  a.tiles_m = (a.M + Sh::BM - 1) / Sh::BM;
  a.tiles_n = (a.N + kSBN - 1) / kSBN;
  const long long tiles = (long long)a.tiles_m * a.tiles_n;
  if (tiles > 0x7fffffffLL) return CC_LADDER_EINVAL;
  a.group_m = a.tiles_m < 16 ? a.tiles_m : 16;
  long long grid = tiles;
  if (EPI == EPI_PACK || EPI == EPI_SYM) {
    if (!a.row_tiles) return CC_LADDER_EINVAL;
    long long needed = 0;
    for (int tm = 0; tm < a.tiles_m; ++tm) {
      const int first = pack_first_tile(tm, Sh::BM, kSBN, a.v);
      needed += first < a.tiles_n ? a.tiles_n - first : 0;
    }
    if (needed <= 0) return CC_LADDER_OK;
    hipLaunchKernelGGL(split_pack_rows_kernel, dim3(1), dim3(1), 0, s,
                       const_cast<int*>(a.row_tiles), a.tiles_m, a.tiles_n, a.v, Sh::BM);
    grid = needed;
  }
  // two-stage shapes run persistent: one workgroup per compute unit
  if (Sh::STAGES == 2 && grid > split_compute_units()) grid = split_compute_units();
  hipLaunchKernelGGL((split_gemm_kernel<S, D, EPI, Sh::W, Sh::BM, Sh::STAGES, Sh::NACC, Sh::NJ>),
                     dim3(static_cast<unsigned>(grid)), dim3(64 * Sh::W), 0, s, a);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

template <int S>
int slice_kc(const double* X, long long ld, int R, int K, const SliceDims& d, __bf16* out, int* ex,
             hipStream_t s) {
  hipLaunchKernelGGL((slice_kc_kernel<S>), dim3(d.rows_pad), dim3(256), 0, s, X, ld, R, K, d.k_pad,
                     out, ex, d.rows_pad);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

template <int S>
int slice_rc(const double* X, long long ld, int R, int K, const SliceDims& d, __bf16* out, int* ex,
             hipStream_t s) {
  if (S != 2)
    hipLaunchKernelGGL(rc_rowmax_kernel, dim3((d.rows_pad + 255) / 256), dim3(256), 0, s, X, ld, R,
                       d.rows_pad, K, ex);
  const long long total = (long long)d.rows_pad * (d.k_pad / 8);
  hipLaunchKernelGGL((slice_rc_kernel<S>), dim3(static_cast<unsigned>((total + 255) / 256)),
                     dim3(256), 0, s, X, ld, R, d.rows_pad, K, d.k_pad, ex, out);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

template <int S, int D>
int split_forward_s(const Plan& pl, const double* L, const double* t, double* R, char* ws,
                    const Tracer& tr, hipStream_t s) {
  const int o = pl.o, v = pl.v, P = pl.P;
  const long long v2 = (long long)v * v;
  // with symmetric vectors the digit rows are the packed vectors' columns {a,c}
  const bool gsym = pl.gsym != 0;
  const long long npv = (long long)v * (v + 1) / 2;
  const SliceDims dL = slice_dims(gsym ? pl.ldg : v2, P);
  const SliceDims dt = slice_dims((long long)o * o, static_cast<int>(v2));
  // integral rows of the largest block: n_a*v, or its packed rows a <= b
  const SliceDims dV = slice_dims(pl.pairsym ? pl.npk : (long long)pl.n_a * v,
                                  static_cast<int>(v2));
  __bf16* Ls = reinterpret_cast<__bf16*>(ws + pl.off_L);
  int* Le = reinterpret_cast<int*>(ws + pl.off_Lexp);
  __bf16* ts = reinterpret_cast<__bf16*>(ws + pl.off_t);
  int* te = reinterpret_cast<int*>(ws + pl.off_texp);
  double* V = reinterpret_cast<double*>(ws + pl.off_V);
  __bf16* Vs = reinterpret_cast<__bf16*>(ws + pl.off_Vs);
  int* Ve = reinterpret_cast<int*>(ws + pl.off_Vexp);
  const long long Lrow = (long long)dL.k_pad * S;  // digits per row of L's buffer

  double* G = gsym ? reinterpret_cast<double*>(ws + pl.off_G) : nullptr;
  tr(CC_LADDER_PHASE_PREP, 0, 0);
  int rc;
  if (gsym) {
    double* Lp = reinterpret_cast<double*>(ws + pl.off_Lp);
    rc = pack_pair_vectors(L, Lp, P, v, pl.ldg, s);
    if (!rc) rc = slice_rc<S>(Lp, pl.ldg, static_cast<int>(npv), P, dL, Ls, Le, s);
  } else {
    rc = slice_rc<S>(L, v2, static_cast<int>(v2), P, dL, Ls, Le, s);
  }
  if (!rc) rc = slice_kc<S>(t, v2, o * o, static_cast<int>(v2), dt, ts, te, s);
  tr(CC_LADDER_PHASE_PREP, 0, 1);
  if (rc) return rc;
  if (gsym) {
    // the whole pair-pair integral G[p][q] = sum_x Lp[x][p] Lp[x][q] from the
    // packed vectors' digits, the tiles on or above the diagonal (each result
    // stored with its mirror); traced as the build of block 0
    SplitArgs gg{};
    gg.A = Ls; gg.ea = Le;
    gg.B = Ls; gg.eb = Le;
    gg.ea_stride = gg.eb_stride = 0;  // one exponent per row
    gg.M = static_cast<int>(npv); gg.N = static_cast<int>(npv); gg.Kp = dL.k_pad;
    gg.C = G; gg.ldc = pl.ldg; gg.v = 1; gg.a0 = 0;
    gg.row_tiles = reinterpret_cast<const int*>(ws + pl.off_tiles);
    tr(CC_LADDER_PHASE_BUILD, 0, 0);
    rc = launch_split_gemm<S, D, EPI_SYM>(gg, s);
    tr(CC_LADDER_PHASE_BUILD, 0, 1);
    if (rc) return rc;
  }
  for (int blk = 0; blk < pl.nblocks; ++blk) {
    int a0, na;
    block_range(pl, blk, &a0, &na);
    if (na <= 0) continue;
    const long long r0 = (long long)a0 * v;  // first (a,c) row of this block
    if (pl.pairsym) {
      // packed rows (a,b), b >= a: columns (b,d) from b = a0 on
      const long long npairs = pair_prefix(a0 + na, v) - pair_prefix(a0, v);
      tr(CC_LADDER_PHASE_BUILD, blk, 0);
      if (gsym) {
        // the block's packed rows gathered from G
        rc = gather_pair_rows(G, pl.ldg, npairs, a0, v, V, s);
      } else {
        SplitArgs b{};
        b.A = Ls + r0 * Lrow; b.ea = Le + r0;
        b.B = Ls + r0 * Lrow; b.eb = Le + r0;
        b.ea_stride = b.eb_stride = 0;
        b.M = na * v; b.N = static_cast<int>((long long)(v - a0) * v); b.Kp = dL.k_pad;
        b.C = V; b.ldc = 0; b.v = v; b.a0 = a0;
        b.row_tiles = reinterpret_cast<const int*>(ws + pl.off_tiles);
        rc = launch_split_gemm<S, D, EPI_PACK>(b, s);
      }
      tr(CC_LADDER_PHASE_BUILD, blk, 1);
      if (rc) return rc;
      tr(CC_LADDER_PHASE_SLICE, blk, 0);
      rc = slice_kc<S>(V, v2, static_cast<int>(npairs), static_cast<int>(v2), dV, Vs, Ve, s);
      tr(CC_LADDER_PHASE_SLICE, blk, 1);
      if (rc) return rc;
      SplitArgs c{};
      c.A = ts; c.ea = te;
      c.B = Vs; c.eb = Ve;
      c.ea_stride = dt.rows_pad;
      c.eb_stride = dV.rows_pad;
      c.M = o * o; c.N = static_cast<int>(npairs); c.Kp = dt.k_pad;
      c.C = R; c.ldc = v2; c.v = v; c.o = o; c.a0 = a0;
      tr(CC_LADDER_PHASE_CONTRACT, blk, 0);
      rc = launch_split_gemm<S, D, EPI_PAIR>(c, s);
      tr(CC_LADDER_PHASE_CONTRACT, blk, 1);
      if (rc) return rc;
      continue;
    }
    SplitArgs b{};
    b.A = Ls + r0 * Lrow; b.ea = Le + r0;
    b.B = Ls; b.eb = Le;
    b.ea_stride = b.eb_stride = 0;  // one exponent per row
    b.M = na * v; b.N = static_cast<int>(v2); b.Kp = dL.k_pad;
    b.C = V; b.ldc = 0; b.v = v;
    tr(CC_LADDER_PHASE_BUILD, blk, 0);
    rc = launch_split_gemm<S, D, EPI_PERM>(b, s);
    tr(CC_LADDER_PHASE_BUILD, blk, 1);
    if (rc) return rc;
    tr(CC_LADDER_PHASE_SLICE, blk, 0);
    rc = slice_kc<S>(V, v2, na * v, static_cast<int>(v2), dV, Vs, Ve, s);
    tr(CC_LADDER_PHASE_SLICE, blk, 1);
    if (rc) return rc;
    SplitArgs c{};
    c.A = ts; c.ea = te;
    c.B = Vs; c.eb = Ve;
    c.ea_stride = dt.rows_pad;  // exponents per (row, chunk)
    c.eb_stride = dV.rows_pad;
    c.M = o * o; c.N = na * v; c.Kp = dt.k_pad;
    c.C = R + r0; c.ldc = v2; c.v = v;
    tr(CC_LADDER_PHASE_CONTRACT, blk, 0);
    rc = launch_split_gemm<S, D, EPI_ACC>(c, s);
    tr(CC_LADDER_PHASE_CONTRACT, blk, 1);
    if (rc) return rc;
  }
  return CC_LADDER_OK;
}

}  // namespace

int split_forward(const Plan& pl, const double* L, const double* t, double* R, char* ws,
                  const Tracer& tr, hipStream_t stream) {
  switch (pl.slices * 10 + pl.split_depth) {
    case 21: return split_forward_s<2, 1>(pl, L, t, R, ws, tr, stream);
    case 22: return split_forward_s<2, 2>(pl, L, t, R, ws, tr, stream);
    case 31: return split_forward_s<3, 1>(pl, L, t, R, ws, tr, stream);
    case 32: return split_forward_s<3, 2>(pl, L, t, R, ws, tr, stream);
    case 41: return split_forward_s<4, 1>(pl, L, t, R, ws, tr, stream);
    case 42: return split_forward_s<4, 2>(pl, L, t, R, ws, tr, stream);
    default: return CC_LADDER_EINVAL;
  }
}

}  // namespace ccl
