// Split-int8 form of the ladder forward: the digit scheme of the split forms
// on the integer matrix cores.
//
// Every operand row (a row of the matrix along its contracted index) gets an
// exponent per chunk of 16384 contracted indices, e with m < 2^e * 127/128 for
// the chunk's largest |x| = m, and each value is cut into S balanced int8
// digits:
//   X = rint(x 2^(7 + 8(S-1) - e)) = sum_{p=0..S-1} d_p 2^(8(S-1-p)),
//   d_p in [-128, 127] taken from the lowest one up (the leading one ends in
//   [-127, 127]), so x = 2^e sum_p d_p 2^-(7+8p) + r with |r| <= 2^(e - 8S - 2).
// Five digits carry 39 bits below each chunk's maximum.  A product of two
// such matrices is, per chunk c,
//   C[m][n] += 2^(eA[m,c] + eB[n,c] - 14) sum_g 2^(-8g) sum_{p+q=g} sum_{k in c} dA_p[m][k] dB_q[n][k],
// keeping the anti-diagonals g = p + q <= S + D - 2 (D = 1: the S(S+1)/2-
// product triangle).  The inner sums run on v_mfma_i32_16x16x64_i8 in int32
// and are exact: a group holds at most S products of magnitude <= 2^14 per
// index, at most 5 * 2^14 * 16384 < 2^31 over a chunk.  So the only rounding
// is the cut of the operands and the float64 drain of each chunk, which goes
// straight into the output (R, or the float64 integral block), about eight
// read-modify-writes of a tile over the 129600-long contraction of the
// o=40 v=360 P=1200 workload; no float64 accumulator stays in registers.
//
// Against the bf16 digits of the split-bf16 form (8 significant bits in 16 bits
// of storage, float32 sums exact only over 256 indices): half the bytes per
// digit, twice the MFMA rate (int8 5.0 POP/s dense against bf16 2.5 PFLOP/s),
// and exact sums over whole chunks.
#include "split.hpp"

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gemm.hpp"

namespace ccl {
namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kIBK = 64;                      // K per stage: one int8 MFMA depth
constexpr int kIRow = kIBK;                   // bytes of one digit row per K-step
constexpr int kIChunkSteps = kI8Chunk / kIBK; // K-steps per exponent chunk and drain
constexpr int kIBM = 128, kIBN = 128;         // workgroup tile
constexpr int kIWaves = 8, kINJ = 2;          // waves per workgroup, 16-column blocks per wave

// Exponent of a chunk whose largest magnitude is m: m < 2^e * 127/128.
__device__ __forceinline__ int i8_exponent(double m) {
  if (!(m > 0.0)) return 0;
  int e;
  (void)frexp(m, &e);  // m < 2^e
  if (m >= ldexp(127.0 / 128.0, e)) ++e;
  return e;
}

// The S digits of x on exponent e (digit 0 the leading one).
template <int S>
__device__ __forceinline__ void i8_digits(double x, int e, int (&d)[S]) {
  long long X = static_cast<long long>(rint(ldexp(x, 7 + 8 * (S - 1) - e)));
#pragma unroll
  for (int p = S - 1; p > 0; --p) {
    const int lo = static_cast<int>((X + 128) & 255) - 128;
    d[p] = lo;
    X = (X - lo) >> 8;  // exact: X - lo is a multiple of 256
  }
  d[0] = static_cast<int>(X);
}

// Digit buffers are [rows][k_pad / 64][S][64] int8: for each 64-deep K-step
// the S slices of one row are adjacent.  Byte offset of digit (p, k) of row r.
template <int S>
__device__ __forceinline__ long long i8_offset(long long r, int k, int Kp, int p) {
  return r * Kp * S + (long long)(k / kIBK) * (S * kIBK) + p * kIBK + (k % kIBK);
}

// Packs byte j of eight digits into one 8-byte word (little-endian order of k).
__device__ __forceinline__ unsigned long long pack8(const int (&v)[8]) {
  unsigned long long w = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) w |= static_cast<unsigned long long>(v[j] & 255) << (8 * j);
  return w;
}

// Rows with the contracted index contiguous, X[r][k] = X[r*ld + k]: one
// workgroup of 256 threads per (row, chunk of kI8Chunk).  Each thread holds 64
// values (eight groups of 8 consecutive k, 2048 apart), the workgroup agrees on
// the chunk's maximum, and every thread writes its digits as 8-byte words.
// Rows past R and indices past K are cut as zeros up to the padded sizes.
template <int S>
__global__ __launch_bounds__(256) void i8_slice_kc_kernel(const double* __restrict__ X, long long ld,
                                                          int R, int K, int Kp, int nch,
                                                          signed char* __restrict__ out,
                                                          int* __restrict__ ex, int ex_stride) {
  const int r = blockIdx.x / nch;
  const int c = blockIdx.x - r * nch;
  const int tid = threadIdx.x;
  const double* row = X + (long long)r * ld;
  const bool vec = r < R && (reinterpret_cast<unsigned long long>(row) & 15) == 0;
  const int kc = c * kI8Chunk;
  double x[8][8];
  double m = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k0 = kc + j * 2048 + tid * 8;
    if (vec && k0 + 8 <= K) {
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const double2 y = *reinterpret_cast<const double2*>(row + k0 + 2 * h);
        x[j][2 * h] = y.x;
        x[j][2 * h + 1] = y.y;
      }
    } else {
#pragma unroll
      for (int h = 0; h < 8; ++h) x[j][h] = (r < R && k0 + h < K) ? row[k0 + h] : 0.0;
    }
#pragma unroll
    for (int h = 0; h < 8; ++h) m = fmax(m, fabs(x[j][h]));
  }
  __shared__ double wmax[4];
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) m = fmax(m, __shfl_xor(m, w, 64));
  if ((tid & 63) == 0) wmax[tid >> 6] = m;
  __syncthreads();
  m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
  const int e = i8_exponent(m);
  if (tid == 0) ex[(long long)c * ex_stride + r] = e;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k0 = kc + j * 2048 + tid * 8;
    if (k0 >= Kp) continue;
    int d[8][S];
#pragma unroll
    for (int h = 0; h < 8; ++h) i8_digits<S>(x[j][h], e, d[h]);
#pragma unroll
    for (int p = 0; p < S; ++p) {
      int v8[8];
#pragma unroll
      for (int h = 0; h < 8; ++h) v8[h] = d[h][p];
      *reinterpret_cast<unsigned long long*>(out + i8_offset<S>(r, k0, Kp, p)) = pack8(v8);
    }
  }
}

// Rows with the row index contiguous, X[r][k] = X[k*ld + r] (the Cholesky
// vectors seen as rows (p,q) along x): exponents per (row, chunk), one thread
// per row, consecutive threads on consecutive rows.
__global__ __launch_bounds__(256) void i8_rowmax_rc_kernel(const double* __restrict__ X,
                                                           long long ld, int R, int Rp, int K,
                                                           int nch, int* __restrict__ ex) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long long)Rp * nch) return;
  const int c = static_cast<int>(idx / Rp);
  const int r = static_cast<int>(idx - (long long)c * Rp);
  double m = 0.0;
  if (r < R) {
    const int k1 = (c + 1) * kI8Chunk < K ? (c + 1) * kI8Chunk : K;
    for (int k = c * kI8Chunk; k < k1; ++k) m = fmax(m, fabs(X[(long long)k * ld + r]));
  }
  ex[(long long)c * Rp + r] = i8_exponent(m);
}

// Digits of row-contiguous rows: one thread per (row, 8 consecutive k).
template <int S>
__global__ __launch_bounds__(256) void i8_slice_rc_kernel(const double* __restrict__ X, long long ld,
                                                          int R, int Rp, int K, int Kp,
                                                          const int* __restrict__ ex,
                                                          signed char* __restrict__ out) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long long)Rp * (Kp / 8)) return;
  const int r = static_cast<int>(idx % Rp);
  const int k0 = static_cast<int>(idx / Rp) * 8;
  const int e = ex[(long long)(k0 / kI8Chunk) * Rp + r];
  int d[8][S];
#pragma unroll
  for (int h = 0; h < 8; ++h) {
    const int k = k0 + h;
    i8_digits<S>((r < R && k < K) ? X[(long long)k * ld + r] : 0.0, e, d[h]);
  }
#pragma unroll
  for (int p = 0; p < S; ++p) {
    int v8[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) v8[h] = d[h][p];
    *reinterpret_cast<unsigned long long*>(out + i8_offset<S>(r, k0, Kp, p)) = pack8(v8);
  }
}

struct I8Args {
  const signed char* A;  // [rows][Kp/64][S][64] digits, row 0 = this product's first row
  const int* ea;         // exponents of A's rows: ea[c * ea_stride + m] for chunk c
  const signed char* B;
  const int* eb;
  int ea_stride, eb_stride;
  int M, N, Kp;
  double* C;             // EPI_ACC: C[m*ldc + n] +=; EPI_PERM: float64 integral block;
                         // EPI_PACK: packed rows a <= b of the block; EPI_PAIR: R (both mirrors);
                         // EPI_SYM: the symmetric product C[m*ldc + n] of one operand with itself
  long long ldc;
  int v;
  int o;                 // EPI_PAIR: occupied count (rows are (i,j))
  int a0;                // EPI_PACK/PAIR: first virtual of the integral block
  const int* row_tiles;  // EPI_PACK/EPI_SYM compact grid: first linear tile of each tile row
  int tiles_m, tiles_n, group_m;
};

__device__ __forceinline__ void i8_wait_vm0() {
  __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));  // vmcnt(0)
}

typedef __attribute__((address_space(3))) void lds_void_i8;

// Digit-pair GEMM on the int8 MFMA.  128 x 128 tiles, 8 waves of 64 x 32
// sub-tiles (4 x 2 blocks of 16 x 16), two LDS stages of S x 256 digit rows of
// 64 bytes (80 KB each at S = 5).  Operands go from global memory straight into
// LDS (global_load_lds_dwordx4: lane l writes 16 bytes at the wave's LDS base +
// 16 l); a 16-row slab of one slice is one load instruction, lane l taking row
// l/4 and physical 16-byte slot l%4, which holds the logical slot
// (l%4) ^ ((row/2)%4) (fragment reads undo the XOR; the same conflict-free
// 64-byte-row swizzle as the bf16 kernel).  Lane l's fragment of a 16-row block
// is the 16 bytes of slot l/16 of row l%16, for A and B alike, so both operands
// enter each MFMA with the same k order.  One int32 sum per anti-diagonal;
// every kI8Chunk contracted indices (and at the end) the sums are scaled and
// added to the output in float64.
template <int S, int D, int EPI, int WAVES, int NJ>
__global__ __launch_bounds__(64 * WAVES, 1) void i8_gemm_kernel(I8Args g) {
  constexpr bool CE = true;  // chunked exponents on both operands
  constexpr int NG = S + D - 1;  // anti-diagonals kept
  constexpr int WCOLS = kIBN / (16 * NJ), MI = kIBM / (16 * (WAVES / WCOLS));
  constexpr int A_BYTES = S * kIBM * kIRow;
  constexpr int B_BYTES = S * kIBN * kIRow;
  constexpr int ASLABS = S * kIBM / 16, BSLABS = S * kIBN / 16;
  constexpr int NLA = ASLABS / WAVES, NLB = BSLABS / WAVES;
  constexpr int STAGES = 2;
  static_assert(ASLABS % WAVES == 0 && BSLABS % WAVES == 0, "slab split");
  static_assert(STAGES * (A_BYTES + B_BYTES) <= 160 * 1024, "LDS");
  static_assert(NG >= 1 && NG <= 2 * S - 1, "anti-diagonals");
  (void)CE;
  __shared__ __attribute__((aligned(1024))) unsigned char lds[STAGES * (A_BYTES + B_BYTES)];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave / WCOLS) * (16 * MI);
  const int wn = (wave % WCOLS) * (16 * NJ);
  // Persistent: workgroup b takes the tiles of linear ids it * G + xcd_linear(b)
  // (G workgroups, one per compute unit), so each XCD walks contiguous runs of
  // the tile order, and the first K-step of its next tile is loaded while the
  // current tile drains (one workgroup fits a compute unit, so nothing else
  // would hide that drain and the next tile's first loads).
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
      tn = pack_first_tile(tm, kIBM, kIBN, g.v) + (lin - g.row_tiles[tm]);
    } else {
      tile_from_linear(lin, ntiles, g.tiles_m, g.group_m, tm, tn);
    }
    // uniform over the workgroup: kept in scalar registers
    m0 = __builtin_amdgcn_readfirstlane(tm * kIBM);
    n0 = __builtin_amdgcn_readfirstlane(tn * kIBN);
  };
  if (lin0 >= ntiles) return;

  const int lrow = lane >> 2;
  const int lslot = (lane & 3) ^ ((lane >> 3) & 3);  // key (row >> 1) & 3
  const long long row_len = (long long)g.Kp * S;     // digit bytes of one row
  const long long loff = (long long)lrow * row_len + lslot * 16;
  // stage of global step gs (steps counted over all tiles of this workgroup)
  auto a_stage = [&](int gs) { return lds + (gs % STAGES) * A_BYTES; };
  auto b_stage = [&](int gs) { return lds + STAGES * A_BYTES + (gs % STAGES) * B_BYTES; };
  auto issue = [&](int m0, int n0, int kt, int gs) {
    const long long ko = (long long)kt * (S * kIBK);
    unsigned char* sa = a_stage(gs);
#pragma unroll
    for (int j = 0; j < NLA; ++j) {
      const int ai = wave * NLA + j, r = ai / S, s = ai % S;
      __builtin_amdgcn_global_load_lds(
          (const void*)(g.A + (long long)(m0 + 16 * r) * row_len + loff + ko + s * kIBK),
          (lds_void_i8*)(sa + (s * kIBM + 16 * r) * kIRow), 16, 0, 0);
    }
    unsigned char* sb = b_stage(gs);
#pragma unroll
    for (int j = 0; j < NLB; ++j) {
      const int bi = wave * NLB + j, r = bi / S, s = bi % S;
      __builtin_amdgcn_global_load_lds(
          (const void*)(g.B + (long long)(n0 + 16 * r) * row_len + loff + ko + s * kIBK),
          (lds_void_i8*)(sb + (s * kIBN + 16 * r) * kIRow), 16, 0, 0);
    }
  };

  const int frag_off = (lane & 15) * kIRow + (((lane >> 4) ^ ((lane >> 1) & 3)) * 16);
  const int nk = g.Kp / kIBK;
  const long long v = g.v;
  if (nk <= 0) return;

  int lin = lin0, m0, n0;
  coords(lin, m0, n0);
  int gbase = 0;  // global step of this tile's first K-step
  issue(m0, n0, 0, 0);
  for (;;) {
    const int lin_next = lin + G;
    const bool more = lin_next < ntiles;
    int m0n = 0, n0n = 0;
    if (more) coords(lin_next, m0n, n0n);
    for (int k0 = 0; k0 < nk; k0 += kIChunkSteps) {
      const int k1 = (k0 + kIChunkSteps) < nk ? (k0 + kIChunkSteps) : nk;
      i32x4 acc[NG][MI][NJ];
#pragma unroll
      for (int q = 0; q < NG; ++q)
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) acc[q][i][j] = i32x4{0, 0, 0, 0};
      for (int kt = k0; kt < k1; ++kt) {
        // step kt's loads are the only ones in flight; once they land and every
        // wave is past the previous step, the other stage takes the next step
        // (this tile's, or the next tile's first)
        i8_wait_vm0();
        __builtin_amdgcn_s_barrier();
        {
          const bool same = kt + 1 < nk;
          if (same || more)
            issue(same ? m0 : m0n, same ? n0 : n0n, same ? kt + 1 : 0, gbase + kt + 1);
        }
        const unsigned char* sa = a_stage(gbase + kt);
        const unsigned char* sb = b_stage(gbase + kt);
        i32x4 fb[S][NJ];
#pragma unroll
        for (int q = 0; q < S; ++q)
#pragma unroll
          for (int j = 0; j < NJ; ++j)
            fb[q][j] = *reinterpret_cast<const i32x4*>(sb + (q * kIBN + wn + 16 * j) * kIRow + frag_off);
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int p = 0; p < S; ++p) {
          if (p >= NG) continue;
          i32x4 fa[MI];
#pragma unroll
          for (int i = 0; i < MI; ++i)
            fa[i] = *reinterpret_cast<const i32x4*>(sa + (p * kIBM + wm + 16 * i) * kIRow + frag_off);
#pragma unroll
          for (int q = 0; q < S; ++q) {
            if (p + q >= NG) continue;
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
              for (int j = 0; j < NJ; ++j)
                acc[p + q][i][j] =
                    __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[i], fb[q][j], acc[p + q][i][j], 0, 0, 0);
          }
        }
        __builtin_amdgcn_s_setprio(0);
      }
      // drain chunk c into the output: 2^(eA + eB - 14) sum_g 2^(-8g) acc_g.
      // The exponents of this lane's 16 rows and NJ columns are loaded together
      // first, from one base each with constant offsets (rows past M and columns
      // past N read the zero-based padding of the exponent tables, which every
      // operand buffer carries past its last tile), so the drain waits on memory
      // once rather than once per element.
      const int c = k0 / kIChunkSteps;
      const bool first = k0 == 0;
      // this lane's first row; opaque to the optimiser, so the row arithmetic of
      // the stores stays here instead of being hoisted into registers held (and
      // spilled) across the K loop
      int mb = m0 + wm + 4 * (lane >> 4);
      asm volatile("" : "+v"(mb));
      const int* ep = g.ea + (long long)c * g.ea_stride + mb;
      const int* fp = g.eb + (long long)c * g.eb_stride + n0 + wn + (lane & 15);
      int erow[MI][4], ecol[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) erow[i][r] = ep[16 * i + r];
#pragma unroll
      for (int j = 0; j < NJ; ++j) ecol[j] = fp[16 * j];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (n >= g.N) continue;
        const int en = ecol[j];
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
            double u = 0.0;
#pragma unroll
            for (int q = NG - 1; q >= 0; --q)
              u = fma(static_cast<double>(acc[q][i][j][r]), 1.0 / static_cast<double>(1ull << (8 * q)),
                      u);
            const double val = ldexp(u, erow[i][r] + en - 14);
            double* C = g.C;
            if (EPI == EPI_ACC) {
              C[(long long)m * g.ldc + n] += val;
            } else if (EPI == EPI_PERM) {
              const int a = m / g.v, x = m - a * g.v;
              double* dst = C + (long long)a * v * v * v + ncol + (long long)x * v;
              *dst = first ? val : *dst + val;
            } else if (EPI == EPI_PACK) {
              const int al = m / g.v, cc = m - al * g.v;
              if (pa < al) continue;
              const long long prow =
                  pair_prefix_d(g.a0 + al, v) - pair_prefix_d(g.a0, v) + (pa - al);
              double* dst = C + prow * v * v + (long long)cc * v + pb;
              *dst = first ? val : *dst + val;
            } else if (EPI == EPI_SYM) {
              // C[m][n] and its mirror C[n][m], from the element on or above the
              // diagonal (A and B are one operand, so the element below the
              // diagonal in a diagonal tile holds the same value)
              if (m > n) continue;
              double* d1 = C + (long long)m * g.ldc + n;
              *d1 = first ? val : *d1 + val;
              if (m < n) {
                double* d2 = C + (long long)n * g.ldc + m;
                *d2 = first ? val : *d2 + val;
              }
            } else {  // EPI_PAIR: R[i][j][a][b] and, for a != b, R[j][i][b][a]
              C[(long long)m * g.ldc + (long long)pa * v + pb] += val;
              if (pa != pb) {
                const int ii = m / g.o, jj = m - ii * g.o;
                C[(long long)(jj * g.o + ii) * g.ldc + (long long)pb * v + pa] += val;
              }
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

// Tile-row offsets of the packed build's compact grid (one thread).
__global__ void i8_pack_rows_kernel(int* row_tiles, int tiles_m, int tiles_n, int v) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int acc = 0;
  for (int tm = 0; tm < tiles_m; ++tm) {
    row_tiles[tm] = acc;
    const int first = pack_first_tile(tm, kIBM, kIBN, v);
    acc += first < tiles_n ? tiles_n - first : 0;
  }
  row_tiles[tiles_m] = acc;
}

// Compute units of the current device (queried once per device).
int i8_compute_units() {
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

template <int S, int D, int EPI>
int launch_i8_gemm(const I8Args& a0, hipStream_t s) {
  I8Args a = a0;
  if (a.M <= 0 || a.N <= 0) return CC_LADDER_OK;
  a.tiles_m = (a.M + kIBM - 1) / kIBM;
  a.tiles_n = (a.N + kIBN - 1) / kIBN;
  const long long tiles = (long long)a.tiles_m * a.tiles_n;
  if (tiles > 0x7fffffffLL) return CC_LADDER_EINVAL;
  a.group_m = a.tiles_m < 16 ? a.tiles_m : 16;
  long long grid = tiles;
  if (EPI == EPI_PACK || EPI == EPI_SYM) {
    if (!a.row_tiles) return CC_LADDER_EINVAL;
    long long needed = 0;
    for (int tm = 0; tm < a.tiles_m; ++tm) {
      const int first = pack_first_tile(tm, kIBM, kIBN, a.v);
      needed += first < a.tiles_n ? a.tiles_n - first : 0;
    }
    if (needed <= 0) return CC_LADDER_OK;
    hipLaunchKernelGGL(i8_pack_rows_kernel, dim3(1), dim3(1), 0, s, const_cast<int*>(a.row_tiles),
                       a.tiles_m, a.tiles_n, a.v);
    grid = needed;
  }
  // one persistent workgroup per compute unit (or per tile, when fewer)
  const long long wgs = grid < i8_compute_units() ? grid : i8_compute_units();
  hipLaunchKernelGGL((i8_gemm_kernel<S, D, EPI, kIWaves, kINJ>), dim3(static_cast<unsigned>(wgs)),
                     dim3(64 * kIWaves), 0, s, a);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

template <int S>
int i8_slice_kc(const double* X, long long ld, int R, int K, const SliceDims& d, signed char* out,
                int* ex, hipStream_t s) {
  const int nch = i8_chunks(d.k_pad);
  const long long grid = (long long)d.rows_pad * nch;
  if (grid > 0x7fffffffLL) return CC_LADDER_EINVAL;
  hipLaunchKernelGGL((i8_slice_kc_kernel<S>), dim3(static_cast<unsigned>(grid)), dim3(256), 0, s, X,
                     ld, R, K, d.k_pad, nch, out, ex, d.rows_pad);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

template <int S>
int i8_slice_rc(const double* X, long long ld, int R, int K, const SliceDims& d, signed char* out,
                int* ex, hipStream_t s) {
  const int nch = i8_chunks(d.k_pad);
  const long long nmax = (long long)d.rows_pad * nch;
  hipLaunchKernelGGL(i8_rowmax_rc_kernel, dim3(static_cast<unsigned>((nmax + 255) / 256)), dim3(256),
                     0, s, X, ld, R, d.rows_pad, K, nch, ex);
  const long long total = (long long)d.rows_pad * (d.k_pad / 8);
  hipLaunchKernelGGL((i8_slice_rc_kernel<S>), dim3(static_cast<unsigned>((total + 255) / 256)),
                     dim3(256), 0, s, X, ld, R, d.rows_pad, K, d.k_pad, ex, out);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

template <int S, int D>
int i8_forward_s(const Plan& pl, const double* L, const double* t, double* R, char* ws,
                 const Tracer& tr, hipStream_t s) {
  const int o = pl.o, v = pl.v, P = pl.P;
  const long long v2 = (long long)v * v;
  // with symmetric vectors the digit rows are the packed vectors' columns {a,c}
  const bool gsym = pl.gsym != 0;
  const long long npv = (long long)v * (v + 1) / 2;
  const SliceDims dL = slice_dims(gsym ? pl.ldg : v2, P);
  const SliceDims dt = slice_dims((long long)o * o, static_cast<int>(v2));
  const SliceDims dV = slice_dims(pl.pairsym ? pl.npk : (long long)pl.n_a * v,
                                  static_cast<int>(v2));
  signed char* Ls = reinterpret_cast<signed char*>(ws + pl.off_L);
  int* Le = reinterpret_cast<int*>(ws + pl.off_Lexp);
  signed char* ts = reinterpret_cast<signed char*>(ws + pl.off_t);
  int* te = reinterpret_cast<int*>(ws + pl.off_texp);
  double* V = reinterpret_cast<double*>(ws + pl.off_V);
  signed char* Vs = reinterpret_cast<signed char*>(ws + pl.off_Vs);
  int* Ve = reinterpret_cast<int*>(ws + pl.off_Vexp);
  const long long Lrow = (long long)dL.k_pad * S;  // digit bytes per row of L's buffer

  double* G = gsym ? reinterpret_cast<double*>(ws + pl.off_G) : nullptr;
  tr(CC_LADDER_PHASE_PREP, 0, 0);
  int rc;
  if (gsym) {
    double* Lp = reinterpret_cast<double*>(ws + pl.off_Lp);
    rc = pack_pair_vectors(L, Lp, P, v, pl.ldg, s);
    if (!rc) rc = i8_slice_rc<S>(Lp, pl.ldg, static_cast<int>(npv), P, dL, Ls, Le, s);
  } else {
    rc = i8_slice_rc<S>(L, v2, static_cast<int>(v2), P, dL, Ls, Le, s);
  }
  if (!rc) rc = i8_slice_kc<S>(t, v2, o * o, static_cast<int>(v2), dt, ts, te, s);
  tr(CC_LADDER_PHASE_PREP, 0, 1);
  if (rc) return rc;
  if (gsym) {
    // the whole pair-pair integral G[p][q] = sum_x Lp[x][p] Lp[x][q] from the
    // packed vectors' digits, the tiles on or above the diagonal (each result
    // stored with its mirror); traced as the build of block 0
    I8Args gg{};
    gg.A = Ls; gg.ea = Le;
    gg.B = Ls; gg.eb = Le;
    gg.ea_stride = gg.eb_stride = dL.rows_pad;
    gg.M = static_cast<int>(npv); gg.N = static_cast<int>(npv); gg.Kp = dL.k_pad;
    gg.C = G; gg.ldc = pl.ldg; gg.v = 1; gg.a0 = 0;
    gg.row_tiles = reinterpret_cast<const int*>(ws + pl.off_tiles);
    tr(CC_LADDER_PHASE_BUILD, 0, 0);
    rc = launch_i8_gemm<S, D, EPI_SYM>(gg, s);
    tr(CC_LADDER_PHASE_BUILD, 0, 1);
    if (rc) return rc;
  }
  for (int blk = 0; blk < pl.nblocks; ++blk) {
    int a0, na;
    block_range(pl, blk, &a0, &na);
    if (na <= 0) continue;
    const long long r0 = (long long)a0 * v;  // first (a,c) row of this block
    const long long nrows = pl.pairsym ? pair_prefix(a0 + na, v) - pair_prefix(a0, v)
                                       : (long long)na * v;
    I8Args b{};
    b.A = Ls + r0 * Lrow; b.ea = Le + r0;
    b.ea_stride = b.eb_stride = dL.rows_pad;
    b.M = na * v; b.Kp = dL.k_pad;
    b.C = V; b.ldc = 0; b.v = v; b.a0 = a0;
    if (gsym) {
      // the block's packed rows gathered from G
      tr(CC_LADDER_PHASE_BUILD, blk, 0);
      rc = gather_pair_rows(G, pl.ldg, nrows, a0, v, V, s);
    } else if (pl.pairsym) {
      // packed rows (a,b), b >= a: columns (b,d) from b = a0 on
      b.B = Ls + r0 * Lrow; b.eb = Le + r0;
      b.N = static_cast<int>((long long)(v - a0) * v);
      b.row_tiles = reinterpret_cast<const int*>(ws + pl.off_tiles);
      tr(CC_LADDER_PHASE_BUILD, blk, 0);
      rc = launch_i8_gemm<S, D, EPI_PACK>(b, s);
    } else {
      b.B = Ls; b.eb = Le;
      b.N = static_cast<int>(v2);
      tr(CC_LADDER_PHASE_BUILD, blk, 0);
      rc = launch_i8_gemm<S, D, EPI_PERM>(b, s);
    }
    tr(CC_LADDER_PHASE_BUILD, blk, 1);
    if (rc) return rc;
    tr(CC_LADDER_PHASE_SLICE, blk, 0);
    rc = i8_slice_kc<S>(V, v2, static_cast<int>(nrows), static_cast<int>(v2), dV, Vs, Ve, s);
    tr(CC_LADDER_PHASE_SLICE, blk, 1);
    if (rc) return rc;
    I8Args c{};
    c.A = ts; c.ea = te;
    c.B = Vs; c.eb = Ve;
    c.ea_stride = dt.rows_pad;
    c.eb_stride = dV.rows_pad;
    c.M = o * o; c.N = static_cast<int>(nrows); c.Kp = dt.k_pad;
    c.v = v; c.o = o; c.a0 = a0; c.ldc = v2;
    tr(CC_LADDER_PHASE_CONTRACT, blk, 0);
    if (pl.pairsym) {
      c.C = R;
      rc = launch_i8_gemm<S, D, EPI_PAIR>(c, s);
    } else {
      c.C = R + r0;
      rc = launch_i8_gemm<S, D, EPI_ACC>(c, s);
    }
    tr(CC_LADDER_PHASE_CONTRACT, blk, 1);
    if (rc) return rc;
  }
  return CC_LADDER_OK;
}

}  // namespace

int split_i8_forward(const Plan& pl, const double* L, const double* t, double* R, char* ws,
                     const Tracer& tr, hipStream_t stream) {
  switch (pl.slices * 10 + pl.split_depth) {
    case 41: return i8_forward_s<4, 1>(pl, L, t, R, ws, tr, stream);
    case 42: return i8_forward_s<4, 2>(pl, L, t, R, ws, tr, stream);
    case 51: return i8_forward_s<5, 1>(pl, L, t, R, ws, tr, stream);
    default: return CC_LADDER_EINVAL;
  }
}

}  // namespace ccl
