// Amplitude-contraction GEMM with direct global->LDS operand loads (gfx950).
//
//   C[m][n] (+)= sum_k A[m*lda + k] B[n*ldb + k]   (both operands KC; EPI_ACC, EPI_PAIR,
//                                                   or EPI_PART: one K-range per workgroup)
//
// 512 threads = 8 wave64s in a 2 x 4 grid over a BM x 256 tile (BM = 128; the
// K-contiguous kernel also 64 and, for float64, 160); each wave owns (BM/2) x 64 =
// BM/32 x 4 MFMA blocks (v_mfma_f64_16x16x4_f64 or v_mfma_f32_16x16x4_f32).
// Every K-step is 128 bytes of each operand row.  Operand slabs of 8 rows go
// from global memory into LDS with global_load_lds_dwordx4 (lane l of a wave
// writes 16 bytes at the wave's LDS base + 16*l): lane l takes row l/8 and
// physical 16-byte slot l%8, which holds the logical k-chunk
// (l%8) ^ ((row/2) % 8).  Fragment reads undo the XOR, so the 16 rows read by
// 16 lanes of one ds_read_b128 land on 16 distinct 4-bank groups.  Three K-steps
// are in flight in a ring of LDS stages; one barrier per K-step.  Rows past M
// or N are clamped onto valid rows (their outputs are never stored); a ragged
// last K-step is loaded through registers with zero fill.
#pragma once

#include "gemm.hpp"

namespace ccl {

constexpr int kDBM = 128, kDBN = 256;
constexpr int kDThreads = 512;
constexpr int kDStages = 3;
constexpr int kDRow = 128;  // bytes of one operand row per K-step

typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ void d_wait_vm(int n) {
  switch (n) {
#define CCL_DVM(N) \
  case N:          \
    __builtin_amdgcn_s_waitcnt(((N)&15) | (7 << 4) | (15 << 8) | (((N) >> 4) << 14)); \
    break;
    CCL_DVM(0) CCL_DVM(5) CCL_DVM(6) CCL_DVM(7)
#undef CCL_DVM
    default:
      __builtin_amdgcn_s_waitcnt(7 << 4 | 15 << 8);
  }
}

// BM = 128 (4 x 4 blocks per wave); for float64 without drains also 160 (5 x 4
// blocks per wave, 156 KB of LDS), whose tiles divide o^2 = 1600 exactly and pad
// 900 and 3600 less; and 64 (2 x 4 blocks per wave) for the remainder rows of a
// product whose last 128-row tile row would be at most half full.
template <class Tr, int EPI, int BM = kDBM>
__global__ __launch_bounds__(kDThreads, 1) void gemm_kc_direct_kernel(GemmArgs<typename Tr::T> g) {
  static_assert(EPI == EPI_ACC || EPI == EPI_PAIR || EPI == EPI_PART || EPI == EPI_PM,
                "K-contiguous epilogues");
  static_assert(BM == kDBM || BM == 64 || (BM == 160 && !Tr::kDrain), "tile heights");
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  using Chunk = typename Tr::Chunk;
  constexpr int CH = Tr::CH;                 // elements per 16 bytes
  constexpr int BK = kDRow / sizeof(T);      // K per step (16 float64 / 32 float32)
  constexpr int MI = BM / 32;                // row blocks per wave (2 wave rows)
  constexpr int A_BYTES = BM * kDRow;        // 8, 16 or 20 KB
  constexpr int B_BYTES = kDBN * kDRow;      // 32 KB
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int A_SLABS = BM / 8, JA = (A_SLABS + 7) / 8;  // 8-row slabs of A; per wave at most JA
  static_assert(kDStages * STAGE <= 160 * 1024, "LDS");
  __shared__ __attribute__((aligned(1024))) unsigned char lds[kDStages * STAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave >> 2) * (BM / 2);
  const int wn = (wave & 3) * 64;
  // slabs this wave loads per stage: A slabs wave + 8j < A_SLABS, and 4 of B
  // (compile-time 5 or 6 when the A slabs split evenly over the 8 waves)
  constexpr bool A_EVEN = A_SLABS % 8 == 0;
  const int LOADS = A_EVEN ? A_SLABS / 8 + 4 : (A_SLABS - wave + 7) / 8 + 4;
  int tm, tn;
  const int nk_all = (g.K + BK - 1) / BK;
  int ks0 = 0, ks1 = nk_all;  // K-steps of this workgroup
  if (EPI == EPI_PART) {
    // grid = tiles x splits; the split is the outer index of the linear id
    const int ntiles = g.tiles_m * g.tiles_n;
    const int id = xcd_linear(blockIdx.x, gridDim.x);
    const int split = id / ntiles;
    tile_from_linear(id - split * ntiles, ntiles, g.tiles_m, g.group_m, tm, tn);
    ks0 = split * g.split_steps;
    ks1 = ks0 + g.split_steps < nk_all ? ks0 + g.split_steps : nk_all;
    g.C = static_cast<double*>(g.C) + split * g.part_stride;
  } else if (g.kband) {
    tile_of_banded(g.kband, blockIdx.x, gridDim.x, g.tiles_m, g.group_m, tm, tn);
  } else {
    tile_of(blockIdx.x, gridDim.x, g.tiles_m, g.group_m, tm, tn);
  }
  const int m0 = tm * BM, n0 = tn * kDBN;
  if (EPI != EPI_PART && g.kband) k_band(g, n0, kDBN, BK, ks0, ks1);

  // Slabs: A rows 8*(wave + 8*j), j < JA; B rows 8*(wave + 8*j), j < 4.  The
  // swizzle of a lane depends on the slab's parity only (slab origin 8*s rows).
  const int lrow = lane >> 3;
  const int sw_even = ((lane & 7) ^ ((lane >> 4) & 7)) * CH;        // slab index even
  const int sw_odd = ((lane & 7) ^ ((4 + (lane >> 4)) & 7)) * CH;   // slab index odd
  const int my_sw = (wave & 1) ? sw_odd : sw_even;  // slabs wave + 8j share the wave's parity
  const T* pa[JA];
  const T* pb[4];
#pragma unroll
  for (int j = 0; j < JA; ++j) {
    int row = m0 + 8 * (wave + 8 * j) + lrow;
    row = row < g.M ? row : g.M - 1;
    pa[j] = g.A + (long long)row * g.lda + my_sw;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int row = n0 + 8 * (wave + 8 * j) + lrow;
    row = row < g.N ? row : g.N - 1;
    pb[j] = g.B + (long long)row * g.ldb + my_sw;
  }
  auto issue = [&](int kt) {
    unsigned char* st = lds + (kt % kDStages) * STAGE;
    const int ko = kt * BK;
#pragma unroll
    for (int j = 0; j < JA; ++j)
      if (A_EVEN || wave + 8 * j < A_SLABS)
        __builtin_amdgcn_global_load_lds((const void*)(pa[j] + ko),
                                         (lds_void*)(st + 8 * (wave + 8 * j) * kDRow), 16, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(pb[j] + ko),
                                       (lds_void*)(st + A_BYTES + 8 * (wave + 8 * j) * kDRow), 16,
                                       0, 0);
  };
  // Ragged last K-step: same LDS image, loaded through registers with zero fill.
  auto issue_tail = [&](int kt) {
    unsigned char* st = lds + (kt % kDStages) * STAGE;
    const int k0 = kt * BK;
    auto one = [&](const T* p, unsigned char* dst) {
      const int kk = k0 + my_sw;  // this lane's first k (p already points my_sw past the row)
      Chunk c;
#pragma unroll
      for (int e = 0; e < CH; ++e) c[e] = (kk + e < g.K) ? p[k0 + e] : T(0);
      *reinterpret_cast<Chunk*>(dst + 16 * lane) = c;
    };
#pragma unroll
    for (int j = 0; j < JA; ++j)
      if (A_EVEN || wave + 8 * j < A_SLABS) one(pa[j], st + 8 * (wave + 8 * j) * kDRow);
#pragma unroll
    for (int j = 0; j < 4; ++j) one(pb[j], st + A_BYTES + 8 * (wave + 8 * j) * kDRow);
    __builtin_amdgcn_s_waitcnt(0xF | (7 << 4) | (3 << 14));  // lgkmcnt(0): the LDS writes landed
  };

  Acc acc[MI][4];
  f64x4 acc64[MI][4];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = Acc{0, 0, 0, 0};
      acc64[i][j] = f64x4{0, 0, 0, 0};
    }

  // fragment: row (lane & 15) of a 16-row block (block origins are multiples
  // of 16, so the row's swizzle is ((lane & 15) >> 1)), logical chunk 4*gi + lane/16
  const int frow = (lane & 15) * kDRow;
  const int fsw = (lane & 15) >> 1;
  const int nk = ks1;        // one past this workgroup's last K-step
  const int nkf = g.K / BK;  // full K-steps; a ragged last one goes through registers
  auto stage_in = [&](int kt) {
    if (kt < nkf)
      issue(kt);
    else
      issue_tail(kt);
  };
  if (ks0 < nk) stage_in(ks0);
  if (ks0 + 1 < nk) stage_in(ks0 + 1);
  for (int k0 = ks0; k0 < nk;) {
    const int kend = (Tr::kDrain && k0 + g.drain_steps < nk) ? k0 + g.drain_steps : nk;
    for (int kt = k0; kt < kend; ++kt) {
      // step kt's direct loads have landed once only step kt+1's remain in flight
      // (a ragged step kt+1 goes through registers and is already complete, and
      // past this workgroup's range nothing more was issued)
      d_wait_vm(kt + 1 < nkf && kt + 1 < nk ? LOADS : 0);
      __builtin_amdgcn_s_barrier();
      if (kt + 2 < nk) stage_in(kt + 2);
      const unsigned char* st = lds + (kt % kDStages) * STAGE;
#pragma unroll
      for (int gi = 0; gi < 2; ++gi) {
        const int chunk = ((4 * gi + (lane >> 4)) ^ fsw) * 16;
        Chunk fa[MI], fb[4];
#pragma unroll
        for (int i = 0; i < MI; ++i)
          fa[i] = *reinterpret_cast<const Chunk*>(st + (wm + 16 * i) * kDRow + frow + chunk);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          fb[j] = *reinterpret_cast<const Chunk*>(st + A_BYTES + (wn + 16 * j) * kDRow + frow + chunk);
#pragma unroll
        for (int e = 0; e < CH; ++e)
#pragma unroll
          for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = Tr::mfma(fa[i][e], fb[j][e], acc[i][j]);
      }
    }
    if (Tr::kDrain) {
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            acc64[i][j][r] += static_cast<double>(acc[i][j][r]);
            acc[i][j][r] = 0;
          }
    }
    k0 = kend;
  }

  const int col = lane & 15;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + wn + 16 * j + col;
    if (n >= g.N) continue;
    const EpiCol ec = epi_col<T, EPI>(g, n);
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + Tr::row_of(lane, r);
        if (m >= g.M) continue;
        const double val = Tr::kDrain ? acc64[i][j][r] : static_cast<double>(acc[i][j][r]);
        epi_store<T, EPI>(g, m, n, ec, val);
      }
  }
}

}  // namespace ccl

namespace ccl {

// Integral-build GEMM with both operands row-contiguous (RC) and direct
// global->LDS loads (gfx950):
//
//   C = perm( sum_k A[k*lda + m] B[k*ldb + n] )          (EPI_PERM store in the operand type)
//
// Same 128 x 256 tile, 8 waves and 3-stage LDS ring as the K-contiguous kernel.
// A stage holds BK rows of k: 128 contiguous m of A and 256 contiguous n of B per
// row, filled 1 KB per wave instruction (lane l writes 16 bytes at +16*l).  An
// MFMA operand needs one value per lane from one k row, so the rows of the 4 x 4
// blocks of a wave are interleaved: block i's row r is wave row pos(i, r) with
// pos = 4r + i (float32) or 32*(i/2) + 2r + (i%2) (float64), making the values a
// lane needs for all four blocks one 16-byte LDS read (two for float64), the 16
// lanes of a k row reading 256 contiguous bytes (no bank conflicts, no swizzle).
// Columns are interleaved the same way, which also makes the values a lane stores
// for the four column blocks adjacent in the output: the permuted epilogue writes
// them with 16-byte stores when v is a multiple of the chunk.  Needs M and N
// multiples of the 16-byte chunk and 16-byte aligned operand rows; rows past M or
// N are clamped onto the last chunk (never stored); a ragged last K-step is
// loaded through registers with zero fill.
template <class Tr>
__device__ __forceinline__ int rc_pos(int i, int r) {
  if constexpr (Tr::CH == 4)
    return 4 * r + i;
  else
    return 32 * (i >> 1) + 2 * r + (i & 1);
}

template <class Tr, int EPI>
__global__ __launch_bounds__(kDThreads, 1) void gemm_rc_direct_kernel(GemmArgs<typename Tr::T> g) {
  static_assert(EPI == EPI_PERM || EPI == EPI_PACK || EPI == EPI_UNPACK || EPI == EPI_SYM,
                "integral-block stores");
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  using Chunk = typename Tr::Chunk;
  constexpr int CH = Tr::CH;
  constexpr int BK = kDRow / sizeof(T);          // 16 float64 / 32 float32 k rows per stage
  constexpr int ROWA = kDBM * sizeof(T);         // bytes of one k row of A (128 m)
  constexpr int ROWB = kDBN * sizeof(T);         // bytes of one k row of B (256 n)
  constexpr int A_BYTES = BK * ROWA;             // 16 KB
  constexpr int B_BYTES = BK * ROWB;             // 32 KB
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int AI = A_BYTES / 1024 / 8;         // 1 KB wave instructions per wave: A (2)
  constexpr int BI = B_BYTES / 1024 / 8;         // B (4)
  constexpr int LOADS = AI + BI;
  constexpr int CPRA = kDBM / CH;                // 16-byte chunks per A row
  constexpr int CPRB = kDBN / CH;                // per B row
  __shared__ __attribute__((aligned(1024))) unsigned char lds[kDStages * STAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave >> 2) * 64;
  const int wn = (wave & 3) * 64;
  int tm, tn;
  if (EPI == EPI_PACK || EPI == EPI_SYM) {
    // compact grid over the tiles on or above the a = b diagonal
    const int id = blockIdx.x;
    int lo = 0, hi = g.tiles_m - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (g.row_tiles[mid] <= id) lo = mid; else hi = mid - 1;
    }
    tm = lo;
    tn = pack_first_tile(tm, kDBM, kDBN, g.v) + (id - g.row_tiles[tm]);
  } else {
    tile_of(blockIdx.x, gridDim.x, g.tiles_m, g.group_m, tm, tn);
  }
  const int m0 = tm * kDBM, n0 = tn * kDBN;

  // Wave instruction q of a stage covers bytes [q KB, q KB + 1 KB) of the A (or B)
  // slab: flattened chunk q*64 + lane -> (k row, chunk).  This lane's k row and
  // source pointer at k = 0 for each of its instructions.
  const T* pa[AI];
  const T* pb[BI];
  int ra[AI], rb[BI];
#pragma unroll
  for (int j = 0; j < AI; ++j) {
    const int flat = (wave + 8 * j) * 64 + lane;
    ra[j] = flat / CPRA;
    int m = m0 + (flat % CPRA) * CH;
    m = m < g.M ? m : g.M - CH;
    pa[j] = g.A + (long long)ra[j] * g.lda + m;
  }
#pragma unroll
  for (int j = 0; j < BI; ++j) {
    const int flat = (wave + 8 * j) * 64 + lane;
    rb[j] = flat / CPRB;
    int n = n0 + (flat % CPRB) * CH;
    n = n < g.N ? n : g.N - CH;
    pb[j] = g.B + (long long)rb[j] * g.ldb + n;
  }
  auto issue = [&](int kt) {
    unsigned char* st = lds + (kt % kDStages) * STAGE;
    const long long ka = (long long)kt * BK * g.lda, kb = (long long)kt * BK * g.ldb;
#pragma unroll
    for (int j = 0; j < AI; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(pa[j] + ka),
                                       (lds_void*)(st + (wave + 8 * j) * 1024), 16, 0, 0);
#pragma unroll
    for (int j = 0; j < BI; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(pb[j] + kb),
                                       (lds_void*)(st + A_BYTES + (wave + 8 * j) * 1024), 16, 0, 0);
  };
  // Ragged last K-step: the same LDS image through registers, k rows >= K zero.
  auto issue_tail = [&](int kt) {
    unsigned char* st = lds + (kt % kDStages) * STAGE;
    const int k0 = kt * BK;
    const long long ka = (long long)k0 * g.lda, kb = (long long)k0 * g.ldb;
#pragma unroll
    for (int j = 0; j < AI; ++j) {
      Chunk c = {};
      if (k0 + ra[j] < g.K) c = *reinterpret_cast<const Chunk*>(pa[j] + ka);
      *reinterpret_cast<Chunk*>(st + (wave + 8 * j) * 1024 + 16 * lane) = c;
    }
#pragma unroll
    for (int j = 0; j < BI; ++j) {
      Chunk c = {};
      if (k0 + rb[j] < g.K) c = *reinterpret_cast<const Chunk*>(pb[j] + kb);
      *reinterpret_cast<Chunk*>(st + A_BYTES + (wave + 8 * j) * 1024 + 16 * lane) = c;
    }
    __builtin_amdgcn_s_waitcnt(0xF | (7 << 4) | (3 << 14));  // lgkmcnt(0): the LDS writes landed
  };

  Acc acc[4][4];
  f64x4 acc64[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = Acc{0, 0, 0, 0};
      acc64[i][j] = f64x4{0, 0, 0, 0};
    }

  // fragment reads: k row (lane / 16) of each 4-deep MFMA step, wave row/column
  // pos(., lane % 16) of the four blocks
  const int kr = lane >> 4;
  const int r16 = lane & 15;
  const int offa = (wm + (CH == 4 ? 4 * r16 : 2 * r16)) * (int)sizeof(T);
  const int offb = (wn + (CH == 4 ? 4 * r16 : 2 * r16)) * (int)sizeof(T);
  const int nk = (g.K + BK - 1) / BK;
  const int nkf = g.K / BK;
  auto stage_in = [&](int kt) {
    if (kt < nkf)
      issue(kt);
    else
      issue_tail(kt);
  };
  stage_in(0);
  if (nk > 1) stage_in(1);
  for (int k0 = 0; k0 < nk;) {
    const int kend = (Tr::kDrain && k0 + g.drain_steps < nk) ? k0 + g.drain_steps : nk;
    for (int kt = k0; kt < kend; ++kt) {
      d_wait_vm(kt + 1 < nkf ? LOADS : 0);
      __builtin_amdgcn_s_barrier();
      if (kt + 2 < nk) stage_in(kt + 2);
      const unsigned char* st = lds + (kt % kDStages) * STAGE;
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const unsigned char* ra_ = st + (4 * kk + kr) * ROWA + offa;
        const unsigned char* rb_ = st + A_BYTES + (4 * kk + kr) * ROWB + offb;
        T fa[4], fb[4];
        if constexpr (CH == 4) {
          const Chunk a = *reinterpret_cast<const Chunk*>(ra_);
          const Chunk b = *reinterpret_cast<const Chunk*>(rb_);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            fa[i] = a[i];
            fb[i] = b[i];
          }
        } else {
          const Chunk a0 = *reinterpret_cast<const Chunk*>(ra_);
          const Chunk a1 = *reinterpret_cast<const Chunk*>(ra_ + 32 * sizeof(T));
          const Chunk b0 = *reinterpret_cast<const Chunk*>(rb_);
          const Chunk b1 = *reinterpret_cast<const Chunk*>(rb_ + 32 * sizeof(T));
          fa[0] = a0[0]; fa[1] = a0[1]; fa[2] = a1[0]; fa[3] = a1[1];
          fb[0] = b0[0]; fb[1] = b0[1]; fb[2] = b1[0]; fb[3] = b1[1];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = Tr::mfma(fa[i], fb[j], acc[i][j]);
      }
    }
    if (Tr::kDrain) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            acc64[i][j][r] += static_cast<double>(acc[i][j][r]);
            acc[i][j][r] = 0;
          }
    }
    k0 = kend;
  }

  // epilogue: column groups of CH adjacent n (blocks j = CH*h .. CH*h + CH - 1).
  // EPI_PERM: m = (a, x), n = (y, d) -> C[a*N*v + y*v^2 + x*v + d];
  // EPI_PACK: m = (a - a0, c), n = (b - a0, d), kept for b >= a, at packed row
  // pair(a, b) - pair(a0, a0): C[row*v^2 + c*v + d];
  // EPI_UNPACK: m = pair(a, b) - pair(a0, a0) (m < m_keep), n = (c, d) ->
  // C[(a - a0)*v^3 + c*v^2 + b*v + d].
  const long long v = g.v;
  const bool vec = (g.v % CH) == 0;
  constexpr int NG = 4 / CH;  // column groups per lane: 1 (float32) or 2 (float64)
  auto dst_of = [&](int m, int n) -> long long {  // -1: not stored
    const int y = n / g.v, d = n - y * g.v;
    if (EPI == EPI_UNPACK) {
      if (m >= g.m_keep) return -1;
      const long long q = pair_prefix_d(g.a0, v) + m;
      const int a = pair_row(q, g.v);
      const int b = a + static_cast<int>(q - pair_prefix_d(a, v));
      return (long long)(a - g.a0) * v * v * v + (long long)y * v * v + (long long)b * v + d;
    }
    const int a = m / g.v, x = m - a * g.v;
    if (EPI == EPI_PERM) return (long long)a * g.N * v + (long long)y * v * v + (long long)x * v + d;
    if (y < a) return -1;
    const long long row = pair_prefix_d(g.a0 + a, v) - pair_prefix_d(g.a0, v) + (y - a);
    return row * v * v + (long long)x * v + d;
  };
#pragma unroll
  for (int h = 0; h < NG; ++h) {
    const int nb = n0 + wn + rc_pos<Tr>(CH * h, r16);  // first column of the group
    if (nb >= g.N) continue;                            // N % CH == 0: whole group out
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + rc_pos<Tr>(i, Tr::row_of(lane, r));
        if (m >= g.M) continue;
        Chunk val;
#pragma unroll
        for (int e = 0; e < CH; ++e) {
          const double s = Tr::kDrain ? acc64[i][CH * h + e][r]
                                      : static_cast<double>(acc[i][CH * h + e][r]);
          val[e] = static_cast<T>(s);
        }
        T* C = static_cast<T*>(g.C);
        if constexpr (EPI == EPI_SYM) {
          // the group's CH adjacent columns, and their mirrors down one column m
          if (g.ldc % CH == 0) {
            *reinterpret_cast<Chunk*>(C + (long long)m * g.ldc + nb) = val;
          } else {
#pragma unroll
            for (int e = 0; e < CH; ++e) C[(long long)m * g.ldc + nb + e] = val[e];
          }
#pragma unroll
          for (int e = 0; e < CH; ++e) C[(long long)(nb + e) * g.ldc + m] = val[e];
          continue;
        }
        if (vec) {
          // the group's CH columns share (y) and are adjacent in d
          const long long o0 = dst_of(m, nb);
          if (o0 >= 0) *reinterpret_cast<Chunk*>(C + o0) = val;
        } else {
#pragma unroll
          for (int e = 0; e < CH; ++e) {
            const long long oe = dst_of(m, nb + e);
            if (oe >= 0) C[oe] = val[e];
          }
        }
      }
  }
}

}  // namespace ccl

namespace ccl {

// Mixed-layout GEMM with direct global->LDS loads (gfx950): A K-contiguous, B
// row-contiguous, float64 accumulation into C:
//
//   C[m*ldc + n] += sum_k A[m*lda + k] B[k*ldb + n]
//
// (the adjoint's dt and second dL term, the hole-hole ladder's contraction).  A is
// staged like the K-contiguous kernel (8-row slabs of 128-byte rows, XOR-swizzled
// chunks), B like the row-contiguous kernel (BK rows of 256 contiguous n, columns
// of a wave's four blocks interleaved).  In MFMA step e of k-group gi, slot j of
// both operands carries k = gi*4*CH + CH*j + e: A's lane reads its CH consecutive
// k once per group, B's lane reads that k row's four (float32) or two-plus-two
// (float64) interleaved columns once per step.  Needs 16-byte aligned rows, N a
// multiple of the 16-byte chunk; rows past M are clamped, columns past N clamped
// onto the last chunk (never stored), a ragged last K-step goes through registers
// with zero fill.
template <class Tr>
__global__ __launch_bounds__(kDThreads, 1) void gemm_kr_direct_kernel(GemmArgs<typename Tr::T> g) {
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  using Chunk = typename Tr::Chunk;
  constexpr int CH = Tr::CH;
  constexpr int BK = kDRow / sizeof(T);          // 16 float64 / 32 float32
  constexpr int ROWB = kDBN * sizeof(T);         // bytes of one k row of B (256 n)
  constexpr int A_BYTES = kDBM * kDRow;          // 16 KB
  constexpr int B_BYTES = BK * ROWB;             // 32 KB
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int AL = kDBM / 8 / 8;               // A: 8-row slabs per wave (2)
  constexpr int BI = B_BYTES / 1024 / 8;         // B: 1 KB instructions per wave (4)
  constexpr int LOADS = AL + BI;
  constexpr int CPRB = kDBN / CH;                // 16-byte chunks per B row
  __shared__ __attribute__((aligned(1024))) unsigned char lds[kDStages * STAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave >> 2) * 64;
  const int wn = (wave & 3) * 64;
  int tm, tn;
  if (g.kband)
    tile_of_banded(g.kband, blockIdx.x, gridDim.x, g.tiles_m, g.group_m, tm, tn);
  else
    tile_of(blockIdx.x, gridDim.x, g.tiles_m, g.group_m, tm, tn);
  const int m0 = tm * kDBM, n0 = tn * kDBN;
  int ks0, ks1;  // this tile's K-steps
  k_band(g, n0, kDBN, BK, ks0, ks1);

  // A: slabs of 8 rows, lane -> row lane/8, physical chunk lane%8 holding
  // logical chunk (lane%8) ^ ((row/2)%8)
  const int lrow = lane >> 3;
  const int sw_even = ((lane & 7) ^ ((lane >> 4) & 7)) * CH;
  const int sw_odd = ((lane & 7) ^ ((4 + (lane >> 4)) & 7)) * CH;
  const int my_sw = (wave & 1) ? sw_odd : sw_even;
  const T* pa[AL];
#pragma unroll
  for (int j = 0; j < AL; ++j) {
    int row = m0 + 8 * (wave + 8 * j) + lrow;
    row = row < g.M ? row : g.M - 1;
    pa[j] = g.A + (long long)row * g.lda + my_sw;
  }
  // B: wave instruction q covers the 1 KB [q KB, q KB + 1 KB) of the stage's B slab
  const T* pb[BI];
  int rb[BI];
#pragma unroll
  for (int j = 0; j < BI; ++j) {
    const int flat = (wave + 8 * j) * 64 + lane;
    rb[j] = flat / CPRB;
    int n = n0 + (flat % CPRB) * CH;
    n = n < g.N ? n : g.N - CH;
    pb[j] = g.B + (long long)rb[j] * g.ldb + n;
  }
  auto issue = [&](int kt) {
    unsigned char* st = lds + (kt % kDStages) * STAGE;
    const int ko = kt * BK;
    const long long kb = (long long)ko * g.ldb;
#pragma unroll
    for (int j = 0; j < AL; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(pa[j] + ko),
                                       (lds_void*)(st + 8 * (wave + 8 * j) * kDRow), 16, 0, 0);
#pragma unroll
    for (int j = 0; j < BI; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(pb[j] + kb),
                                       (lds_void*)(st + A_BYTES + (wave + 8 * j) * 1024), 16, 0, 0);
  };
  auto issue_tail = [&](int kt) {
    unsigned char* st = lds + (kt % kDStages) * STAGE;
    const int k0 = kt * BK;
#pragma unroll
    for (int j = 0; j < AL; ++j) {
      const int kk = k0 + my_sw;  // this lane's first k
      Chunk c;
#pragma unroll
      for (int e = 0; e < CH; ++e) c[e] = (kk + e < g.K) ? pa[j][k0 + e] : T(0);
      *reinterpret_cast<Chunk*>(st + 8 * (wave + 8 * j) * kDRow + 16 * lane) = c;
    }
    const long long kb = (long long)k0 * g.ldb;
#pragma unroll
    for (int j = 0; j < BI; ++j) {
      Chunk c = {};
      if (k0 + rb[j] < g.K) c = *reinterpret_cast<const Chunk*>(pb[j] + kb);
      *reinterpret_cast<Chunk*>(st + A_BYTES + (wave + 8 * j) * 1024 + 16 * lane) = c;
    }
    __builtin_amdgcn_s_waitcnt(0xF | (7 << 4) | (3 << 14));  // lgkmcnt(0): the LDS writes landed
  };

  Acc acc[4][4];
  f64x4 acc64[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = Acc{0, 0, 0, 0};
      acc64[i][j] = f64x4{0, 0, 0, 0};
    }

  const int frow = (lane & 15) * kDRow;
  const int fsw = (lane & 15) >> 1;
  const int slot = lane >> 4;
  const int r16 = lane & 15;
  const int offb = (wn + (CH == 4 ? 4 * r16 : 2 * r16)) * (int)sizeof(T);
  const int nk = ks1;
  const int nkf = g.K / BK;
  auto stage_in = [&](int kt) {
    if (kt < nkf)
      issue(kt);
    else
      issue_tail(kt);
  };
  stage_in(ks0);
  if (ks0 + 1 < nk) stage_in(ks0 + 1);
  for (int k0 = ks0; k0 < nk;) {
    const int kend = (Tr::kDrain && k0 + g.drain_steps < nk) ? k0 + g.drain_steps : nk;
    for (int kt = k0; kt < kend; ++kt) {
      // step kt's direct loads have landed once only step kt+1's remain in flight
      d_wait_vm(kt + 1 < nkf && kt + 1 < nk ? LOADS : 0);
      __builtin_amdgcn_s_barrier();
      if (kt + 2 < nk) stage_in(kt + 2);
      const unsigned char* st = lds + (kt % kDStages) * STAGE;
#pragma unroll
      for (int gi = 0; gi < 2; ++gi) {
        const int chunk = ((4 * gi + slot) ^ fsw) * 16;
        Chunk fa[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          fa[i] = *reinterpret_cast<const Chunk*>(st + (wm + 16 * i) * kDRow + frow + chunk);
#pragma unroll
        for (int e = 0; e < CH; ++e) {
          // k row gi*4*CH + CH*slot + e of B, this lane's interleaved columns
          const unsigned char* rb_ = st + A_BYTES + (4 * CH * gi + CH * slot + e) * ROWB + offb;
          T fb[4];
          if constexpr (CH == 4) {
            const Chunk b = *reinterpret_cast<const Chunk*>(rb_);
#pragma unroll
            for (int j = 0; j < 4; ++j) fb[j] = b[j];
          } else {
            const Chunk b0 = *reinterpret_cast<const Chunk*>(rb_);
            const Chunk b1 = *reinterpret_cast<const Chunk*>(rb_ + 32 * sizeof(T));
            fb[0] = b0[0]; fb[1] = b0[1]; fb[2] = b1[0]; fb[3] = b1[1];
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = Tr::mfma(fa[i][e], fb[j], acc[i][j]);
        }
      }
    }
    if (Tr::kDrain) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            acc64[i][j][r] += static_cast<double>(acc[i][j][r]);
            acc[i][j][r] = 0;
          }
    }
    k0 = kend;
  }

  double* C = static_cast<double*>(g.C);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + wn + rc_pos<Tr>(j, r16);
    if (n >= g.N) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + Tr::row_of(lane, r);
        if (m >= g.M) continue;
        C[(long long)m * g.ldc + n] +=
            g.alpha * (Tr::kDrain ? acc64[i][j][r] : static_cast<double>(acc[i][j][r]));
      }
  }
}

}  // namespace ccl
