// Amplitude-contraction GEMM with direct global->LDS operand loads (gfx950).
//
//   C[m][n] (+)= sum_k A[m*lda + k] B[n*ldb + k]   (both operands KC; EPI_ACC, EPI_PAIR,
//                                                   or EPI_PART: one K-range per workgroup)
//
// 512 threads = 8 wave64s in a 2 x 4 grid over a 128 x 256 tile; each wave owns
// 64 x 64 = 4 x 4 MFMA blocks (v_mfma_f64_16x16x4_f64 or v_mfma_f32_16x16x4_f32).
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
    CCL_DVM(0) CCL_DVM(6)
#undef CCL_DVM
    default:
      __builtin_amdgcn_s_waitcnt(7 << 4 | 15 << 8);
  }
}

template <class Tr, int EPI>
__global__ __launch_bounds__(kDThreads, 1) void gemm_kc_direct_kernel(GemmArgs<typename Tr::T> g) {
  static_assert(EPI == EPI_ACC || EPI == EPI_PAIR || EPI == EPI_PART, "K-contiguous epilogues");
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  using Chunk = typename Tr::Chunk;
  constexpr int CH = Tr::CH;                 // elements per 16 bytes
  constexpr int BK = kDRow / sizeof(T);      // K per step (16 float64 / 32 float32)
  constexpr int A_BYTES = kDBM * kDRow;      // 16 KB
  constexpr int B_BYTES = kDBN * kDRow;      // 32 KB
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int LOADS = (kDBM + kDBN) / 8 / 8;  // 8-row slabs per wave per stage (= 6)
  __shared__ __attribute__((aligned(1024))) unsigned char lds[kDStages * STAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave >> 2) * 64;
  const int wn = (wave & 3) * 64;
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
  } else {
    tile_of(blockIdx.x, gridDim.x, g.tiles_m, g.group_m, tm, tn);
  }
  const int m0 = tm * kDBM, n0 = tn * kDBN;

  // Slabs: A rows 8*(wave + 8*j), j < 2; B rows 8*(wave + 8*j), j < 4.  The
  // swizzle of a lane depends on the slab's parity only (slab origin 8*s rows).
  const int lrow = lane >> 3;
  const int sw_even = ((lane & 7) ^ ((lane >> 4) & 7)) * CH;        // slab index even
  const int sw_odd = ((lane & 7) ^ ((4 + (lane >> 4)) & 7)) * CH;   // slab index odd
  const int my_sw = (wave & 1) ? sw_odd : sw_even;  // slabs wave + 8j share the wave's parity
  const T* pa[2];
  const T* pb[4];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
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
    for (int j = 0; j < 2; ++j)
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
    for (int j = 0; j < 2; ++j) one(pa[j], st + 8 * (wave + 8 * j) * kDRow);
#pragma unroll
    for (int j = 0; j < 4; ++j) one(pb[j], st + A_BYTES + 8 * (wave + 8 * j) * kDRow);
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
        Chunk fa[4], fb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          fa[i] = *reinterpret_cast<const Chunk*>(st + (wm + 16 * i) * kDRow + frow + chunk);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          fb[j] = *reinterpret_cast<const Chunk*>(st + A_BYTES + (wn + 16 * j) * kDRow + frow + chunk);
#pragma unroll
        for (int e = 0; e < CH; ++e)
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = Tr::mfma(fa[i][e], fb[j][e], acc[i][j]);
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

  const int col = lane & 15;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + wn + 16 * j + col;
    if (n >= g.N) continue;
    const EpiCol ec = epi_col<T, EPI>(g, n);
#pragma unroll
    for (int i = 0; i < 4; ++i)
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
