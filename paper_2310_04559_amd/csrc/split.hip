// Split-bf16 form of the ladder forward.
//
// Every operand row (a row of the matrix along its contracted index) gets one
// exponent e with max|x| < 2^e, and is cut into S balanced base-256 digits:
//   x = 2^e * sum_{p=1..S} d_p 2^(-8p) + r,   d_1 in [-256, 256], d_p in [-128, 128] (p > 1),
// |r| <= 2^(e - 8S - 1).  Digits are integers, exact in bf16.  A product of two
// such matrices is
//   C[m][n] = 2^(eA[m] + eB[n]) sum_{g} 2^(-8g) sum_{p+q=g} sum_k dA_p[m][k] dB_q[n][k],
// keeping the anti-diagonals g = p + q <= S + D (D = 1: the S(S+1)/2-product
// triangle; D = 2 adds the next anti-diagonal).  Each inner
// sum is a sum of integer products; over K-chunks of 128 every partial sum of
// one group stays below 2^24, so the bf16 MFMA's float32 accumulation is exact
// and each chunk is drained into float64.  The two contractions then run as:
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

constexpr int kSBM = 64;    // workgroup tile rows (M)
constexpr int kSBN = 128;   // workgroup tile columns (N)
constexpr int kSBK = 32;    // K per stage = one bf16 MFMA depth
constexpr int kChunkSteps = 4;  // K-steps per exact float32 chunk (128 contracted indices)

// Balanced base-256 digits of y in (-1, 1): writes S bf16 digits, most significant first.
template <int S>
__device__ __forceinline__ void digits(double y, __bf16 (&d)[S]) {
#pragma unroll
  for (int p = 0; p < S; ++p) {
    y *= 256.0;
    const double q = rint(y);
    y -= q;
    d[p] = static_cast<__bf16>(static_cast<float>(q));
  }
}

// ---------------------------------------------------------------------------
// slicing
// ---------------------------------------------------------------------------

// Rows with the contracted index contiguous: X[r][k] = X[r*ld + k], r < R, k < K.
// One workgroup per output row (R_pad rows, the padding rows get zero digits).
template <int S>
__global__ __launch_bounds__(256) void slice_kc_kernel(const double* __restrict__ X, long long ld,
                                                       int R, int K, int Kp, long long sstride,
                                                       __bf16* __restrict__ out, int* __restrict__ ex) {
  const int r = blockIdx.x;
  const int tid = threadIdx.x;
  const double* row = X + (long long)r * ld;
  double m = 0.0;
  if (r < R)
    for (int k = tid; k < K; k += 256) m = fmax(m, fabs(row[k]));
  __shared__ double red[256];
  red[tid] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  int e = 0;
  if (red[0] > 0.0) (void)frexp(red[0], &e);  // max|x| < 2^e
  if (tid == 0) ex[r] = e;
  for (int k0 = tid * 8; k0 < Kp; k0 += 256 * 8) {
    __bf16 d[8][S];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + j;
      const double x = (r < R && k < K) ? row[k] : 0.0;
      digits<S>(ldexp(x, -e), d[j]);
    }
#pragma unroll
    for (int p = 0; p < S; ++p) {
      bf16x8 v;
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = d[j][p];
      *reinterpret_cast<bf16x8*>(out + p * sstride + (long long)r * Kp + k0) = v;
    }
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
                                                       int R, int Rp, int K, int Kp, long long sstride,
                                                       const int* __restrict__ ex,
                                                       __bf16* __restrict__ out) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long total = (long long)Rp * (Kp / 8);
  if (idx >= total) return;
  const int r = static_cast<int>(idx % Rp);
  const int k0 = static_cast<int>(idx / Rp) * 8;
  const int e = ex[r];
  __bf16 d[8][S];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = k0 + j;
    const double x = (r < R && k < K) ? X[(long long)k * ld + r] : 0.0;
    digits<S>(ldexp(x, -e), d[j]);
  }
#pragma unroll
  for (int p = 0; p < S; ++p) {
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = d[j][p];
    *reinterpret_cast<bf16x8*>(out + p * sstride + (long long)r * Kp + k0) = v;
  }
}

// ---------------------------------------------------------------------------
// slice-pair GEMM
// ---------------------------------------------------------------------------

struct SplitArgs {
  const __bf16* A;   // [S][rows][Kp] digits, row 0 = this product's first row
  long long sa;      // slice stride of A
  const int* ea;     // exponents of A's rows (same row origin)
  const __bf16* B;
  long long sb;
  const int* eb;
  int M, N, Kp;
  void* C;           // EPI_ACC: float64 C[m*ldc + n] +=; EPI_PERM: float64 integral block
  long long ldc;
  int v;
  int tiles_m, tiles_n, group_m;
};

// 256 threads = 4 waves in 2x2; wave tile 32 x 64 = 2 x 4 blocks of 16x16.
// Slice products (p, q) (0-based) are kept when p + q < S + D - 1: D = 1 is the
// triangle p'+q' <= S+1 of 1-based slices, D = 2 adds its next anti-diagonal.
//
// Operand tiles go from global memory straight into LDS (global_load_lds_dwordx4:
// lane l of a wave writes 16 bytes at the wave's LDS base + 16*l), three K-steps
// in flight in a ring of LDS stages, one barrier per K-step.  A 16-row slab of a
// slice is one load instruction: lane l takes row l/4 and physical 16-byte slot
// l%4, which holds the logical k-chunk (l%4) ^ ((row/2)%4); fragment reads undo the
// XOR.  Keying on row/2 (pairs of 64-byte rows share a key) makes the 16-byte
// fragment reads free of bank conflicts on gfx950; keying on row/4, or no
// swizzle, costs one extra LDS cycle per read (measured with the hardware's
// bank-conflict counter on a read-pattern probe).
constexpr int kStages = 3;
constexpr int kRowBytes = kSBK * 2;  // 64 bytes: one 32-deep row of bf16 digits

typedef __attribute__((address_space(3))) void lds_void_t;

__device__ __forceinline__ void wait_vm(int n) {
  // s_waitcnt with vmcnt = n (0..63); lgkmcnt and expcnt left unconstrained
  switch (n) {
#define CCL_VM(N) \
  case N:         \
    __builtin_amdgcn_s_waitcnt(((N)&15) | (7 << 4) | (15 << 8) | (((N) >> 4) << 14)); \
    break;
    CCL_VM(0) CCL_VM(6) CCL_VM(9) CCL_VM(12)
#undef CCL_VM
    default:
      __builtin_amdgcn_s_waitcnt(7 << 4 | 15 << 8);
  }
}

template <int S, int D, int EPI>
__global__ __launch_bounds__(256, 1) void split_gemm_kernel(SplitArgs g) {
  constexpr int NG = S + D - 1;                          // anti-diagonals kept
  constexpr int A_BYTES = S * kSBM * kRowBytes;          // one stage of A digits
  constexpr int B_BYTES = S * kSBN * kRowBytes;
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int LOADS = 3 * S;                           // load instructions per wave per stage
  static_assert(kStages * STAGE <= 160 * 1024, "LDS");
  __shared__ __attribute__((aligned(1024))) unsigned char lds[kStages * STAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave >> 1) * 32;
  const int wn = (wave & 1) * 64;
  int tm, tn;
  tile_of(blockIdx.x, gridDim.x, g.tiles_m, g.group_m, tm, tn);
  const int m0 = tm * kSBM, n0 = tn * kSBN;

  // this lane's element offset inside any 16-row slab (row lane/4, swizzled chunk)
  const int lrow = lane >> 2;
  const int lchunk = (lane & 3) ^ ((lane >> 3) & 3);  // key (row >> 1) & 3
  const long long loff = (long long)lrow * g.Kp + lchunk * 8;
  const __bf16* pa = g.A + (long long)(m0 + 16 * wave) * g.Kp + loff;
  const __bf16* pb = g.B + (long long)(n0 + 16 * wave) * g.Kp + loff;
  const long long b_half = 64LL * g.Kp;
  // LDS byte offsets (wave-uniform) of this wave's slabs inside a stage
  const int la = 16 * wave * kRowBytes;
  const int lb = A_BYTES + 16 * wave * kRowBytes;

  auto issue = [&](int kt) {
    unsigned char* st = lds + (kt % kStages) * STAGE;
    const int ko = kt * kSBK;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      __builtin_amdgcn_global_load_lds((const void*)(pa + s * g.sa + ko),
                                       (lds_void_t*)(st + la + s * kSBM * kRowBytes), 16, 0, 0);
#pragma unroll
      for (int h = 0; h < 2; ++h)
        __builtin_amdgcn_global_load_lds(
            (const void*)(pb + s * g.sb + h * b_half + ko),
            (lds_void_t*)(st + lb + (s * kSBN + 64 * h) * kRowBytes), 16, 0, 0);
    }
  };

  f64x4 acc64[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc64[i][j] = f64x4{0, 0, 0, 0};

  // fragment read: row (lane & 15) of a 16-row block, logical chunk lane >> 4
  const int frag_off = (lane & 15) * kRowBytes + (((lane >> 4) ^ ((lane >> 1) & 3)) * 16);
  const int nk = g.Kp / kSBK;
  issue(0);
  if (nk > 1) issue(1);
  // One exact chunk (kChunkSteps K-steps) per trip: its float32 anti-diagonal
  // sums start at zero, stay in MFMA accumulators and are drained at its end.
  for (int k0 = 0; k0 < nk; k0 += kChunkSteps) {
    f32x4 acc[NG][2][4];
#pragma unroll
    for (int q = 0; q < NG; ++q)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[q][i][j] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < kChunkSteps; ++u) {
      const int kt = k0 + u;
      if (kt < nk) {
        wait_vm(kt + 1 < nk ? LOADS : 0);  // this wave's loads of step kt have landed
        __builtin_amdgcn_s_barrier();      // ... and every wave's; step kt-1 is consumed
        if (kt + 2 < nk) issue(kt + 2);
        const unsigned char* st = lds + (kt % kStages) * STAGE;
        bf16x8 fa[S][2], fb[S][4];
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
          for (int i = 0; i < 2; ++i)
            fa[s][i] = *reinterpret_cast<const bf16x8*>(
                st + (s * kSBM + wm + 16 * i) * kRowBytes + frag_off);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            fb[s][j] = *reinterpret_cast<const bf16x8*>(
                st + A_BYTES + (s * kSBN + wn + 16 * j) * kRowBytes + frag_off);
        }
#pragma unroll
        for (int p = 0; p < S; ++p)
#pragma unroll
          for (int q = 0; q < S; ++q) {
            if (p + q > NG - 1) continue;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j)
                acc[p + q][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    fa[p][i], fb[q][j], acc[p + q][i][j], 0, 0, 0);
          }
      }
    }
    // exact float32 anti-diagonal sums -> float64, scaled by 2^(-8*(q+2))
    double scale = 1.0 / 65536.0;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc64[i][j][r] = fma(static_cast<double>(acc[q][i][j][r]), scale, acc64[i][j][r]);
      scale *= 1.0 / 256.0;
    }
  }

  // Epilogue: lane holds column lane%16, rows 4*(lane/16)+r of each block.
  const long long v = g.v;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + wn + 16 * j + (lane & 15);
    if (n >= g.N) continue;
    const int en = g.eb[n];
    long long ncol = n;
    if (EPI == EPI_PERM) {
      const int y = n / g.v, d = n - y * g.v;
      ncol = (long long)y * v * v + d;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        if (m >= g.M) continue;
        const double val = ldexp(acc64[i][j][r], g.ea[m] + en);
        if (EPI == EPI_ACC) {
          static_cast<double*>(g.C)[(long long)m * g.ldc + n] += val;
        } else {
          const int a = m / g.v, x = m - a * g.v;
          static_cast<double*>(g.C)[(long long)a * v * v * v + ncol + (long long)x * v] = val;
        }
      }
  }
}

// Same product with 8 waves: waves w and w+4 own the same 32 x 64 sub-tile; wave
// w accumulates the anti-diagonals [0, G0) (slices below G0 only), wave w+4 the
// anti-diagonals [G0, NG).  Each half fits 256 registers, so two waves share a
// SIMD and hide each other's LDS and memory latency; their float64 partial sums
// are added through LDS before the epilogue.
template <int S, int D>
struct GroupSplit {
  static constexpr int NG = S + D - 1;
  static constexpr int pairs(int q) { return (q < S ? q + 1 : 2 * S - 1 - q); }
  static constexpr int count(int lo, int hi) { return lo >= hi ? 0 : pairs(lo) + count(lo + 1, hi); }
  static constexpr int larger(int g) { return count(0, g) > count(g, NG) ? count(0, g) : count(g, NG); }
  // split point in [1, NG) that minimises the larger half's products
  static constexpr int pick(int g, int best) {
    return g >= NG ? best : pick(g + 1, larger(g) < larger(best) ? g : best);
  }
  static constexpr int G0 = pick(1, 1);
  static_assert(G0 >= 1 && G0 < NG, "both halves hold products");
};

template <int S, int D, int EPI>
__global__ __launch_bounds__(512, 1) void split_gemm2_kernel(SplitArgs g) {
  constexpr int NG = S + D - 1;
  constexpr int G0 = GroupSplit<S, D>::G0;
  constexpr int A_BYTES = S * kSBM * kRowBytes;
  constexpr int B_BYTES = S * kSBN * kRowBytes;
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int ASLABS = S * kSBM / 16, BSLABS = S * kSBN / 16;  // 16-row slabs per stage
  constexpr int LOADS = (ASLABS + BSLABS) / 8;                    // per wave
  static_assert((ASLABS % 8) == 0 && (BSLABS % 8) == 0, "slab split");
  static_assert(kStages * STAGE <= 160 * 1024, "LDS");
  static_assert(4 * 64 * 32 * 8 <= kStages * STAGE, "reduction buffer");
  __shared__ __attribute__((aligned(1024))) unsigned char lds[kStages * STAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int sub = wave & 3, half = wave >> 2;
  const int wm = (sub >> 1) * 32;
  const int wn = (sub & 1) * 64;
  int tm, tn;
  tile_of(blockIdx.x, gridDim.x, g.tiles_m, g.group_m, tm, tn);
  const int m0 = tm * kSBM, n0 = tn * kSBN;

  const int lrow = lane >> 2;
  const int lchunk = (lane & 3) ^ ((lane >> 3) & 3);  // key (row >> 1) & 3
  const long long loff = (long long)lrow * g.Kp + lchunk * 8;
  auto issue = [&](int kt) {
    unsigned char* st = lds + (kt % kStages) * STAGE;
    const int ko = kt * kSBK;
#pragma unroll
    for (int j = 0; j < ASLABS / 8; ++j) {
      const int ai = wave + 8 * j, s = ai / (kSBM / 16), r = ai % (kSBM / 16);
      __builtin_amdgcn_global_load_lds(
          (const void*)(g.A + s * g.sa + (long long)(m0 + 16 * r) * g.Kp + loff + ko),
          (lds_void_t*)(st + (s * kSBM + 16 * r) * kRowBytes), 16, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < BSLABS / 8; ++j) {
      const int bi = wave + 8 * j, s = bi / (kSBN / 16), r = bi % (kSBN / 16);
      __builtin_amdgcn_global_load_lds(
          (const void*)(g.B + s * g.sb + (long long)(n0 + 16 * r) * g.Kp + loff + ko),
          (lds_void_t*)(st + A_BYTES + (s * kSBN + 16 * r) * kRowBytes), 16, 0, 0);
    }
  };

  f64x4 acc64[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc64[i][j] = f64x4{0, 0, 0, 0};

  const int frag_off = (lane & 15) * kRowBytes + (((lane >> 4) ^ ((lane >> 1) & 3)) * 16);
  const int nk = g.Kp / kSBK;

  // One exact chunk of this wave's anti-diagonals [LO, HI) (slices < SL needed).
  auto run_chunk = [&](int k0, auto lo_c, auto hi_c) {
    constexpr int LO = decltype(lo_c)::value, HI = decltype(hi_c)::value;
    constexpr int SL = (HI - 1) < S ? HI : S;  // slices with index < SL can appear
    f32x4 acc[HI - LO][2][4];
#pragma unroll
    for (int q = 0; q < HI - LO; ++q)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[q][i][j] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < kChunkSteps; ++u) {
      const int kt = k0 + u;
      if (kt < nk) {
        wait_vm(kt + 1 < nk ? LOADS : 0);
        __builtin_amdgcn_s_barrier();
        if (kt + 2 < nk) issue(kt + 2);
        const unsigned char* st = lds + (kt % kStages) * STAGE;
        bf16x8 fa[SL][2], fb[SL][4];
#pragma unroll
        for (int sl = 0; sl < SL; ++sl) {
#pragma unroll
          for (int i = 0; i < 2; ++i)
            fa[sl][i] = *reinterpret_cast<const bf16x8*>(
                st + (sl * kSBM + wm + 16 * i) * kRowBytes + frag_off);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            fb[sl][j] = *reinterpret_cast<const bf16x8*>(
                st + A_BYTES + (sl * kSBN + wn + 16 * j) * kRowBytes + frag_off);
        }
#pragma unroll
        for (int p = 0; p < SL; ++p)
#pragma unroll
          for (int q = 0; q < SL; ++q) {
            if (p + q < LO || p + q >= HI) continue;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j)
                acc[p + q - LO][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    fa[p][i], fb[q][j], acc[p + q - LO][i][j], 0, 0, 0);
          }
      }
    }
    double scale = 1.0 / 65536.0;
#pragma unroll
    for (int q = 0; q < LO; ++q) scale *= 1.0 / 256.0;
#pragma unroll
    for (int q = 0; q < HI - LO; ++q) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc64[i][j][r] = fma(static_cast<double>(acc[q][i][j][r]), scale, acc64[i][j][r]);
      scale *= 1.0 / 256.0;
    }
  };

  issue(0);
  if (nk > 1) issue(1);
  for (int k0 = 0; k0 < nk; k0 += kChunkSteps) {
    if (half == 0)
      run_chunk(k0, std::integral_constant<int, 0>{}, std::integral_constant<int, G0>{});
    else
      run_chunk(k0, std::integral_constant<int, G0>{}, std::integral_constant<int, NG>{});
  }

  // add the upper anti-diagonals' sums (waves 4..7) into waves 0..3
  __builtin_amdgcn_s_barrier();  // every wave is done reading the operand stages
  // lane-contiguous: each store or load of the 64 lanes touches 512 consecutive bytes
  double* red = reinterpret_cast<double*>(lds) + sub * 64 * 32 + lane;
  if (half == 1) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[((i * 4 + j) * 4 + r) * 64] = acc64[i][j][r];
  }
  __syncthreads();
  if (half == 1) return;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[i][j][r] += red[((i * 4 + j) * 4 + r) * 64];

  const long long v = g.v;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + wn + 16 * j + (lane & 15);
    if (n >= g.N) continue;
    const int en = g.eb[n];
    long long ncol = n;
    if (EPI == EPI_PERM) {
      const int y = n / g.v, d = n - y * g.v;
      ncol = (long long)y * v * v + d;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        if (m >= g.M) continue;
        const double val = ldexp(acc64[i][j][r], g.ea[m] + en);
        if (EPI == EPI_ACC) {
          static_cast<double*>(g.C)[(long long)m * g.ldc + n] += val;
        } else {
          const int a = m / g.v, x = m - a * g.v;
          static_cast<double*>(g.C)[(long long)a * v * v * v + ncol + (long long)x * v] = val;
        }
      }
  }
}

template <int S, int D, int EPI>
int launch_split_gemm(const SplitArgs& a0, hipStream_t s) {
  SplitArgs a = a0;
  if (a.M <= 0 || a.N <= 0) return CC_LADDER_OK;
  a.tiles_m = (a.M + kSBM - 1) / kSBM;
  a.tiles_n = (a.N + kSBN - 1) / kSBN;
  const long long tiles = (long long)a.tiles_m * a.tiles_n;
  if (tiles > 0x7fffffffLL) return CC_LADDER_EINVAL;
  a.group_m = a.tiles_m < 16 ? a.tiles_m : 16;
  if constexpr (S == 4)  // enough products for both halves of the 8-wave kernel
    hipLaunchKernelGGL((split_gemm2_kernel<S, D, EPI>), dim3(static_cast<unsigned>(tiles)),
                       dim3(512), 0, s, a);
  else
    hipLaunchKernelGGL((split_gemm_kernel<S, D, EPI>), dim3(static_cast<unsigned>(tiles)),
                       dim3(256), 0, s, a);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

template <int S>
int slice_kc(const double* X, long long ld, int R, int K, const SliceDims& d, __bf16* out, int* ex,
             hipStream_t s) {
  hipLaunchKernelGGL((slice_kc_kernel<S>), dim3(d.rows_pad), dim3(256), 0, s, X, ld, R, K, d.k_pad,
                     (long long)d.rows_pad * d.k_pad, out, ex);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

template <int S>
int slice_rc(const double* X, long long ld, int R, int K, const SliceDims& d, __bf16* out, int* ex,
             hipStream_t s) {
  hipLaunchKernelGGL(rc_rowmax_kernel, dim3((d.rows_pad + 255) / 256), dim3(256), 0, s, X, ld, R,
                     d.rows_pad, K, ex);
  const long long total = (long long)d.rows_pad * (d.k_pad / 8);
  hipLaunchKernelGGL((slice_rc_kernel<S>), dim3(static_cast<unsigned>((total + 255) / 256)),
                     dim3(256), 0, s, X, ld, R, d.rows_pad, K, d.k_pad,
                     (long long)d.rows_pad * d.k_pad, ex, out);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

template <int S, int D>
int split_forward_s(const Plan& pl, const double* L, const double* t, double* R, char* ws,
                    const Tracer& tr, hipStream_t s) {
  const int o = pl.o, v = pl.v, P = pl.P;
  const long long v2 = (long long)v * v;
  const SliceDims dL = slice_dims(static_cast<long long>(v2), P);
  const SliceDims dt = slice_dims((long long)o * o, static_cast<int>(v2));
  const SliceDims dV = slice_dims((long long)pl.n_a * v, static_cast<int>(v2));
  __bf16* Ls = reinterpret_cast<__bf16*>(ws + pl.off_L);
  int* Le = reinterpret_cast<int*>(ws + pl.off_Lexp);
  __bf16* ts = reinterpret_cast<__bf16*>(ws + pl.off_t);
  int* te = reinterpret_cast<int*>(ws + pl.off_texp);
  double* V = reinterpret_cast<double*>(ws + pl.off_V);
  __bf16* Vs = reinterpret_cast<__bf16*>(ws + pl.off_Vs);
  int* Ve = reinterpret_cast<int*>(ws + pl.off_Vexp);
  const long long sL = (long long)dL.rows_pad * dL.k_pad;
  const long long st = (long long)dt.rows_pad * dt.k_pad;
  const long long sV = (long long)dV.rows_pad * dV.k_pad;

  tr(CC_LADDER_PHASE_PREP, 0, 0);
  int rc = slice_rc<S>(L, v2, static_cast<int>(v2), P, dL, Ls, Le, s);
  if (!rc) rc = slice_kc<S>(t, v2, o * o, static_cast<int>(v2), dt, ts, te, s);
  tr(CC_LADDER_PHASE_PREP, 0, 1);
  if (rc) return rc;
  for (int a0 = 0, blk = 0; a0 < v; a0 += pl.n_a, ++blk) {
    const int na = (v - a0) < pl.n_a ? (v - a0) : pl.n_a;
    const long long r0 = (long long)a0 * v;  // first (a,c) row of this block
    SplitArgs b{};
    b.A = Ls + r0 * dL.k_pad; b.sa = sL; b.ea = Le + r0;
    b.B = Ls; b.sb = sL; b.eb = Le;
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
    c.A = ts; c.sa = st; c.ea = te;
    c.B = Vs; c.sb = sV; c.eb = Ve;
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
