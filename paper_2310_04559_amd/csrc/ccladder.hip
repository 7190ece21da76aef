// C ABI of the MI355X ladder library: argument checks, planning, scratch,
// and the stream-ordered schedule of the MFMA kernels.
//
// Forward (eq. cholesky + eq. vfunction), per block A of first virtuals:
//   build    V_A[a][b][c][d] = sum_x L[x][a][c] L[x][b][d]     GEMM M=(a,c) N=(b,d) K=x
//   contract R[(ij)][(a b)] += sum_(cd) t[(ij)][(cd)] V_A[(ab)][(cd)]   GEMM M=ij N=(a,b) K=(c,d)
// Adjoint, per block, with V_A rebuilt:
//   dt[(ij)][(cd)] += sum_(a in A, b) lam[(ij)][(ab)] V_A[(ab)][(cd)]
//   W'_A[a][c][b][d] = sum_(ij) lam[(ij)][(ab)] t[(ij)][(cd)]
//   dL[x][(a c)]  += sum_(bd) L[x][(bd)] W'_A[(ac)][(bd)]          (a in A)
//   dL[x][(b d)]  += sum_(a in A, c) L[x][(ac)] W'_A[(ac)][(bd)]
// Occupied intermediates (eqs. vfunction3/vfunction4), per block of first index p:
//   build    G[p][y][x][d] = sum_x' Lrow[x'][p][x] L_ov[x'][y][d]   GEMM M=(p,x) N=(y,d) K=x'
//   contract Z[(ij)][(p y)] += sum_(xd) t'[(ij)][(xd)] G[(py)][(xd)]
// ijkl: Lrow = L_ov, t' = t; ijbk: Lrow = L, t' = t with c and d swapped, since
// G[b][k][d][c] = (bd|kc) carries its last two indices in (d, c) order.
// Exchange partner (eq. vfunction2): the same schedule on t with c and d swapped,
// since sum_(cd) (ad|bc) t[i][j][c][d] = sum_(cd) (ac|bd) t[i][j][d][c]; the
// adjoint's dt comes back with the swap undone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "ccladder.h"
#include "gemm.hpp"
#include "gemm_direct.hpp"
#include "plan.h"
#include "split.hpp"

namespace ccl {
namespace {

#define CCL_HIP(expr)                                  \
  do {                                                 \
    if ((expr) != hipSuccess) return CC_LADDER_EHIP;   \
  } while (0)

// ---------------------------------------------------------------------------
// device checks
// ---------------------------------------------------------------------------

std::mutex g_dev_mu;
int g_dev_ok[64];  // 0 unknown, 1 gfx950, -1 other

int check_device() {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return CC_LADDER_ENODEV;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return CC_LADDER_ENODEV;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if (g_dev_ok[dev] == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return CC_LADDER_ENODEV;
    g_dev_ok[dev] = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : -1;
  }
  return g_dev_ok[dev] == 1 ? CC_LADDER_OK : CC_LADDER_ENODEV;
}

// ---------------------------------------------------------------------------
// GEMM launch
// ---------------------------------------------------------------------------

template <class T>
bool vec_ok(const T* p, long long ld) {
  constexpr int per16 = 16 / sizeof(T);
  return (reinterpret_cast<uintptr_t>(p) % 16) == 0 && (ld % per16) == 0;
}

// Products with both operands K-contiguous and 16-byte aligned rows take the
// direct-to-LDS kernel (128 x 256 tiles, 8 waves); everything else the
// register-staged family.
template <class Tr, int EPI>
bool launch_kc_direct(const GemmArgs<typename Tr::T>& g0, hipStream_t stream, int* rc) {
  if (!vec_ok(g0.A, g0.lda) || !vec_ok(g0.B, g0.ldb)) return false;
  GemmArgs<typename Tr::T> g = g0;
  // the tiling whose grids finish first: 160-row tiles (float64), or 128-row
  // tiles plus a 64-row launch over the remainder rows (plain or pair-mirrored
  // accumulation, whose rows can be offset)
  constexpr bool kTall = !Tr::kDrain;
  constexpr bool kSplit = EPI == EPI_ACC || EPI == EPI_PAIR || EPI == EPI_PM;
  long long main_rows = g.M;
  const int bm = choose_kc_tiling(g.M, g.N, kTall, kSplit, &main_rows);
  auto launch = [&](auto kernel, const GemmArgs<typename Tr::T>& a, int rows_per_tile) {
    GemmArgs<typename Tr::T> b = a;
    b.tiles_m = (b.M + rows_per_tile - 1) / rows_per_tile;
    b.tiles_n = (b.N + kDBN - 1) / kDBN;
    b.group_m = b.tiles_m < 16 ? b.tiles_m : 16;
    const long long tiles = (long long)b.tiles_m * b.tiles_n;
    hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(tiles)), dim3(kDThreads), 0, stream, b);
  };
  if ((long long)((g.M + 63) / 64) * ((g.N + kDBN - 1) / kDBN) > 0x7fffffffLL) return false;
  if (bm == 160) {
    if constexpr (kTall) launch(gemm_kc_direct_kernel<Tr, EPI, 160>, g, 160);
  } else if (bm == 64) {
    if constexpr (kSplit) {
      GemmArgs<typename Tr::T> rest = g;
      g.M = static_cast<int>(main_rows);
      rest.M -= g.M;
      rest.A += main_rows * g.lda;
      if constexpr (EPI == EPI_PAIR || EPI == EPI_PM)
        rest.m_off = g.m_off + g.M;  // the mirrored store needs the global (i,j) row
      else
        rest.C = static_cast<double*>(g.C) + main_rows * g.ldc;
      launch(gemm_kc_direct_kernel<Tr, EPI>, g, kDBM);
      launch(gemm_kc_direct_kernel<Tr, EPI, 64>, rest, 64);
    }
  } else {
    launch(gemm_kc_direct_kernel<Tr, EPI>, g, kDBM);
  }
  *rc = hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
  return true;
}

// Offsets of the packed build's compact grid: row_tiles[tm] = number of needed
// tiles in tile rows before tm (one thread; a few thousand rows at most).
__global__ void pack_rows_kernel(int* row_tiles, int tiles_m, int tiles_n, int v, int bm, int bn) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int acc = 0;
  for (int tm = 0; tm < tiles_m; ++tm) {
    row_tiles[tm] = acc;
    const int first = pack_first_tile(tm, bm, bn, v);
    acc += first < tiles_n ? tiles_n - first : 0;
  }
  row_tiles[tiles_m] = acc;
}

// Integral builds (both operands row-contiguous, permuted or packed store) take
// the direct-to-LDS RC kernel when rows are whole 16-byte chunks and aligned.
template <class Tr, int EPI>
bool launch_rc_direct(const GemmArgs<typename Tr::T>& g0, hipStream_t stream, int* rc) {
  constexpr int CH = Tr::CH;
  if (!vec_ok(g0.A, g0.lda) || !vec_ok(g0.B, g0.ldb)) return false;
  if (g0.M % CH != 0 || g0.N % CH != 0 || g0.K <= 0) return false;
  GemmArgs<typename Tr::T> g = g0;
  g.tiles_m = (g.M + kDBM - 1) / kDBM;
  g.tiles_n = (g.N + kDBN - 1) / kDBN;
  long long grid = (long long)g.tiles_m * g.tiles_n;
  if (grid > 0x7fffffffLL) return false;
  g.group_m = g.tiles_m < 16 ? g.tiles_m : 16;
  if (EPI == EPI_PACK || EPI == EPI_SYM) {
    if (!g.row_tiles) return false;
    long long needed = 0;
    for (int tm = 0; tm < g.tiles_m; ++tm) {
      const int first = pack_first_tile(tm, kDBM, kDBN, g.v);
      needed += first < g.tiles_n ? g.tiles_n - first : 0;
    }
    if (needed <= 0) {
      *rc = CC_LADDER_OK;
      return true;
    }
    hipLaunchKernelGGL(pack_rows_kernel, dim3(1), dim3(1), 0, stream,
                       const_cast<int*>(g.row_tiles), g.tiles_m, g.tiles_n, g.v, kDBM, kDBN);
    grid = needed;
  }
  hipLaunchKernelGGL((gemm_rc_direct_kernel<Tr, EPI>), dim3(static_cast<unsigned>(grid)),
                     dim3(kDThreads), 0, stream, g);
  *rc = hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
  return true;
}

// K-contiguous A times row-contiguous B, float64 accumulation: the mixed
// direct-to-LDS kernel when rows are aligned and N is whole 16-byte chunks.
template <class Tr>
bool launch_kr_direct(const GemmArgs<typename Tr::T>& g0, hipStream_t stream, int* rc) {
  if (!vec_ok(g0.A, g0.lda) || !vec_ok(g0.B, g0.ldb)) return false;
  if (g0.N % Tr::CH != 0 || g0.K <= 0) return false;
  GemmArgs<typename Tr::T> g = g0;
  g.tiles_m = (g.M + kDBM - 1) / kDBM;
  g.tiles_n = (g.N + kDBN - 1) / kDBN;
  const long long tiles = (long long)g.tiles_m * g.tiles_n;
  if (tiles > 0x7fffffffLL) return false;
  g.group_m = g.tiles_m < 16 ? g.tiles_m : 16;
  hipLaunchKernelGGL((gemm_kr_direct_kernel<Tr>), dim3(static_cast<unsigned>(tiles)),
                     dim3(kDThreads), 0, stream, g);
  *rc = hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
  return true;
}

template <class Tr, int LA, int LB, int EPI>
int launch_gemm(const typename Tr::T* A, long long lda, const typename Tr::T* B, long long ldb,
                void* C, long long ldc, int M, int N, int K, int v, int drain_steps,
                hipStream_t stream, int o = 0, int a0 = 0, int* row_tiles = nullptr,
                double alpha = 1.0, int pm = 0, int kband = 0, int m_keep = 0) {
  if (M <= 0 || N <= 0 || K <= 0) return CC_LADDER_OK;
  GemmArgs<typename Tr::T> g;
  g.alpha = alpha;
  g.pm = pm;
  g.kband = kband;
  g.m_keep = m_keep;
  g.A = A; g.lda = lda;
  g.B = B; g.ldb = ldb;
  g.C = C; g.ldc = ldc;
  g.M = M; g.N = N; g.K = K;
  g.v = v;
  g.o = o;
  g.a0 = a0;
  g.row_tiles = row_tiles;
  g.drain_steps = drain_steps > 0 ? drain_steps : 1;
  if constexpr (LA == RC && LB == RC &&
                (EPI == EPI_PERM || EPI == EPI_PACK || EPI == EPI_UNPACK || EPI == EPI_SYM) &&
                Tr::kDirectRC) {
    int rc = CC_LADDER_OK;
    if (launch_rc_direct<Tr, EPI>(g, stream, &rc)) return rc;
  }
  g.tiles_m = (M + kBM - 1) / kBM;
  g.tiles_n = (N + kBN - 1) / kBN;
  const long long tiles = (long long)g.tiles_m * g.tiles_n;
  if (tiles > 0x7fffffffLL) return CC_LADDER_EINVAL;
  // Bands of up to 16 tile rows: co-resident tiles of one XCD then share
  // both their row panels and a few column panels.
  g.group_m = g.tiles_m < 16 ? g.tiles_m : 16;
  dim3 grid(static_cast<unsigned>(tiles));
  if (EPI == EPI_PACK || EPI == EPI_SYM) {
    if (!row_tiles) return CC_LADDER_EINVAL;
    // the compact grid's size is the sum over tile rows of the needed columns
    long long needed = 0;
    for (int tm = 0; tm < g.tiles_m; ++tm) {
      const int first = pack_first_tile(tm, kBM, kBN, v);
      needed += first < g.tiles_n ? g.tiles_n - first : 0;
    }
    if (needed <= 0) return CC_LADDER_OK;
    hipLaunchKernelGGL(pack_rows_kernel, dim3(1), dim3(1), 0, stream, row_tiles, g.tiles_m,
                       g.tiles_n, v, kBM, kBN);
    grid = dim3(static_cast<unsigned>(needed));
  }
  if constexpr (LA == KC && LB == KC && (EPI == EPI_ACC || EPI == EPI_PAIR || EPI == EPI_PM) &&
                Tr::kDirectKC) {
    int rc = CC_LADDER_OK;
    if (launch_kc_direct<Tr, EPI>(g, stream, &rc)) return rc;
  }
  if constexpr (LA == KC && LB == RC && EPI == EPI_ACC && Tr::kDirectKR) {
    int rc = CC_LADDER_OK;
    if (launch_kr_direct<Tr>(g, stream, &rc)) return rc;
  }
  const dim3 block(kThreads);
  if (vec_ok(A, lda) && vec_ok(B, ldb))
    hipLaunchKernelGGL((gemm_kernel<Tr, LA, LB, EPI, true>), grid, block, 0, stream, g);
  else
    hipLaunchKernelGGL((gemm_kernel<Tr, LA, LB, EPI, false>), grid, block, 0, stream, g);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

// C[m*ldc + n] += sum_s part[s*stride + m*N + n], the split partials summed in
// order of s (the same order for every element, whatever the tiling).
__global__ __launch_bounds__(256) void part_reduce_kernel(const double* __restrict__ part, int S,
                                                          long long stride, int N, long long MN,
                                                          double* __restrict__ C, long long ldc) {
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < MN; e += step) {
    double acc = part[e];
    for (int q = 1; q < S; ++q) acc += part[q * stride + e];
    const long long m = e / N;
    C[m * ldc + (e - m * N)] += acc;
  }
}

// C[m*ldc + n] += sum_k A[m*lda + k] B[n*ldb + k] with K cut into `splits`
// ranges of whole K-steps, one workgroup per (tile, range), float64 partials in
// `part` (splits * M * N) and an ordered reduction.  For products whose tile grid
// alone leaves compute units idle (small M x N, long K).  Falls back to the plain
// product when there is one range or the operands do not suit the direct kernel.
template <class Tr>
int launch_contract_split(const typename Tr::T* A, long long lda, const typename Tr::T* B,
                          long long ldb, double* C, long long ldc, int M, int N, int K, int splits,
                          double* part, int drain_steps, hipStream_t stream) {
  if (M <= 0 || N <= 0 || K <= 0) return CC_LADDER_OK;
  if (splits <= 1 || !part || !vec_ok(A, lda) || !vec_ok(B, ldb))
    return launch_gemm<Tr, KC, KC, EPI_ACC>(A, lda, B, ldb, C, ldc, M, N, K, 0, drain_steps, stream);
  GemmArgs<typename Tr::T> g;
  g.alpha = 1.0;
  g.A = A; g.lda = lda;
  g.B = B; g.ldb = ldb;
  g.C = part; g.ldc = N;
  g.M = M; g.N = N; g.K = K;
  g.v = 0; g.o = 0; g.a0 = 0; g.row_tiles = nullptr;
  g.tiles_m = (M + kDBM - 1) / kDBM;
  g.tiles_n = (N + kDBN - 1) / kDBN;
  g.group_m = g.tiles_m < 16 ? g.tiles_m : 16;
  g.drain_steps = drain_steps > 0 ? drain_steps : 1;
  const int bk = kDRow / static_cast<int>(sizeof(typename Tr::T));
  const int nk = (K + bk - 1) / bk;
  g.split_steps = (nk + splits - 1) / splits;
  const int S = (nk + g.split_steps - 1) / g.split_steps;  // non-empty ranges
  g.part_stride = (long long)M * N;
  const long long grid = (long long)g.tiles_m * g.tiles_n * S;
  if (grid > 0x7fffffffLL) return CC_LADDER_EINVAL;
  hipLaunchKernelGGL((gemm_kc_direct_kernel<Tr, EPI_PART>), dim3(static_cast<unsigned>(grid)),
                     dim3(kDThreads), 0, stream, g);
  const long long MN = (long long)M * N;
  const long long blocks = std::min<long long>((MN + 255) / 256, 4096);
  hipLaunchKernelGGL(part_reduce_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                     static_cast<const double*>(part), S, g.part_stride, N, MN, C, ldc);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

// ---------------------------------------------------------------------------
// operand preparation and reductions
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void to_f32_kernel(const double* __restrict__ x,
                                                     float* __restrict__ y, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    y[i] = static_cast<float>(x[i]);  // round to nearest even
}

int to_f32(const double* x, float* y, size_t n, hipStream_t s) {
  if (!n) return CC_LADDER_OK;
  const long long blocks = std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(to_f32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, x, y,
                     static_cast<long long>(n));
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

// y[m][d][c] = x[m][c][d] for o^2 matrices m of v x v, through a 32 x 32 LDS
// tile so that both the read and the write of a tile row are coalesced.  One
// workgroup per (matrix, tile) pair, grid-stride.  Out is double or float
// (the float32 form swaps while converting, round to nearest even).
constexpr int kSwapTile = 32;

template <typename Out>
__global__ __launch_bounds__(256) void swap_cd_kernel(const double* __restrict__ x,
                                                      Out* __restrict__ y, int v, long long nmat,
                                                      int tiles) {
  __shared__ double tile[kSwapTile][kSwapTile + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows of 32 lanes
  const long long per_mat = (long long)tiles * tiles;
  const long long v2 = (long long)v * v;
  for (long long w = blockIdx.x; w < nmat * per_mat; w += gridDim.x) {
    const long long m = w / per_mat;
    const int r = static_cast<int>(w - m * per_mat);
    const int c0 = (r / tiles) * kSwapTile, d0 = (r % tiles) * kSwapTile;
    const double* xm = x + m * v2;
    Out* ym = y + m * v2;
#pragma unroll
    for (int k = ty; k < kSwapTile; k += 8) {
      const int c = c0 + k, d = d0 + tx;
      if (c < v && d < v) tile[k][tx] = xm[(long long)c * v + d];
    }
    __syncthreads();
#pragma unroll
    for (int k = ty; k < kSwapTile; k += 8) {
      const int d = d0 + k, c = c0 + tx;
      if (c < v && d < v) ym[(long long)d * v + c] = static_cast<Out>(tile[tx][k]);
    }
    __syncthreads();
  }
}

template <typename Out>
int swap_cd(const double* x, Out* y, int o, int v, hipStream_t s) {
  const long long nmat = (long long)o * o;
  const int tiles = (v + kSwapTile - 1) / kSwapTile;
  const long long work = nmat * tiles * tiles;
  const long long blocks = std::min<long long>(work, 16384);
  hipLaunchKernelGGL(swap_cd_kernel<Out>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, x,
                     y, v, nmat, tiles);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

__global__ __launch_bounds__(256) void fill_zero_kernel(double* __restrict__ x, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = 0.0;
}

int fill_zero(double* x, long long n, hipStream_t s) {
  if (n <= 0) return CC_LADDER_OK;
  const long long blocks = std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, x, n);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

// Pair-symmetric adjoint, per block: lamP[(ij)][q] = w lam[(ij)][(a,b)] for the
// block's packed pairs q -> (a, b) (a in the block, b >= a), w = 1/2 when a == b,
// row stride ldp; the pad columns [npairs, ldp) are zero.
template <typename T>
__global__ __launch_bounds__(256) void gather_pairs_kernel(const T* __restrict__ lam,
                                                           T* __restrict__ lamP, int o2, int v,
                                                           int a0, long long npairs, long long ldp) {
  const long long n = (long long)o2 * ldp;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long v2 = (long long)v * v;
  const long long base = pair_prefix_d(a0, v);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const long long row = e / ldp, q = e - row * ldp;
    if (q >= npairs) {
      lamP[e] = T(0);
      continue;
    }
    const int a = pair_row(base + q, v);
    const int b = a + static_cast<int>(base + q - pair_prefix_d(a, v));
    const T x = lam[row * v2 + (long long)a * v + b];
    lamP[e] = (a == b) ? x * T(0.5) : x;
  }
}

// Rows (a - a0, c) of a half-written adjoint block W[na][v][v][v] (only b >= a
// stored by the packed product): zeros at b in [max(0, a - s), a), the rows next
// to the diagonal that the K-banded products still read.
template <typename T>
__global__ __launch_bounds__(256) void zero_band_kernel(T* __restrict__ W, int na, int v, int a0,
                                                        int s) {
  const long long v2 = (long long)v * v;
  const long long rows = (long long)na * v;
  for (long long r = blockIdx.x; r < rows; r += gridDim.x) {
    const int a = a0 + static_cast<int>(r / v);
    const int b0 = a - s > 0 ? a - s : 0;
    T* row = W + r * v2;
    for (long long e = (long long)b0 * v + threadIdx.x; e < (long long)a * v; e += blockDim.x)
      row[e] = T(0);
  }
}

// dt[i][j][c][d] += B[i][j][c][d] + B[j][i][d][c], the mirror read through a
// 32 x 32 LDS tile so that both reads and the update are coalesced.
__global__ __launch_bounds__(256) void mirror_add_kernel(const double* __restrict__ B,
                                                         double* __restrict__ dt, int o, int v,
                                                         int tiles) {
  __shared__ double tile[kSwapTile][kSwapTile + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const long long per_mat = (long long)tiles * tiles;
  const long long nmat = (long long)o * o;
  const long long v2 = (long long)v * v;
  for (long long w = blockIdx.x; w < nmat * per_mat; w += gridDim.x) {
    const long long m = w / per_mat;
    const int i = static_cast<int>(m / o), j = static_cast<int>(m - (long long)i * o);
    const long long mp = (long long)j * o + i;
    const int r = static_cast<int>(w - m * per_mat);
    const int c0 = (r / tiles) * kSwapTile, d0 = (r % tiles) * kSwapTile;
#pragma unroll
    for (int k = ty; k < kSwapTile; k += 8) {  // rows d, columns c of the mirror matrix
      const int d = d0 + k, c = c0 + tx;
      if (c < v && d < v) tile[k][tx] = B[mp * v2 + (long long)d * v + c];
    }
    __syncthreads();
#pragma unroll
    for (int k = ty; k < kSwapTile; k += 8) {  // rows c, columns d of this matrix
      const int c = c0 + k, d = d0 + tx;
      if (c < v && d < v) {
        const long long e = m * v2 + (long long)c * v + d;
        dt[e] += B[e] + tile[tx][k];
      }
    }
    __syncthreads();
  }
}

// In place W <- W + W^T for a square n x n matrix (row stride n): one workgroup
// per pair of 32 x 32 tiles P <= Q reads both tiles through LDS and writes both
// sums, so every element is read and written once and no two workgroups touch
// the same element.
template <typename T>
__global__ __launch_bounds__(256) void sym_add_kernel(T* __restrict__ W, long long n, int tiles) {
  __shared__ double a[kSwapTile][kSwapTile + 1], b[kSwapTile][kSwapTile + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const long long npairs = (long long)tiles * (tiles + 1) / 2;
  for (long long w = blockIdx.x; w < npairs; w += gridDim.x) {
    const int P = pair_row(w, tiles);
    const int Q = P + static_cast<int>(w - pair_prefix_d(P, tiles));
    const long long p0 = (long long)P * kSwapTile, q0 = (long long)Q * kSwapTile;
#pragma unroll
    for (int k = ty; k < kSwapTile; k += 8) {
      // a[k][tx] = W[p0+k][q0+tx], b[k][tx] = W[q0+k][p0+tx]
      a[k][tx] = (p0 + k < n && q0 + tx < n) ? static_cast<double>(W[(p0 + k) * n + q0 + tx]) : 0.0;
      b[k][tx] = (q0 + k < n && p0 + tx < n) ? static_cast<double>(W[(q0 + k) * n + p0 + tx]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = ty; k < kSwapTile; k += 8) {
      // W[p0+k][q0+tx] = a[k][tx] + b[tx][k]; W[q0+k][p0+tx] = b[k][tx] + a[tx][k]
      if (p0 + k < n && q0 + tx < n) W[(p0 + k) * n + q0 + tx] = static_cast<T>(a[k][tx] + b[tx][k]);
      if (P != Q && q0 + k < n && p0 + tx < n)
        W[(q0 + k) * n + p0 + tx] = static_cast<T>(b[k][tx] + a[tx][k]);
    }
    __syncthreads();
  }
}

template <typename T>
int sym_add(T* W, long long n, hipStream_t s) {
  const int tiles = static_cast<int>((n + kSwapTile - 1) / kSwapTile);
  const long long work = (long long)tiles * (tiles + 1) / 2;
  const long long blocks = std::min<long long>(work, 65536);
  hipLaunchKernelGGL((sym_add_kernel<T>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, W, n,
                     tiles);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

int mirror_add(const double* B, double* dt, int o, int v, hipStream_t s) {
  const int tiles = (v + kSwapTile - 1) / kSwapTile;
  const long long work = (long long)o * o * tiles * tiles;
  const long long blocks = std::min<long long>(work, 16384);
  hipLaunchKernelGGL(mirror_add_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, B, dt,
                     o, v, tiles);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

// Symmetric and antisymmetric combinations of the v x v matrices X[r] of a set
// of rows, over the pairs of their two indices:
//   plus [rp][k(c,d)] = X[c][d] + X[d][c] for c < d,  wdiag * X[c][c] for c = d
//   minus[rm][k'(c,d)] = sm * (X[c][d] - X[d][c])      for c < d
// with k(c,d) = prefix_v(c) + d - c numbering the pairs c <= d and k'(c,d) =
// prefix_{v-1}(c) + d - c - 1 the pairs c < d.  Rows:
//   AMPS: the pairs (i, j), i <= j, of o; X = t[i][j]; rp = the pair index, rm
//         its index among the pairs i < j (none for i = j)
//   INTS: the packed integral rows (a, b), a <= b, a from a0; X = row r of the
//         block; rp = r, rm = the local index among the pairs a < b (none for a = b)
// One workgroup per (row, tile pair C <= D of 32 x 32 tiles): both tiles X[C][D]
// and X[D][C] go through LDS, so reads and writes run along contiguous d.
enum { PM_AMPS = 0, PM_INTS = 1 };

template <int MODE, typename In, typename Out>
__global__ __launch_bounds__(256) void pm_rows_kernel(const In* __restrict__ X, long long nrows,
                                                      int n, int a0, int v, int tiles,
                                                      Out* __restrict__ plus, long long ldp,
                                                      Out* __restrict__ minus, long long ldm,
                                                      double wdiag, double sm) {
  __shared__ double xs[kSwapTile][kSwapTile + 1], ys[kSwapTile][kSwapTile + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const long long ntp = (long long)tiles * (tiles + 1) / 2;
  const long long v2 = (long long)v * v;
  for (long long w = blockIdx.x; w < nrows * ntp; w += gridDim.x) {
    const long long r = w / ntp;
    const int tp = static_cast<int>(w - r * ntp);
    const int C = pair_row(tp, tiles);
    const int D = C + static_cast<int>(tp - pair_prefix_d(C, tiles));
    const int c0 = C * kSwapTile, d0 = D * kSwapTile;
    long long src, rm;
    if (MODE == PM_AMPS) {
      const int i = pair_row(r, n);
      const int j = i + static_cast<int>(r - pair_prefix_d(i, n));
      src = (long long)i * n + j;
      rm = i < j ? pair_prefix_d(i, n - 1) + (j - i - 1) : -1;
    } else {
      const long long q = pair_prefix_d(a0, v) + r;
      const int a = pair_row(q, v);
      const int b = a + static_cast<int>(q - pair_prefix_d(a, v));
      src = r;
      rm = a < b ? pair_prefix_d(a, v - 1) - pair_prefix_d(a0, v - 1) + (b - a - 1) : -1;
    }
    const In* x = X + src * v2;
#pragma unroll
    for (int k = ty; k < kSwapTile; k += 8) {
      const int c = c0 + k, d = d0 + tx;  // xs[k][tx] = X[c0+k][d0+tx]
      xs[k][tx] = (c < v && d < v) ? static_cast<double>(x[(long long)c * v + d]) : 0.0;
      const int dd = d0 + k, cc = c0 + tx;  // ys[k][tx] = X[d0+k][c0+tx]
      ys[k][tx] = (dd < v && cc < v) ? static_cast<double>(x[(long long)dd * v + cc]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = ty; k < kSwapTile; k += 8) {
      const int c = c0 + k, d = d0 + tx;
      if (c < v && d < v && c <= d) {
        const double xcd = xs[k][tx], xdc = ys[tx][k];
        const long long kp = pair_prefix_d(c, v) + (d - c);
        plus[r * ldp + kp] = static_cast<Out>(c == d ? wdiag * xcd : xcd + xdc);
        if (rm >= 0 && c < d) {
          const long long km = pair_prefix_d(c, v - 1) + (d - c - 1);
          minus[rm * ldm + km] = static_cast<Out>(sm * (xcd - xdc));
        }
      }
    }
    __syncthreads();
  }
}

template <int MODE, typename In, typename Out>
int pm_rows(const In* X, long long nrows, int n, int a0, int v, Out* plus, long long ldp,
            Out* minus, long long ldm, double wdiag, double sm, hipStream_t s) {
  if (nrows <= 0) return CC_LADDER_OK;
  const int tiles = (v + kSwapTile - 1) / kSwapTile;
  const long long work = nrows * ((long long)tiles * (tiles + 1) / 2);
  const long long blocks = std::min<long long>(work, 65536);
  hipLaunchKernelGGL((pm_rows_kernel<MODE, In, Out>), dim3(static_cast<unsigned>(blocks)), dim3(256),
                     0, s, X, nrows, n, a0, v, tiles, plus, ldp, minus, ldm, wdiag, sm);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

// Symmetric vectors: Lp[x][pair(a,c)] = L[x][a][c] for a <= c (pair(a,c) =
// prefix_v(a) + c - a), row stride ldg, the pad columns [v(v+1)/2, ldg) zero.
// One workgroup per (x, a): contiguous reads and writes along c.
template <typename Out>
__global__ __launch_bounds__(256) void pack_sym_kernel(const double* __restrict__ L,
                                                       Out* __restrict__ Lp, int P, int v,
                                                       long long ldg) {
  const long long v2 = (long long)v * v;
  const long long npv = (long long)v * (v + 1) / 2;
  for (long long r = blockIdx.x; r < (long long)P * v; r += gridDim.x) {
    const long long x = r / v;
    const int a = static_cast<int>(r - x * v);
    const double* src = L + x * v2 + (long long)a * v;
    Out* dst = Lp + x * ldg + pair_prefix_d(a, v) - a;  // dst[c] = Lp[x][pair(a, c)]
    for (int c = a + static_cast<int>(threadIdx.x); c < v; c += blockDim.x)
      dst[c] = static_cast<Out>(src[c]);
    if (a == v - 1)
      for (long long e = npv + threadIdx.x; e < ldg; e += blockDim.x) Lp[x * ldg + e] = Out(0);
  }
}

// A block's integral rows, gathered from the whole pair-pair integral G of
// symmetric vectors (G[p][q] = G[q][p], p, q unordered pairs): the rows (a, b),
// a <= b, a from a0, of X_ab[c][d] = (ac|bd) = G[{a,c}][{b,d}], either whole
// (GATHER_ROWS: plus[r][c*v + d], the packed block of the pair-symmetric
// forward and adjoint) or combined into plus/minus exactly as in pm_rows
// (GATHER_PM: wdiag 2, sm 1).
// Work item w = (tile pair C <= D, row r), the row inner: workgroups that run
// together on one XCD take consecutive rows, the same a with consecutive b.
// Every element of the two 32 x 32 tiles is read in an orientation of G that
// keeps 32 lanes on one contiguous run where one exists: along d in row {a,c}
// when d >= b; along c in row {b,d} when d < b and c >= a; otherwise (c < a,
// d < b) element by element, where neighbouring rows b share the cache lines.
enum { GATHER_PM = 0, GATHER_ROWS = 1 };

template <int MODE, typename T>
__global__ __launch_bounds__(256) void pm_gather_kernel(const T* __restrict__ G, long long ldg,
                                                        long long nrows, int a0, int v, int tiles,
                                                        T* __restrict__ plus, long long ldp,
                                                        T* __restrict__ minus, long long ldm) {
  __shared__ double xs[kSwapTile][kSwapTile + 1], ys[kSwapTile][kSwapTile + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const long long ntp = (long long)tiles * (tiles + 1) / 2;
  const long long work = nrows * ntp;
  auto pp = [&](long long x) { return pair_prefix_d(x, v); };
  for (long long w = xcd_linear(blockIdx.x, gridDim.x); w < work; w += gridDim.x) {
    const long long tp = w / nrows, r = w - tp * nrows;
    const int C = pair_row(tp, tiles);
    const int D = C + static_cast<int>(tp - pair_prefix_d(C, tiles));
    const int c0 = C * kSwapTile, d0 = D * kSwapTile;
    const long long q = pp(a0) + r;
    const int a = pair_row(q, v);
    const int b = a + static_cast<int>(q - pp(a));
    const long long rm = a < b ? pair_prefix_d(a, v - 1) - pair_prefix_d(a0, v - 1) + (b - a - 1) : -1;
    // S[k][l] = X_ab[r0 + k][s0 + l]
    auto load = [&](double (*S)[kSwapTile + 1], int r0, int s0) {
#pragma unroll
      for (int k = ty; k < kSwapTile; k += 8) {
        const int c = r0 + k, d = s0 + tx;
        double x = 0.0;
        if (c < v && d < v) {
          if (d >= b) {
            const long long pac = a <= c ? pp(a) + c - a : pp(c) + a - c;
            x = static_cast<double>(G[pac * ldg + pp(b) + d - b]);
          } else if (c < a) {
            x = static_cast<double>(G[(pp(c) + a - c) * ldg + pp(d) + b - d]);
          }
        }
        if (!(c < v && d < v) || d >= b || c < a) S[k][tx] = x;
      }
#pragma unroll
      for (int l = ty; l < kSwapTile; l += 8) {
        const int c = r0 + tx, d = s0 + l;
        if (c < v && d < v && d < b && c >= a)
          S[tx][l] = static_cast<double>(G[(pp(d) + b - d) * ldg + pp(a) + c - a]);
      }
    };
    load(xs, c0, d0);
    if (MODE == GATHER_PM || D != C) load(ys, d0, c0);
    __syncthreads();
    if (MODE == GATHER_ROWS) {
      // X[C][D] and X[D][C] along contiguous d
      T* row = plus + r * ldp;
#pragma unroll
      for (int k = ty; k < kSwapTile; k += 8) {
        if (c0 + k < v && d0 + tx < v)
          row[(long long)(c0 + k) * v + d0 + tx] = static_cast<T>(xs[k][tx]);
        if (D != C && d0 + k < v && c0 + tx < v)
          row[(long long)(d0 + k) * v + c0 + tx] = static_cast<T>(ys[k][tx]);
      }
    } else {
#pragma unroll
      for (int k = ty; k < kSwapTile; k += 8) {
        const int c = c0 + k, d = d0 + tx;
        if (c < v && d < v && c <= d) {
          const double xcd = xs[k][tx], xdc = ys[tx][k];
          const long long kp = pp(c) + (d - c);
          plus[r * ldp + kp] = static_cast<T>(c == d ? 2.0 * xcd : xcd + xdc);
          if (rm >= 0 && c < d) {
            const long long km = pair_prefix_d(c, v - 1) + (d - c - 1);
            minus[rm * ldm + km] = static_cast<T>(xcd - xdc);
          }
        }
      }
    }
    __syncthreads();
  }
}

template <int MODE, typename T>
int pm_gather(const T* G, long long ldg, long long nrows, int a0, int v, T* plus, long long ldp,
              T* minus, long long ldm, hipStream_t s) {
  if (nrows <= 0) return CC_LADDER_OK;
  const int tiles = (v + kSwapTile - 1) / kSwapTile;
  const long long work = nrows * ((long long)tiles * (tiles + 1) / 2);
  const long long blocks = std::min<long long>(work, 65536);
  hipLaunchKernelGGL((pm_gather_kernel<MODE, T>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                     s, G, ldg, nrows, a0, v, tiles, plus, ldp, minus, ldm);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

// Symmetric vectors: G[p][q] = sum_x Lp[x][p] Lp[x][q] over the unordered pairs,
// the tiles on or above the diagonal (each stored with its mirror), traced as
// the build of block 0.
template <class Tr>
int build_pair_integral(const Plan& pl, const typename Tr::T* Lp, typename Tr::T* G,
                        int* row_tiles, const Tracer& tr, hipStream_t s) {
  const int drain = Tr::kDrain ? pl.k_chunk / Tr::BK : 0;
  const int n = static_cast<int>(pl.ldg);
  tr(CC_LADDER_PHASE_BUILD, 0, 0);
  const int rc = launch_gemm<Tr, RC, RC, EPI_SYM>(Lp, pl.ldg, Lp, pl.ldg, G, pl.ldg, n, n, pl.P, 1,
                                                  drain, s, 0, 0, row_tiles);
  tr(CC_LADDER_PHASE_BUILD, 0, 1);
  return rc;
}

template <typename Out>
int pack_sym(const double* L, Out* Lp, int P, int v, long long ldg, hipStream_t s) {
  const long long blocks = std::min<long long>((long long)P * v, 65536);
  hipLaunchKernelGGL((pack_sym_kernel<Out>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                     L, Lp, P, v, ldg);
  return hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
}

constexpr int kRedBlocks = 1024;

__global__ __launch_bounds__(256) void reduce_partial_kernel(const double* __restrict__ x,
                                                             const double* __restrict__ y,
                                                             long long n, double* part) {
  double sxy = 0.0, syy = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double yi = y[i];
    sxy = fma(x[i], yi, sxy);
    syy = fma(yi, yi, syy);
  }
  __shared__ double s1[256], s2[256];
  s1[threadIdx.x] = sxy;
  s2[threadIdx.x] = syy;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1[0];
    part[2 * blockIdx.x + 1] = s2[0];
  }
}

__global__ __launch_bounds__(256) void reduce_final_kernel(const double* __restrict__ part, int nb,
                                                           double* out) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  __shared__ double s1[256], s2[256];
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s1[0];
    out[1] = s2[0];
  }
}

// ---------------------------------------------------------------------------
// scratch
// ---------------------------------------------------------------------------

struct Scratch {
  char* base = nullptr;
  bool owned = false;
  hipStream_t stream = nullptr;
  ~Scratch() {
    if (owned && base) (void)hipFreeAsync(base, stream);
  }
};

size_t default_budget() {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return 0;
  const size_t half = free_b / 2;
  const size_t cap = static_cast<size_t>(128) << 30;
  return half < cap ? half : cap;
}

// The caller's workspace when given (it must hold the plan), else a stream-
// ordered allocation released when `ws` goes out of scope.
int take_scratch(const Plan& plan, hipStream_t stream, const cc_ladder_opts* opts, Scratch* ws) {
  if (opts && opts->workspace) {
    if (opts->workspace_bytes < plan.bytes) return CC_LADDER_ENOMEM;
    ws->base = static_cast<char*>(opts->workspace);
    return CC_LADDER_OK;
  }
  void* p = nullptr;
  const hipError_t e = hipMallocAsync(&p, plan.bytes ? plan.bytes : 256, stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? CC_LADDER_ENOMEM : CC_LADDER_EHIP;
  }
  ws->base = static_cast<char*>(p);
  ws->owned = true;
  ws->stream = stream;
  return CC_LADDER_OK;
}

// Planning, device check and scratch of a ladder call, in this order: with a
// caller workspace the plan (sized to it) and the workspace's overlap with the
// call's arrays are settled on the host before any device call; otherwise the
// budget (the caller's, or half the free device memory) needs the device first.
int plan_and_scratch(int o, int v, int P, int precision, int backward, hipStream_t stream,
                     const cc_ladder_opts* opts, const Operand* ops, int nops, Plan* plan,
                     Scratch* ws) {
  int rc;
  if (opts && opts->workspace) {
    rc = make_plan(o, v, P, precision, backward, opts->workspace_bytes, opts, plan);
    if (rc) return rc;
    rc = check_workspace(opts, plan->bytes, ops, nops);
    if (rc) return rc;
    rc = check_device();
    if (rc) return rc;
  } else {
    rc = check_device();
    if (rc) return rc;
    const size_t budget = (opts && opts->hbm_budget) ? opts->hbm_budget : default_budget();
    if (!budget) return CC_LADDER_EHIP;
    rc = make_plan(o, v, P, precision, backward, budget, opts, plan);
    if (rc) return rc;
  }
  return take_scratch(*plan, stream, opts, ws);
}

// Symmetry check of nmat v x v matrices: out[0] = max |x[m][c][d] - x[m'][d][c]|
// with partner m' = (j, i) of m = (i, j) over o x o when o > 0 (the pair
// symmetry of t or lam), m' = m when o == 0 (each matrix symmetric: the
// Cholesky vectors); out[1] = max |x|; as the bit patterns of non-negative
// doubles (ordered like the values, so an integer maximum combines them).  out
// must be zero on entry.
__global__ __launch_bounds__(256) void pair_asym_kernel(const double* __restrict__ x, long long nmat,
                                                        int o, int v, unsigned long long* out) {
  const long long v2 = (long long)v * v;
  const long long n = nmat * v2;
  const long long stride = (long long)gridDim.x * blockDim.x;
  double dmax = 0.0, xmax = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const long long m = e / v2, cd = e - m * v2;
    long long partner = m;
    if (o > 0) {
      const long long i = m / o, j = m - i * o;
      partner = j * o + i;
    }
    const long long c = cd / v, d = cd - c * v;
    const double a = x[e];
    const double b = x[partner * v2 + d * v + c];
    dmax = fmax(dmax, fabs(a - b));
    xmax = fmax(xmax, fabs(a));
  }
  __shared__ double s1[256], s2[256];
  s1[threadIdx.x] = dmax;
  s2[threadIdx.x] = xmax;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + w]);
      s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(s1[0])));
    atomicMax(out + 1, static_cast<unsigned long long>(__double_as_longlong(s2[0])));
  }
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  if (static_cast<int>(threadIdx.x) < n) p[threadIdx.x] = 0ull;
}

// CC_LADDER_CHECK_SYMMETRY: returns CC_LADDER_EINVAL when some pair of x differs
// by more than 2^-40 max|x| (synchronises the stream to read the result).
int check_symmetric(const double* x, long long nmat, int o, int v, unsigned long long* buf,
                    hipStream_t s) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, buf, 2);
  const long long n = nmat * v * v;
  const long long blocks = std::min<long long>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(pair_asym_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, x,
                     nmat, o, v, buf);
  if (hipGetLastError() != hipSuccess) return CC_LADDER_EHIP;
  unsigned long long h[2] = {0, 0};
  CCL_HIP(hipMemcpyAsync(h, buf, sizeof(h), hipMemcpyDeviceToHost, s));
  CCL_HIP(hipStreamSynchronize(s));
  double d, m;
  std::memcpy(&d, &h[0], sizeof(double));
  std::memcpy(&m, &h[1], sizeof(double));
  return d <= std::ldexp(m, -40) ? CC_LADDER_OK : CC_LADDER_EINVAL;
}

// t or lam against its pair transpose x[j][i][d][c]
int check_pair_symmetric(const double* x, int o, int v, unsigned long long* buf, hipStream_t s) {
  return check_symmetric(x, (long long)o * o, o, v, buf, s);
}

// the Cholesky vectors against their transposes L[x][c][a]
int check_vectors_symmetric(const double* L, int P, int v, unsigned long long* buf, hipStream_t s) {
  return check_symmetric(L, P, 0, v, buf, s);
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------

template <class Tr>
int forward_blocks(const Plan& pl, const typename Tr::T* L, const typename Tr::T* t, double* R,
                   typename Tr::T* V, int* row_tiles, const Tracer& tr, hipStream_t s,
                   const typename Tr::T* Lp = nullptr, typename Tr::T* G = nullptr) {
  const int o = pl.o, v = pl.v, P = pl.P;
  const long long v2 = (long long)v * v;
  const int drain = Tr::kDrain ? pl.k_chunk / Tr::BK : 0;
  if (pl.gsym) {
    const int rc = build_pair_integral<Tr>(pl, Lp, G, row_tiles, tr, s);
    if (rc) return rc;
  }
  for (int blk = 0; blk < pl.nblocks; ++blk) {
    int a0, na;
    block_range(pl, blk, &a0, &na);
    if (na <= 0) continue;
    if (pl.pairsym) {
      // packed rows (a,b), a in the block, b >= a: columns (b,d) from b = a0 on
      // (or, with symmetric vectors, gathered from the pair-pair integral)
      const long long off = (long long)a0 * v;
      const long long npairs = pair_prefix(a0 + na, v) - pair_prefix(a0, v);
      tr(CC_LADDER_PHASE_BUILD, blk, 0);
      int rc = pl.gsym ? pm_gather<GATHER_ROWS>(static_cast<const typename Tr::T*>(G), pl.ldg,
                                                npairs, a0, v, V, v2,
                                                static_cast<typename Tr::T*>(nullptr), 0, s)
                       : launch_gemm<Tr, RC, RC, EPI_PACK>(L + off, v2, L + off, v2, V, 0, na * v,
                                                           static_cast<int>((long long)(v - a0) * v),
                                                           P, v, drain, s, o, a0, row_tiles);
      tr(CC_LADDER_PHASE_BUILD, blk, 1);
      if (rc) return rc;
      // R[(ij)][(ab)] and R[(ji)][(ba)] += t[(ij)][(cd)] . V_A[pair(a,b)][(cd)]
      tr(CC_LADDER_PHASE_CONTRACT, blk, 0);
      rc = launch_gemm<Tr, KC, KC, EPI_PAIR>(t, v2, V, v2, R, v2, o * o, static_cast<int>(npairs),
                                             static_cast<int>(v2), v, drain, s, o, a0);
      tr(CC_LADDER_PHASE_CONTRACT, blk, 1);
      if (rc) return rc;
      continue;
    }
    // V_A[a][b][c][d]: rows (a,c) of L's block, columns (b,d) of L, K = x
    tr(CC_LADDER_PHASE_BUILD, blk, 0);
    int rc = launch_gemm<Tr, RC, RC, EPI_PERM>(L + (long long)a0 * v, v2, L, v2, V, 0, na * v,
                                               static_cast<int>(v2), P, v, drain, s);
    tr(CC_LADDER_PHASE_BUILD, blk, 1);
    if (rc) return rc;
    // R[(ij)][a0*v + (a,b)] += t[(ij)][(cd)] . V_A[(ab)][(cd)]
    tr(CC_LADDER_PHASE_CONTRACT, blk, 0);
    rc = launch_gemm<Tr, KC, KC, EPI_ACC>(t, v2, V, v2, R + (long long)a0 * v, v2, o * o, na * v,
                                          static_cast<int>(v2), v, drain, s);
    tr(CC_LADDER_PHASE_CONTRACT, blk, 1);
    if (rc) return rc;
  }
  return CC_LADDER_OK;
}

// Forward over the symmetric and antisymmetric combinations (pair-symmetric t):
// per block, the packed integral rows a <= b are built as in the pair-symmetric
// forward, combined into V+ (a <= b, c <= d) and V- (a < b, c < d), and
// contracted with t+ (rows i <= j) and t- (rows i < j); each product adds half
// its result to R at the four (i,j)/(a,b) mirrors.
template <class Tr>
int forward_blocks_pm(const Plan& pl, const typename Tr::T* L, const typename Tr::T* Tp,
                      const typename Tr::T* Tm, double* R, typename Tr::T* V,
                      typename Tr::T* Vp, typename Tr::T* Vm, int* row_tiles, const Tracer& tr,
                      hipStream_t s, const typename Tr::T* Lp = nullptr,
                      typename Tr::T* G = nullptr) {
  const int o = pl.o, v = pl.v, P = pl.P;
  const long long v2 = (long long)v * v;
  const int drain = Tr::kDrain ? pl.k_chunk / Tr::BK : 0;
  const int mp = o * (o + 1) / 2, mm = o * (o - 1) / 2;
  const int kp = static_cast<int>((long long)v * (v + 1) / 2);
  const int km = static_cast<int>((long long)v * (v - 1) / 2);
  if (pl.gsym) {
    const int rc = build_pair_integral<Tr>(pl, Lp, G, row_tiles, tr, s);
    if (rc) return rc;
  }
  for (int blk = 0; blk < pl.nblocks; ++blk) {
    int a0, na;
    block_range(pl, blk, &a0, &na);
    if (na <= 0) continue;
    const long long off = (long long)a0 * v;
    const long long np = pair_prefix(a0 + na, v) - pair_prefix(a0, v);
    const long long nm = np - na;
    tr(CC_LADDER_PHASE_BUILD, blk, 0);
    int rc;
    if (pl.gsym) {
      rc = pm_gather<GATHER_PM>(static_cast<const typename Tr::T*>(G), pl.ldg, np, a0, v, Vp,
                                pl.ldp, Vm, pl.ldm, s);
    } else {
      rc = launch_gemm<Tr, RC, RC, EPI_PACK>(L + off, v2, L + off, v2, V, 0, na * v,
                                             static_cast<int>((long long)(v - a0) * v), P, v,
                                             drain, s, o, a0, row_tiles);
      if (!rc)
        rc = pm_rows<PM_INTS>(V, np, v, a0, v, Vp, pl.ldp, Vm, pl.ldm, 2.0, 1.0, s);
    }
    tr(CC_LADDER_PHASE_BUILD, blk, 1);
    if (rc) return rc;
    tr(CC_LADDER_PHASE_CONTRACT, blk, 0);
    rc = launch_gemm<Tr, KC, KC, EPI_PM>(Tp, pl.ldp, Vp, pl.ldp, R, v2, mp, static_cast<int>(np), kp,
                                         v, drain, s, o, a0, nullptr, 0.5, 1);
    if (!rc)
      rc = launch_gemm<Tr, KC, KC, EPI_PM>(Tm, pl.ldm, Vm, pl.ldm, R, v2, mm, static_cast<int>(nm),
                                           km, v, drain, s, o, a0, nullptr, 0.5, 2);
    tr(CC_LADDER_PHASE_CONTRACT, blk, 1);
    if (rc) return rc;
  }
  return CC_LADDER_OK;
}

template <class Tr>
int backward_blocks(const Plan& pl, const typename Tr::T* L, const typename Tr::T* t,
                    const typename Tr::T* lam, double* dL, double* dt, char* base,
                    const Tracer& tr, hipStream_t s, const typename Tr::T* Lp = nullptr,
                    typename Tr::T* G = nullptr) {
  using T = typename Tr::T;
  const int o = pl.o, v = pl.v, P = pl.P;
  const long long v2 = (long long)v * v;
  const int drain = Tr::kDrain ? pl.k_chunk / Tr::BK : 0;
  T* V = reinterpret_cast<T*>(base + pl.off_V);
  T* W = reinterpret_cast<T*>(base + pl.off_W);
  const bool sym = pl.pairsym_adj != 0;
  // pair-symmetric t and lam: dt = B + mirror(B) with B over the packed rows a <= b
  double* Bacc = sym ? reinterpret_cast<double*>(base + pl.off_B) : nullptr;
  T* lamP = sym ? reinterpret_cast<T*>(base + pl.off_lamP) : nullptr;
  int* row_tiles = sym ? reinterpret_cast<int*>(base + pl.off_tiles) : nullptr;
  if (sym) {
    int rc = fill_zero(Bacc, (long long)o * o * v2, s);
    if (!rc && pl.gsym) rc = build_pair_integral<Tr>(pl, Lp, G, row_tiles, tr, s);
    if (rc) return rc;
  }
  for (int blk = 0; blk < pl.nblocks; ++blk) {
    int a0, na;
    block_range(pl, blk, &a0, &na);
    if (na <= 0) continue;
    const long long off = (long long)a0 * v;
    // pair-symmetric: the block's packed pairs (a, b), a <= b, and lamP's row stride
    const long long npairs = pair_prefix(a0 + na, v) - pair_prefix(a0, v);
    const long long ldp = (npairs + 3) / 4 * 4;
    int rc;
    if (sym) {
      tr(CC_LADDER_PHASE_BUILD, blk, 0);
      rc = pl.gsym ? pm_gather<GATHER_ROWS>(static_cast<const T*>(G), pl.ldg, npairs, a0, v, V, v2,
                                            static_cast<T*>(nullptr), 0, s)
                   : launch_gemm<Tr, RC, RC, EPI_PACK>(L + off, v2, L + off, v2, V, 0, na * v,
                                                       static_cast<int>((long long)(v - a0) * v), P,
                                                       v, drain, s, o, a0, row_tiles);
      tr(CC_LADDER_PHASE_BUILD, blk, 1);
      if (rc) return rc;
      // B[(ij)][(cd)] += sum_(ab packed) w lam[(ij)][(ab)] V_A[pair(a,b)][(cd)]
      tr(CC_LADDER_PHASE_DT, blk, 0);
      const long long n = (long long)o * o * npairs;
      const long long blocks = std::min<long long>((n + 255) / 256, 8192);
      hipLaunchKernelGGL((gather_pairs_kernel<T>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                         s, lam, lamP, o * o, v, a0, npairs, ldp);
      rc = hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
      if (!rc)
        rc = launch_gemm<Tr, KC, RC, EPI_ACC>(lamP, ldp, V, v2, Bacc, v2, o * o,
                                              static_cast<int>(v2), static_cast<int>(npairs), v,
                                              drain, s);
      tr(CC_LADDER_PHASE_DT, blk, 1);
      if (rc) return rc;
    } else {
      tr(CC_LADDER_PHASE_BUILD, blk, 0);
      rc = launch_gemm<Tr, RC, RC, EPI_PERM>(L + off, v2, L, v2, V, 0, na * v,
                                             static_cast<int>(v2), P, v, drain, s);
      tr(CC_LADDER_PHASE_BUILD, blk, 1);
      if (rc) return rc;
      // dt[(ij)][(cd)] += lam[(ij)][a0*v + (ab)] . V_A[(ab)][(cd)]
      tr(CC_LADDER_PHASE_DT, blk, 0);
      rc = launch_gemm<Tr, KC, RC, EPI_ACC>(lam + off, v2, V, v2, dt, v2, o * o,
                                            static_cast<int>(v2), na * v, v, drain, s);
      tr(CC_LADDER_PHASE_DT, blk, 1);
      if (rc) return rc;
    }
    // W'_A[a][c][b][d] = sum_(ij) lam[(ij)][a0*v + (ab)] t[(ij)][(cd)]
    tr(CC_LADDER_PHASE_W, blk, 0);
    if (sym) {
      // With pair-symmetric t and lam, W[b,d,a,c] = W[a,c,b,d]: only the half
      // Wh over the packed pairs b >= a is formed (the diagonal a == b halved by
      // lamP's weights), so that W = Wh + Wh^T.  The K-banded dL products read
      // up to `band` rows b below the diagonal: those are zeroed.
      const int band = (kDBN - 2 + v) / v + (32 - 2 + v) / v;
      const long long rows = (long long)na * v;
      hipLaunchKernelGGL((zero_band_kernel<T>), dim3(static_cast<unsigned>(std::min<long long>(rows, 16384))),
                         dim3(256), 0, s, W, na, v, a0, band);
      rc = hipGetLastError() == hipSuccess ? CC_LADDER_OK : CC_LADDER_EHIP;
      if (!rc)
        rc = launch_gemm<Tr, RC, RC, EPI_UNPACK>(lamP, ldp, t, v2, W, 0, static_cast<int>(ldp),
                                                 static_cast<int>(v2), o * o, v, drain, s, 0, a0,
                                                 nullptr, 1.0, 0, 0, static_cast<int>(npairs));
    } else {
      rc = launch_gemm<Tr, RC, RC, EPI_PERM>(lam + off, v2, t, v2, W, 0, na * v,
                                             static_cast<int>(v2), o * o, v, drain, s);
    }
    tr(CC_LADDER_PHASE_W, blk, 1);
    if (rc) return rc;
    tr(CC_LADDER_PHASE_DL, blk, 0);
    if (sym) {
      // Each dL term of W = Wh + Wh^T is the first term of Wh plus the second
      // of Wh, and the two terms of W are equal: dL += 2 (first + second), with
      // the K ranges cut to Wh's non-zero half (b >= a).
      // dL[x][a0*v + (ac)] += 2 L[x][(bd), b >= a] . Wh[(ac)][(bd)]
      rc = launch_gemm<Tr, KC, KC, EPI_ACC>(L, v2, W, v2, dL + off, v2, P, na * v,
                                            static_cast<int>(v2), v, drain, s, 0, a0, nullptr,
                                            2.0, 0, 1);
      // dL[x][(bd), b >= a0] += 2 L[x][a0*v + (ac), a <= b] . Wh[(ac)][(bd)]
      if (!rc)
        rc = launch_gemm<Tr, KC, RC, EPI_ACC>(L + off, v2, W + off, v2, dL + off, v2, P,
                                              static_cast<int>((long long)(v - a0) * v), na * v,
                                              v, drain, s, 0, a0, nullptr, 2.0, 0, 2);
    } else if (na == v) {
      // one block holds all of W' = [(ac)][(bd)]: the two terms are one product
      // with its symmetric part, dL[x][p] += sum_q L[x][q] (W'[p][q] + W'[q][p])
      rc = sym_add(W, v2, s);
      if (!rc)
        rc = launch_gemm<Tr, KC, KC, EPI_ACC>(L, v2, W, v2, dL, v2, P, static_cast<int>(v2),
                                              static_cast<int>(v2), v, drain, s);
    } else {
      // dL[x][a0*v + (ac)] += L[x][(bd)] . W'_A[(ac)][(bd)]
      rc = launch_gemm<Tr, KC, KC, EPI_ACC>(L, v2, W, v2, dL + off, v2, P, na * v,
                                            static_cast<int>(v2), v, drain, s);
      // dL[x][(bd)] += L[x][a0*v + (ac)] . W'_A[(ac)][(bd)]
      if (!rc)
        rc = launch_gemm<Tr, KC, RC, EPI_ACC>(L + off, v2, W, v2, dL, v2, P, static_cast<int>(v2),
                                              na * v, v, drain, s);
    }
    tr(CC_LADDER_PHASE_DL, blk, 1);
    if (rc) return rc;
  }
  if (sym) {
    // dt[i][j][c][d] += B[i][j][c][d] + B[j][i][d][c]
    tr(CC_LADDER_PHASE_DT, pl.nblocks, 0);
    const int rc = mirror_add(Bacc, dt, o, v, s);
    tr(CC_LADDER_PHASE_DT, pl.nblocks, 1);
    if (rc) return rc;
  }
  return CC_LADDER_OK;
}

// Occupied intermediates: Z[(ij)][(p, y)] += sum_(x,d) t[(ij)][(x,d)] G[(p,y)][(x,d)],
// G built per block of first indices p from rows (p, x) of Lrow ([P][n_first*v],
// leading dimension ld_row) and columns (y, d) of L_ov ([P][o*v]).
template <class Tr>
int intermediate_blocks(const Plan& pl, const typename Tr::T* Lrow, long long ld_row,
                        const typename Tr::T* Lov, const typename Tr::T* t, double* Z,
                        typename Tr::T* V, double* part, const Tracer& tr, hipStream_t s) {
  const int o = pl.o, v = pl.v, P = pl.P;
  const long long v2 = (long long)v * v;
  const int n_first = pl.op == kOpIjkl ? o : v;
  const long long ld_out = (long long)n_first * o;
  const int drain = Tr::kDrain ? pl.k_chunk / Tr::BK : 0;
  for (int p0 = 0, blk = 0; p0 < n_first; p0 += pl.n_a, ++blk) {
    const int np = (n_first - p0) < pl.n_a ? (n_first - p0) : pl.n_a;
    tr(CC_LADDER_PHASE_BUILD, blk, 0);
    int rc = launch_gemm<Tr, RC, RC, EPI_PERM>(Lrow + (long long)p0 * v, ld_row, Lov,
                                               (long long)o * v, V, 0, np * v, o * v, P, v, drain,
                                               s);
    tr(CC_LADDER_PHASE_BUILD, blk, 1);
    if (rc) return rc;
    tr(CC_LADDER_PHASE_CONTRACT, blk, 0);
    rc = launch_contract_split<Tr>(t, v2, V, v2, Z + (long long)p0 * o, ld_out, o * o, np * o,
                                   static_cast<int>(v2), pl.k_splits, part, drain, s);
    tr(CC_LADDER_PHASE_CONTRACT, blk, 1);
    if (rc) return rc;
  }
  return CC_LADDER_OK;
}

// Hole-hole ladder, per block of occupied i:
//   build    W[i][j][k][l] = sum_x L_oo[x][i][k] L_oo[x][j][l]    GEMM M=(i,k) N=(j,l) K=x
//   contract R[(i j)][(ab)] += sum_(kl) W[(ij)][(kl)] t[(kl)][(ab)]  GEMM M=(i,j) N=(a,b) K=(k,l)
template <class Tr>
int hole_blocks(const Plan& pl, const typename Tr::T* Loo, const typename Tr::T* t, double* R,
                typename Tr::T* W, const Tracer& tr, hipStream_t s) {
  const int o = pl.o, v = pl.v, P = pl.P;
  const long long o2 = (long long)o * o, v2 = (long long)v * v;
  const int drain = Tr::kDrain ? pl.k_chunk / Tr::BK : 0;
  for (int i0 = 0, blk = 0; i0 < o; i0 += pl.n_a, ++blk) {
    const int ni = (o - i0) < pl.n_a ? (o - i0) : pl.n_a;
    tr(CC_LADDER_PHASE_BUILD, blk, 0);
    int rc = launch_gemm<Tr, RC, RC, EPI_PERM>(Loo + (long long)i0 * o, o2, Loo, o2, W, 0, ni * o,
                                               static_cast<int>(o2), P, o, drain, s);
    tr(CC_LADDER_PHASE_BUILD, blk, 1);
    if (rc) return rc;
    tr(CC_LADDER_PHASE_CONTRACT, blk, 0);
    rc = launch_gemm<Tr, KC, RC, EPI_ACC>(W, o2, t, v2, R + (long long)i0 * o * v2, v2, ni * o,
                                          static_cast<int>(v2), static_cast<int>(o2), v, drain, s);
    tr(CC_LADDER_PHASE_CONTRACT, blk, 1);
    if (rc) return rc;
  }
  return CC_LADDER_OK;
}

// Shared body of the occupied-index terms: the two intermediates (Lrow is L_ov
// for ijkl, L for ijbk) and the hole-hole ladder (Lrow = Lov = L_oo, Z = R).
int intermediate_call(int which, int o, int v, int P, const double* Lrow, const double* Lov,
                      const double* t, double* Z, int precision, hipStream_t stream,
                      const cc_ladder_opts* opts) {
  int rc = check_dims(o, v, P);
  if (rc) return rc;
  rc = check_precision_opts(precision, opts);
  if (rc) return rc;
  if (!Lrow || !Lov || !t || !Z) return CC_LADDER_EINVAL;
  const bool ijkl = which == CC_INTERMEDIATE_IJKL;
  const bool hole = which == CC_HOLE_LADDER;
  const long long n_first = which == CC_INTERMEDIATE_IJBK ? v : o;
  const size_t nt = (size_t)o * o * v * v * sizeof(double);
  const size_t nov = (size_t)P * o * (hole ? o : v) * sizeof(double);
  const size_t nrow = hole ? nov : (size_t)P * n_first * v * sizeof(double);
  const size_t nz = hole ? nt : (size_t)o * o * n_first * o * sizeof(double);
  if (overlaps(Z, nz, t, nt) || overlaps(Z, nz, Lov, nov) || overlaps(Z, nz, Lrow, nrow))
    return CC_LADDER_EINVAL;
  if (precision == CC_LADDER_SPLIT_BF16 || precision == CC_LADDER_SPLIT_INT8 ||
      (opts && opts->flags))
    return CC_LADDER_EUNSUPPORTED;
  Plan pl;
  Scratch ws;
  if (opts && opts->workspace) {
    rc = make_plan_intermediate(which, o, v, P, precision, opts->workspace_bytes, opts, &pl);
    if (rc) return rc;
    const Operand ops[4] = {{Lrow, nrow}, {Lov, nov}, {t, nt}, {Z, nz}};
    rc = check_workspace(opts, pl.bytes, ops, 4);
    if (rc) return rc;
    rc = check_device();
    if (rc) return rc;
  } else {
    rc = check_device();
    if (rc) return rc;
    const size_t budget = (opts && opts->hbm_budget) ? opts->hbm_budget : default_budget();
    if (!budget) return CC_LADDER_EHIP;
    rc = make_plan_intermediate(which, o, v, P, precision, budget, opts, &pl);
    if (rc) return rc;
  }
  rc = take_scratch(pl, stream, opts, &ws);
  if (rc) return rc;
  char* base = ws.base;
  const Tracer tr(opts, stream);
  if (hole) {
    if (precision == CC_LADDER_FP64)
      return hole_blocks<TrF64>(pl, Lov, t, Z, reinterpret_cast<double*>(base + pl.off_V), tr,
                                stream);
    float* Loo32 = reinterpret_cast<float*>(base + pl.off_L);
    float* t32 = reinterpret_cast<float*>(base + pl.off_t);
    tr(CC_LADDER_PHASE_PREP, 0, 0);
    rc = to_f32(Lov, Loo32, (size_t)P * o * o, stream);
    if (!rc) rc = to_f32(t, t32, (size_t)o * o * v * v, stream);
    tr(CC_LADDER_PHASE_PREP, 0, 1);
    if (rc) return rc;
    return hole_blocks<TrF32>(pl, Loo32, t32, Z, reinterpret_cast<float*>(base + pl.off_V), tr,
                              stream);
  }
  const long long ld_row = n_first * v;
  double* part = pl.k_splits > 1 ? reinterpret_cast<double*>(base + pl.off_part) : nullptr;
  if (precision == CC_LADDER_FP64) {
    if (!ijkl) {
      double* tx = reinterpret_cast<double*>(base + pl.off_tx);
      tr(CC_LADDER_PHASE_PREP, 0, 0);
      rc = swap_cd(t, tx, o, v, stream);
      tr(CC_LADDER_PHASE_PREP, 0, 1);
      if (rc) return rc;
      t = tx;
    }
    return intermediate_blocks<TrF64>(pl, Lrow, ld_row, Lov, t, Z,
                                      reinterpret_cast<double*>(base + pl.off_V), part, tr, stream);
  }
  float* Lov32 = reinterpret_cast<float*>(base + pl.off_L);
  float* Lrow32 = ijkl ? Lov32 : reinterpret_cast<float*>(base + pl.off_L2);
  float* t32 = reinterpret_cast<float*>(base + pl.off_t);
  tr(CC_LADDER_PHASE_PREP, 0, 0);
  rc = to_f32(Lov, Lov32, (size_t)P * o * v, stream);
  if (!rc && !ijkl) rc = to_f32(Lrow, Lrow32, (size_t)P * v * v, stream);
  if (!rc) rc = ijkl ? to_f32(t, t32, (size_t)o * o * v * v, stream) : swap_cd(t, t32, o, v, stream);
  tr(CC_LADDER_PHASE_PREP, 0, 1);
  if (rc) return rc;
  return intermediate_blocks<TrF32>(pl, Lrow32, ld_row, Lov32, t32, Z,
                                    reinterpret_cast<float*>(base + pl.off_V), part, tr, stream);
}

}  // namespace
}  // namespace ccl

using namespace ccl;

namespace ccl {
namespace {

// The forward once its plan and scratch (`base`) are settled.
int residual_body(const Plan& pl, const double* L, const double* t, double* R, int precision,
                  char* base, const cc_ladder_opts* opts, hipStream_t stream) {
  const int o = pl.o, v = pl.v, P = pl.P;
  int rc;
  if (pl.check_sym) {
    unsigned long long* buf = reinterpret_cast<unsigned long long*>(base + pl.off_check);
    rc = check_pair_symmetric(t, o, v, buf, stream);
    if (!rc && opts && (opts->flags & CC_LADDER_SYMMETRIC_VECTORS))
      rc = check_vectors_symmetric(L, P, v, buf, stream);
    if (rc) return rc;
  }
  const Tracer tr(opts, stream);
  if (pl.pm) {
    // t+ and t- (the exchange partner's amplitudes give t+ and -t-), then the blocks
    const double sm = pl.exchange ? -1.0 : 1.0;
    const long long mp = (long long)o * (o + 1) / 2;
    tr(CC_LADDER_PHASE_PREP, 0, 0);
    if (precision == CC_LADDER_FP64) {
      double* Tp = reinterpret_cast<double*>(base + pl.off_Tp);
      double* Tm = reinterpret_cast<double*>(base + pl.off_Tm);
      double* Lp = pl.gsym ? reinterpret_cast<double*>(base + pl.off_Lp) : nullptr;
      rc = pm_rows<PM_AMPS>(t, mp, o, 0, v, Tp, pl.ldp, Tm, pl.ldm, 1.0, sm, stream);
      if (!rc && pl.gsym) rc = pack_sym(L, Lp, P, v, pl.ldg, stream);
      tr(CC_LADDER_PHASE_PREP, 0, 1);
      if (rc) return rc;
      return forward_blocks_pm<TrF64>(pl, L, Tp, Tm, R, reinterpret_cast<double*>(base + pl.off_V),
                                      reinterpret_cast<double*>(base + pl.off_Vp),
                                      reinterpret_cast<double*>(base + pl.off_Vm),
                                      reinterpret_cast<int*>(base + pl.off_tiles), tr, stream, Lp,
                                      pl.gsym ? reinterpret_cast<double*>(base + pl.off_G) : nullptr);
    }
    if (precision != CC_LADDER_FP32) return CC_LADDER_EUNSUPPORTED;
    float* Tp = reinterpret_cast<float*>(base + pl.off_Tp);
    float* Tm = reinterpret_cast<float*>(base + pl.off_Tm);
    float* L32 = pl.gsym ? nullptr : reinterpret_cast<float*>(base + pl.off_L);
    float* Lp = pl.gsym ? reinterpret_cast<float*>(base + pl.off_Lp) : nullptr;
    rc = pl.gsym ? pack_sym(L, Lp, P, v, pl.ldg, stream) : to_f32(L, L32, (size_t)P * v * v, stream);
    if (!rc) rc = pm_rows<PM_AMPS>(t, mp, o, 0, v, Tp, pl.ldp, Tm, pl.ldm, 1.0, sm, stream);
    tr(CC_LADDER_PHASE_PREP, 0, 1);
    if (rc) return rc;
    return forward_blocks_pm<TrF32>(pl, L32, Tp, Tm, R, reinterpret_cast<float*>(base + pl.off_V),
                                    reinterpret_cast<float*>(base + pl.off_Vp),
                                    reinterpret_cast<float*>(base + pl.off_Vm),
                                    reinterpret_cast<int*>(base + pl.off_tiles), tr, stream, Lp,
                                    pl.gsym ? reinterpret_cast<float*>(base + pl.off_G) : nullptr);
  }
  if (pl.exchange && precision != CC_LADDER_FP32) {
    // the exchange partner is the ladder of the swapped amplitudes
    double* tx = reinterpret_cast<double*>(base + pl.off_tx);
    tr(CC_LADDER_PHASE_PREP, 0, 0);
    rc = swap_cd(t, tx, o, v, stream);
    tr(CC_LADDER_PHASE_PREP, 0, 1);
    if (rc) return rc;
    t = tx;
  }
  switch (precision) {
    case CC_LADDER_FP64: {
      double* Lp = pl.gsym ? reinterpret_cast<double*>(base + pl.off_Lp) : nullptr;
      if (pl.gsym) {
        tr(CC_LADDER_PHASE_PREP, 0, 0);
        rc = pack_sym(L, Lp, P, v, pl.ldg, stream);
        tr(CC_LADDER_PHASE_PREP, 0, 1);
        if (rc) return rc;
      }
      return forward_blocks<TrF64>(pl, L, t, R, reinterpret_cast<double*>(base + pl.off_V),
                                   reinterpret_cast<int*>(base + pl.off_tiles), tr, stream, Lp,
                                   pl.gsym ? reinterpret_cast<double*>(base + pl.off_G) : nullptr);
    }
    case CC_LADDER_FP32: {
      // (with symmetric vectors the build reads only the packed float32 vectors)
      float* L32 = pl.gsym ? nullptr : reinterpret_cast<float*>(base + pl.off_L);
      float* t32 = reinterpret_cast<float*>(base + pl.off_t);
      float* Lp = pl.gsym ? reinterpret_cast<float*>(base + pl.off_Lp) : nullptr;
      tr(CC_LADDER_PHASE_PREP, 0, 0);
      rc = pl.gsym ? pack_sym(L, Lp, P, v, pl.ldg, stream) : to_f32(L, L32, (size_t)P * v * v, stream);
      if (!rc)
        rc = pl.exchange ? swap_cd(t, t32, o, v, stream) : to_f32(t, t32, (size_t)o * o * v * v, stream);
      tr(CC_LADDER_PHASE_PREP, 0, 1);
      if (rc) return rc;
      return forward_blocks<TrF32>(pl, L32, t32, R, reinterpret_cast<float*>(base + pl.off_V),
                                   reinterpret_cast<int*>(base + pl.off_tiles), tr, stream, Lp,
                                   pl.gsym ? reinterpret_cast<float*>(base + pl.off_G) : nullptr);
    }
    case CC_LADDER_SPLIT_BF16:
      return split_forward(pl, L, t, R, base, tr, stream);
    case CC_LADDER_SPLIT_INT8:
      return split_i8_forward(pl, L, t, R, base, tr, stream);
    default:
      return CC_LADDER_EINVAL;
  }
}

}  // namespace

int pack_pair_vectors(const double* L, double* Lp, int P, int v, long long ldg, hipStream_t s) {
  return pack_sym(L, Lp, P, v, ldg, s);
}

int gather_pair_rows(const double* G, long long ldg, long long nrows, int a0, int v, double* rows,
                     hipStream_t s) {
  return pm_gather<GATHER_ROWS>(G, ldg, nrows, a0, v, rows, (long long)v * v,
                                static_cast<double*>(nullptr), 0, s);
}

int ladder_forward_planned(const Plan& pl, const double* L, const double* t, double* R,
                           int precision, char* base, const cc_ladder_opts* opts,
                           hipStream_t stream) {
  return residual_body(pl, L, t, R, precision, base, opts, stream);
}

int device_ok() { return check_device(); }

}  // namespace ccl

extern "C" int cc_ladder_residual(int o, int v, int P, const double* L, const double* t,
                                  double* R, int precision, hipStream_t stream,
                                  const cc_ladder_opts* opts) {
  Operand ops[3];
  int rc = check_residual_args(o, v, P, L, t, R, precision, opts, ops);
  if (rc) return rc;
  Plan pl;
  Scratch ws;
  rc = plan_and_scratch(o, v, P, precision, 0, stream, opts, ops, 3, &pl, &ws);
  if (rc) return rc;
  return residual_body(pl, L, t, R, precision, ws.base, opts, stream);
}

namespace ccl {
namespace {

// Scratch of cc_ladder_residual_noalloc.  Each device holds its own copy of
// this array from the library's load until the process ends.  In host code the
// name is a host-side stand-in, never a device address: the device address
// comes from hipGetSymbolAddress, once per device, and only that pointer is
// handed to kernels.
static __device__ __align__(256) unsigned char scratch[CC_LADDER_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
char* g_scratch_ptr[64];  // device address of `scratch` per device, null until looked up

// The current device's copy of `scratch` (looked up on its first use there).
int noalloc_scratch(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return CC_LADDER_ENODEV;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return CC_LADDER_EHIP;
    }
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return CC_LADDER_OK;
}

}  // namespace
}  // namespace ccl

extern "C" int cc_ladder_residual_noalloc(int o, int v, int P, const double* L, const double* t,
                                          double* R, int precision, hipStream_t stream,
                                          const cc_ladder_opts* opts) {
  Operand ops[3];
  int rc = check_residual_args(o, v, P, L, t, R, precision, opts, ops);
  if (rc) return rc;
  // the scratch is the static array: no caller workspace, and no flag whose
  // work reads a result back to the host
  if (opts && (opts->workspace || opts->workspace_bytes ||
               (opts->flags & CC_LADDER_CHECK_SYMMETRY)))
    return CC_LADDER_EINVAL;
  const size_t cap = CC_LADDER_NOALLOC_SCRATCH_BYTES;
  const size_t budget = (opts && opts->hbm_budget && opts->hbm_budget < cap) ? opts->hbm_budget : cap;
  Plan pl;
  rc = make_plan(o, v, P, precision, 0, budget, opts, &pl);
  if (rc) return rc;
  if (pl.bytes > cap) return CC_LADDER_ENOMEM;
  rc = check_device();
  if (rc) return rc;
  char* base = nullptr;
  rc = noalloc_scratch(&base);
  if (rc) return rc;
  return residual_body(pl, L, t, R, precision, base, opts, stream);
}

extern "C" int cc_ladder_backward(int o, int v, int P, const double* L, const double* t,
                                  const double* lam, double* dL, double* dt, int precision,
                                  hipStream_t stream, const cc_ladder_opts* opts) {
  Operand ops[5];
  int rc = check_backward_args(o, v, P, L, t, lam, dL, dt, precision, opts, ops);
  if (rc) return rc;
  if (precision == CC_LADDER_SPLIT_BF16 || precision == CC_LADDER_SPLIT_INT8)
    return CC_LADDER_EUNSUPPORTED;
  Plan pl;
  Scratch ws;
  rc = plan_and_scratch(o, v, P, precision, 1, stream, opts, ops, 5, &pl, &ws);
  if (rc) return rc;
  char* base = ws.base;
  if (pl.check_sym) {
    unsigned long long* buf = reinterpret_cast<unsigned long long*>(base + pl.off_check);
    rc = check_pair_symmetric(t, o, v, buf, stream);
    if (!rc) rc = check_pair_symmetric(lam, o, v, buf, stream);
    if (!rc && opts && (opts->flags & CC_LADDER_SYMMETRIC_VECTORS))
      rc = check_vectors_symmetric(L, P, v, buf, stream);
    if (rc) return rc;
  }
  const Tracer tr(opts, stream);
  // exchange: gradients of the ladder at the swapped amplitudes; dt is
  // accumulated in swapped order in scratch and swapped back at the end
  double* dtx = pl.exchange ? reinterpret_cast<double*>(base + pl.off_dtx) : dt;
  if (pl.exchange) {
    tr(CC_LADDER_PHASE_PREP, 0, 0);
    rc = swap_cd(dt, dtx, o, v, stream);
    if (!rc && precision == CC_LADDER_FP64) {
      rc = swap_cd(t, reinterpret_cast<double*>(base + pl.off_tx), o, v, stream);
      t = reinterpret_cast<const double*>(base + pl.off_tx);
    }
    tr(CC_LADDER_PHASE_PREP, 0, 1);
    if (rc) return rc;
  }
  if (precision == CC_LADDER_FP64) {
    double* Lp = pl.gsym ? reinterpret_cast<double*>(base + pl.off_Lp) : nullptr;
    if (pl.gsym) {
      tr(CC_LADDER_PHASE_PREP, 0, 0);
      rc = pack_sym(L, Lp, P, v, pl.ldg, stream);
      tr(CC_LADDER_PHASE_PREP, 0, 1);
      if (rc) return rc;
    }
    rc = backward_blocks<TrF64>(pl, L, t, lam, dL, dtx, base, tr, stream, Lp,
                                pl.gsym ? reinterpret_cast<double*>(base + pl.off_G) : nullptr);
  } else {
    float* L32 = reinterpret_cast<float*>(base + pl.off_L);
    float* t32 = reinterpret_cast<float*>(base + pl.off_t);
    float* lam32 = reinterpret_cast<float*>(base + pl.off_lam);
    float* Lp = pl.gsym ? reinterpret_cast<float*>(base + pl.off_Lp) : nullptr;
    tr(CC_LADDER_PHASE_PREP, 0, 0);
    rc = to_f32(L, L32, (size_t)P * v * v, stream);
    if (!rc)
      rc = pl.exchange ? swap_cd(t, t32, o, v, stream) : to_f32(t, t32, (size_t)o * o * v * v, stream);
    if (!rc) rc = to_f32(lam, lam32, (size_t)o * o * v * v, stream);
    if (!rc && pl.gsym) rc = pack_sym(L, Lp, P, v, pl.ldg, stream);
    tr(CC_LADDER_PHASE_PREP, 0, 1);
    if (rc) return rc;
    rc = backward_blocks<TrF32>(pl, L32, t32, lam32, dL, dtx, base, tr, stream, Lp,
                                pl.gsym ? reinterpret_cast<float*>(base + pl.off_G) : nullptr);
  }
  if (rc || !pl.exchange) return rc;
  tr(CC_LADDER_PHASE_PREP, 1, 0);
  rc = swap_cd(dtx, dt, o, v, stream);
  tr(CC_LADDER_PHASE_PREP, 1, 1);
  return rc;
}

extern "C" int cc_ladder_reduce(int o, int v, const double* x, const double* y, double* out_dev,
                                hipStream_t stream) {
  if (o <= 0 || v <= 0 || o > 46340 || v > 46340) return CC_LADDER_EINVAL;
  if (!x || !y || !out_dev) return CC_LADDER_EINVAL;
  const long long n = (long long)o * o * v * v;
  if (overlaps(out_dev, 2 * sizeof(double), x, n * sizeof(double)) ||
      overlaps(out_dev, 2 * sizeof(double), y, n * sizeof(double)))
    return CC_LADDER_EINVAL;
  int rc = check_device();
  if (rc) return rc;
  const long long want = (n + 255) / 256;
  const int nb = static_cast<int>(want < kRedBlocks ? want : kRedBlocks);
  void* part = nullptr;
  if (hipMallocAsync(&part, 2 * sizeof(double) * nb, stream) != hipSuccess) {
    (void)hipGetLastError();
    return CC_LADDER_ENOMEM;
  }
  hipLaunchKernelGGL(reduce_partial_kernel, dim3(nb), dim3(256), 0, stream, x, y, n,
                     static_cast<double*>(part));
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, stream,
                     static_cast<const double*>(part), nb, out_dev);
  const bool ok = hipGetLastError() == hipSuccess;
  (void)hipFreeAsync(part, stream);
  return ok ? CC_LADDER_OK : CC_LADDER_EHIP;
}

extern "C" int cc_ladder_workspace_query(int o, int v, int P, int precision, int backward,
                                         size_t hbm_budget, const cc_ladder_opts* opts,
                                         size_t* bytes, int* a_block) {
  if (!bytes || !a_block) return CC_LADDER_EINVAL;
  Plan pl;
  const int rc = make_plan(o, v, P, precision, backward, hbm_budget, opts, &pl);
  if (rc) return rc;
  *bytes = pl.bytes;
  *a_block = pl.n_a;
  return CC_LADDER_OK;
}

extern "C" int cc_intermediate_ijkl(int o, int v, int P, const double* L_ov, const double* t,
                                    double* X, int precision, hipStream_t stream,
                                    const cc_ladder_opts* opts) {
  return intermediate_call(CC_INTERMEDIATE_IJKL, o, v, P, L_ov, L_ov, t, X, precision, stream,
                           opts);
}

extern "C" int cc_intermediate_ijbk(int o, int v, int P, const double* L, const double* L_ov,
                                    const double* t, double* Y, int precision, hipStream_t stream,
                                    const cc_ladder_opts* opts) {
  return intermediate_call(CC_INTERMEDIATE_IJBK, o, v, P, L, L_ov, t, Y, precision, stream, opts);
}

extern "C" int cc_hole_ladder(int o, int v, int P, const double* L_oo, const double* t, double* R,
                              int precision, hipStream_t stream, const cc_ladder_opts* opts) {
  return intermediate_call(CC_HOLE_LADDER, o, v, P, L_oo, L_oo, t, R, precision, stream, opts);
}

extern "C" int cc_intermediate_workspace_query(int which, int o, int v, int P, int precision,
                                               size_t hbm_budget, const cc_ladder_opts* opts,
                                               size_t* bytes, int* block) {
  if (!bytes || !block) return CC_LADDER_EINVAL;
  Plan pl;
  const int rc = make_plan_intermediate(which, o, v, P, precision, hbm_budget, opts, &pl);
  if (rc) return rc;
  *bytes = pl.bytes;
  *block = pl.n_a;
  return CC_LADDER_OK;
}

extern "C" const char* cc_ladder_strerror(int code) {
  switch (code) {
    case CC_LADDER_OK: return "success";
    case CC_LADDER_EINVAL: return "invalid argument (dimension, pointer, aliasing, precision or option)";
    case CC_LADDER_ENOMEM: return "scratch does not fit the budget or the workspace";
    case CC_LADDER_ENODEV: return "no gfx950 device is current";
    case CC_LADDER_EHIP: return "HIP runtime error";
    case CC_LADDER_EUNSUPPORTED: return "request not supported by the library";
    default: return "unknown error code";
  }
}
