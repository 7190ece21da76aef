// Split-bf16 form of the ladder forward (operands cut into exponent-aligned
// bf16 slices; slice products on bf16 MFMA).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace ccl {

// Geometry of a digit buffer [rows_pad][k_pad / 32][S][32] (the S slices of a
// row's 32-deep K-step adjacent): rows padded so that every workgroup tile of a
// product stays inside it, the contracted index to whole 32-deep MFMA steps
// (zero digits in the padding).
struct SliceDims {
  int rows_pad;
  int k_pad;
};

// Contracted indices per exponent of the contraction's digit rows, which is
// also the length of one float32 chunk of the slice-pair GEMM: 256 for four
// slices and the hi/lo split, whose exact groups (the leading two
// anti-diagonals, partial sums of at most 256 * 2^16 = 2^24) stay exact over
// 256 indices; 128 for three slices, whose third anti-diagonal would not.
constexpr int exp_chunk_len(int slices) { return slices == 3 ? 128 : 256; }
inline int exp_chunks(int k_pad, int slices) {
  return (k_pad + exp_chunk_len(slices) - 1) / exp_chunk_len(slices);
}

// Contracted indices per exponent and per exact int32 chunk of the split-int8
// form (a group of at most 5 products of int8 digits stays below
// 5 * 2^14 * 16384 < 2^31).
constexpr int kI8Chunk = 16384;
inline int i8_chunks(int k_pad) { return k_pad > 0 ? (k_pad + kI8Chunk - 1) / kI8Chunk : 1; }

inline SliceDims slice_dims(long long rows, int K) {
  SliceDims d;
  d.rows_pad = static_cast<int>((rows + 127) / 128 * 128 + 128);
  d.k_pad = (K + 63) / 64 * 64;
  return d;
}

// Symmetric vectors (defined with the float64 path): Lp[x][pair(a,c)] =
// L[x][a][c] for a <= c (row stride ldg, pads zero), and the block's packed
// rows X_ab[c][d] = G[{a,c}][{b,d}] (a <= b, a from a0; row stride v^2)
// gathered from the whole pair-pair integral G (row stride ldg).
int pack_pair_vectors(const double* L, double* Lp, int P, int v, long long ldg, hipStream_t s);
int gather_pair_rows(const double* G, long long ldg, long long nrows, int a0, int v, double* rows,
                     hipStream_t s);

int split_forward(const Plan& pl, const double* L, const double* t, double* R, char* ws,
                  const Tracer& tr, hipStream_t stream);
int split_i8_forward(const Plan& pl, const double* L, const double* t, double* R, char* ws,
                     const Tracer& tr, hipStream_t stream);

}  // namespace ccl
