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

// Contracted indices per exponent of the contraction's digit rows (one exact
// float32 chunk of the slice-pair GEMM).
constexpr int kExpChunk = 128;
inline int exp_chunks(int k_pad) { return (k_pad + kExpChunk - 1) / kExpChunk; }

inline SliceDims slice_dims(long long rows, int K) {
  SliceDims d;
  d.rows_pad = static_cast<int>((rows + 127) / 128 * 128 + 128);
  d.k_pad = (K + 63) / 64 * 64;
  return d;
}

int split_forward(const Plan& pl, const double* L, const double* t, double* R, char* ws,
                  const Tracer& tr, hipStream_t stream);

}  // namespace ccl
