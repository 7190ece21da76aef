// Split-bf16 form of the ladder forward (operands cut into exponent-aligned
// bf16 slices; slice products on bf16 MFMA).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace ccl {

int split_forward(const Plan& pl, const double* L, const double* t, double* R, char* ws,
                  const Tracer& tr, hipStream_t stream);

}  // namespace ccl
