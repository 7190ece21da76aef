// Split-bf16 form: not built yet.
#include "split.hpp"

namespace ccl {

int split_forward(const Plan&, const double*, const double*, double*, char*, const Tracer&,
                  hipStream_t) {
  return CC_LADDER_EUNSUPPORTED;
}

}  // namespace ccl
