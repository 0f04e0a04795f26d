// Split-precision product (INT8 slices on the matrix cores); see split.h.
#include "split.h"

namespace rfk {

int split_init(SplitPlan& sp, const refine_matrix&, int, int, const Prob&, Prob*, hipStream_t) {
  sp = SplitPlan();
  return REFINE_EINVAL;
}

hipError_t split_product(SplitPlan&, const Prob*, hipStream_t) { return hipErrorNotSupported; }

void split_free(SplitPlan& sp) { sp = SplitPlan(); }

}  // namespace rfk
