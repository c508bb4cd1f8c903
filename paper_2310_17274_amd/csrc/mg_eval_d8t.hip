// Evaluation kernel instantiations: chain depth 8, serial chain = false.
#include "mg_eval.h"

namespace mg {
hipError_t launch_eval_d8t(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s) {
  return launch_eval_shape<8, false>(a, grid_x, cand, grad, s);
}
}  // namespace mg
