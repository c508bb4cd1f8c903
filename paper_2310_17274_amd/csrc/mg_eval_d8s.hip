// Evaluation kernel instantiations: chain depth 8, serial chain = true.
#include "mg_eval.h"

namespace mg {
hipError_t launch_eval_d8s(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s) {
  return launch_eval_shape<8, true>(a, grid_x, cand, grad, s);
}
}  // namespace mg
