// Evaluation kernel instantiations: chain depth 16, serial chain = true.
#include "mg_eval.h"

namespace mg {
hipError_t launch_eval_d16s(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s) {
  return launch_eval_shape<16, true>(a, grid_x, cand, grad, s);
}
}  // namespace mg
