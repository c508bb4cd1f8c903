// Evaluation kernel instantiations: 8 lanes per evaluation, 4 sphere slots per link.
#include "mg_eval.h"

namespace mg {
hipError_t launch_eval_l8s4(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s) {
  return launch_eval_shape<8, 4>(a, grid_x, cand, grad, s);
}
}  // namespace mg
