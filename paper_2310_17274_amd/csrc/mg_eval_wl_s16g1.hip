// Evaluation kernel instantiations, wave-per-link layout: 16 sphere slots per
// lane, 1 slot group per wave.
#include "mg_eval_wl.h"

namespace mg {
MG_WL_LAUNCHER(16, 1) { return launch_eval_wl_g<16, 1>(a, grid_x, slices, cand, grad, s, fs); }
}  // namespace mg
