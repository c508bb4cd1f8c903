// Evaluation kernel instantiations, wave-per-link layout: 4 sphere slots per
// lane, 4 slot groups per wave.
#include "mg_eval_wl.h"

namespace mg {
MG_WL_LAUNCHER(4, 4) { return launch_eval_wl_g<4, 4>(a, grid_x, slices, cand, grad, s, fs); }
}  // namespace mg
