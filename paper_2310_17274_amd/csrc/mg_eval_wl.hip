// Evaluation kernel, wave-per-link layout: choice of the instantiation.
#include "mg_eval_wl.h"

namespace mg {
hipError_t launch_eval_wl(const EvalArgs& a, int grid_x, int slices, bool cand, bool grad, hipStream_t s,
                          const SelFuse* fs) {
  // sphere slots per lane: all of a link's, half with two waves per link
  // or two slot groups per wave, a quarter with four slot groups
  const int per = a.wl.groups == 4 ? a.wl.maxs / 4
                  : (a.wl.halves == 2 || a.wl.groups == 2) ? a.wl.maxs / 2 : a.wl.maxs;
  if (a.wl.groups == 4) {
    if (per == 2) return launch_eval_wl_s2g4(a, grid_x, slices, cand, grad, s, fs);
    if (per == 4) return launch_eval_wl_s4g4(a, grid_x, slices, cand, grad, s, fs);
    return hipErrorInvalidValue;
  }
  if (a.wl.groups == 2) {
    if (per == 2) return launch_eval_wl_s2g2(a, grid_x, slices, cand, grad, s, fs);
    if (per == 4) return launch_eval_wl_s4g2(a, grid_x, slices, cand, grad, s, fs);
    if (per == 8) return launch_eval_wl_s8g2(a, grid_x, slices, cand, grad, s, fs);
    return hipErrorInvalidValue;
  }
  if (a.wl.groups != 1) return hipErrorInvalidValue;
  if (per == 2) return launch_eval_wl_s2g1(a, grid_x, slices, cand, grad, s, fs);
  if (per == 4) return launch_eval_wl_s4g1(a, grid_x, slices, cand, grad, s, fs);
  if (per == 8) return launch_eval_wl_s8g1(a, grid_x, slices, cand, grad, s, fs);
  if (per == 16) return launch_eval_wl_s16g1(a, grid_x, slices, cand, grad, s, fs);
  return hipErrorInvalidValue;
}
}  // namespace mg
