// select_kernel instantiations for PL = 16 vector elements per lane with the
// fused L-BFGS step over up to 16 history pairs.
#include "mg_solver.h"

namespace mg {
hipError_t launch_select_p16_long(const SelectArgs& a, const LbfgsArgs& la, int KP, bool V4, hipStream_t s) {
  const dim3 grid(a.n_seeds);
  if (V4) {
    if (KP == 4) select_kernel<16, kMaxHist, true, 4, true><<<grid, kWave, 0, s>>>(a, la);
    else if (KP == 8) select_kernel<16, kMaxHist, true, 8, true><<<grid, kWave, 0, s>>>(a, la);
    else select_kernel<16, kMaxHist, true, 16, true><<<grid, kWave, 0, s>>>(a, la);
  } else {
    if (KP == 4) select_kernel<16, kMaxHist, true, 4, false><<<grid, kWave, 0, s>>>(a, la);
    else if (KP == 8) select_kernel<16, kMaxHist, true, 8, false><<<grid, kWave, 0, s>>>(a, la);
    else select_kernel<16, kMaxHist, true, 16, false><<<grid, kWave, 0, s>>>(a, la);
  }
  return hipGetLastError();
}
}  // namespace mg
