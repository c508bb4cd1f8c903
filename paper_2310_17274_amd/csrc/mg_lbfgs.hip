// Standalone L-BFGS kernel instantiations and the select launcher's choice
// of its instantiation unit.
#include "mg_solver.h"

namespace mg {
namespace {
template <int MH>
hipError_t launch_lbfgs_h(const LbfgsArgs& a, int max_n, hipStream_t s) {
  const dim3 grid(a.n_seeds);
  const bool v4 = rows_v4(a.uniform_T, a.dof) && (a.rows * a.dof) % 4 == 0 && aligned16(a.x) && aligned16(a.g) &&
                  aligned16(a.S) && aligned16(a.Y) && aligned16(a.x_prev) && aligned16(a.g_prev) && aligned16(a.dir);
  if (max_n <= 64) lbfgs_kernel<1, MH, false><<<grid, kWave, 0, s>>>(a);
  else if (max_n <= 128) lbfgs_kernel<2, MH, false><<<grid, kWave, 0, s>>>(a);
  else if (max_n <= 256 && v4) lbfgs_kernel<4, MH, true><<<grid, kWave, 0, s>>>(a);
  else if (max_n <= 256) lbfgs_kernel<4, MH, false><<<grid, kWave, 0, s>>>(a);
  else if (max_n <= 512 && v4) lbfgs_kernel<8, MH, true><<<grid, kWave, 0, s>>>(a);
  else if (max_n <= 512) lbfgs_kernel<8, MH, false><<<grid, kWave, 0, s>>>(a);
  else if (v4) lbfgs_kernel<16, MH, true><<<grid, kWave, 0, s>>>(a);
  else lbfgs_kernel<16, MH, false><<<grid, kWave, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lbfgs(const LbfgsArgs& a, int max_n, hipStream_t s) {
  if (a.m <= 4) return launch_lbfgs_h<4>(a, max_n, s);
  return launch_lbfgs_h<kMaxHist>(a, max_n, s);
}
hipError_t launch_select(const SelectArgs& a, int max_n, const LbfgsArgs* fuse, hipStream_t s) {
  if (max_n <= 32) return launch_select_packed(a, max_n, fuse, s);
  if (max_n <= 64) return launch_select_p1(a, fuse, s);
  if (max_n <= 128) return launch_select_p2(a, fuse, s);
  if (max_n <= 256) return launch_select_p4(a, fuse, s);
  if (max_n <= 512) return launch_select_p8(a, fuse, s);
  return launch_select_p16(a, fuse, s);
}

}  // namespace mg
