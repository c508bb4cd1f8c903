// select_kernel instantiations for PL = 2 vector elements per lane.
#include "mg_solver.h"

namespace mg {
namespace {
template <int PL, int KP, bool V4>
hipError_t launch_select_k(const SelectArgs& a, const LbfgsArgs* la, hipStream_t s) {
  const dim3 grid(a.n_seeds);
  if (!la) select_kernel<PL, 4, false, KP, V4><<<grid, kWave, 0, s>>>(a, LbfgsArgs{});
  else if (la->m <= 4) select_kernel<PL, 4, true, KP, V4><<<grid, kWave, 0, s>>>(a, *la);
  else select_kernel<PL, kMaxHist, true, KP, V4><<<grid, kWave, 0, s>>>(a, *la);
  return hipGetLastError();
}

bool select_v4(const SelectArgs& a, const LbfgsArgs* la) {
  bool ok = rows_v4(a.uniform_T, a.dof) && aligned16(a.x) && aligned16(a.d) && aligned16(a.g0) &&
            aligned16(a.x_out) && aligned16(a.g_out) && aligned16(a.best_x) && aligned16(a.grad_e);
  if (la)
    ok = ok && aligned16(la->S) && aligned16(la->Y) && aligned16(la->x_prev) && aligned16(la->g_prev) &&
         aligned16(la->dir) && (la->rows * la->dof) % 4 == 0;
  return ok;
}

template <int PL>
hipError_t launch_select_pl(const SelectArgs& a, const LbfgsArgs* la, hipStream_t s) {
  if (a.K < 1 || a.K > kMaxK) return hipErrorInvalidValue;
  if constexpr (PL >= 4) {
    if (select_v4(a, la)) {
      if (a.K <= 4) return launch_select_k<PL, 4, true>(a, la, s);
      if (a.K <= 8) return launch_select_k<PL, 8, true>(a, la, s);
      return launch_select_k<PL, 16, true>(a, la, s);
    }
  }
  if (a.K <= 4) return launch_select_k<PL, 4, false>(a, la, s);
  if (a.K <= 8) return launch_select_k<PL, 8, false>(a, la, s);
  return launch_select_k<PL, 16, false>(a, la, s);
}

}  // namespace

hipError_t launch_select_p2(const SelectArgs& a, const LbfgsArgs* la, hipStream_t s) {
  return launch_select_pl<2>(a, la, s);
}
}  // namespace mg
