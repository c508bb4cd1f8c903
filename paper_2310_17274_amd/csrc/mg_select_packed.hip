// select_kernel instantiations with several seeds per wavefront (PL = 1,
// W = 8, 16 or 32 lanes per seed): row blocks of at most 32 floats, where
// one wavefront per seed would leave most of its lanes idle.
#include "mg_solver.h"

namespace mg {
namespace {
template <int KP, int W>
hipError_t launch_select_w(const SelectArgs& a, const LbfgsArgs* la, hipStream_t s) {
  constexpr int spw = kWave / W;
  const dim3 grid((a.n_seeds + spw - 1) / spw);
  if (!la) select_kernel<1, 4, false, KP, false, W><<<grid, kWave, 0, s>>>(a, LbfgsArgs{});
  else if (la->m <= 4) select_kernel<1, 4, true, KP, false, W><<<grid, kWave, 0, s>>>(a, *la);
  else select_kernel<1, kMaxHist, true, KP, false, W><<<grid, kWave, 0, s>>>(a, *la);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_select_packed(const SelectArgs& a, int max_n, const LbfgsArgs* la, hipStream_t s) {
  if (a.K < 1 || a.K > kMaxK || max_n > 32 || a.n_seeds < 1) return hipErrorInvalidValue;
  // the narrowest group that holds the block and one lane per candidate
  const int need = max_n > a.K ? max_n : a.K;
  if (need <= 8) return a.K <= 4 ? launch_select_w<4, 8>(a, la, s) : launch_select_w<8, 8>(a, la, s);
  if (need <= 16) {
    if (a.K <= 4) return launch_select_w<4, 16>(a, la, s);
    if (a.K <= 8) return launch_select_w<8, 16>(a, la, s);
    return launch_select_w<16, 16>(a, la, s);
  }
  if (a.K <= 4) return launch_select_w<4, 32>(a, la, s);
  if (a.K <= 8) return launch_select_w<8, 32>(a, la, s);
  return launch_select_w<16, 32>(a, la, s);
}
}  // namespace mg
