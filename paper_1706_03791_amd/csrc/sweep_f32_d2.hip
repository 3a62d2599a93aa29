// Sweep kernel variants for element type float, 2-D fields.
#include "sweep_launch.hpp"

namespace szh {
hipError_t sweep_f32_d2(int nl, bool comp, int cw, const SweepArgs& a, int grid, hipStream_t st) {
  return launch_sweep_t<float, 2>(nl, comp, cw, a, grid, st);
}
}  // namespace szh
