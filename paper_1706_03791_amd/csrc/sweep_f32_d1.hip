// Sweep kernel variants for element type float, 1-D fields.
#include "sweep_launch.hpp"

namespace szh {
hipError_t sweep_f32_d1(int nl, bool comp, int cw, const SweepArgs& a, int grid, hipStream_t st) {
  return launch_sweep_t<float, 1>(nl, comp, cw, a, grid, st);
}
}  // namespace szh
