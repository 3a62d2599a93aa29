// Sweep kernel variants for element type double, 1-D fields.
#include "sweep_launch.hpp"

namespace szh {
hipError_t sweep_f64_d1(int nl, bool comp, int cw, const SweepArgs& a, int grid, hipStream_t st) {
  return launch_sweep_t<double, 1>(nl, comp, cw, a, grid, st);
}
}  // namespace szh
