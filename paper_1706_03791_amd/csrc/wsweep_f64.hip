// Wave-tiled sweep variants for element type double (3-D fields, one layer).
#include "sweep_launch.hpp"

namespace szh {
hipError_t wsweep_f64(bool comp, int cw, const WArgs& a, int grid, hipStream_t st) {
  return launch_wsweep_t<double>(comp, cw, a, grid, st);
}
}  // namespace szh
