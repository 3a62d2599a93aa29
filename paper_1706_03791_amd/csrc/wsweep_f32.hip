// Wave-tiled sweep variants for element type float (3-D fields, one layer).
#include "sweep_launch.hpp"

namespace szh {
hipError_t wsweep_f32(bool comp, int cw, const WArgs& a, int grid, hipStream_t st) {
  return launch_wsweep_t<float>(comp, cw, a, grid, st);
}
}  // namespace szh
