// Wave-tiled sweep variants for element type float (2-D and 3-D fields, one layer).
#include "sweep_launch.hpp"

namespace szh {
hipError_t wsweep_f32(bool comp, int cw, int nw, int az, const WArgs& a, int grid, hipStream_t st) {
  return launch_wsweep_t<float>(comp, cw, nw, az, a, grid, st);
}
}  // namespace szh
