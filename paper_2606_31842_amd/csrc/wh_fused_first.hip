// Instantiations of the temporally blocked 2D kernel for the first launch of a wave solve.
#include "wh_fused_kernel.h"

namespace wh {

void launch_fused2d_first(bool f32, int k, int shape, bool varc, bool force, FusedDev& d, hipStream_t s) {
  launch_fused2d_phase<kPhaseFirst>(f32, k, shape, varc, force, d, s);
}

}  // namespace wh
