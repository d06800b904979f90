// mtvd_3d.hip -- 3D sweep kernels (placeholder until the 3D kernels land).
#include "mtvd_launch.h"

namespace mtvd {

hipError_t launch_sweep_3d(int, const Coef&, Shared*, const double*, int, int, bool,
                           const double*, double*, int, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace mtvd
