// mtvd_launch.h -- host-side launchers of the sweep kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "mtvd_device.h"

namespace mtvd {

// one directional operator L_axis(tau) in 2D (axis 0 = x, 2 = z)
hipError_t launch_sweep_2d(int axis, const Coef& c, Shared* sh, const double* zr, int slot,
                           int first, bool fuse, const double* X, double* Y, int kc,
                           hipStream_t s);
int strips_2d(int nx);

// one directional operator L_axis(tau) in 3D (axis 0 = x, 1 = y, 2 = z)
hipError_t launch_sweep_3d(int axis, const Coef& c, Shared* sh, const double* zr, int slot,
                           int first, bool fuse, const double* X, double* Y, int kc,
                           hipStream_t s);

}  // namespace mtvd
