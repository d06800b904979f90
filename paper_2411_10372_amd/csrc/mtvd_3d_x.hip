// mtvd_3d_x.hip -- L_x in 3D (flux across lanes, march z, waves along y)
// and the per-axis dispatch of the 3D operators.
#include "mtvd_3d.h"

namespace mtvd {

hipError_t launch_sweep_3d_x(const Coef& c, Shared* sh, const double* zr, int slot, int first,
                             int fo, const double* X, double* Y, int kc, hipStream_t s) {
  const int nstrips = strips_3d(c.nx);
  const int nbb = (c.ny + kPer - 1) / kPer;
  const int nch = (c.nz + kc - 1) / kc;
  const long long nblk = (long long)nstrips * nbb * nch;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblk), block(64 * kNW);
#define MTVD_LF(F, T) sweep_lf3d<F, T><<<grid, block, 0, s>>>(c, sh, zr, slot, first, X, Y, kc, nstrips, nbb)
  if (c.stretched) {
    if (fo == 2) MTVD_LF(2, true); else if (fo == 1) MTVD_LF(1, true); else MTVD_LF(0, true);
  } else {
    if (fo == 2) MTVD_LF(2, false); else if (fo == 1) MTVD_LF(1, false); else MTVD_LF(0, false);
  }
#undef MTVD_LF
  return hipGetLastError();
}

hipError_t launch_sweep_3d(int axis, const Coef& c, Shared* sh, const double* zr, int slot,
                           int first, bool fuse, const double* X, double* Y, int kc,
                           hipStream_t s) {
  // the lane part of an address within a z plane is a 32-bit byte offset
  if ((unsigned long long)c.plane * sizeof(double) >= (1ull << 32)) return hipErrorInvalidValue;
  const int fo = fuse ? (c.dt_rule ? 2 : 1) : 0;
  if (axis == 0) return launch_sweep_3d_x(c, sh, zr, slot, first, fo, X, Y, kc, s);
  if (axis == 1) return launch_sweep_3d_y(c, sh, zr, slot, first, fo, X, Y, kc, s);
  return launch_sweep_3d_z(c, sh, zr, slot, first, fo, X, Y, kc, s);
}

}  // namespace mtvd
