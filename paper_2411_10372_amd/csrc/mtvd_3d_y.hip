// mtvd_3d_y.hip -- L_y in 3D (flux along the march in y, waves along z;
// plate rows copied through).
#include "mtvd_3d.h"

namespace mtvd {

hipError_t launch_sweep_3d_y(const Coef& c, Shared* sh, const double* zr, int slot, int first,
                             int fo, const double* X, double* Y, int kc, hipStream_t s) {
  const int nstrips = strips_3d(c.nx);
  const int nbb = (c.nz + kPer - 1) / kPer;
  const int nch = (c.ny + kc - 1) / kc;
  const long long nblk = (long long)nstrips * nbb * nch;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblk), block(64 * kNW);
#define MTVD_MY(F, T) sweep_mf3d<1, F, true, T><<<grid, block, 0, s>>>(c, sh, zr, slot, first, X, Y, kc, nstrips, nbb, 0, c.ny)
  if (c.stretched) {
    if (fo == 2) MTVD_MY(2, true); else if (fo == 1) MTVD_MY(1, true); else MTVD_MY(0, true);
  } else {
    if (fo == 2) MTVD_MY(2, false); else if (fo == 1) MTVD_MY(1, false); else MTVD_MY(0, false);
  }
#undef MTVD_MY
  return hipGetLastError();
}

}  // namespace mtvd
