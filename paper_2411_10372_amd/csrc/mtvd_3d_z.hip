// mtvd_3d_z.hip -- L_z in 3D (flux along the march in z, plates, waves
// along y).  Built without fused multiply-adds: its plate rows and the rows
// between run two separately compiled copies of the same arithmetic, and
// with every expression rounded as written both copies give the same bits,
// so results do not depend on the rows per wave.
#include "mtvd_3d.h"

namespace mtvd {

hipError_t launch_sweep_3d_z(const Coef& c, Shared* sh, const double* zr, int slot, int first,
                             int fo, const double* X, double* Y, int kc, hipStream_t s) {
  const int nstrips = strips_3d(c.nx);
  const int nbb = (c.ny + kPer - 1) / kPer;
  const dim3 block(64 * kNW);
  // The kPlate rows next to each plate run the copy with the plate and wall
  // code (its registers spill) in launches of their own; the rows between
  // (output rows >= 4 and <= M-4, so no stage reaches a plate) run the copy
  // without it in chunks of kc.  The launches of one operator are
  // independent (disjoint output rows); only the first one does the step's
  // bookkeeping (time, dt, the next slot).
  constexpr int kPlate = 8;
  int fst = first;
  hipError_t e = hipSuccess;
  auto run = [&](int r0, int r1, int k, bool pl) {
    if (r1 <= r0 || e != hipSuccess) return;
    const long long nck = (r1 - r0 + k - 1) / k;
    const long long nblk = (long long)nstrips * nbb * nck;
    if (nblk > 0x7fffffffLL) {
      e = hipErrorInvalidValue;
      return;
    }
    const dim3 g((unsigned)nblk);
#define MTVD_MF(F, P, T) sweep_mf3d<2, F, P, T><<<g, block, 0, s>>>(c, sh, zr, slot, fst, X, Y, k, nstrips, nbb, r0, r1)
#define MTVD_MF_F(P, T) \
  do { if (fo == 2) MTVD_MF(2, P, T); else if (fo == 1) MTVD_MF(1, P, T); else MTVD_MF(0, P, T); } while (0)
    if (c.stretched) {
      if (pl) MTVD_MF_F(true, true); else MTVD_MF_F(false, true);
    } else {
      if (pl) MTVD_MF_F(true, false); else MTVD_MF_F(false, false);
    }
#undef MTVD_MF_F
#undef MTVD_MF
    fst = 0;
    e = hipGetLastError();
  };
  if (c.nz > 2 * kPlate) {
    run(0, kPlate, kPlate, true);
    run(kPlate, c.nz - kPlate, kc, false);
    run(c.nz - kPlate, c.nz, kPlate, true);
  } else {
    run(0, c.nz, kc, true);
  }
  return e;
}

}  // namespace mtvd
