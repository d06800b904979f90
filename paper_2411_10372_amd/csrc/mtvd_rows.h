// mtvd_rows.h -- the default rows per wave of the sweep launches (how many
// rows of its march each wave takes): the launch shape of the 2D and 3D
// operators and of the batch, chosen from the grid and the device's
// resident waves.  Kept apart from the rest of the host code because the
// committed kernel profiles depend on it.
#pragma once

#include <vector>

#include "mtvd_device.h"
#include "mtvd_launch.h"

namespace mtvd {

// slots: resident waves of the 2D sweep kernel of `axis` (wave_slots_2d)
inline int default_rows_for(const Coef& cf, int slots, int axis) {
  long long kc;
  if (cf.ndim == 2) {
    // the fewest rows per wave that keep the whole launch in one round of
    // the device's resident waves: long marches (less halo re-reading per
    // row) and no partly filled last round
    const long long cols = (long long)strips_2d(cf.nx);
    long long chunks = slots > 0 ? slots / cols : 1;
    if (chunks < 1) chunks = 1;
    kc = (cf.nz + chunks - 1) / chunks;
    // small grids: at least 2 rows (more, shorter waves measured faster
    // down to 2 at 512x128, where every launch is latency-bound)
    if (kc < 2) kc = 2;
    if (kc > 64) kc = 64;
  } else {
    // 3D, blocks of 8 waves (L_x and L_z march z, L_y marches y): L_x and
    // L_y half the marched extent up to 128 rows; L_z, whose 8 rows next to
    // each plate run in launches of their own, the rows between in equal
    // chunks of at most 80 (tall grids) or a quarter of nz (short ones).
    // Measured at 1024x1024x256: L_x fastest at 128 (5% ahead of the
    // whole extent), L_y at 128, L_z at 80 (3 x 80 rows; 2% ahead of
    // 5 x 48, 4-7% ahead of 32 and 64); uneven splits are slow.
    const long long len = (axis == 1) ? cf.ny : cf.nz;
    if (axis == 0 || axis == 1) {
      kc = len / 2 < 128 ? len / 2 : 128;
    } else if (len >= 128) {
      const long long mid = len - 16, nch = (mid + 79) / 80;
      kc = (mid + nch - 1) / nch;
    } else {
      kc = len / 4 < 48 ? len / 4 : 48;
    }
    if (kc < 4) kc = 4;
  }
  return (int)kc;
}

// The default rows per wave of a batch operator: the smallest bound k >= 4
// for which the launch -- every box's column strips times its chunks of at
// most k rows -- fits the device's resident waves in one round (a second,
// partly filled round would cost as much as a full one), every box's rows
// split into equal chunks of at most k.  64 at most.
inline int batch_default_k(const std::vector<Coef>& cs, int slots) {
  if (slots <= 0) return 32;
  for (int k = 4; k < 64; ++k) {
    long long w = 0;
    for (const auto& c : cs) w += (long long)strips_2d(c.nx) * ((c.nz + k - 1) / k);
    if (w <= slots) return k;
  }
  return 64;
}

inline int batch_rows(const Coef& c, int kc, int kdef) {
  if (kc > 0) return kc;
  const int n = (c.nz + kdef - 1) / kdef;   // chunks of at most kdef rows
  return (c.nz + n - 1) / n;
}

}  // namespace mtvd
