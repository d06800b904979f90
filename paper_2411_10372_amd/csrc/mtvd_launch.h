// mtvd_launch.h -- host-side launchers of the sweep kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "mtvd_adjoint.h"
#include "mtvd_device.h"

namespace mtvd {

// one directional operator L_axis(tau) in 2D (axis 0 = x, 2 = z)
hipError_t launch_sweep_2d(int axis, const Coef& c, Shared* sh, const double* zr, int slot,
                           int first, bool fuse, const double* X, double* Y, int kc,
                           hipStream_t s);
int strips_2d(int nx);
// waves of the 2D sweep kernel of `axis` to fill the device with: those it
// keeps resident at once, at most two per SIMD (0 if the runtime cannot say)
int wave_slots_2d(int axis, bool fuse);

// all boxes of a batch, one directional operator (2D), one launch
hipError_t launch_batch_2d(int axis, const BoxDesc* boxes, const int4* items, int nitems,
                           Shared* shs, const double* zarena, int slot, int first, bool fuse,
                           const double* X, double* Y, hipStream_t s);

// one directional operator L_axis(tau) in 3D (axis 0 = x, 1 = y, 2 = z)
hipError_t launch_sweep_3d(int axis, const Coef& c, Shared* sh, const double* zr, int slot,
                           int first, bool fuse, const double* X, double* Y, int kc,
                           hipStream_t s);

// reverse of one 2D operator L_axis(dt_frozen/2) at A.X, in two parts:
// launch_adj_fw fills the forward values A.P, A.S, A.XP, A.PP of A.X (it
// needs no cotangent); launch_adj_rev then takes A.Xb = J^T A.Yb + nu_w
// dNu_mean/dX (A.X) (nu_w = 0: no objective term; eps: the Nusselt
// number's eps), and A.MU and A.KB accumulate the mu and K cotangents.
// With next_axis >= 0 the same launch also fills the forward values of the
// operator reversed next (axis next_axis, state F.X) into F.P, F.S, F.XP,
// F.PP, which must not alias A's.
hipError_t launch_adj_fw(int axis, const adj::AC& c, const adj::Arr& A, const Shared* sh,
                         hipStream_t s);
hipError_t launch_adj_rev(int axis, const adj::AC& c, const adj::Arr& A, const Shared* sh,
                          double nu_w, double eps, int next_axis, const adj::Arr& F,
                          hipStream_t s);
hipError_t launch_fill(double* a, long long n, double v, hipStream_t s);
hipError_t launch_ra_reduce(long long cnt, const double* MU, const double* KB, double s_mu,
                            double s_K, double* out, hipStream_t s);
// acc[0] += w Nu_mean(X) (2D)
hipError_t launch_nu_obj(const Coef& c, const double* zr, const double* X, double w, double* acc,
                         hipStream_t s);
// xb += w dNu_mean/dX (2D)
hipError_t launch_nu_vjp(const adj::AC& ac, const Coef& c, const double* zr, const double* X,
                         double w, double* xb, hipStream_t s);
hipError_t launch_init_theta(const Coef& c, const double* zr, const double* theta, double* X,
                             hipStream_t s);
hipError_t launch_grad_theta(const Coef& c, const double* X0, const double* xb, double* gt,
                             hipStream_t s);

// analysis row means (Sec. 4): out[q nz + k], q < kNumProfiles, from
// per-segment partials part[nz][nb][kNumProfiles]
constexpr int kNumProfiles = 10;
// Node heights of the z grid (uniform k/M, or the tanh grid of stretch s).
std::vector<double> grid_heights(double s, int nz);

hipError_t launch_profiles(const Coef& c, const double* zr, const double* X, double* part,
                           int nb, double* out, hipStream_t s);

}  // namespace mtvd
