// mtvd_adjoint.hip -- kernels of the reverse pass of a 2D time step with a
// frozen dt: the four stages of each directional operator's reverse
// (functions of mtvd_adjoint.h, one kernel per stage), the objective (the mean plate
// Nusselt number, accumulated over steps), its cotangent, the initial state
// from a temperature perturbation and the perturbation's cotangent.
//
// Paper: Tiwari, Sharma & Verma, arXiv:2411.10372: Sec. 3.1 (the operator
// reversed), Sec. 2 (initial state, mean_Nu).
#include "mtvd_adjoint.h"
#include "mtvd_device.h"
#include "mtvd_launch.h"

namespace mtvd {

using adj::AC;
using adj::Arr;

namespace {

enum Stage { kFwAll, kRvTc, kRvPred, kRvPrim };

constexpr int kBlk = 256;

// AX: the operator's axis as a compile-time constant, so that every axis
// test of the stage functions folds away
template <int ST, int AX>
__global__ __launch_bounds__(kBlk) void adj_stage(AC c, Arr A, const Shared* sh) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= c.cnt) return;
  c.axis = AX;
  c.iha = AX == 0 ? c.ihx : c.ihz;
  c.tau = 0.5 * sh->dt_frozen;
  c.lm = c.tau * c.iha;
  const int i = (int)(t % c.nx), k = (int)(t / c.nx);
  switch (ST) {
    case kFwAll: adj::fw_all(c, A, i, k); break;
    case kRvTc: adj::rv_tc(c, A, i, k); break;
    case kRvPred: adj::rv_pred(c, A, i, k); break;
    default: adj::rv_prim(c, A, i, k); break;
  }
}

// out[0] += s_mu * sum(MU) + s_K * sum(KB); one block, fixed order
__global__ __launch_bounds__(1024) void ra_reduce_kernel(long long cnt, const double* MU,
                                                         const double* KB, double s_mu,
                                                         double s_K, double* out) {
  __shared__ double sm[1024], sk[1024];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (long long n = t; n < cnt; n += 1024) {
    a += MU[n];
    b += KB[n];
  }
  sm[t] = a;
  sk[t] = b;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) {
      sm[t] += sm[t + w];
      sk[t] += sk[t + w];
    }
    __syncthreads();
  }
  if (t == 0) *out += sm[0] * s_mu + sk[0] * s_K;
}

__global__ void fill_kernel(double* a, long long n, double v) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) a[t] = v;
}

__device__ __forceinline__ double node_T(const Coef& c, const double* X, long long n, double z) {
  const double rho = X[n];
  const double ri = 1.0 / rho;
  const double ux = X[n + c.cnt] * ri, uz = X[n + 2 * c.cnt] * ri;
  return (X[n + 3 * c.cnt] * ri - 0.5 * (ux * ux + uz * uz) - c.g * z) * c.icv;
}

// Rows read by mean_Nu and the weights of their mean temperatures:
// Nu_mean = (Nu(z=0) + Nu(z=1))/2 with Nu = -(dT/dz + D)/eps and one-sided
// second-order dT/dz of the row means (weights -3, 4, -1 and 1, -4, 3, over
// 2 dz).
__device__ __forceinline__ void nu_rows(const Coef& c, int r, int* row, double* wgt) {
  const int rows[6] = {0, 1, 2, c.M - 2, c.M - 1, c.M};
  const double w[6] = {-3.0, 4.0, -1.0, 1.0, -4.0, 3.0};
  *row = rows[r];
  *wgt = w[r];
}

// acc[0] += w * Nu_mean(X): one wave per row that Nu_mean reads (6 waves).
// Each lane sums the temperatures of nodes lane, lane + 64, ... in that
// order, the wave adds its 64 partial sums by a fixed butterfly, and the
// first thread combines the six row means: a fixed order of operations, so
// repeated runs give the same bits.
__global__ __launch_bounds__(6 * 64) void nu_obj_kernel(Coef c, const double* zr,
                                                        const double* __restrict__ X, double w,
                                                        double* acc) {
  __shared__ double rows[6];
  const int r = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int k;
  double wr;
  nu_rows(c, r, &k, &wr);
  const double z = zr[k];
  const long long base = (long long)k * c.nx;
  double s = 0.0;
#pragma unroll 8
  for (int i = lane; i < c.nx; i += 64) s += node_T(c, X, base + i, z);
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) rows[r] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tm[6];
    for (int q = 0; q < 6; ++q) tm[q] = rows[q] / (double)c.nx;
    const double gb = ((-3.0 * tm[0] + 4.0 * tm[1]) - tm[2]) * (0.5 * c.ihz);
    const double gt = ((3.0 * tm[5] - 4.0 * tm[4]) + tm[3]) * (0.5 * c.ihz);
    const double nub = -(gb + c.D) / c.eps, nut = -(gt + c.D) / c.eps;
    acc[0] += w * (0.5 * (nub + nut));
  }
}

// xb += w dNu_mean/dX.  One thread per node of a row slot r; a row that two
// slots share (nz = 5) is handled by its first slot with the summed weight.
__global__ void nu_vjp_kernel(AC ac, Coef c, const double* zr, const double* X, double w,
                              double* xb) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 6LL * c.nx) return;
  const int r = (int)(t / c.nx), i = (int)(t % c.nx);
  int k;
  double wr;
  nu_rows(c, r, &k, &wr);
  for (int q = 0; q < r; ++q) {
    int kq;
    double wq;
    nu_rows(c, q, &kq, &wq);
    if (kq == k) return;
  }
  for (int q = r + 1; q < 6; ++q) {
    int kq;
    double wq;
    nu_rows(c, q, &kq, &wq);
    if (kq == k) wr += wq;
  }
  // d Nu_mean / d T(i, k) = -(1/(2 eps)) wr (1/(2 dz)) / nx
  const double Tb = w * (-0.5 / c.eps) * wr * (0.5 * c.ihz) / (double)c.nx;
  const long long n = (long long)k * c.nx + i;
  double x[4], xbn[4];
  const double qb[4] = {0.0, 0.0, Tb, 0.0};
  adj::ld4(X, c.cnt, n, x);
  adj::ld4(xb, c.cnt, n, xbn);
  adj::prim_vjp(ac, x, zr[k], qb, xbn);
  adj::st4(xb, c.cnt, n, xbn);
}

// X0: the conduction state of the initial-state kernel with T0 + theta on
// interior rows (theta may be null: no perturbation)
__global__ void init_theta_kernel(Coef c, const double* zr, const double* theta, double* X) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= c.cnt) return;
  const int k = (int)(n / c.plane);
  const double z = zr[k];
  const double T0 = 1.0 - c.init_delta * z;
  const double rho = pow(T0, c.init_expo);
  double T = T0;
  if (theta && k > 0 && k < c.M) T = T0 + theta[n];
  X[n] = rho;
  X[n + c.cnt] = 0.0;
  X[n + 2 * c.cnt] = 0.0;
  X[n + 3 * c.cnt] = rho * (c.cv * T + c.g * z);
}

// dJ/dtheta = dJ/dE rho c_v on interior rows (E = rho (c_v T + g z), rho
// does not depend on theta), 0 on the plates
__global__ void grad_theta_kernel(Coef c, const double* X0, const double* xb, double* gt) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= c.cnt) return;
  const int k = (int)(n / c.plane);
  gt[n] = (k > 0 && k < c.M) ? xb[n + 3 * c.cnt] * X0[n] * c.cv : 0.0;
}

unsigned blocks_for(long long n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_adj_fw(int axis, const AC& c0, const Arr& A, const Shared* sh,
                         hipStream_t s) {
  AC c = c0;
  c.axis = axis;
  c.iha = axis == 0 ? c.ihx : c.ihz;
  const unsigned g = blocks_for(c.cnt, kBlk);
  if (axis == 0)
    adj_stage<kFwAll, 0><<<g, kBlk, 0, s>>>(c, A, sh);
  else
    adj_stage<kFwAll, 2><<<g, kBlk, 0, s>>>(c, A, sh);
  return hipGetLastError();
}

hipError_t launch_adj_rev(int axis, const AC& c0, const Arr& A, const Shared* sh,
                          hipStream_t s) {
  AC c = c0;
  c.axis = axis;
  c.iha = axis == 0 ? c.ihx : c.ihz;
  const unsigned g = blocks_for(c.cnt, kBlk);
  if (axis == 0) {
    adj_stage<kRvTc, 0><<<g, kBlk, 0, s>>>(c, A, sh);
    adj_stage<kRvPred, 0><<<g, kBlk, 0, s>>>(c, A, sh);
    adj_stage<kRvPrim, 0><<<g, kBlk, 0, s>>>(c, A, sh);
  } else {
    adj_stage<kRvTc, 2><<<g, kBlk, 0, s>>>(c, A, sh);
    adj_stage<kRvPred, 2><<<g, kBlk, 0, s>>>(c, A, sh);
    adj_stage<kRvPrim, 2><<<g, kBlk, 0, s>>>(c, A, sh);
  }
  return hipGetLastError();
}

hipError_t launch_fill(double* a, long long n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_kernel<<<blocks_for(n, 256), 256, 0, s>>>(a, n, v);
  return hipGetLastError();
}

hipError_t launch_ra_reduce(long long cnt, const double* MU, const double* KB, double s_mu,
                            double s_K, double* out, hipStream_t s) {
  ra_reduce_kernel<<<1, 1024, 0, s>>>(cnt, MU, KB, s_mu, s_K, out);
  return hipGetLastError();
}

hipError_t launch_nu_obj(const Coef& c, const double* zr, const double* X, double w, double* acc,
                         hipStream_t s) {
  nu_obj_kernel<<<1, 6 * 64, 0, s>>>(c, zr, X, w, acc);
  return hipGetLastError();
}

hipError_t launch_nu_vjp(const AC& ac, const Coef& c, const double* zr, const double* X,
                         double w, double* xb, hipStream_t s) {
  nu_vjp_kernel<<<blocks_for(6LL * c.nx, 256), 256, 0, s>>>(ac, c, zr, X, w, xb);
  return hipGetLastError();
}

hipError_t launch_init_theta(const Coef& c, const double* zr, const double* theta, double* X,
                             hipStream_t s) {
  init_theta_kernel<<<blocks_for(c.cnt, 256), 256, 0, s>>>(c, zr, theta, X);
  return hipGetLastError();
}

hipError_t launch_grad_theta(const Coef& c, const double* X0, const double* xb, double* gt,
                             hipStream_t s) {
  grad_theta_kernel<<<blocks_for(c.cnt, 256), 256, 0, s>>>(c, X0, xb, gt);
  return hipGetLastError();
}

}  // namespace mtvd
