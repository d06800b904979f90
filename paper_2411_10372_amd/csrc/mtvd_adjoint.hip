// mtvd_adjoint.hip -- kernels of the reverse pass of a 2D time step with a
// frozen dt: each directional operator's forward values and its reverse
// (the functions of mtvd_adjoint.h: one kernel for the forward values, one
// for the three cotangent stages fused over tiles), the objective (the
// mean plate Nusselt number, accumulated over steps), its cotangent, the
// initial state from a temperature perturbation and the perturbation's
// cotangent.
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

constexpr int kBlk = 256;

// The operator's forward values (fw_all), one thread per node.  AX: the
// operator's axis as a compile-time constant, so that every axis test of
// the stage functions folds away.
template <int AX>
__global__ __launch_bounds__(kBlk) void adj_fw_kernel(AC c, Arr A, const Shared* sh) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= c.cnt) return;
  c.axis = AX;
  c.iha = AX == 0 ? c.ihx : c.ihz;
  c.tau = 0.5 * sh->dt_frozen;
  c.lm = c.tau * c.iha;
  const int i = (int)(t % c.nx), k = (int)(t / c.nx);
  adj::fw_all(c, A, i, k);
}

// The reverse of one operator in one kernel: the three cotangent stages
// over a tile of kTA x kTB output nodes per block, their intermediate
// values in shared memory (the tiled pass of mtvd_adjoint.h; thread t
// computes node t of each stage's region).  tiles_b = tiles across the
// axis; block q < ntiles takes tile (q / tiles_b, q % tiles_b) (along,
// across).  With AXF >= 0 the blocks from ntiles on fill, for the operator
// to be reversed next (axis AXF, state F.X), its forward values F.P, F.S,
// F.XP, F.PP: independent work that keeps the CUs busy while the tiles
// wait on memory, and leaves those values in the caches for the next
// launch.  40 KiB of shared memory and at most 168 VGPRs (three waves per
// SIMD) let three blocks share a CU: 768 blocks at once, more than the
// ~520 tiles (+ 128 forward-value blocks) of a 512 x 128 grid, which then
// run in a single round.
template <int AX, int AXF>
__global__ __launch_bounds__(adj::kNT, 3) void adj_rev_fused(AC c, Arr A, const Shared* sh,
                                                              int tiles_b, int ntiles,
                                                              double nu_a, Arr F) {
  __shared__ double L[adj::kTileDoubles];
  c.tau = 0.5 * sh->dt_frozen;
  if (AXF >= 0 && (int)blockIdx.x >= ntiles) {
    AC cf = c;
    cf.axis = AXF;
    cf.iha = AXF == 0 ? c.ihx : c.ihz;
    cf.lm = cf.tau * cf.iha;
    const long long stride = (long long)(gridDim.x - ntiles) * adj::kNT;
    for (long long n = (long long)(blockIdx.x - ntiles) * adj::kNT + threadIdx.x; n < c.cnt;
         n += stride)
      adj::fw_all(cf, F, (int)(n % c.nx), (int)(n / c.nx));
    return;
  }
  c.axis = AX;
  c.iha = AX == 0 ? c.ihx : c.ihz;
  c.lm = c.tau * c.iha;
  const int a0 = (int)(blockIdx.x / tiles_b) * adj::kTA, b0 = (int)(blockIdx.x % tiles_b) * adj::kTB;
  const int t = threadIdx.x;
  adj::tile_tc(c, A, L, a0, b0, t);
  __syncthreads();
  adj::PredOut o;
  const bool put = t < adj::kNP && adj::tile_pred(c, A, L, a0, b0, t, o);
  __syncthreads();
  if (put) adj::tile_pred_put(L, t, o);
  __syncthreads();
  if (t < adj::kNO) adj::tile_prim(c, A, L, a0, b0, t, nu_a);
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
    adj_fw_kernel<0><<<g, kBlk, 0, s>>>(c, A, sh);
  else
    adj_fw_kernel<2><<<g, kBlk, 0, s>>>(c, A, sh);
  return hipGetLastError();
}

hipError_t launch_adj_rev(int axis, const AC& c0, const Arr& A, const Shared* sh, double nu_w,
                          double eps, int next_axis, const Arr& F, hipStream_t s) {
  const double nu_a = nu_w == 0.0 ? 0.0 : nu_w * (-0.5 / eps);
  AC c = c0;
  c.axis = axis;
  c.iha = axis == 0 ? c.ihx : c.ihz;
  const int na = axis == 0 ? c.nx : c.nz, nb = axis == 0 ? c.nz : c.nx;
  const int ta = (na + adj::kTA - 1) / adj::kTA, tb = (nb + adj::kTB - 1) / adj::kTB;
  const int nt = ta * tb;
  // forward-value blocks: up to 128, a node per thread and round
  const long long fwb = (c.cnt + adj::kNT - 1) / adj::kNT;
  const int nf = next_axis < 0 ? 0 : (int)(fwb < 128 ? fwb : 128);
  const unsigned g = (unsigned)(nt + nf);
  if (axis == 0) {
    if (next_axis == 2)
      adj_rev_fused<0, 2><<<g, adj::kNT, 0, s>>>(c, A, sh, tb, nt, nu_a, F);
    else if (next_axis == 0)
      adj_rev_fused<0, 0><<<g, adj::kNT, 0, s>>>(c, A, sh, tb, nt, nu_a, F);
    else
      adj_rev_fused<0, -1><<<g, adj::kNT, 0, s>>>(c, A, sh, tb, nt, nu_a, F);
  } else {
    if (next_axis == 0)
      adj_rev_fused<2, 0><<<g, adj::kNT, 0, s>>>(c, A, sh, tb, nt, nu_a, F);
    else if (next_axis == 2)
      adj_rev_fused<2, 2><<<g, adj::kNT, 0, s>>>(c, A, sh, tb, nt, nu_a, F);
    else
      adj_rev_fused<2, -1><<<g, adj::kNT, 0, s>>>(c, A, sh, tb, nt, nu_a, F);
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
