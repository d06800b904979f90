// mtvd_analysis.hip -- the analysis quantities of the paper's Secs. 4-6 as
// row means on the device: <T>_A, <rho>_A, <|u|^2>_A, <rho u_z T_sa>_A,
// <(rho u_z)^2>_A, <T_sa^2>_A and the z-momentum terms F_n = rho (u.grad)
// u_z, F_p = -dp/dz, F_b = rho g, F_v = d_i tau_iz; and, on the host, the
// snapshot scalars made from them (Re, Sec. 2; the correlation C, Sec.
// 6.2; the volume means of the momentum terms, Sec. 6.1) and the
// boundary-layer thicknesses of a profile (Sec. 5).
//
// Discretisation (the paper gives none for these diagnostics): central
// second-order differences along x, y (periodic) and on interior rows;
// second-order one-sided first derivatives on the plates ((-3, 4, -1) /
// (2 dz) at z = 0, (3, -4, 1) / (2 dz) at z = 1); second derivatives (1, -2,
// 1) / h^2, on the plates (2, -5, 4, -1) / dz^2; the mixed derivative of
// div u is the z operator applied to each row's central x (and y)
// difference; F_v = mu (lap u_z + (1 + lambda) d_z div u), which is
// d_i tau_iz for the constant mu of these units.
//
// Paper: Tiwari, Sharma & Verma, arXiv:2411.10372, Sec. 2 (Re, T_A, rho_A)
// Secs. 4-5 (profiles, boundary layers), Sec. 6.1 (momentum balance) and
// Sec. 6.2 (C(Ra)).
#include <math.h>

#include "../../include/mtvd.h"
#include "mtvd_device.h"
#include "mtvd_launch.h"

namespace mtvd {

namespace {

constexpr int kProfBlock = 256;

struct P6 {
  double rho, ux, uy, uz, T, p;
};

__device__ __forceinline__ int wrapi(int v, int n) {
  int m = v % n;
  return m < 0 ? m + n : m;
}

// primitives of node (i, j, k); i, j wrap (periodic sides)
__device__ __forceinline__ P6 prim_at(const Coef& c, const double* zr,
                                      const double* __restrict__ X, int i, int j, int k) {
  const long long n = ((long long)k * (c.ndim == 3 ? c.ny : 1) + wrapi(j, c.ndim == 3 ? c.ny : 1)) *
                          c.nx + wrapi(i, c.nx);
  const int fz = c.nf - 2;
  P6 q;
  q.rho = X[n];
  q.ux = X[n + c.cnt] / q.rho;
  q.uy = (c.ndim == 3) ? X[n + 2 * c.cnt] / q.rho : 0.0;
  q.uz = X[n + fz * c.cnt] / q.rho;
  const double u2 = (q.ux * q.ux + q.uy * q.uy) + q.uz * q.uz;
  q.T = (X[n + (c.nf - 1) * c.cnt] / q.rho - 0.5 * u2 - c.g * zr[k]) / c.cv;
  q.p = c.a * q.rho * q.T;
  return q;
}

// the ten quantities of node (i, j, k), in the order of the output rows
__device__ void node_quantities(const Coef& c, const double* zr, const double* __restrict__ X,
                                int i, int j, int k, double v[10]) {
  const double hx = c.hx, hz = c.hz;
  const P6 q = prim_at(c, zr, X, i, j, k);
  const P6 xm = prim_at(c, zr, X, i - 1, j, k), xp = prim_at(c, zr, X, i + 1, j, k);
  const double dx_uz = (xp.uz - xm.uz) / (2.0 * hx);
  const double dxx_uz = (xp.uz - 2.0 * q.uz + xm.uz) / (hx * hx);
  double dy_uz = 0.0, dyy_uz = 0.0;
  if (c.ndim == 3) {
    const double hy = c.hy;
    const P6 ym = prim_at(c, zr, X, i, j - 1, k), yp = prim_at(c, zr, X, i, j + 1, k);
    dy_uz = (yp.uz - ym.uz) / (2.0 * hy);
    dyy_uz = (yp.uz - 2.0 * q.uz + ym.uz) / (hy * hy);
  }
  // horizontal divergence of the row r (central differences)
  auto dxy = [&](int r) -> double {
    double s = (prim_at(c, zr, X, i + 1, j, r).ux - prim_at(c, zr, X, i - 1, j, r).ux) / (2.0 * hx);
    if (c.ndim == 3)
      s = s + (prim_at(c, zr, X, i, j + 1, r).uy - prim_at(c, zr, X, i, j - 1, r).uy) /
                  (2.0 * c.hy);
    return s;
  };
  const int M = c.M;
  double dz_uz, dz_p, dzz_uz, dz_dxy;
  if (c.stretched) {
    // the same stencils on the node heights (metric table): first
    // derivatives over the same stencil of z, second derivatives by the
    // three-point weights inside and the four-point Lagrange weights at a
    // plate
    const double* m = c.zm + (size_t)k * kZM;
    if (k == 0 || k == M) {
      const int sg = (k == 0) ? 1 : -1;
      const P6 a1 = prim_at(c, zr, X, i, j, k + sg), a2 = prim_at(c, zr, X, i, j, k + 2 * sg),
               a3 = prim_at(c, zr, X, i, j, k + 3 * sg);
      const double iw = m[kZM_IWALL];
      const double s3 = (double)sg * 3.0;   // -3, 4, -1 at the bottom; 3, -4, 1 at the top
      dz_uz = (-s3 * q.uz + sg * 4.0 * a1.uz - sg * a2.uz) * iw;
      dz_p = (-s3 * q.p + sg * 4.0 * a1.p - sg * a2.p) * iw;
      dzz_uz = ((m[kZM_D2] * q.uz + m[kZM_D2 + 1] * a1.uz) + m[kZM_D2 + 2] * a2.uz) +
               m[kZM_D2 + 3] * a3.uz;
      dz_dxy = (-s3 * dxy(k) + sg * 4.0 * dxy(k + sg) - sg * dxy(k + 2 * sg)) * iw;
    } else {
      const P6 zm = prim_at(c, zr, X, i, j, k - 1), zp = prim_at(c, zr, X, i, j, k + 1);
      const double ic = m[kZM_ICEN];
      dz_uz = (zp.uz - zm.uz) * ic;
      dz_p = (zp.p - zm.p) * ic;
      dzz_uz = (m[kZM_D2] * zm.uz + m[kZM_D2 + 1] * q.uz) + m[kZM_D2 + 2] * zp.uz;
      dz_dxy = (dxy(k + 1) - dxy(k - 1)) * ic;
    }
  } else if (k == 0) {
    const P6 a1 = prim_at(c, zr, X, i, j, 1), a2 = prim_at(c, zr, X, i, j, 2),
             a3 = prim_at(c, zr, X, i, j, 3);
    dz_uz = (-3.0 * q.uz + 4.0 * a1.uz - a2.uz) / (2.0 * hz);
    dz_p = (-3.0 * q.p + 4.0 * a1.p - a2.p) / (2.0 * hz);
    dzz_uz = (2.0 * q.uz - 5.0 * a1.uz + 4.0 * a2.uz - a3.uz) / (hz * hz);
    dz_dxy = (-3.0 * dxy(0) + 4.0 * dxy(1) - dxy(2)) / (2.0 * hz);
  } else if (k == M) {
    const P6 a1 = prim_at(c, zr, X, i, j, M - 1), a2 = prim_at(c, zr, X, i, j, M - 2),
             a3 = prim_at(c, zr, X, i, j, M - 3);
    dz_uz = (3.0 * q.uz - 4.0 * a1.uz + a2.uz) / (2.0 * hz);
    dz_p = (3.0 * q.p - 4.0 * a1.p + a2.p) / (2.0 * hz);
    dzz_uz = (2.0 * q.uz - 5.0 * a1.uz + 4.0 * a2.uz - a3.uz) / (hz * hz);
    dz_dxy = (3.0 * dxy(M) - 4.0 * dxy(M - 1) + dxy(M - 2)) / (2.0 * hz);
  } else {
    const P6 zm = prim_at(c, zr, X, i, j, k - 1), zp = prim_at(c, zr, X, i, j, k + 1);
    dz_uz = (zp.uz - zm.uz) / (2.0 * hz);
    dz_p = (zp.p - zm.p) / (2.0 * hz);
    dzz_uz = (zp.uz - 2.0 * q.uz + zm.uz) / (hz * hz);
    dz_dxy = (dxy(k + 1) - dxy(k - 1)) / (2.0 * hz);
  }
  const double u2 = (q.ux * q.ux + q.uy * q.uy) + q.uz * q.uz;
  const double Tsa = q.T - (1.0 - c.D * zr[k]);
  const double ruz = q.rho * q.uz;
  const double adv = (c.ndim == 3) ? (q.ux * dx_uz + q.uy * dy_uz) + q.uz * dz_uz
                                   : q.ux * dx_uz + q.uz * dz_uz;
  const double lap = (c.ndim == 3) ? (dxx_uz + dyy_uz) + dzz_uz : dxx_uz + dzz_uz;
  v[0] = q.T;
  v[1] = q.rho;
  v[2] = u2;
  v[3] = ruz * Tsa;
  v[4] = ruz * ruz;
  v[5] = Tsa * Tsa;
  v[6] = q.rho * adv;
  v[7] = -dz_p;
  v[8] = q.rho * c.g;
  v[9] = c.mu * (lap + (1.0 + c.lam) * (dz_dxy + dzz_uz));
}

// per-row partial sums over one segment of a row; fixed-order tree
__global__ __launch_bounds__(kProfBlock) void profile_rows_kernel(Coef c, const double* zr,
                                                                  const double* __restrict__ X,
                                                                  double* part, int nb) {
  __shared__ double red[kNumProfiles][kProfBlock];
  const int k = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
  const long long seg = (c.plane + nb - 1) / nb;
  const long long lo = (long long)b * seg;
  const long long hi = min(lo + seg, c.plane);
  double acc[kNumProfiles];
  for (int q = 0; q < kNumProfiles; ++q) acc[q] = 0.0;
  for (long long e = lo + t; e < hi; e += kProfBlock) {
    double v[kNumProfiles];
    node_quantities(c, zr, X, (int)(e % c.nx), (int)(e / c.nx), k, v);
    for (int q = 0; q < kNumProfiles; ++q) acc[q] += v[q];
  }
  for (int q = 0; q < kNumProfiles; ++q) red[q][t] = acc[q];
  __syncthreads();
  for (int w = kProfBlock / 2; w > 0; w >>= 1) {
    if (t < w)
      for (int q = 0; q < kNumProfiles; ++q) red[q][t] += red[q][t + w];
    __syncthreads();
  }
  if (t < kNumProfiles) part[((size_t)k * nb + b) * kNumProfiles + t] = red[t][0];
}

// out[q nz + k] = (sum over the row's segments, in order) / nodes per row
__global__ void profile_final_kernel(Coef c, const double* part, int nb, double* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kNumProfiles * c.nz) return;
  const int q = t / c.nz, k = t % c.nz;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[((size_t)k * nb + b) * kNumProfiles + q];
  out[t] = s / (double)c.plane;
}

}  // namespace

hipError_t launch_profiles(const Coef& c, const double* zr, const double* X, double* part,
                           int nb, double* out, hipStream_t s) {
  dim3 grid(nb, c.nz);
  profile_rows_kernel<<<grid, kProfBlock, 0, s>>>(c, zr, X, part, nb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = kNumProfiles * c.nz;
  profile_final_kernel<<<(n + 255) / 256, 256, 0, s>>>(c, part, nb, out);
  return hipGetLastError();
}

}  // namespace mtvd

// ---------------------------------------------------------------------------
// host only: what the profile rows give for one snapshot

namespace {

// <f>_V of a row-mean profile: trapezoid in z over a box of height 1 (on a
// stretched grid with the dual cells of the node heights z as weights)
double volume_mean(const double* v, int nz, const double* z) {
  const int M = nz - 1;
  if (z) {
    double s = 0.5 * (z[1] - z[0]) * v[0];
    for (int k = 1; k < M; ++k) s += 0.5 * (z[k + 1] - z[k - 1]) * v[k];
    return s + 0.5 * (z[M] - z[M - 1]) * v[M];
  }
  double s = 0.5 * v[0];
  for (int k = 1; k < M; ++k) s += v[k];
  s += 0.5 * v[M];
  return s / (double)M;
}

// slopes between rows and their midpoints: the boundary-layer crossings
// (uniform rows when z is null)
void bl_crossings(const double* tmean, const double* z, int nz, double D, double rtol,
                  double* lam_b, double* lam_t) {
  const int M = nz - 1;
  const double hz = 1.0 / (double)M;
  const double thr = -(1.0 + rtol) * D;
  auto slope = [&](int k) {
    return z ? (tmean[k + 1] - tmean[k]) / (z[k + 1] - z[k]) : (tmean[k + 1] - tmean[k]) / hz;
  };
  auto zmid = [&](int k) { return z ? 0.5 * (z[k] + z[k + 1]) : ((double)k + 0.5) * hz; };
  // from the bottom plate up
  *lam_b = -1.0;
  for (int k = 0; k < M; ++k) {
    if (slope(k) >= thr) {
      if (k == 0) {
        *lam_b = zmid(0);
      } else {
        const double f = (thr - slope(k - 1)) / (slope(k) - slope(k - 1));
        *lam_b = zmid(k - 1) + f * (zmid(k) - zmid(k - 1));
      }
      break;
    }
  }
  // from the top plate down, measured from the top
  *lam_t = -1.0;
  for (int k = M - 1; k >= 0; --k) {
    if (slope(k) >= thr) {
      double zc;
      if (k == M - 1) {
        zc = zmid(M - 1);
      } else {
        const double f = (thr - slope(k + 1)) / (slope(k) - slope(k + 1));
        zc = zmid(k + 1) + f * (zmid(k) - zmid(k + 1));
      }
      *lam_t = 1.0 - zc;
      break;
    }
  }
}

}  // namespace

extern "C" {

int mtvd_analysis_from_profiles(const mtvd_params* p, const double* prof, size_t count,
                                mtvd_analysis* out, double* tsa_z, double* drho_z, double* U_z) {
  if (!p || !prof || !out || p->nz < 5 || !(p->Ra > 0.0) || !(p->Pr > 0.0) ||
      !(p->gamma > 1.0) || !(p->stretch >= 0.0) || !(p->stretch <= 10.0))
    return MTVD_EINVAL;
  const int nz = p->nz;
  if (count < (size_t)mtvd::kNumProfiles * (size_t)nz) return MTVD_ESIZE;
  const std::vector<double> zg = mtvd::grid_heights(p->stretch, nz);
  const double* zw = p->stretch > 0.0 ? zg.data() : nullptr;
  double V[mtvd::kNumProfiles];
  for (int q = 0; q < mtvd::kNumProfiles; ++q) V[q] = volume_mean(prof + (size_t)q * nz, nz, zw);
  out->u2 = V[2];
  out->rho_uz_Tsa = V[3];
  out->rho_uz2 = V[4];
  out->Tsa2 = V[5];
  out->Fn = V[6];
  out->Fp = V[7];
  out->Fb = V[8];
  out->Fv = V[9];
  // Re = sqrt(Ra/Pr) U with U the rms velocity (Sec. 2)
  out->Re = sqrt(p->Ra / p->Pr) * sqrt(V[2]);
  // C = <rho u_z T_sa> / sqrt(<(rho u_z)^2> <T_sa^2>) (Sec. 6.2)
  const double den = sqrt(V[4] * V[5]);
  out->C = den > 0.0 ? V[3] / den : 0.0;
  const double beta = 1.0 / (p->gamma - 1.0);
  for (int k = 0; k < nz; ++k) {
    const double z = zg[k];
    if (tsa_z) tsa_z[k] = prof[k] - (1.0 - p->D * z);
    if (drho_z) drho_z[k] = prof[(size_t)nz + k] - pow(1.0 - p->D * z, beta);
    if (U_z) U_z[k] = sqrt(prof[(size_t)2 * nz + k]);
  }
  return MTVD_OK;
}

int mtvd_bl_thickness(const double* tmean, int32_t nz, double D, double rtol, double* lam_b,
                      double* lam_t) {
  if (!tmean || !lam_b || !lam_t || nz < 3 || !(D > 0.0) || !(rtol >= 0.0))
    return MTVD_EINVAL;
  bl_crossings(tmean, nullptr, nz, D, rtol, lam_b, lam_t);
  return MTVD_OK;
}

int mtvd_bl_thickness_grid(const double* tmean, const double* z, int32_t nz, double D,
                           double rtol, double* lam_b, double* lam_t) {
  if (!tmean || !z || !lam_b || !lam_t || nz < 3 || !(D > 0.0) || !(rtol >= 0.0))
    return MTVD_EINVAL;
  for (int k = 0; k + 1 < nz; ++k)
    if (!(z[k + 1] > z[k])) return MTVD_EINVAL;
  bl_crossings(tmean, z, nz, D, rtol, lam_b, lam_t);
  return MTVD_OK;
}

}  // extern "C"
