// mtvd_api.hip -- the C ABI (include/mtvd.h): parameter checks, buffer
// binding, the per-step launch sequence, and the initial-state, dt and
// diagnostics kernels.
//
// Paper: Tiwari, Sharma & Verma, arXiv:2411.10372.  Initial state: the
// conduction profile between plates at T = 1 and 1 - eps - D (Sec. 2) in
// hydrostatic balance; step composition: Sec. 3.1 (time_step);
// diagnostics: Sec. 2 (volume_Nu, mean_Nu).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mtvd.h"
#include "mtvd_device.h"
#include "mtvd_launch.h"
#include "mtvd_rows.h"

using namespace mtvd;

// ---------------------------------------------------------------------------
// workspace layout (bytes; every region 256-aligned)

namespace {

constexpr size_t kAlign = 256;
constexpr int kDiagBlock = 256;
constexpr int kDiagVals = 8;   // per-row sums kept per block
constexpr int kDiagOut = 32;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t shared, zrow, zmet, part, out, ppart, pout, total;
  int diag_nb;  // blocks per row of the diagnostics reduction
};

Layout layout_of(const mtvd_params* p) {
  Layout L;
  long long plane = (long long)p->nx * (p->ndim == 3 ? p->ny : 1);
  // about 16 elements per thread per block, at most 1024 blocks per row
  long long nb = (plane + kDiagBlock * 16 - 1) / (kDiagBlock * 16);
  if (nb < 1) nb = 1;
  if (nb > 1024) nb = 1024;
  L.diag_nb = (int)nb;
  size_t off = 0;
  L.shared = off;
  off = align_up(off + sizeof(Shared));
  L.zrow = off;
  off = align_up(off + sizeof(double) * (size_t)p->nz);
  L.zmet = off;   // metric table of a stretched grid (empty when uniform)
  if (p->stretch > 0.0) off = align_up(off + sizeof(double) * (size_t)p->nz * kZM);
  L.part = off;
  off = align_up(off + sizeof(double) * (size_t)p->nz * (size_t)nb * kDiagVals);
  L.out = off;
  off = align_up(off + sizeof(double) * kDiagOut);
  L.ppart = off;   // analysis row partials, then the row means
  off = align_up(off + sizeof(double) * (size_t)p->nz * (size_t)nb * kNumProfiles);
  L.pout = off;
  off = align_up(off + sizeof(double) * (size_t)p->nz * kNumProfiles);
  L.total = off;
  return L;
}

}  // namespace

// ---------------------------------------------------------------------------
// kernels

namespace mtvd {

// z_k = k / M exactly as a correctly rounded quotient, so both plates sit
// at 0 and 1
__global__ void zrow_kernel(int nz, double* zr) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nz) zr[k] = (double)k / (double)(nz - 1);
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t n) {
  // n-th output of SplitMix64 from `seed` (Steele, Lea & Flood 2014)
  uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Initial state: T0 = 1 - (eps+D) z, rho = T0^(m-1) (hydrostatic for T0),
// u = 0, uniform noise of amplitude noise_amp on interior T, E = rho(c_v T
// + g z).  One thread per node; the canonical linear index selects the
// noise draw.
__global__ void init_kernel(Coef c, const double* __restrict__ zr, double* __restrict__ X) {
  long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= c.cnt) return;
  int k = (int)(n / c.plane);
  double z = zr[k];
  double T0 = 1.0 - c.init_delta * z;
  double rho = pow(T0, c.init_expo);
  double T = T0;
  if (k > 0 && k < c.M && c.noise_amp != 0.0) {
    uint64_t r = splitmix64(c.seed, (uint64_t)n + 1);
    double U = (double)(r >> 11) * 0x1.0p-53;
    T = T + c.noise_amp * (2.0 * U - 1.0);
  }
  X[n] = rho;
  for (int f = 1; f < c.nf - 1; ++f) X[n + f * c.cnt] = 0.0;
  X[n + (c.nf - 1) * c.cnt] = rho * (c.cv * T + c.g * z);
}

__global__ void clear_slot_kernel(Shared* sh, int slot) {
  if (threadIdx.x < kMaxParts * 4) sh->smax[slot][threadIdx.x >> 2][threadIdx.x & 3] = 0ull;
}

__global__ void set_scalars_kernel(Shared* sh, double time, int clear_flags) {
  if (threadIdx.x == 0) {
    sh->time = time;
    sh->dt_last = 0.0;
    if (clear_flags) sh->flags = 0u;
  }
}

// max over nodes of |u_a| + c into slot, and the non-finite / positivity
// flag
__global__ __launch_bounds__(256) void dt_kernel(Coef c, Shared* sh, const double* zr,
                                                 int slot, const double* __restrict__ X) {
  double m[3] = {0.0, 0.0, 0.0};
  double md = INFINITY;      // min of rho h^2 (dt_rule = 1)
  bool bad = false;
  const int fz = c.nf - 2;   // rho u_z slot
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < c.cnt;
       n += (long long)gridDim.x * blockDim.x) {
    int k = (int)(n / c.plane);
    double rho = X[n];
    double ri = 1.0 / rho;
    double ux = X[n + c.cnt] * ri;
    double uy = (c.ndim == 3) ? X[n + 2 * c.cnt] * ri : 0.0;
    double uz = X[n + fz * c.cnt] * ri;
    double ke = 0.5 * ((ux * ux + uy * uy) + uz * uz);
    double T = (X[n + (c.nf - 1) * c.cnt] * ri - ke - c.g * zr[k]) * c.icv;
    double cs = sqrt(c.gam_a * T);
    double sx = fabs(ux) + cs, sy = fabs(uy) + cs, sz = fabs(uz) + cs;
    if (c.stretched) sz *= c.zm[(size_t)k * kZM + kZM_IHMIN];   // (|u_z| + c)/h_z,k
    m[0] = fmax(m[0], sx);
    m[1] = fmax(m[1], sy);
    m[2] = fmax(m[2], sz);
    if (c.dt_rule) md = fmin(md, rho * diff_h2(c, k));
    if (!(rho > 0.0) || !(T > 0.0) || !(sx < INFINITY) || !(sy < INFINITY) ||
        !(sz < INFINITY))
      bad = true;
  }
  for (int a = 0; a < 3; ++a) m[a] = wave_max(m[a]);
  if (c.dt_rule) md = wave_min(md);
  unsigned long long anybad = __ballot(bad);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&sh->smax[slot][max_part()][0], d2u(m[0]));
    if (c.ndim == 3) atomicMax(&sh->smax[slot][max_part()][1], d2u(m[1]));
    atomicMax(&sh->smax[slot][max_part()][2], d2u(m[2]));
    if (c.dt_rule) fold_rho_h2(sh, slot, max_part(), md);
    if (anybad) atomicOr(&sh->flags, 1u);
  }
}

__global__ void freeze_dt_kernel(Coef c, Shared* sh, int slot) {
  if (threadIdx.x == 0) {
    Coef cc = c;
    cc.dt_mode = 0;
    sh->dt_frozen = cc.stretched ? step_dt<true>(cc, sh, slot) : step_dt<false>(cc, sh, slot);
  }
}

// Per-row partial sums of rho, rho|u|^2/2, E, rho u_z T_sa, rho u_z |u|^2,
// T over one segment of a row; fixed-order tree reduction.
__global__ __launch_bounds__(kDiagBlock) void diag_rows_kernel(Coef c, const double* zr,
                                                               const double* __restrict__ X,
                                                               double* part, int nb,
                                                               Shared* sh) {
  __shared__ double red[kDiagVals][kDiagBlock];
  const int k = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
  const long long seg = (c.plane + nb - 1) / nb;
  const long long lo = (long long)b * seg;
  const long long hi = min(lo + seg, c.plane);
  const double z = zr[k];
  const double TA = 1.0 - c.D * z;   // adiabatic T_A (Sec. 2)
  const int fz = c.nf - 2;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  bool bad = false;
  for (long long e = lo + t; e < hi; e += kDiagBlock) {
    long long n = (long long)k * c.plane + e;
    double rho = X[n];
    double ri = 1.0 / rho;
    double ux = X[n + c.cnt] * ri;
    double uy = (c.ndim == 3) ? X[n + 2 * c.cnt] * ri : 0.0;
    double uz = X[n + fz * c.cnt] * ri;
    double uu = (ux * ux + uy * uy) + uz * uz;
    double E = X[n + (c.nf - 1) * c.cnt];
    double T = (E * ri - 0.5 * uu - c.g * z) * c.icv;
    acc[0] += rho;
    acc[1] += 0.5 * rho * uu;
    acc[2] += E;
    acc[3] += rho * uz * (T - TA);
    acc[4] += rho * uz * uu;
    acc[5] += T;
    if (!(rho > 0.0) || !(T > 0.0) || !(fabs(E) < INFINITY)) bad = true;
  }
  for (int q = 0; q < 6; ++q) red[q][t] = acc[q];
  __syncthreads();
  for (int w = kDiagBlock / 2; w > 0; w >>= 1) {
    if (t < w)
      for (int q = 0; q < 6; ++q) red[q][t] += red[q][t + w];
    __syncthreads();
  }
  if (t < 6) part[((size_t)k * nb + b) * kDiagVals + t] = red[t][0];
  if (bad) atomicOr(&sh->flags, 1u);
}

// Weighted totals (trapezoid in z) and the Nusselt numbers.  One block.
__global__ __launch_bounds__(kDiagBlock) void diag_final_kernel(Coef c, const double* part,
                                                                int nb, double* out) {
  __shared__ double red[5][kDiagBlock];
  const int t = threadIdx.x;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int k = t; k < c.nz; k += kDiagBlock) {
    // trapezoid weights in units of dz; a stretched grid's dual cells
    double w = c.stretched ? c.zm[(size_t)k * kZM + kZM_W] * c.ihz
                           : (k == 0 || k == c.M) ? 0.5 : 1.0;
    for (int q = 0; q < 5; ++q) {
      double s = 0.0;
      for (int b = 0; b < nb; ++b) s += part[((size_t)k * nb + b) * kDiagVals + q];
      acc[q] += w * s;
    }
  }
  for (int q = 0; q < 5; ++q) red[q][t] = acc[q];
  __syncthreads();
  for (int w = kDiagBlock / 2; w > 0; w >>= 1) {
    if (t < w)
      for (int q = 0; q < 5; ++q) red[q][t] += red[q][t + w];
    __syncthreads();
  }
  if (t == 0) {
    double dV = c.hx * c.hz * ((c.ndim == 3) ? c.hy : 1.0);
    double V = (c.ndim == 3) ? (c.hx * c.nx) * (c.hy * c.ny) : c.hx * c.nx;
    int rows[6] = {0, 1, 2, c.M - 2, c.M - 1, c.M};
    double tm[6];
    for (int i = 0; i < 6; ++i) {
      double s = 0.0;
      for (int b = 0; b < nb; ++b) s += part[((size_t)rows[i] * nb + b) * kDiagVals + 5];
      tm[i] = s / (double)c.plane;
    }
    double mass = red[0][0] * dV, kin = red[1][0] * dV, Etot = red[2][0] * dV;
    double nuc = c.sRP / c.eps * (red[3][0] * dV / V);
    double nuk = c.D * c.sRP / 2.0 * (red[4][0] * dV / V);
    double ib = 0.5 * c.ihz, it = 0.5 * c.ihz;
    if (c.stretched) {   // the plate stencils applied to the heights divide
      ib = c.zm[kZM_IWALL];
      it = c.zm[(size_t)c.M * kZM + kZM_IWALL];
    }
    double gb = ((-3.0 * tm[0] + 4.0 * tm[1]) - tm[2]) * ib;
    double gt = ((3.0 * tm[5] - 4.0 * tm[4]) + tm[3]) * it;
    double nub = -(gb + c.D) / c.eps, nut = -(gt + c.D) / c.eps;
    out[0] = mass;
    out[1] = kin;
    out[2] = Etot;
    out[3] = nub;
    out[4] = nut;
    out[5] = 0.5 * (nub + nut);
    out[6] = (1.0 + nuc) + nuk;
    out[7] = nuc;
    out[8] = nuk;
    for (int i = 0; i < 6; ++i) out[9 + i] = tm[i];
  }
}

// Heights of the nz rows: uniform k/M, or the tanh grid of the stretch
// parameter s, z_k = (1 + tanh(s (2k - M)/M) / tanh s) / 2, whose quotient
// is exactly -1 and 1 at the ends (tanh is odd), so the plates sit at 0, 1.
std::vector<double> grid_heights(double s, int nz) {
  const int M = nz - 1;
  std::vector<double> z(nz);
  if (!(s > 0.0)) {
    for (int k = 0; k < nz; ++k) z[k] = (double)k / (double)M;
    return z;
  }
  const double ts = tanh(s);
  for (int k = 0; k < nz; ++k) {
    const double xi = (2.0 * (double)k - (double)M) / (double)M;
    z[k] = 0.5 * (1.0 + tanh(s * xi) / ts);
  }
  return z;
}

}  // namespace mtvd

// ---------------------------------------------------------------------------
// context

struct mtvd_ctx {
  mtvd_params p;
  Coef c;
  Layout L;
  hipStream_t stream;
  int device;
  double* buf[2];
  unsigned char* ws;
  int cur;        // buffer holding the current state
  int slot;       // max slot holding the dt of the next step
  int64_t step;
  bool bound, have_state;
  int rows_x, rows_z;
  int slots_x, slots_z;   // resident waves of the 2D sweep kernels
  bool timing;
  struct Rec { int axis; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  std::string err;
};

namespace {

int set_err(mtvd_ctx* c, int code, const char* what) {
  if (c) c->err = what;
  return code;
}

int hip_fail(mtvd_ctx* c, hipError_t e, const char* where) {
  if (c) {
    c->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  return MTVD_EHIP;
}

#define HIPCHK(ctx, expr)                               \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
  } while (0)

// The per-row metric table of a stretched grid (kZM doubles per row, the
// kZM_* slots): reciprocals of the face, centred and dual-cell spans, the
// face length, the narrowest face of each node and the two plate stencils.
std::vector<double> grid_metrics(const std::vector<double>& z) {
  const int nz = (int)z.size(), M = nz - 1;
  std::vector<double> m((size_t)nz * kZM, 0.0);
  for (int k = 0; k < nz; ++k) {
    double* r = &m[(size_t)k * kZM];
    if (k < M) {
      r[kZM_HF] = z[k + 1] - z[k];
      r[kZM_IHF] = 1.0 / r[kZM_HF];
    }
    double w, hmin;
    if (k == 0) {
      w = 0.5 * (z[1] - z[0]);
      hmin = z[1] - z[0];
      r[kZM_IWALL] = 1.0 / ((-3.0 * z[0] + 4.0 * z[1]) - z[2]);
    } else if (k == M) {
      w = 0.5 * (z[M] - z[M - 1]);
      hmin = z[M] - z[M - 1];
      r[kZM_IWALL] = 1.0 / ((3.0 * z[M] - 4.0 * z[M - 1]) + z[M - 2]);
    } else {
      w = 0.5 * (z[k + 1] - z[k - 1]);
      hmin = fmin(z[k] - z[k - 1], z[k + 1] - z[k]);
      r[kZM_ICEN] = 1.0 / (z[k + 1] - z[k - 1]);
    }
    r[kZM_W] = w;
    r[kZM_IW] = 1.0 / w;
    r[kZM_IHMIN] = 1.0 / hmin;
    if (k == 0 || k == M) {
      // L_j''(z_plate) of the cubic through the plate and three rows:
      // 2 sum_{l != j} (x0 - z_l) / prod_{l != j} (z_j - z_l)
      const int sgn = (k == 0) ? 1 : -1;
      double zs[4];
      for (int j = 0; j < 4; ++j) zs[j] = z[k + sgn * j];
      for (int j = 0; j < 4; ++j) {
        double num = 0.0, den = 1.0;
        for (int l = 0; l < 4; ++l)
          if (l != j) {
            num += zs[0] - zs[l];
            den *= zs[j] - zs[l];
          }
        r[kZM_D2 + j] = 2.0 * num / den;
      }
    } else {
      const double hm = z[k] - z[k - 1], hp = z[k + 1] - z[k];
      r[kZM_D2 + 0] = 2.0 / (hm * (hm + hp));
      r[kZM_D2 + 1] = -2.0 / (hm * hp);
      r[kZM_D2 + 2] = 2.0 / (hp * (hm + hp));
    }
  }
  return m;
}

// The checks with their reason as a string literal (no allocation).
int validate_c(const mtvd_params* p, const char** why) {
  if (!p) { *why = "null params"; return MTVD_EINVAL; }
  if (p->ndim != 2 && p->ndim != 3) { *why = "ndim must be 2 or 3"; return MTVD_EINVAL; }
  if (p->nx < 1 || p->nz < 5 || (p->ndim == 3 && p->ny < 1)) {
    *why = "grid too small (nx >= 1, ny >= 1, nz >= 5)";
    return MTVD_EINVAL;
  }
  if (p->ndim == 2 && p->ny != 1) { *why = "ny must be 1 in 2D"; return MTVD_EINVAL; }
  double nodes = (double)p->nx * (double)p->ny * (double)p->nz;
  if (nodes * (p->ndim + 2) > 9.0e18 / 8 || p->nz > (1 << 30)) {
    *why = "grid too large";
    return MTVD_EINVAL;
  }
  if (!(p->gamma > 1.0) || !(p->eps > 0.0) || !(p->D > 0.0) || !(p->Ra > 0.0) ||
      !(p->Pr > 0.0) || !(p->aspect > 0.0) || !(p->noise_amp >= 0.0) ||
      !(p->gravity_scale >= 0.0) || !isfinite(p->bulk_coef) || !isfinite(p->Ra)) {
    *why = "physical parameters out of range";
    return MTVD_EINVAL;
  }
  if (!(1.0 - (p->eps + p->D) > 0.0)) { *why = "top plate temperature 1-eps-D <= 0"; return MTVD_EINVAL; }
  if (p->dt_mode != 0 && p->dt_mode != 1) { *why = "dt_mode must be 0 or 1"; return MTVD_EINVAL; }
  if (p->limiter_form != 0 && p->limiter_form != 1) { *why = "limiter_form must be 0 or 1"; return MTVD_EINVAL; }
  if (p->sweep_order != 0 && p->sweep_order != 1) { *why = "sweep_order must be 0 or 1"; return MTVD_EINVAL; }
  if (p->tvd_on != 0 && p->tvd_on != 1) { *why = "tvd_on must be 0 or 1"; return MTVD_EINVAL; }
  if (p->wall_order != 1 && p->wall_order != 2) { *why = "wall_order must be 1 or 2"; return MTVD_EINVAL; }
  if (p->dt_rule != 0 && p->dt_rule != 1) { *why = "dt_rule must be 0 or 1"; return MTVD_EINVAL; }
  if (!(p->stretch >= 0.0) || !(p->stretch <= 10.0)) { *why = "stretch must lie in [0, 10]"; return MTVD_EINVAL; }
  if (p->stretch > 0.0 && p->ndim == 3 && p->nz > 2048) {
    *why = "a stretched 3D grid has at most 2048 rows";   // the L_z kernels keep the heights in LDS
    return MTVD_EINVAL;
  }
  if (!(p->cfl > 0.0) || !(p->cfl <= 1.0)) { *why = "cfl must lie in (0, 1]"; return MTVD_ESTABILITY; }
  // dt_rule = 1 keeps every diffusion number at most cfl/2 by itself
  if (p->dt_rule == 1) return MTVD_OK;
  // diffusion number of the initial state (the acoustic limit sets dt):
  // max(mu(2+|lambda|), K/c_v) * tau / (rho_min h_min^2) <= 1/2
  double hx = p->aspect / p->nx, hz = 1.0 / (p->nz - 1);
  if (p->stretch > 0.0) {
    std::vector<double> z = grid_heights(p->stretch, p->nz);
    hz = z[1] - z[0];   // the tanh grid's narrowest face sits at a plate
  }
  double hmin = fmin(hx, hz);
  if (p->ndim == 3) hmin = fmin(hmin, p->aspect / p->ny);
  double Delta = p->eps + p->D;
  double m = p->gamma * p->D / ((p->gamma - 1.0) * Delta);
  double expo = p->gravity_scale * m - 1.0;
  double rho_min = fmin(1.0, pow(1.0 - Delta, expo));
  double a = (p->gamma - 1.0) / (p->gamma * p->eps * p->D);
  double cmax = sqrt(p->gamma * a * (1.0 + p->noise_amp));
  double tau = 0.5 * p->cfl * hmin / cmax;
  double mu = sqrt(p->Pr / p->Ra);
  double K = 1.0 / (p->eps * p->D * sqrt(p->Ra * p->Pr));
  double cv = 1.0 / (p->gamma * p->eps * p->D);
  double nu = fmax(mu * (2.0 + fabs(p->bulk_coef)), K / cv) * tau / (rho_min * hmin * hmin);
  if (!(nu <= 0.5)) { *why = "diffusion number above 1/2 for this grid and Ra"; return MTVD_ESTABILITY; }
  return MTVD_OK;
}

int validate(const mtvd_params* p, std::string* why) {
  const char* w = "";
  int rc = validate_c(p, &w);
  *why = w;
  return rc;
}

Coef make_coef(const mtvd_params* p) {
  Coef c;
  memset(&c, 0, sizeof(c));
  c.ndim = p->ndim;
  c.nf = p->ndim + 2;
  c.nx = p->nx;
  c.ny = (p->ndim == 3) ? p->ny : 1;
  c.nz = p->nz;
  c.M = p->nz - 1;
  c.plane = (long long)c.nx * c.ny;
  c.cnt = c.plane * c.nz;
  c.hx = p->aspect / p->nx;
  c.hy = (p->ndim == 3) ? p->aspect / p->ny : 1.0;
  c.hz = 1.0 / (double)(p->nz - 1);
  c.ihx = 1.0 / c.hx;
  c.ihy = 1.0 / c.hy;
  c.ihz = 1.0 / c.hz;
  c.gamma = p->gamma;
  c.cv = 1.0 / (p->gamma * p->eps * p->D);
  c.icv = p->gamma * p->eps * p->D;
  c.a = (p->gamma - 1.0) / (p->gamma * p->eps * p->D);
  c.gam_a = p->gamma * c.a;
  c.g = p->gravity_scale / p->eps;
  c.mu = sqrt(p->Pr / p->Ra);
  c.K = 1.0 / (p->eps * p->D * sqrt(p->Ra * p->Pr));
  c.lam = p->bulk_coef;
  c.Tb = 1.0;
  c.Tt = 1.0 - (p->eps + p->D);
  c.cfl = p->cfl;
  c.D = p->D;
  c.eps = p->eps;
  c.sRP = sqrt(p->Ra * p->Pr);
  c.init_delta = p->eps + p->D;
  double m = p->gamma * p->D / ((p->gamma - 1.0) * c.init_delta);
  c.init_expo = p->gravity_scale * m - 1.0;
  c.noise_amp = p->noise_amp;
  c.seed = p->seed;
  c.limiter_form = p->limiter_form;
  c.tvd_on = p->tvd_on;
  c.wall_order = p->wall_order;
  c.dt_mode = p->dt_mode;
  c.dt_rule = p->dt_rule;
  c.kappa = fmax(c.mu * (2.0 + fabs(c.lam)), c.K / c.cv);
  c.hmh = (p->ndim == 3) ? fmin(c.hx, c.hy) : c.hx;
  c.hm2 = fmin(c.hmh, c.hz) * fmin(c.hmh, c.hz);
  c.stretched = p->stretch > 0.0;
  c.zm = nullptr;   // set when the workspace is bound
  return c;
}

Shared* shared_of(mtvd_ctx* c) { return (Shared*)(c->ws + c->L.shared); }
double* zrow_of(mtvd_ctx* c) { return (double*)(c->ws + c->L.zrow); }

int default_rows(const mtvd_ctx* c, int axis) {
  return default_rows_for(c->c, axis == 2 ? c->slots_z : c->slots_x, axis);
}

hipError_t take_event(mtvd_ctx* c, hipEvent_t* ev) {
  if (!c->pool.empty()) {
    *ev = c->pool.back();
    c->pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(ev);
}

hipError_t sweep_launch(mtvd_ctx* c, int axis, int first, bool fuse) {
  const double* X = c->buf[c->cur];
  double* Y = c->buf[c->cur ^ 1];
  int kc = (axis == 2) ? c->rows_z : c->rows_x;
  if (kc <= 0) kc = default_rows(c, axis);
  hipError_t e;
  mtvd_ctx::Rec rec{axis, nullptr, nullptr};
  if (c->timing) {
    if ((e = take_event(c, &rec.a)) != hipSuccess) return e;
    if ((e = take_event(c, &rec.b)) != hipSuccess) return e;
    if ((e = hipEventRecord(rec.a, c->stream)) != hipSuccess) return e;
  }
  if (c->c.ndim == 2)
    e = launch_sweep_2d(axis, c->c, shared_of(c), zrow_of(c), c->slot, first, fuse, X, Y, kc,
                        c->stream);
  else
    e = launch_sweep_3d(axis, c->c, shared_of(c), zrow_of(c), c->slot, first, fuse, X, Y, kc,
                        c->stream);
  if (e == hipSuccess) c->cur ^= 1;
  if (c->timing) {
    hipError_t e2 = hipEventRecord(rec.b, c->stream);
    if (e == hipSuccess) e = e2;
    c->recs.push_back(rec);
  }
  return e;
}

// dt of the current state into the current slot (and the frozen dt)
int refresh_dt(mtvd_ctx* c) {
  Shared* sh = shared_of(c);
  clear_slot_kernel<<<1, 64, 0, c->stream>>>(sh, c->slot);
  HIPCHK(c, hipGetLastError());
  long long blocks = (c->c.cnt + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  dt_kernel<<<(int)blocks, 256, 0, c->stream>>>(c->c, sh, zrow_of(c), c->slot,
                                                c->buf[c->cur]);
  HIPCHK(c, hipGetLastError());
  if (c->p.dt_mode == 1) {
    freeze_dt_kernel<<<1, 64, 0, c->stream>>>(c->c, sh, c->slot);
    HIPCHK(c, hipGetLastError());
  }
  return MTVD_OK;
}

// max over the partial maxima of a slot, as step_dt takes it on the device
void host_slot_max(const Shared& hs, int slot, double S[3]) {
  for (int a = 0; a < 3; ++a) {
    unsigned long long m = 0ull;
    for (int q = 0; q < kMaxParts; ++q) m = hs.smax[slot][q][a] > m ? hs.smax[slot][q][a] : m;
    memcpy(&S[a], &m, sizeof(double));
  }
}

// dt of the step a slot's maxima give, the same arithmetic as step_dt on
// the device (entry 3: the complement of the minimum of rho h^2)
double host_dt(const Coef& c, const Shared& hs, int slot) {
  double S[3];
  host_slot_max(hs, slot, S);
  double m = fmin(c.hx / S[0], (c.stretched ? 1.0 : c.hz) / S[2]);
  if (c.ndim == 3) m = fmin(m, c.hy / S[1]);
  if (c.dt_rule) {
    unsigned long long b = 0ull;
    for (int q = 0; q < kMaxParts; ++q) b = hs.smax[slot][q][3] > b ? hs.smax[slot][q][3] : b;
    b = ~b;
    double rh2;
    memcpy(&rh2, &b, sizeof(double));
    m = fmin(m, rh2 / c.kappa);
  }
  return c.cfl * m;
}

int read_flags(mtvd_ctx* c, unsigned int* flags) {
  HIPCHK(c, hipMemcpyAsync(flags, &shared_of(c)->flags, sizeof(unsigned int),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MTVD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

void mtvd_default_params(mtvd_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->ndim = 2;
  p->nx = 256;
  p->ny = 1;
  p->nz = 64;
  p->aspect = 4.0;
  p->gamma = 1.4;
  p->Pr = 1.0;
  p->Ra = 1e6;
  p->eps = 0.1;
  p->D = 0.4;
  p->cfl = 0.5;
  p->seed = 0;
  p->noise_amp = 1e-3;
  p->dt_mode = 0;
  p->bulk_coef = -2.0 / 3.0;
  p->limiter_form = 0;
  p->sweep_order = 0;
  p->tvd_on = 1;
  p->gravity_scale = 1.0;
  p->wall_order = 2;
}

int mtvd_grid_heights(const mtvd_params* p, double* z, size_t count) {
  std::string why;
  int rc = validate(p, &why);
  if (rc != MTVD_OK && rc != MTVD_ESTABILITY) return rc;
  if (!z) return MTVD_EINVAL;
  if (count < (size_t)p->nz) return MTVD_ESIZE;
  std::vector<double> h = grid_heights(p->stretch, p->nz);
  for (int k = 0; k < p->nz; ++k) z[k] = h[k];
  return MTVD_OK;
}

int mtvd_state_bytes(const mtvd_params* p, size_t* state_bytes, size_t* workspace_bytes) {
  std::string why;
  int rc = validate(p, &why);
  if (rc != MTVD_OK && rc != MTVD_ESTABILITY) return rc;
  Layout L = layout_of(p);
  size_t nodes = (size_t)p->nx * (size_t)(p->ndim == 3 ? p->ny : 1) * (size_t)p->nz;
  if (state_bytes) *state_bytes = nodes * (size_t)(p->ndim + 2) * sizeof(double);
  if (workspace_bytes) *workspace_bytes = L.total;
  return MTVD_OK;
}

int mtvd_create(const mtvd_params* p, void* hip_stream, mtvd_ctx** out) {
  if (!out) return MTVD_EINVAL;
  *out = nullptr;
  std::string why;
  int rc = validate(p, &why);
  if (rc != MTVD_OK) {
    fprintf(stderr, "mtvd_create: %s\n", why.c_str());
    return rc;
  }
  mtvd_ctx* c = new (std::nothrow) mtvd_ctx();
  if (!c) return MTVD_EINVAL;
  c->p = *p;
  c->c = make_coef(p);
  c->L = layout_of(p);
  c->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return MTVD_EHIP;
  }
  c->buf[0] = c->buf[1] = nullptr;
  c->ws = nullptr;
  c->cur = 0;
  c->slot = 0;
  c->step = 0;
  c->bound = c->have_state = false;
  c->rows_x = c->rows_z = 0;
  c->slots_x = c->slots_z = 0;
  if (c->c.ndim == 2) {
    c->slots_x = wave_slots_2d(0, false);
    c->slots_z = wave_slots_2d(2, false);
  }
  c->timing = false;
  *out = c;
  return MTVD_OK;
}

int mtvd_bind(mtvd_ctx* c, double* buf_a, double* buf_b, void* workspace) {
  if (!c) return MTVD_EINVAL;
  if (!buf_a || !buf_b || !workspace) return set_err(c, MTVD_ESIZE, "null buffer");
  if (buf_a == buf_b || (void*)buf_a == workspace || (void*)buf_b == workspace)
    return set_err(c, MTVD_ESIZE, "buffers must be distinct");
  if (((uintptr_t)buf_a | (uintptr_t)buf_b | (uintptr_t)workspace) % kAlign)
    return set_err(c, MTVD_ESIZE, "buffers must be 256-byte aligned");
  c->buf[0] = buf_a;
  c->buf[1] = buf_b;
  c->ws = (unsigned char*)workspace;
  c->cur = 0;
  c->slot = 0;
  c->bound = true;
  c->have_state = false;
  HIPCHK(c, hipMemsetAsync(c->ws, 0, c->L.total, c->stream));
  if (c->c.stretched) {
    // heights and metrics of the tanh grid, made on the host (the same
    // libm tanh for every row) and copied once
    std::vector<double> z = grid_heights(c->p.stretch, c->c.nz);
    std::vector<double> m = grid_metrics(z);
    double* zm = (double*)(c->ws + c->L.zmet);
    HIPCHK(c, hipMemcpyAsync(zrow_of(c), z.data(), sizeof(double) * z.size(),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(zm, m.data(), sizeof(double) * m.size(), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->c.zm = zm;
  } else {
    zrow_kernel<<<(c->c.nz + 255) / 256, 256, 0, c->stream>>>(c->c.nz, zrow_of(c));
    HIPCHK(c, hipGetLastError());
  }
  return MTVD_OK;
}

int mtvd_init_state(mtvd_ctx* c) {
  if (!c) return MTVD_EINVAL;
  if (!c->bound) return set_err(c, MTVD_ESTATE, "mtvd_bind first");
  c->cur = 0;
  c->slot = 0;
  c->step = 0;
  long long blocks = (c->c.cnt + 255) / 256;
  init_kernel<<<(unsigned)blocks, 256, 0, c->stream>>>(c->c, zrow_of(c), c->buf[0]);
  HIPCHK(c, hipGetLastError());
  set_scalars_kernel<<<1, 64, 0, c->stream>>>(shared_of(c), 0.0, 1);
  HIPCHK(c, hipGetLastError());
  int rc = refresh_dt(c);
  if (rc) return rc;
  c->have_state = true;
  return MTVD_OK;
}

int mtvd_step(mtvd_ctx* c, int32_t nsteps) {
  if (!c) return MTVD_EINVAL;
  if (nsteps < 0) return set_err(c, MTVD_EINVAL, "nsteps < 0");
  if (!c->have_state) return set_err(c, MTVD_ESTATE, "no state: mtvd_init_state or mtvd_set_state first");
  // L_x L_y L_z L_x L_y L_z, rightmost first (Sec. 3.1, time_step)
  static const int o2[2][4] = {{2, 0, 2, 0}, {2, 0, 0, 2}};
  static const int o3[2][6] = {{2, 1, 0, 2, 1, 0}, {2, 1, 0, 0, 1, 2}};
  const int ns = (c->c.ndim == 3) ? 6 : 4;
  const int* order = (c->c.ndim == 3) ? o3[c->p.sweep_order] : o2[c->p.sweep_order];
  const bool track = (c->p.dt_mode == 0);
  for (int s = 0; s < nsteps; ++s) {
    for (int o = 0; o < ns; ++o) {
      hipError_t e = sweep_launch(c, order[o], o == 0 ? 1 : 0, track && o == ns - 1);
      if (e != hipSuccess) return hip_fail(c, e, "sweep launch");
    }
    if (track) c->slot ^= 1;
    c->step += 1;
  }
  return MTVD_OK;
}

int mtvd_sweep(mtvd_ctx* c, int32_t axis) {
  if (!c) return MTVD_EINVAL;
  if (!c->have_state) return set_err(c, MTVD_ESTATE, "no state");
  if (axis < 0 || axis > 2 || (axis == 1 && c->c.ndim != 3))
    return set_err(c, MTVD_EINVAL, "bad axis");
  if (c->p.dt_mode == 0) {
    int rc = refresh_dt(c);
    if (rc) return rc;
  }
  hipError_t e = sweep_launch(c, axis, 0, false);
  if (e != hipSuccess) return hip_fail(c, e, "sweep launch");
  // the next step's dt belongs to the new state
  if (c->p.dt_mode == 0) return refresh_dt(c);
  return MTVD_OK;
}

int mtvd_diagnostics(mtvd_ctx* c, mtvd_diag* out) {
  if (!c || !out) return MTVD_EINVAL;
  if (!c->have_state) return set_err(c, MTVD_ESTATE, "no state");
  Shared* sh = shared_of(c);
  double* part = (double*)(c->ws + c->L.part);
  double* dout = (double*)(c->ws + c->L.out);
  dim3 grid(c->L.diag_nb, c->c.nz);
  diag_rows_kernel<<<grid, kDiagBlock, 0, c->stream>>>(c->c, zrow_of(c), c->buf[c->cur], part,
                                                       c->L.diag_nb, sh);
  HIPCHK(c, hipGetLastError());
  diag_final_kernel<<<1, kDiagBlock, 0, c->stream>>>(c->c, part, c->L.diag_nb, dout);
  HIPCHK(c, hipGetLastError());
  double host[kDiagOut];
  Shared hs;
  HIPCHK(c, hipMemcpyAsync(host, dout, sizeof(double) * 15, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&hs, sh, sizeof(Shared), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  memset(out, 0, sizeof(*out));
  out->step = c->step;
  out->time = hs.time;
  if (c->p.dt_mode == 1) {
    out->dt = hs.dt_frozen;
  } else {
    out->dt = host_dt(c->c, hs, c->slot);
  }
  out->mass = host[0];
  out->kinetic = host[1];
  out->total_energy = host[2];
  out->nu_bottom = host[3];
  out->nu_top = host[4];
  out->nu_mean = host[5];
  out->nu_bulk = host[6];
  out->nu_conv = host[7];
  out->nu_kin = host[8];
  for (int i = 0; i < 6; ++i) out->tmean[i] = host[9 + i];
  out->flags = (int32_t)hs.flags;
  return hs.flags ? MTVD_ENONFINITE : MTVD_OK;
}

int mtvd_profiles(mtvd_ctx* c, double* out, size_t count) {
  if (!c || !out) return MTVD_EINVAL;
  if (!c->have_state) return set_err(c, MTVD_ESTATE, "no state");
  const size_t n = (size_t)kNumProfiles * (size_t)c->c.nz;
  if (count < n) return set_err(c, MTVD_ESIZE, "profile array too small");
  double* part = (double*)(c->ws + c->L.ppart);
  double* dout = (double*)(c->ws + c->L.pout);
  hipError_t e = launch_profiles(c->c, zrow_of(c), c->buf[c->cur], part, c->L.diag_nb, dout,
                                 c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "profiles launch");
  HIPCHK(c, hipMemcpyAsync(out, dout, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  unsigned int flags = 0;
  int rc = read_flags(c, &flags);
  if (rc) return rc;
  return flags ? MTVD_ENONFINITE : MTVD_OK;
}

int mtvd_get_state(mtvd_ctx* c, double* host, size_t count) {
  if (!c || !host) return MTVD_EINVAL;
  if (!c->have_state) return set_err(c, MTVD_ESTATE, "no state");
  if (count != (size_t)c->c.cnt * c->c.nf) return set_err(c, MTVD_ESIZE, "count mismatch");
  HIPCHK(c, hipMemcpyAsync(host, c->buf[c->cur], sizeof(double) * count, hipMemcpyDeviceToHost,
                           c->stream));
  unsigned int flags = 0;
  int rc = read_flags(c, &flags);
  if (rc) return rc;
  return flags ? MTVD_ENONFINITE : MTVD_OK;
}

int mtvd_set_state(mtvd_ctx* c, const double* host, size_t count, double time, int64_t step) {
  if (!c || !host) return MTVD_EINVAL;
  if (!c->bound) return set_err(c, MTVD_ESTATE, "mtvd_bind first");
  if (count != (size_t)c->c.cnt * c->c.nf) return set_err(c, MTVD_ESIZE, "count mismatch");
  c->cur = 0;
  c->slot = 0;
  HIPCHK(c, hipMemcpyAsync(c->buf[0], host, sizeof(double) * count, hipMemcpyHostToDevice,
                           c->stream));
  set_scalars_kernel<<<1, 64, 0, c->stream>>>(shared_of(c), time, 1);
  HIPCHK(c, hipGetLastError());
  int rc = refresh_dt(c);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->step = step;
  c->have_state = true;
  return MTVD_OK;
}

int mtvd_current(const mtvd_ctx* c, int32_t* which) {
  if (!c || !which) return MTVD_EINVAL;
  *which = c->cur;
  return MTVD_OK;
}

int mtvd_sync(mtvd_ctx* c) {
  if (!c) return MTVD_EINVAL;
  if (!c->bound) return MTVD_OK;
  unsigned int flags = 0;
  int rc = read_flags(c, &flags);
  if (rc) return rc;
  return flags ? MTVD_ENONFINITE : MTVD_OK;
}

int mtvd_set_tiling(mtvd_ctx* c, int32_t rows_x, int32_t rows_z) {
  if (!c || rows_x < 0 || rows_z < 0) return MTVD_EINVAL;
  c->rows_x = rows_x;
  c->rows_z = rows_z;
  return MTVD_OK;
}

int mtvd_set_timing(mtvd_ctx* c, int32_t enable) {
  if (!c) return MTVD_EINVAL;
  c->timing = enable != 0;
  return MTVD_OK;
}

int mtvd_kernel_times(mtvd_ctx* c, double ms[3], int64_t counts[3]) {
  if (!c || !ms || !counts) return MTVD_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto& r : c->recs) {
    float t = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&t, r.a, r.b));
    ms[r.axis] += t;
    counts[r.axis] += 1;
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
  return MTVD_OK;
}

int mtvd_destroy(mtvd_ctx* c) {
  if (!c) return MTVD_OK;
  for (auto& r : c->recs) {
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  for (auto ev : c->pool) (void)hipEventDestroy(ev);
  delete c;
  return MTVD_OK;
}

const char* mtvd_strerror(int status) {
  switch (status) {
    case MTVD_OK: return "ok";
    case MTVD_EINVAL: return "invalid argument";
    case MTVD_ESIZE: return "buffer size, alignment or count";
    case MTVD_ESTABILITY: return "cfl or diffusion-number limit";
    case MTVD_ESTATE: return "call out of order";
    case MTVD_ENONFINITE: return "non-finite or non-positive rho/T on the device";
    case MTVD_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* mtvd_last_error(const mtvd_ctx* c) { return c ? c->err.c_str() : ""; }

}  // extern "C"

// ---------------------------------------------------------------------------
// batches of independent 2D boxes

struct mtvd_batch {
  int nbox;
  std::vector<mtvd_params> p;
  std::vector<Coef> c;
  std::vector<long long> off;     // state offset of each box (doubles)
  std::vector<int> zoff;          // plate-table offset of each box
  std::vector<int> kcx, kcz;      // rows per wave (0 = default)
  int kdef_x, kdef_z;             // the default's row bound per operator
  hipStream_t stream;
  hipStream_t cap;                // private stream for graph capture
  int device;
  double* buf[2];
  unsigned char* ws;
  int cur, slot;
  std::vector<int64_t> step;
  bool bound, have_state, items_dirty;
  size_t state_doubles;
  size_t o_sh, o_desc, o_items, o_z, o_part, o_out, total;
  int items_cap;                  // capacity of each item list
  int nitems_x, nitems_z;
  int diag_nb_max;
  hipGraphExec_t g2[2];
  bool have_g2[2];
  std::string err;
};

namespace {

int berr(mtvd_batch* b, int code, const std::string& what) {
  if (b) b->err = what;
  return code;
}

#define BHIP(b, expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return berr(b, MTVD_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// item capacity: every box at the smallest tiling (4 rows per wave)
int item_capacity(const std::vector<Coef>& cs) {
  long long n = 0;
  for (const auto& c : cs) n += (long long)strips_2d(c.nx) * ((c.nz + 3) / 4);
  return (int)n;
}

struct BatchLayout {
  size_t o_sh, o_desc, o_items, o_z, o_part, o_out, total, state_doubles;
  std::vector<long long> off;
  std::vector<int> zoff;
  int items_cap, diag_nb_max;
};

BatchLayout batch_layout(const mtvd_params* ps, int nbox, const std::vector<Coef>& cs) {
  BatchLayout L;
  size_t so = 0;
  int zo = 0;
  int nbmax = 1;
  int nzmax = 1;
  for (int b = 0; b < nbox; ++b) {
    L.off.push_back((long long)so);
    L.zoff.push_back(zo);
    so += (size_t)cs[b].nf * (size_t)cs[b].cnt;
    so = (so + 31) / 32 * 32;                 // 256-byte boundary per box
    zo += cs[b].nz;
    Layout l1 = layout_of(&ps[b]);
    if (l1.diag_nb > nbmax) nbmax = l1.diag_nb;
    if (cs[b].nz > nzmax) nzmax = cs[b].nz;
  }
  L.state_doubles = so;
  L.items_cap = item_capacity(cs);
  L.diag_nb_max = nbmax;
  size_t off = 0;
  L.o_sh = off;
  off = align_up(off + sizeof(Shared) * (size_t)nbox);
  L.o_desc = off;
  off = align_up(off + sizeof(BoxDesc) * (size_t)nbox);
  L.o_items = off;
  off = align_up(off + sizeof(int4) * 2 * (size_t)L.items_cap);
  L.o_z = off;
  off = align_up(off + sizeof(double) * (size_t)zo);
  L.o_part = off;
  off = align_up(off + sizeof(double) * (size_t)nzmax * nbmax * kDiagVals);
  L.o_out = off;
  off = align_up(off + sizeof(double) * kDiagOut);
  L.total = off;
  return L;
}

Shared* bsh(mtvd_batch* b) { return (Shared*)(b->ws + b->o_sh); }
double* bz(mtvd_batch* b) { return (double*)(b->ws + b->o_z); }

// descriptor table and the two work lists (largest boxes first)
int upload_items(mtvd_batch* b) {
  std::vector<BoxDesc> d(b->nbox);
  std::vector<int> order(b->nbox);
  for (int i = 0; i < b->nbox; ++i) {
    order[i] = i;
    memset(&d[i], 0, sizeof(BoxDesc));
    d[i].c = b->c[i];
    d[i].off = b->off[i];
    d[i].zoff = b->zoff[i];
    d[i].kc_x = batch_rows(b->c[i], b->kcx[i], b->kdef_x);
    d[i].kc_z = batch_rows(b->c[i], b->kcz[i], b->kdef_z);
    d[i].nstrips = strips_2d(b->c[i].nx);
  }
  for (int i = 1; i < b->nbox; ++i)
    for (int j = i; j > 0 && b->c[order[j]].cnt > b->c[order[j - 1]].cnt; --j)
      std::swap(order[j], order[j - 1]);
  std::vector<int4> items[2];
  for (int a = 0; a < 2; ++a) {
    for (int ib : order) {
      int kc = a == 0 ? d[ib].kc_x : d[ib].kc_z;
      int nch = (b->c[ib].nz + kc - 1) / kc;
      for (int ch = 0; ch < nch; ++ch)
        for (int st = 0; st < d[ib].nstrips; ++st)
          items[a].push_back(make_int4(ib, st, ch, (st == 0 && ch == 0) ? 1 : 0));
    }
    if ((int)items[a].size() > b->items_cap)
      return berr(b, MTVD_EINVAL, "work list larger than its capacity");
  }
  b->nitems_x = (int)items[0].size();
  b->nitems_z = (int)items[1].size();
  int4* dev = (int4*)(b->ws + b->o_items);
  BHIP(b, hipMemcpyAsync(b->ws + b->o_desc, d.data(), sizeof(BoxDesc) * b->nbox,
                         hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipMemcpyAsync(dev, items[0].data(), sizeof(int4) * b->nitems_x,
                         hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipMemcpyAsync(dev + b->items_cap, items[1].data(), sizeof(int4) * b->nitems_z,
                         hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  for (int a = 0; a < 2; ++a)
    if (b->have_g2[a]) {
      (void)hipGraphExecDestroy(b->g2[a]);
      b->have_g2[a] = false;
    }
  b->items_dirty = false;
  return MTVD_OK;
}

// one step of every box on stream s, with the given max slot
hipError_t batch_step_on(mtvd_batch* b, hipStream_t s, int slot) {
  static const int o2[2][4] = {{2, 0, 2, 0}, {2, 0, 0, 2}};
  const int* order = o2[b->p[0].sweep_order];
  const bool track = b->p[0].dt_mode == 0;
  const BoxDesc* desc = (const BoxDesc*)(b->ws + b->o_desc);
  const int4* items = (const int4*)(b->ws + b->o_items);
  int cur = b->cur;
  for (int o = 0; o < 4; ++o) {
    int ax = order[o];
    const int4* it = ax == 0 ? items : items + b->items_cap;
    int n = ax == 0 ? b->nitems_x : b->nitems_z;
    hipError_t e = launch_batch_2d(ax, desc, it, n, bsh(b), bz(b), slot, o == 0 ? 1 : 0,
                                   track && o == 3, b->buf[cur], b->buf[cur ^ 1], s);
    if (e != hipSuccess) return e;
    cur ^= 1;
  }
  return hipSuccess;
}

int batch_refresh_dt(mtvd_batch* b, int box) {
  Shared* sh = bsh(b) + box;
  const Coef& c = b->c[box];
  clear_slot_kernel<<<1, 64, 0, b->stream>>>(sh, b->slot);
  BHIP(b, hipGetLastError());
  long long blocks = (c.cnt + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  dt_kernel<<<(int)blocks, 256, 0, b->stream>>>(c, sh, bz(b) + b->zoff[box], b->slot,
                                                b->buf[b->cur] + b->off[box]);
  BHIP(b, hipGetLastError());
  if (b->p[box].dt_mode == 1) {
    freeze_dt_kernel<<<1, 64, 0, b->stream>>>(c, sh, b->slot);
    BHIP(b, hipGetLastError());
  }
  return MTVD_OK;
}

// The rules every box of a batch must meet: valid parameters (a diffusion
// number above 1/2 is tolerated where only sizes are asked for), 2D, and the
// dt_mode and sweep_order of the first box.
int batch_check(const mtvd_params* boxes, int nbox, bool sizes_only, std::string* why) {
  if (!boxes || nbox < 1) {
    *why = "no boxes";
    return MTVD_EINVAL;
  }
  for (int i = 0; i < nbox; ++i) {
    std::string w;
    int rc = validate(&boxes[i], &w);
    if (rc != MTVD_OK && !(sizes_only && rc == MTVD_ESTABILITY)) {
      *why = "box " + std::to_string(i) + ": " + w;
      return rc;
    }
    if (boxes[i].ndim != 2) {
      *why = "box " + std::to_string(i) + ": batches hold 2D boxes only";
      return MTVD_EINVAL;
    }
    if (boxes[i].stretch != 0.0) {
      *why = "box " + std::to_string(i) + ": batches use the uniform z grid";
      return MTVD_EINVAL;
    }
    if (boxes[i].dt_mode != boxes[0].dt_mode || boxes[i].sweep_order != boxes[0].sweep_order) {
      *why = "box " + std::to_string(i) + ": dt_mode and sweep_order differ from box 0";
      return MTVD_EINVAL;
    }
  }
  return MTVD_OK;
}

}  // namespace

extern "C" {

int mtvd_batch_bytes(const mtvd_params* boxes, int32_t nbox, size_t* state_bytes,
                     size_t* workspace_bytes) {
  std::string why;
  int rc = batch_check(boxes, nbox, true, &why);
  if (rc != MTVD_OK) return rc;
  std::vector<Coef> cs;
  for (int i = 0; i < nbox; ++i) cs.push_back(make_coef(&boxes[i]));
  BatchLayout L = batch_layout(boxes, nbox, cs);
  if (state_bytes) *state_bytes = L.state_doubles * sizeof(double);
  if (workspace_bytes) *workspace_bytes = L.total;
  return MTVD_OK;
}

int mtvd_batch_create(const mtvd_params* boxes, int32_t nbox, void* hip_stream,
                      mtvd_batch** out) {
  if (!out) return MTVD_EINVAL;
  *out = nullptr;
  std::string why;
  int rc = batch_check(boxes, nbox, false, &why);
  if (rc != MTVD_OK) {
    fprintf(stderr, "mtvd_batch_create: %s\n", why.c_str());
    return rc;
  }
  mtvd_batch* b = new (std::nothrow) mtvd_batch();
  if (!b) return MTVD_EINVAL;
  b->nbox = nbox;
  for (int i = 0; i < nbox; ++i) {
    b->p.push_back(boxes[i]);
    b->c.push_back(make_coef(&boxes[i]));
  }
  BatchLayout L = batch_layout(boxes, nbox, b->c);
  b->off = L.off;
  b->zoff = L.zoff;
  b->kcx.assign(nbox, 0);
  b->kcz.assign(nbox, 0);
  b->kdef_x = batch_default_k(b->c, wave_slots_2d(0, false));
  b->kdef_z = batch_default_k(b->c, wave_slots_2d(2, false));
  b->o_sh = L.o_sh;
  b->o_desc = L.o_desc;
  b->o_items = L.o_items;
  b->o_z = L.o_z;
  b->o_part = L.o_part;
  b->o_out = L.o_out;
  b->total = L.total;
  b->items_cap = L.items_cap;
  b->diag_nb_max = L.diag_nb_max;
  b->state_doubles = L.state_doubles;
  b->stream = (hipStream_t)hip_stream;
  b->buf[0] = b->buf[1] = nullptr;
  b->ws = nullptr;
  b->cur = b->slot = 0;
  b->step.assign(nbox, 0);
  b->bound = b->have_state = false;
  b->items_dirty = true;
  b->nitems_x = b->nitems_z = 0;
  b->have_g2[0] = b->have_g2[1] = false;
  if (hipGetDevice(&b->device) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return MTVD_EHIP;
  }
  *out = b;
  return MTVD_OK;
}

int mtvd_batch_bind(mtvd_batch* b, double* buf_a, double* buf_b, void* workspace) {
  if (!b) return MTVD_EINVAL;
  if (!buf_a || !buf_b || !workspace || buf_a == buf_b)
    return berr(b, MTVD_ESIZE, "null or repeated buffer");
  if (((uintptr_t)buf_a | (uintptr_t)buf_b | (uintptr_t)workspace) % kAlign)
    return berr(b, MTVD_ESIZE, "buffers must be 256-byte aligned");
  b->buf[0] = buf_a;
  b->buf[1] = buf_b;
  b->ws = (unsigned char*)workspace;
  b->cur = b->slot = 0;
  b->bound = true;
  b->have_state = false;
  BHIP(b, hipMemsetAsync(b->ws, 0, b->o_items, b->stream));
  for (int i = 0; i < b->nbox; ++i) {
    zrow_kernel<<<(b->c[i].nz + 255) / 256, 256, 0, b->stream>>>(b->c[i].nz, bz(b) + b->zoff[i]);
    BHIP(b, hipGetLastError());
  }
  return upload_items(b);
}

int mtvd_batch_offset(const mtvd_batch* b, int32_t box, size_t* offset) {
  if (!b || !offset || box < 0 || box >= b->nbox) return MTVD_EINVAL;
  *offset = (size_t)b->off[box];
  return MTVD_OK;
}

int mtvd_batch_init_state(mtvd_batch* b) {
  if (!b) return MTVD_EINVAL;
  if (!b->bound) return berr(b, MTVD_ESTATE, "mtvd_batch_bind first");
  b->cur = b->slot = 0;
  for (int i = 0; i < b->nbox; ++i) {
    const Coef& c = b->c[i];
    init_kernel<<<(unsigned)((c.cnt + 255) / 256), 256, 0, b->stream>>>(
        c, bz(b) + b->zoff[i], b->buf[0] + b->off[i]);
    BHIP(b, hipGetLastError());
    set_scalars_kernel<<<1, 64, 0, b->stream>>>(bsh(b) + i, 0.0, 1);
    BHIP(b, hipGetLastError());
    int rc = batch_refresh_dt(b, i);
    if (rc) return rc;
    b->step[i] = 0;
  }
  b->have_state = true;
  return MTVD_OK;
}

int mtvd_batch_step(mtvd_batch* b, int32_t nsteps) {
  if (!b) return MTVD_EINVAL;
  if (nsteps < 0) return berr(b, MTVD_EINVAL, "nsteps < 0");
  if (!b->have_state) return berr(b, MTVD_ESTATE, "no state");
  if (b->items_dirty) {
    int rc = upload_items(b);
    if (rc) return rc;
  }
  const bool track = b->p[0].dt_mode == 0;
  int left = nsteps;
  while (left >= 2) {
    int s0 = b->slot;
    if (!b->have_g2[s0]) {
      hipGraph_t g;
      BHIP(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
      hipError_t e1 = batch_step_on(b, b->cap, s0);
      hipError_t e2 = batch_step_on(b, b->cap, track ? (s0 ^ 1) : s0);
      hipError_t e3 = hipStreamEndCapture(b->cap, &g);
      if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
        return berr(b, MTVD_EHIP, "graph capture failed");
      hipError_t e4 = hipGraphInstantiate(&b->g2[s0], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e4 != hipSuccess) return berr(b, MTVD_EHIP, "graph instantiate failed");
      b->have_g2[s0] = true;
    }
    BHIP(b, hipGraphLaunch(b->g2[s0], b->stream));
    left -= 2;
    for (auto& s : b->step) s += 2;
  }
  if (left == 1) {
    BHIP(b, batch_step_on(b, b->stream, b->slot));
    if (track) b->slot ^= 1;
    for (auto& s : b->step) s += 1;
  }
  return MTVD_OK;
}

int mtvd_batch_diagnostics(mtvd_batch* b, int32_t box, mtvd_diag* out) {
  if (!b || !out || box < 0 || box >= b->nbox) return MTVD_EINVAL;
  if (!b->have_state) return berr(b, MTVD_ESTATE, "no state");
  const Coef& c = b->c[box];
  Layout l1 = layout_of(&b->p[box]);
  double* part = (double*)(b->ws + b->o_part);
  double* dout = (double*)(b->ws + b->o_out);
  Shared* sh = bsh(b) + box;
  dim3 grid(l1.diag_nb, c.nz);
  diag_rows_kernel<<<grid, kDiagBlock, 0, b->stream>>>(c, bz(b) + b->zoff[box],
                                                       b->buf[b->cur] + b->off[box], part,
                                                       l1.diag_nb, sh);
  BHIP(b, hipGetLastError());
  diag_final_kernel<<<1, kDiagBlock, 0, b->stream>>>(c, part, l1.diag_nb, dout);
  BHIP(b, hipGetLastError());
  double host[kDiagOut];
  Shared hs;
  BHIP(b, hipMemcpyAsync(host, dout, sizeof(double) * 15, hipMemcpyDeviceToHost, b->stream));
  BHIP(b, hipMemcpyAsync(&hs, sh, sizeof(Shared), hipMemcpyDeviceToHost, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  memset(out, 0, sizeof(*out));
  out->step = b->step[box];
  out->time = hs.time;
  if (b->p[box].dt_mode == 1) {
    out->dt = hs.dt_frozen;
  } else {
    out->dt = host_dt(c, hs, b->slot);
  }
  out->mass = host[0];
  out->kinetic = host[1];
  out->total_energy = host[2];
  out->nu_bottom = host[3];
  out->nu_top = host[4];
  out->nu_mean = host[5];
  out->nu_bulk = host[6];
  out->nu_conv = host[7];
  out->nu_kin = host[8];
  for (int i = 0; i < 6; ++i) out->tmean[i] = host[9 + i];
  out->flags = (int32_t)hs.flags;
  return hs.flags ? MTVD_ENONFINITE : MTVD_OK;
}

int mtvd_batch_get_state(mtvd_batch* b, int32_t box, double* host, size_t count) {
  if (!b || !host || box < 0 || box >= b->nbox) return MTVD_EINVAL;
  if (!b->have_state) return berr(b, MTVD_ESTATE, "no state");
  const Coef& c = b->c[box];
  if (count != (size_t)c.cnt * c.nf) return berr(b, MTVD_ESIZE, "count mismatch");
  BHIP(b, hipMemcpyAsync(host, b->buf[b->cur] + b->off[box], sizeof(double) * count,
                         hipMemcpyDeviceToHost, b->stream));
  unsigned int flags = 0;
  BHIP(b, hipMemcpyAsync(&flags, &(bsh(b) + box)->flags, sizeof(unsigned int),
                         hipMemcpyDeviceToHost, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  return flags ? MTVD_ENONFINITE : MTVD_OK;
}

int mtvd_batch_set_state(mtvd_batch* b, int32_t box, const double* host, size_t count,
                         double time, int64_t step) {
  if (!b || !host || box < 0 || box >= b->nbox) return MTVD_EINVAL;
  if (!b->bound) return berr(b, MTVD_ESTATE, "mtvd_batch_bind first");
  if (!b->have_state) return berr(b, MTVD_ESTATE, "mtvd_batch_init_state first");
  const Coef& c = b->c[box];
  if (count != (size_t)c.cnt * c.nf) return berr(b, MTVD_ESIZE, "count mismatch");
  BHIP(b, hipMemcpyAsync(b->buf[b->cur] + b->off[box], host, sizeof(double) * count,
                         hipMemcpyHostToDevice, b->stream));
  set_scalars_kernel<<<1, 64, 0, b->stream>>>(bsh(b) + box, time, 1);
  BHIP(b, hipGetLastError());
  int rc = batch_refresh_dt(b, box);
  if (rc) return rc;
  BHIP(b, hipStreamSynchronize(b->stream));
  b->step[box] = step;
  return MTVD_OK;
}

int mtvd_batch_current(const mtvd_batch* b, int32_t* which) {
  if (!b || !which) return MTVD_EINVAL;
  *which = b->cur;
  return MTVD_OK;
}

int mtvd_batch_set_tiling(mtvd_batch* b, int32_t box, int32_t rows_x, int32_t rows_z) {
  if (!b || box < 0 || box >= b->nbox || rows_x < 0 || rows_z < 0) return MTVD_EINVAL;
  b->kcx[box] = rows_x;
  b->kcz[box] = rows_z;
  b->items_dirty = true;
  return MTVD_OK;
}

int mtvd_batch_get_tiling(const mtvd_batch* b, int32_t box, int32_t* rows_x,
                          int32_t* rows_z) {
  if (!b || box < 0 || box >= b->nbox || !rows_x || !rows_z) return MTVD_EINVAL;
  *rows_x = batch_rows(b->c[box], b->kcx[box], b->kdef_x);
  *rows_z = batch_rows(b->c[box], b->kcz[box], b->kdef_z);
  return MTVD_OK;
}

int mtvd_batch_autotune(mtvd_batch* b, void* scratch, int32_t trial_steps) {
  if (!b || !scratch || trial_steps < 1) return MTVD_EINVAL;
  if (!b->have_state) return berr(b, MTVD_ESTATE, "no state");
  if ((uintptr_t)scratch % kAlign) return berr(b, MTVD_ESIZE, "scratch must be 256-byte aligned");
  const size_t sbytes = b->state_doubles * sizeof(double);
  const size_t shbytes = sizeof(Shared) * (size_t)b->nbox;
  static_assert(sizeof(Shared) <= 2048, "the documented scratch size per box");
  unsigned char* sc = (unsigned char*)scratch;
  // save the state (current buffer), the per-box scalars and the slot
  BHIP(b, hipMemcpyAsync(sc, b->buf[b->cur], sbytes, hipMemcpyDeviceToDevice, b->stream));
  BHIP(b, hipMemcpyAsync(sc + sbytes, bsh(b), shbytes, hipMemcpyDeviceToDevice, b->stream));
  const int cur0 = b->cur, slot0 = b->slot;
  std::vector<int64_t> step0 = b->step;
  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0));
  BHIP(b, hipEventCreate(&e1));
  auto restore = [&]() -> int {
    b->cur = cur0;
    b->slot = slot0;
    b->step = step0;
    BHIP(b, hipMemcpyAsync(b->buf[b->cur], sc, sbytes, hipMemcpyDeviceToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(bsh(b), sc + sbytes, shbytes, hipMemcpyDeviceToDevice, b->stream));
    return MTVD_OK;
  };
  auto trial = [&](float* ms) -> int {
    int rc = restore();
    if (rc) return rc;
    rc = upload_items(b);
    if (rc) return rc;
    float best = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      BHIP(b, hipEventRecord(e0, b->stream));
      for (int s = 0; s < trial_steps; ++s) {
        BHIP(b, batch_step_on(b, b->stream, b->slot));
        if (b->p[0].dt_mode == 0) b->slot ^= 1;
      }
      BHIP(b, hipEventRecord(e1, b->stream));
      BHIP(b, hipEventSynchronize(e1));
      float t = 0.0f;
      BHIP(b, hipEventElapsedTime(&t, e0, e1));
      if (t < best) best = t;
    }
    *ms = best;
    return MTVD_OK;
  };
  static const int cand[5] = {4, 8, 16, 32, 64};
  std::vector<int> done(b->nbox, 0);
  for (int i = 0; i < b->nbox; ++i) {
    if (done[i]) continue;
    std::vector<int> same;
    for (int j = 0; j < b->nbox; ++j)
      if (b->c[j].nx == b->c[i].nx && b->c[j].nz == b->c[i].nz) same.push_back(j);
    for (int axis = 0; axis < 2; ++axis) {   // 0: rows of L_z, 1: rows of L_x
      int bestk = 0;
      float bestt = 1e30f;
      const int kd = batch_rows(b->c[i], 0, axis == 0 ? b->kdef_z : b->kdef_x);
      for (int ci = -1; ci < 5; ++ci) {
        const int k = ci < 0 ? kd : cand[ci];
        if (k > b->c[i].nz || (ci >= 0 && k == kd)) continue;
        for (int j : same) (axis == 0 ? b->kcz[j] : b->kcx[j]) = k;
        float t;
        int rc = trial(&t);
        if (rc) return rc;
        if (t < bestt) {
          bestt = t;
          bestk = k;
        }
      }
      for (int j : same) (axis == 0 ? b->kcz[j] : b->kcx[j]) = bestk;
    }
    for (int j : same) done[j] = 1;
  }
  int rc = restore();
  if (rc) return rc;
  rc = upload_items(b);
  if (rc) return rc;
  BHIP(b, hipStreamSynchronize(b->stream));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return MTVD_OK;
}

int mtvd_batch_destroy(mtvd_batch* b) {
  if (!b) return MTVD_OK;
  for (int a = 0; a < 2; ++a)
    if (b->have_g2[a]) (void)hipGraphExecDestroy(b->g2[a]);
  (void)hipStreamDestroy(b->cap);
  delete b;
  return MTVD_OK;
}

const char* mtvd_batch_last_error(const mtvd_batch* b) { return b ? b->err.c_str() : ""; }

}  // extern "C"

// ---------------------------------------------------------------------------
// adjoint of the time-averaged mean Nusselt number (2D, frozen dt)
//
// J = (1/N) sum_{n=1..N} Nu_mean(X_n), X_n = S^n(X_0), X_0 = X_0(theta),
// S one step with a fixed dt.  The forward pass keeps X at steps 0, E, 2E, ...
// (E = checkpoint interval); the backward pass recomputes one interval at a
// time with the forward kernels, keeping every operator's input, and runs
// the operators' reverses from the last step to the first.

// events in each of the forward pass's two rings (more than the batches in
// flight, so that a wait always finds the record it means)
constexpr int kNuEvents = 8;
static_assert(kNuEvents > 4, "the forward pass keeps up to 4 batches in flight");

struct mtvd_adj {
  mtvd_params p;
  Coef c;                 // dt_mode = 1
  adj::AC ac;
  int nsteps, every, nseg, kc;
  hipStream_t stream;
  hipStream_t side;       // recomputes the next segment while one is reversed
  hipEvent_t rec_done[2], rev_done[2];
  // forward pass: a batch of steps done on the stream / its objective terms
  // added on the side stream (rings of kNuEvents)
  hipEvent_t fwd_done[kNuEvents], nu_done[kNuEvents];
  unsigned char* ws;
  double *zr, *acc, *ckpt, *segs[2], *fw[2], *tmp[2], *cot[2];
  Shared* sh;
  adj::Arr A;
  size_t total;
  bool bound, have_fwd, have_bwd;
  double gmu, gK;         // Jbar dJ/dmu*, Jbar dJ/dK* of the latest backward pass
  std::string err;
};

namespace {

int aerr(mtvd_adj* a, int code, const std::string& what) {
  if (a) a->err = what;
  return code;
}

#define AHIP(a, expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess)                                                      \
      return aerr(a, MTVD_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kFwDoubles = 13;   // P (4), S (1), XP (4), PP (4) per node

// the forward-value arrays in ring slot b (operator q of an interval uses
// slot q & 1: each reverse launch reads its own slot and fills the other
// for the operator reversed after it)
void fw_slice(const mtvd_adj* a, int b, adj::Arr* A) {
  const size_t one = (size_t)a->c.cnt;
  double* base = a->fw[b];
  A->P = base;
  A->XP = base + 4 * one;
  A->PP = base + 8 * one;
  A->S = base + 12 * one;
}

// byte offsets of the adjoint workspace (or, with base set, its pointers)
size_t adj_layout(mtvd_adj* a, unsigned char* base) {
  const long long cnt = a->c.cnt;
  const size_t S = sizeof(double) * 4 * (size_t)cnt, one = sizeof(double) * (size_t)cnt;
  size_t off = 0;
  auto take = [&](size_t bytes) -> unsigned char* {
    unsigned char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  a->sh = (Shared*)take(sizeof(Shared));
  a->zr = (double*)take(sizeof(double) * a->c.nz);
  a->acc = (double*)take(sizeof(double) * 8);
  a->ckpt = (double*)take(S * a->nseg);
  // two segment buffers: one is reversed while the other is recomputed
  for (int q = 0; q < 2; ++q) a->segs[q] = (double*)take(S * 4 * (size_t)a->every);
  for (int q = 0; q < 2; ++q) a->tmp[q] = (double*)take(S);
  for (int q = 0; q < 2; ++q) a->cot[q] = (double*)take(S);
  // forward values (P, S, XP, PP: 13 doubles per node) of two operators:
  // the one being reversed and the next
  for (int q = 0; q < 2; ++q) a->fw[q] = (double*)take(kFwDoubles * one);
  adj::Arr& A = a->A;
  A.P = A.XP = A.PP = A.S = nullptr;   // set per operator (fw_slice)
  // the cotangent stages keep their intermediate values on chip
  A.XPb = A.PPb = A.PB = A.DPb = A.DB = A.SB = nullptr;
  A.MU = (double*)take(one);
  A.KB = (double*)take(one);
  A.zr = a->zr;
  return off;
}

int adj_check(const mtvd_params* p, int32_t nsteps, int32_t every, std::string* why) {
  int rc = validate(p, why);
  if (rc != MTVD_OK) return rc;
  if (p->ndim != 2) { *why = "the adjoint is 2D only"; return MTVD_EINVAL; }
  if (p->limiter_form != 0) { *why = "the adjoint reverses the printed limiter form (limiter_form 0) only"; return MTVD_EINVAL; }
  if (p->stretch != 0.0) { *why = "the adjoint needs the uniform z grid"; return MTVD_EINVAL; }
  if (nsteps < 1) { *why = "nsteps must be >= 1"; return MTVD_EINVAL; }
  if (every < 1) { *why = "checkpoint interval must be >= 1"; return MTVD_EINVAL; }
  return MTVD_OK;
}

void adj_shape(mtvd_adj* a, const mtvd_params* p, int32_t nsteps, int32_t every) {
  a->p = *p;
  a->p.dt_mode = 1;
  a->c = make_coef(&a->p);
  a->nsteps = nsteps;
  a->every = every > nsteps ? nsteps : every;
  a->nseg = (nsteps + a->every - 1) / a->every;
  // rows per wave of the forward sweeps as for a single box: fill the
  // resident wave slots in one round, 2..64 rows
  const long long cols = (long long)strips_2d(a->c.nx);
  const int slots = wave_slots_2d(0, false);
  long long chunks = slots > 0 ? slots / cols : 1;
  if (chunks < 1) chunks = 1;
  long long kc = (a->c.nz + chunks - 1) / chunks;
  a->kc = (int)(kc < 2 ? 2 : (kc > 64 ? 64 : kc));
  adj::AC& ac = a->ac;
  memset(&ac, 0, sizeof(ac));
  const Coef& c = a->c;
  ac.nx = c.nx;
  ac.nz = c.nz;
  ac.M = c.M;
  ac.cnt = c.cnt;
  ac.ihx = c.ihx;
  ac.ihz = c.ihz;
  ac.cv = c.cv;
  ac.icv = c.icv;
  ac.a = c.a;
  ac.gam_a = c.gam_a;
  ac.g = c.g;
  ac.mu = c.mu;
  ac.K = c.K;
  ac.lam = c.lam;
  ac.Tb = c.Tb;
  ac.Tt = c.Tt;
  ac.wall_order = c.wall_order;
  ac.tvd_on = c.tvd_on;
  ac.limiter_form = c.limiter_form;
}

const int kOrder2[2][4] = {{2, 0, 2, 0}, {2, 0, 0, 2}};

hipError_t adj_fwd_step(mtvd_adj* a, const double* in, double* out) {
  // the step's operators in order, through tmp[0], tmp[1], tmp[0]
  const int* o = kOrder2[a->p.sweep_order];
  const double* X[4] = {in, a->tmp[0], a->tmp[1], a->tmp[0]};
  double* Y[4] = {a->tmp[0], a->tmp[1], a->tmp[0], out};
  for (int s = 0; s < 4; ++s) {
    hipError_t e = launch_sweep_2d(o[s], a->c, a->sh, a->zr, 0, 0, false, X[s], Y[s], a->kc,
                                   a->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

int mtvd_adj_bytes(const mtvd_params* p, int32_t nsteps, int32_t every, size_t* workspace_bytes) {
  std::string why;
  int rc = adj_check(p, nsteps, every, &why);
  if (rc != MTVD_OK) return rc;
  mtvd_adj a;
  adj_shape(&a, p, nsteps, every);
  if (workspace_bytes) *workspace_bytes = adj_layout(&a, nullptr);
  return MTVD_OK;
}

int mtvd_adj_create(const mtvd_params* p, int32_t nsteps, int32_t every, void* hip_stream,
                    mtvd_adj** out) {
  if (!out) return MTVD_EINVAL;
  *out = nullptr;
  std::string why;
  int rc = adj_check(p, nsteps, every, &why);
  if (rc != MTVD_OK) {
    fprintf(stderr, "mtvd_adj_create: %s\n", why.c_str());
    return rc;
  }
  mtvd_adj* a = new (std::nothrow) mtvd_adj();
  if (!a) return MTVD_EINVAL;
  adj_shape(a, p, nsteps, every);
  a->total = adj_layout(a, nullptr);
  a->stream = (hipStream_t)hip_stream;
  a->side = nullptr;
  for (int q = 0; q < 2; ++q) a->rec_done[q] = a->rev_done[q] = nullptr;
  for (int q = 0; q < kNuEvents; ++q) a->fwd_done[q] = a->nu_done[q] = nullptr;
  // default priority, as the caller's stream; events without timing
  bool ok = hipStreamCreateWithFlags(&a->side, hipStreamNonBlocking) == hipSuccess;
  for (int q = 0; q < 2 && ok; ++q)
    ok = hipEventCreateWithFlags(&a->rec_done[q], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&a->rev_done[q], hipEventDisableTiming) == hipSuccess;
  for (int q = 0; q < kNuEvents && ok; ++q)
    ok = hipEventCreateWithFlags(&a->fwd_done[q], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&a->nu_done[q], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    mtvd_adj_destroy(a);
    fprintf(stderr, "mtvd_adj_create: stream or event creation failed\n");
    return MTVD_EHIP;
  }
  a->ws = nullptr;
  a->bound = a->have_fwd = a->have_bwd = false;
  a->gmu = a->gK = 0.0;
  *out = a;
  return MTVD_OK;
}

int mtvd_adj_bind(mtvd_adj* a, void* workspace) {
  if (!a) return MTVD_EINVAL;
  if (!workspace) return aerr(a, MTVD_ESIZE, "null workspace");
  if ((uintptr_t)workspace % kAlign) return aerr(a, MTVD_ESIZE, "workspace must be 256-byte aligned");
  a->ws = (unsigned char*)workspace;
  adj_layout(a, a->ws);
  AHIP(a, launch_fill((double*)a->sh, sizeof(Shared) / sizeof(double), 0.0, a->stream));
  zrow_kernel<<<(a->c.nz + 255) / 256, 256, 0, a->stream>>>(a->c.nz, a->zr);
  AHIP(a, hipGetLastError());
  a->bound = true;
  a->have_fwd = a->have_bwd = false;
  return MTVD_OK;
}

int mtvd_adj_forward(mtvd_adj* a, const double* theta, double dt, double* J, double* dt_used) {
  if (!a) return MTVD_EINVAL;
  if (!a->bound) return aerr(a, MTVD_ESTATE, "mtvd_adj_bind first");
  if (!(dt >= 0.0) || !isfinite(dt)) return aerr(a, MTVD_EINVAL, "dt must be finite and >= 0");
  a->have_fwd = a->have_bwd = false;
  const size_t S = 4 * (size_t)a->c.cnt;
  AHIP(a, launch_init_theta(a->c, a->zr, theta, a->ckpt, a->stream));
  if (dt > 0.0) {
    AHIP(a, launch_fill(&a->sh->dt_frozen, 1, dt, a->stream));
  } else {
    clear_slot_kernel<<<1, 64, 0, a->stream>>>(a->sh, 0);
    AHIP(a, hipGetLastError());
    long long blocks = (a->c.cnt + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    dt_kernel<<<(int)blocks, 256, 0, a->stream>>>(a->c, a->sh, a->zr, 0, a->ckpt);
    AHIP(a, hipGetLastError());
    freeze_dt_kernel<<<1, 64, 0, a->stream>>>(a->c, a->sh, 0);
    AHIP(a, hipGetLastError());
  }
  AHIP(a, launch_fill(a->acc, 8, 0.0, a->stream));
  const double w = 1.0 / (double)a->nsteps;
  // The step states go to the checkpoints or to a ring of R states (the
  // first interval buffer, unused until the backward pass), so that the
  // objective's terms can follow on the side stream, in step order, K
  // steps at a time: the stream records fwd_done after a batch, the side
  // stream waits for it, adds the batch's terms and records nu_done; a
  // batch's ring slots are rewritten only after the side stream has read
  // them (the stream waits for the nu_done of the batch D before it).
  // At 512 x 128 the forward pass took 14.8 ms with batches of 25 steps
  // (200-state ring), 15.0 ms with 50, and 15.4 ms with a ring of 16
  // states kept in the caches and batches of 8: a hand-over costs more
  // than the ring's traffic to memory.
  const int R = 4 * a->every;
  const int K = R / 2 < 25 ? (R / 2 < 1 ? 1 : R / 2) : 25;
  const int D = R / K < 4 ? R / K : 4;               // batches in flight, < kNuEvents
  auto state_out = [&](int n) -> double* {           // X_{n+1}
    const int nn = n + 1;
    if (nn % a->every == 0 && nn / a->every < a->nseg) return a->ckpt + S * (nn / a->every);
    return a->segs[0] + S * (size_t)(n % R);
  };
  AHIP(a, hipEventRecord(a->fwd_done[kNuEvents - 1], a->stream));
  AHIP(a, hipStreamWaitEvent(a->side, a->fwd_done[kNuEvents - 1], 0));   // after the fill above
  const double* in = a->ckpt;
  for (int m = 0, n0 = 0; n0 < a->nsteps; ++m, n0 += K) {
    const int n1 = n0 + K < a->nsteps ? n0 + K : a->nsteps;
    if (m >= D) AHIP(a, hipStreamWaitEvent(a->stream, a->nu_done[(m - D) % kNuEvents], 0));
    for (int n = n0; n < n1; ++n) {
      double* out = state_out(n);
      AHIP(a, adj_fwd_step(a, in, out));
      in = out;
    }
    AHIP(a, hipEventRecord(a->fwd_done[m % kNuEvents], a->stream));
    AHIP(a, hipStreamWaitEvent(a->side, a->fwd_done[m % kNuEvents], 0));
    for (int n = n0; n < n1; ++n)
      AHIP(a, launch_nu_obj(a->c, a->zr, state_out(n), w, a->acc, a->side));
    AHIP(a, hipEventRecord(a->nu_done[m % kNuEvents], a->side));
  }
  AHIP(a, hipEventRecord(a->nu_done[0], a->side));
  AHIP(a, hipStreamWaitEvent(a->stream, a->nu_done[0], 0));
  double host[2];
  AHIP(a, hipMemcpyAsync(&host[0], a->acc, sizeof(double), hipMemcpyDeviceToHost, a->stream));
  AHIP(a, hipMemcpyAsync(&host[1], &a->sh->dt_frozen, sizeof(double), hipMemcpyDeviceToHost,
                         a->stream));
  AHIP(a, hipStreamSynchronize(a->stream));
  if (J) *J = host[0];
  if (dt_used) *dt_used = host[1];
  if (!isfinite(host[0])) return aerr(a, MTVD_ENONFINITE, "non-finite objective");
  a->have_fwd = true;
  return MTVD_OK;
}

int mtvd_adj_backward(mtvd_adj* a, double Jbar, double* grad_x0, double* grad_theta,
                      double* grad_ra) {
  if (!a) return MTVD_EINVAL;
  if (!a->have_fwd) return aerr(a, MTVD_ESTATE, "mtvd_adj_forward first");
  if (!isfinite(Jbar)) return aerr(a, MTVD_EINVAL, "non-finite cotangent");
  const long long cnt = a->c.cnt;
  const size_t S = 4 * (size_t)cnt;
  const int* o = kOrder2[a->p.sweep_order];
  const double w = Jbar / (double)a->nsteps;
  AHIP(a, launch_fill(a->A.MU, cnt, 0.0, a->stream));
  AHIP(a, launch_fill(a->A.KB, cnt, 0.0, a->stream));
  AHIP(a, launch_fill(a->acc + 1, 1, 0.0, a->stream));
  // Segment seg's 4m operator inputs are recomputed from its checkpoint
  // into segs[b] on the side stream while the main stream reverses the
  // segment after it from segs[b ^ 1]; events order each buffer's
  // recompute before its reverse and its reverse before its next recompute.
  // The forward values an operator's reverse reads are filled by the
  // reverse launch before it (launch_adj_rev's next operator), the
  // segment's last operator's by a launch of their own.
  auto seg_len = [&](int seg) {
    const int s0 = seg * a->every;
    return (a->nsteps - s0 < a->every) ? a->nsteps - s0 : a->every;
  };
  auto recompute = [&](int seg, int b) -> hipError_t {
    const double* base = a->ckpt + S * seg;
    const int m = seg_len(seg);
    for (int j = 0; j < m; ++j)
      for (int s = 0; s < 4; ++s) {
        const int q = 4 * j + s;
        const double* in = q == 0 ? base : a->segs[b] + S * (size_t)(q - 1);
        hipError_t e = launch_sweep_2d(o[s], a->c, a->sh, a->zr, 0, 0, false, in,
                                       a->segs[b] + S * (size_t)q, a->kc, a->side);
        if (e != hipSuccess) return e;
      }
    return hipEventRecord(a->rec_done[b], a->side);
  };
  // the side stream starts after everything the caller queued before
  AHIP(a, hipEventRecord(a->rev_done[0], a->stream));
  AHIP(a, hipEventRecord(a->rev_done[1], a->stream));
  AHIP(a, hipStreamWaitEvent(a->side, a->rev_done[0], 0));
  AHIP(a, recompute(a->nseg - 1, 0));
  int cur = 0;   // cot[cur] holds the running cotangent
  for (int seg = a->nseg - 1; seg >= 0; --seg) {
    const int b = (a->nseg - 1 - seg) & 1;
    if (seg >= 1) {
      AHIP(a, hipStreamWaitEvent(a->side, a->rev_done[b ^ 1], 0));
      AHIP(a, recompute(seg - 1, b ^ 1));
    }
    AHIP(a, hipStreamWaitEvent(a->stream, a->rec_done[b], 0));
    const int s0 = seg * a->every;
    const int m = seg_len(seg);
    double* base = a->ckpt + S * seg;
    auto state = [&](int q) -> double* { return q == 0 ? base : a->segs[b] + S * (size_t)(q - 1); };
    {
      adj::Arr A = a->A;
      A.X = state(4 * m - 1);
      fw_slice(a, (4 * m - 1) & 1, &A);
      AHIP(a, launch_adj_fw(o[3], a->ac, A, a->sh, a->stream));
    }
    for (int j = m - 1; j >= 0; --j) {
      const int n = s0 + j + 1;   // the step maps X_{n-1} to X_n
      if (n == a->nsteps) {
        AHIP(a, launch_fill(a->cot[cur], (long long)S, 0.0, a->stream));
        AHIP(a, launch_nu_vjp(a->ac, a->c, a->zr, state(4 * m), w, a->cot[cur], a->stream));
      }
      for (int s = 3; s >= 0; --s) {
        const int q = 4 * j + s;
        adj::Arr A = a->A;
        A.X = state(q);
        fw_slice(a, q & 1, &A);
        A.Yb = a->cot[cur];
        A.Xb = a->cot[cur ^ 1];
        // the step's first operator reads the state X_{n-1}: its reverse
        // also adds the objective's cotangent at X_{n-1} (none at X_0)
        const double nu_w = (s == 0 && n - 1 >= 1) ? w : 0.0;
        // and fills the forward values of operator q - 1 of the segment
        adj::Arr F = a->A;
        int next_axis = -1;
        if (q >= 1) {
          F.X = state(q - 1);
          fw_slice(a, (q - 1) & 1, &F);
          next_axis = o[(q - 1) & 3];
        }
        AHIP(a, launch_adj_rev(o[s], a->ac, A, a->sh, nu_w, a->c.eps, next_axis, F, a->stream));
        cur ^= 1;
      }
    }
    AHIP(a, hipEventRecord(a->rev_done[b], a->stream));
  }
  if (grad_x0)
    AHIP(a, hipMemcpyAsync(grad_x0, a->cot[cur], sizeof(double) * S, hipMemcpyDeviceToDevice,
                           a->stream));
  if (grad_theta) AHIP(a, launch_grad_theta(a->c, a->ckpt, a->cot[cur], grad_theta, a->stream));
  // mu = sqrt(Pr/Ra), K = 1/(eps D sqrt(Ra Pr)): d/dRa = -mu/(2 Ra), -K/(2 Ra)
  const double Ra = a->p.Ra;
  AHIP(a, launch_fill(a->acc + 2, 2, 0.0, a->stream));
  AHIP(a, launch_ra_reduce(cnt, a->A.MU, a->A.KB, -a->c.mu / (2.0 * Ra), -a->c.K / (2.0 * Ra),
                           a->acc + 1, a->stream));
  AHIP(a, launch_ra_reduce(cnt, a->A.MU, a->A.KB, 1.0, 0.0, a->acc + 2, a->stream));
  AHIP(a, launch_ra_reduce(cnt, a->A.MU, a->A.KB, 0.0, 1.0, a->acc + 3, a->stream));
  double g3[3] = {0.0, 0.0, 0.0};
  AHIP(a, hipMemcpyAsync(g3, a->acc + 1, 3 * sizeof(double), hipMemcpyDeviceToHost, a->stream));
  AHIP(a, hipStreamSynchronize(a->stream));
  if (grad_ra) *grad_ra = g3[0];
  a->gmu = g3[1];
  a->gK = g3[2];
  a->have_bwd = true;
  if (!isfinite(g3[0])) return aerr(a, MTVD_ENONFINITE, "non-finite gradient");
  return MTVD_OK;
}

int mtvd_adj_coef_grads(const mtvd_adj* a, double* grad_mu, double* grad_K) {
  if (!a || !grad_mu || !grad_K) return MTVD_EINVAL;
  if (!a->have_bwd) return MTVD_ESTATE;
  *grad_mu = a->gmu;
  *grad_K = a->gK;
  return MTVD_OK;
}

int mtvd_adj_destroy(mtvd_adj* a) {
  if (!a) return MTVD_OK;
  if (a->side) {
    (void)hipStreamSynchronize(a->side);
    (void)hipStreamDestroy(a->side);
  }
  for (int q = 0; q < 2; ++q) {
    if (a->rec_done[q]) (void)hipEventDestroy(a->rec_done[q]);
    if (a->rev_done[q]) (void)hipEventDestroy(a->rev_done[q]);
  }
  for (int q = 0; q < kNuEvents; ++q) {
    if (a->fwd_done[q]) (void)hipEventDestroy(a->fwd_done[q]);
    if (a->nu_done[q]) (void)hipEventDestroy(a->nu_done[q]);
  }
  delete a;
  return MTVD_OK;
}

const char* mtvd_adj_last_error(const mtvd_adj* a) { return a ? a->err.c_str() : ""; }

}  // extern "C"

// ---------------------------------------------------------------------------
// The step without a context or a caller workspace (for callers that cannot
// allocate).  Its scratch -- the scalars the kernels share (Shared) and the
// row heights -- lives in this array, one copy per GPU, held until the
// process ends; host code reaches it only through the device address that
// hipGetSymbolAddress returns for the current device.

namespace {

constexpr size_t kNoallocShared = (sizeof(Shared) + kAlign - 1) / kAlign * kAlign;
constexpr size_t kNoallocBytes = kNoallocShared + sizeof(double) * MTVD_NOALLOC_MAX_NZ;
static_assert(kNoallocBytes == MTVD_NOALLOC_SCRATCH_BYTES, "scratch size in the header");

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices];   // device address of `scratch` per device

// the current device's copy of `scratch`, looked up once per device
hipError_t scratch_of_current(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[dev] = (unsigned char*)ptr;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

int mtvd_step_noalloc(const mtvd_params* p, double* buf_a, double* buf_b, int32_t nsteps,
                      void* hip_stream, int32_t* which) {
  if (!p || !buf_a || !buf_b || !which) return MTVD_EINVAL;
  if (nsteps < 0) return MTVD_EINVAL;
  if (p->stretch != 0.0) {
    fprintf(stderr, "mtvd_step_noalloc: uniform z grids only (stretch = 0)\n");
    return MTVD_EINVAL;
  }
  if (p->nz > MTVD_NOALLOC_MAX_NZ) {
    fprintf(stderr, "mtvd_step_noalloc: nz = %d exceeds the scratch limit of %d rows\n", p->nz,
            MTVD_NOALLOC_MAX_NZ);
    return MTVD_ESIZE;
  }
  const char* why = "";
  int rc = validate_c(p, &why);
  if (rc != MTVD_OK) {
    fprintf(stderr, "mtvd_step_noalloc: %s\n", why);
    return rc;
  }
  if (buf_a == buf_b) return MTVD_ESIZE;
  if (((uintptr_t)buf_a | (uintptr_t)buf_b) % kAlign) return MTVD_ESIZE;
  unsigned char* base = nullptr;
  if (scratch_of_current(&base) != hipSuccess) return MTVD_EHIP;
  Shared* sh = (Shared*)base;
  double* zr = (double*)(base + kNoallocShared);
  hipStream_t st = (hipStream_t)hip_stream;
  const Coef c = make_coef(p);
  // clear the scalars with a kernel (no memset node if the caller captures
  // this into a graph), then the row heights, time 0, and the dt of the
  // state in buf_a, as mtvd_set_state does
  hipError_t e = launch_fill((double*)sh, (long long)(sizeof(Shared) / sizeof(double)), 0.0, st);
  if (e != hipSuccess) return MTVD_EHIP;
  zrow_kernel<<<(c.nz + 255) / 256, 256, 0, st>>>(c.nz, zr);
  set_scalars_kernel<<<1, 64, 0, st>>>(sh, 0.0, 1);
  clear_slot_kernel<<<1, 64, 0, st>>>(sh, 0);
  long long blocks = (c.cnt + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  dt_kernel<<<(int)blocks, 256, 0, st>>>(c, sh, zr, 0, buf_a);
  if (p->dt_mode == 1) freeze_dt_kernel<<<1, 64, 0, st>>>(c, sh, 0);
  if (hipGetLastError() != hipSuccess) return MTVD_EHIP;
  // the steps, as mtvd_step
  static const int o2[2][4] = {{2, 0, 2, 0}, {2, 0, 0, 2}};
  static const int o3[2][6] = {{2, 1, 0, 2, 1, 0}, {2, 1, 0, 0, 1, 2}};
  const int ns = (c.ndim == 3) ? 6 : 4;
  const int* order = (c.ndim == 3) ? o3[p->sweep_order] : o2[p->sweep_order];
  const bool track = (p->dt_mode == 0);
  int kcs[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a)
    kcs[a] = default_rows_for(c, c.ndim == 2 ? wave_slots_2d(a, false) : 0, a);
  double* buf[2] = {buf_a, buf_b};
  int cur = 0, slot = 0;
  for (int s = 0; s < nsteps; ++s) {
    for (int o = 0; o < ns; ++o) {
      const int axis = order[o];
      const int first = (o == 0) ? 1 : 0;
      const bool fuse = track && o == ns - 1;
      e = (c.ndim == 2)
              ? launch_sweep_2d(axis, c, sh, zr, slot, first, fuse, buf[cur], buf[cur ^ 1],
                                kcs[axis], st)
              : launch_sweep_3d(axis, c, sh, zr, slot, first, fuse, buf[cur], buf[cur ^ 1],
                                kcs[axis], st);
      if (e != hipSuccess) return MTVD_EHIP;
      cur ^= 1;
    }
    if (track) slot ^= 1;
  }
  *which = cur;
  return MTVD_OK;
}

}  // extern "C"
