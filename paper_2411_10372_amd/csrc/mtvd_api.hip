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

#include <new>
#include <string>
#include <vector>

#include "../../include/mtvd.h"
#include "mtvd_device.h"
#include "mtvd_launch.h"

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
  size_t shared, zrow, part, out, total;
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
  L.part = off;
  off = align_up(off + sizeof(double) * (size_t)p->nz * (size_t)nb * kDiagVals);
  L.out = off;
  off = align_up(off + sizeof(double) * kDiagOut);
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
  if (threadIdx.x < 4) sh->smax[slot][threadIdx.x] = 0ull;
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
    m[0] = fmax(m[0], sx);
    m[1] = fmax(m[1], sy);
    m[2] = fmax(m[2], sz);
    if (!(rho > 0.0) || !(T > 0.0) || !(sx < INFINITY) || !(sy < INFINITY) ||
        !(sz < INFINITY))
      bad = true;
  }
  for (int a = 0; a < 3; ++a) m[a] = wave_max(m[a]);
  unsigned long long anybad = __ballot(bad);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&sh->smax[slot][0], d2u(m[0]));
    if (c.ndim == 3) atomicMax(&sh->smax[slot][1], d2u(m[1]));
    atomicMax(&sh->smax[slot][2], d2u(m[2]));
    if (anybad) atomicOr(&sh->flags, 1u);
  }
}

__global__ void freeze_dt_kernel(Coef c, Shared* sh, int slot) {
  if (threadIdx.x == 0) {
    Coef cc = c;
    cc.dt_mode = 0;
    sh->dt_frozen = step_dt(cc, sh, slot);
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
    double w = (k == 0 || k == c.M) ? 0.5 : 1.0;
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
    double gb = ((-3.0 * tm[0] + 4.0 * tm[1]) - tm[2]) * (0.5 * c.ihz);
    double gt = ((3.0 * tm[5] - 4.0 * tm[4]) + tm[3]) * (0.5 * c.ihz);
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

int validate(const mtvd_params* p, std::string* why) {
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
  if (!(p->cfl > 0.0) || !(p->cfl <= 1.0)) { *why = "cfl must lie in (0, 1]"; return MTVD_ESTABILITY; }
  // diffusion number of the initial state (the acoustic limit sets dt):
  // max(mu(2+|lambda|), K/c_v) * tau / (rho_min h_min^2) <= 1/2
  double hx = p->aspect / p->nx, hz = 1.0 / (p->nz - 1);
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
  return c;
}

Shared* shared_of(mtvd_ctx* c) { return (Shared*)(c->ws + c->L.shared); }
double* zrow_of(mtvd_ctx* c) { return (double*)(c->ws + c->L.zrow); }

int default_rows(const mtvd_ctx* c) {
  long long kc;
  if (c->c.ndim == 2) {
    // about four waves per SIMD (1024 SIMDs) when the grid allows it
    long long cols = (long long)strips_2d(c->c.nx);
    kc = cols * c->c.nz / 4096;
  } else {
    // 3D: blocks of 8 waves; a quarter of the marched extent, 4..32 rows
    kc = c->c.nz / 4;
    if (kc > 32) kc = 32;
  }
  if (kc < 4) kc = 4;
  if (kc > 64) kc = 64;
  return (int)kc;
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
  if (kc <= 0) kc = default_rows(c);
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
  zrow_kernel<<<(c->c.nz + 255) / 256, 256, 0, c->stream>>>(c->c.nz, zrow_of(c));
  HIPCHK(c, hipGetLastError());
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
    // the same arithmetic as step_dt on the device
    double S[3];
    for (int a = 0; a < 3; ++a) memcpy(&S[a], &hs.smax[c->slot][a], sizeof(double));
    double m = fmin(c->c.hx / S[0], c->c.hz / S[2]);
    if (c->c.ndim == 3) m = fmin(m, c->c.hy / S[1]);
    out->dt = c->c.cfl * m;
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
