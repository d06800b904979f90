// mtvd_device.h -- device-side pieces shared by the MacCormack-TVD kernels.
//
// Equations: Tiwari, Sharma & Verma, arXiv:2411.10372, Sec. 2 (p, E, tau_ij
// of the nondimensional equations) and Sec. 3.1 (fluxes F_alpha, the TVD
// coefficient G, phi and C).  All arithmetic is FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mtvd {

// Constants of one problem, passed by value to every kernel.
struct Coef {
  int nx, ny, nz, M;            // M = nz - 1
  int ndim, nf;
  long long plane;              // nx * ny
  long long cnt;                // nodes = plane * nz (field stride)
  double hx, hy, hz;            // spacings
  double ihx, ihy, ihz;         // 1/h
  double gamma, cv, icv;        // c_v = 1/(gamma eps D), icv = 1/c_v
  double a;                     // p = a rho T, a = (gamma-1)/(gamma eps D)
  double gam_a;                 // c^2 = gamma a T
  double g;                     // gravity: momentum source -g rho, E has g z
  double mu, K, lam;            // sqrt(Pr/Ra), 1/(eps D sqrt(Ra Pr)), bulk coef
  double Tb, Tt;                // plate temperatures 1 and 1 - (eps + D)
  double cfl;
  double D, eps, sRP;           // D, eps, sqrt(Ra Pr) (diagnostics)
  double init_delta, init_expo; // T0 = 1 - delta z, rho0 = T0^expo
  double noise_amp;
  uint64_t seed;
  int limiter_form, tvd_on, wall_order, dt_mode;
  // dt_rule = 1: dt also keeps every node's diffusion number at most cfl/2,
  // dt <= cfl rho h^2 / kappa, kappa = max(mu (2 + |lambda|), K/c_v), h the
  // node's smallest spacing (hm2 = h^2 on a uniform grid; hmh the smaller
  // horizontal spacing)
  int dt_rule;
  double kappa, hm2, hmh;
  // tanh-stretched z grid: per-row metric table of kZM doubles per row
  // (see the kZM_* slots), device memory in the workspace; null when uniform
  int stretched;
  const double* zm;
};

// Slots of a row's entry in the metric table of a stretched grid.  Every
// z difference divides by the same difference of the node heights; the
// table holds the reciprocals (and the two lengths the TVD flux and the
// volume weights use).
constexpr int kZM = 16;
constexpr int kZM_IHF = 0;    // 1/(z_k+1 - z_k), face k+1/2 (rows 0..M-1)
constexpr int kZM_ICEN = 1;   // 1/(z_k+1 - z_k-1), centred span (rows 1..M-1)
constexpr int kZM_IW = 2;     // 1/w_k, w_k the dual cell (half a face at a plate)
constexpr int kZM_HF = 3;     // z_k+1 - z_k
constexpr int kZM_IHMIN = 4;  // 1/min of the node's faces (dt)
constexpr int kZM_IWALL = 5;  // row 0: 1/(-3 z0 + 4 z1 - z2); row M: 1/(3 zM - 4 zM-1 + zM-2)
constexpr int kZM_W = 6;      // w_k (volume weight)
// second z derivative (analysis): inside, the three-point weights of rows
// k-1, k, k+1; at a plate, the four-point one-sided Lagrange weights of the
// plate and the three rows next to it (nearest first)
constexpr int kZM_D2 = 7;     // slots 7..9 inside, 7..10 on the plates

__device__ __forceinline__ double zmet(const Coef& c, int k, int slot) {
  return c.zm[k * kZM + slot];
}

// Partial maxima per step slot: the blocks of a launch fold into
// kMaxParts addresses (block index mod kMaxParts) instead of one, so the
// device-scope atomics of thousands of waves do not queue on a single
// address; readers take the max over the parts.
constexpr int kMaxParts = 16;

// Scalars the kernels share through the workspace.
struct Shared {
  unsigned long long smax[2][kMaxParts][4];  // max over nodes of |u_a| + c
                                  // (bit patterns of positive doubles), two
                                  // step slots of kMaxParts partial maxima
  double time;                    // simulated time of the current state
  double dt_last;                 // dt used by the latest step
  double dt_frozen;               // dt when dt_mode = 1
  unsigned int flags;             // bit 0: non-finite / non-positive seen
  unsigned int pad[9];            // 1088 bytes per box in a batch
};

// the part a block folds into
__device__ __forceinline__ int max_part() { return (int)(blockIdx.x % kMaxParts); }

// Work index of this block, XCD-aware.  The dispatcher hands consecutive
// blocks to the 8 XCDs in turn, and each XCD has its own L2; this bijection
// of [0, nblocks) gives every XCD a contiguous range of work indices, so
// blocks that share halo rows, planes and cache lines run on the same L2 at
// about the same time instead of fetching the shared data once per XCD.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block() {
  const int b = (int)blockIdx.x, G = (int)gridDim.x;
  const int x = b % kXcds, k = b / kXcds;
  const int q = G / kXcds, r = G % kXcds;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// One box of a batch: its constants, the offset of its state in the state
// arenas (field stride c.cnt from there), of its plate table in the z
// arena, and its rows per wave for each operator.
struct BoxDesc {
  Coef c;
  long long off;
  int zoff;
  int kc_x, kc_z;
  int nstrips;
  int pad[2];
};

__device__ __forceinline__ double u2d(unsigned long long b) {
  return __longlong_as_double((long long)b);
}
__device__ __forceinline__ unsigned long long d2u(double d) {
  return (unsigned long long)__double_as_longlong(d);
}

// dt of the current step from the maxima in `slot` (or the frozen value):
// dt = cfl * min_a h_a / max_nodes(|u_a| + c), the same number as the
// minimum over nodes of h_a/(|u_a| + c) because division by a positive
// number is monotone.
__device__ __forceinline__ double slot_max(const Shared* sh, int slot, int a) {
  // positive doubles order as their bit patterns
  unsigned long long m = 0ull;
  for (int q = 0; q < kMaxParts; ++q) m = max(m, sh->smax[slot][q][a]);
  return u2d(m);
}

// Slot entry 3 (dt_rule = 1) holds the minimum over nodes of rho h^2 as
// the bitwise complement of its bit pattern: complements of positive
// doubles order in reverse, so the same atomic max that folds the other
// entries folds this minimum (and a cleared entry, 0, lies below them all).
__device__ __forceinline__ double slot_min_rho_h2(const Shared* sh, int slot) {
  unsigned long long m = 0ull;
  for (int q = 0; q < kMaxParts; ++q) m = max(m, sh->smax[slot][q][3]);
  return u2d(~m);
}

// STR: a stretched z grid, whose z slot holds max (|u_z| + c)/h_z,k already
template <bool STR = false>
__device__ __forceinline__ double step_dt(const Coef& c, const Shared* sh, int slot) {
  if (c.dt_mode) return sh->dt_frozen;
  double m = c.hx / slot_max(sh, slot, 0);
  double mz = (STR ? 1.0 : c.hz) / slot_max(sh, slot, 2);
  m = fmin(m, mz);
  if (c.ndim == 3) m = fmin(m, c.hy / slot_max(sh, slot, 1));
  // the minimum over nodes of rho h^2 / kappa is (min rho h^2) / kappa:
  // division by the positive constant kappa is monotone
  if (c.dt_rule) m = fmin(m, slot_min_rho_h2(sh, slot) / c.kappa);
  return c.cfl * m;
}

// h^2 of a node of row k for the diffusion part of dt: its smallest
// spacing, on a stretched grid the narrower of its z faces (a plate node
// has one)
__device__ __forceinline__ double diff_h2(const Coef& c, int k) {
  if (!c.stretched) return c.hm2;
  const double hz = (k == 0)      ? c.zm[kZM_HF]
                    : (k == c.M) ? c.zm[(c.M - 1) * kZM + kZM_HF]
                                 : fmin(c.zm[(k - 1) * kZM + kZM_HF], c.zm[k * kZM + kZM_HF]);
  const double h = fmin(c.hmh, hz);
  return h * h;
}

// ---- 2D node values -------------------------------------------------------

struct N2 { double r, mx, mz, E; };
struct P2 { double ux, uz, T, p; };

__device__ __forceinline__ N2 operator-(const N2& a, const N2& b) {
  return N2{a.r - b.r, a.mx - b.mx, a.mz - b.mz, a.E - b.E};
}

// 1/x from the hardware estimate and two Newton steps (error within an ulp
// for the normal, finite, positive arguments the kernels pass)
__device__ __forceinline__ double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// sqrt(y) for normal positive y: reciprocal square-root estimate, one
// coupled Newton step on (s, h) = (y r, r/2) and a final residual
// correction (Goldschmidt); within an ulp.  Non-positive or non-finite y
// gives a non-finite or zero result, which the positivity checks flag.
__device__ __forceinline__ double fsqrt(double y) {
  double r = __builtin_amdgcn_rsq(y);
  double s = y * r;
  double h = 0.5 * r;
  double e = fma(-s, h, 0.5);
  s = fma(s, e, s);
  h = fma(h, e, h);
  double d = fma(-s, s, y);
  return fma(d, h, s);
}

// lane i <- lane i-1 (wave_shr:1) and lane i <- lane i+1 (wave_shl:1) for a
// double; the lane without a source reads 0 (bound_ctrl; it is always a
// halo lane), so no old value has to be set up first
__device__ __forceinline__ double lane_from_below(double v) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_mov_dpp((int)b, 0x138, 0xf, 0xf, true);
  int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_from_above(double v) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_mov_dpp((int)b, 0x130, 0xf, 0xf, true);
  int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// primitives (Sec. 2): u = m/rho, T = (E/rho - |u|^2/2 - g z)/c_v, p = a rho T
__device__ __forceinline__ P2 prim2(const Coef& c, const N2& x, double z) {
  double ri = frcp(x.r);
  P2 q;
  q.ux = x.mx * ri;
  q.uz = x.mz * ri;
  double ke = 0.5 * (q.ux * q.ux + q.uz * q.uz);
  q.T = (x.E * ri - ke - c.g * z) * c.icv;
  q.p = c.a * x.r * q.T;
  return q;
}

// sound speed c = sqrt(gamma p / rho) = sqrt(gamma a T)
__device__ __forceinline__ double sound(const Coef& c, double T) {
  return fsqrt(c.gam_a * T);
}

// Flux along z (Sec. 3.1 F_3; tau_zz, tau_xz of Sec. 2) given the inner
// z-derivatives (dzux, dzuz, dzT) and central x-derivatives (dxux, dxuz).
__device__ __forceinline__ N2 flux_z2(const Coef& c, const N2& x, const P2& q,
                                      double dzux, double dzuz, double dzT,
                                      double dxux, double dxuz) {
  double div = dxux + dzuz;
  double tzz = c.mu * ((dzuz + dzuz) + c.lam * div);
  double txz = c.mu * (dzux + dxuz);
  N2 F;
  F.r = x.mz;
  F.mx = x.mx * q.uz - txz;
  F.mz = (x.mz * q.uz - tzz) + q.p;
  F.E = (q.uz * (x.E + q.p) - c.K * dzT) - (q.ux * txz + q.uz * tzz);
  return F;
}

// Flux along x (Sec. 3.1 F_1; tau_xx, tau_zx of Sec. 2) given the inner
// x-derivatives and central z-derivatives.
__device__ __forceinline__ N2 flux_x2(const Coef& c, const N2& x, const P2& q,
                                      double dxux, double dxuz, double dxT,
                                      double dzux, double dzuz) {
  double div = dxux + dzuz;
  double txx = c.mu * ((dxux + dxux) + c.lam * div);
  double tzx = c.mu * (dxuz + dzux);
  N2 F;
  F.r = x.mx;
  F.mx = (x.mx * q.ux - txx) + q.p;
  F.mz = x.mz * q.ux - tzx;
  F.E = (q.ux * (x.E + q.p) - c.K * dxT) - (q.ux * txx + q.uz * tzx);
  return F;
}

// phi(x) = max(0, min(2x, 1))  (Sec. 3.1)
__device__ __forceinline__ double phi(double x) { return fmax(0.0, fmin(2.0 * x, 1.0)); }

// TVD coefficient G of the face between two nodes (Sec. 3.1): a_m, a_p are
// the dot products dX_{-1/2}.dX_{+1/2} and dX_{+1/2}.dX_{+3/2}, den the
// squared norm of dX_{+1/2}; Co = lam_h * max(|u|+c) over the two nodes.  A
// face with den == 0 has no TVD flux.
__device__ __forceinline__ double tvd_G(const Coef& c, double a_m, double a_p,
                                        double den, double Co) {
  if (den == 0.0) return 0.0;
  double C = (Co <= 0.5) ? Co * (1.0 - Co) : 0.25;
  double id = frcp(den);
  if (c.limiter_form == 0) {
    return 0.5 * C * (1.0 - phi(a_m * id + a_p * id));
  }
  return 0.5 * C * (1.0 - phi(a_m * id)) + 0.5 * C * (1.0 - phi(a_p * id));
}

__device__ __forceinline__ double dot2(const N2& a, const N2& b) {
  return ((a.r * b.r + a.mx * b.mx) + a.mz * b.mz) + a.E * b.E;
}

// wave-wide max and min (64 lanes)
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// fold the minimum of rho h^2 into slot entry 3 of part `part` (one lane)
__device__ __forceinline__ void fold_rho_h2(Shared* sh, int slot, int part, double md) {
  atomicMax(&sh->smax[slot][part][3], ~d2u(md));
}

}  // namespace mtvd
