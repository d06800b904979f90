// mtvd_2d.hip -- fused predictor/corrector/TVD kernels of one directional
// operator L_a(tau) in 2D (Sec. 3.1 of arXiv:2411.10372: predictor with
// backward flux differences, corrector with forward differences of the
// predicted fluxes, average plus the TVD term).
//
// Launch shape (both directions): one wave of 64 lanes owns a strip of 60
// output columns plus two halo columns on each side (lane l <-> column
// i0 - 2 + l, periodic) and marches up a chunk of rows.  Values along z
// stay in registers in rings of period 4 (the march is unrolled by 4 so
// every ring index is a compile-time constant); values along x move between
// neighbouring lanes with DPP wave shifts.  Rows are prefetched two
// iterations ahead, with their heights z_k, so a wave's loads overlap its own
// arithmetic.  Each sweep reads and writes the state once: 4 fields x 8 B in,
// 4 x 8 B out per node, plus halo re-reads that hit in L2.
#include "mtvd_device.h"
#include "mtvd_launch.h"

namespace mtvd {

constexpr int kStrip = 60;   // output columns per wave

struct Cols {
  int col;        // this lane's (wrapped) column
  bool out;       // lane writes its column
};

__device__ __forceinline__ Cols lane_cols(const Coef& c, int strip, int lane) {
  Cols r;
  int i0 = strip * kStrip;
  int i = i0 - 2 + lane;
  int m = i % c.nx;
  r.col = (m < 0) ? m + c.nx : m;
  r.out = lane >= 2 && lane < 62 && (i0 + lane - 2) < c.nx;
  return r;
}

__device__ __forceinline__ N2 load2(const Coef& c, const double* __restrict__ X,
                                    int k, int col) {
  long long n = (long long)k * c.nx + col;
  N2 v;
  v.r = X[n];
  v.mx = X[n + c.cnt];
  v.mz = X[n + 2 * c.cnt];
  v.E = X[n + 3 * c.cnt];
  return v;
}

__device__ __forceinline__ void store2(const Coef& c, double* __restrict__ Y, int k,
                                       int col, const N2& v) {
  long long n = (long long)k * c.nx + col;
  Y[n] = v.r;
  Y[n + c.cnt] = v.mx;
  Y[n + 2 * c.cnt] = v.mz;
  Y[n + 3 * c.cnt] = v.E;
}

// value of the next lane up (i+1) / down (i-1)
__device__ __forceinline__ double up(double v) { return lane_from_above(v); }
__device__ __forceinline__ double dn(double v) { return lane_from_below(v); }
__device__ __forceinline__ N2 up(const N2& v) { return N2{up(v.r), up(v.mx), up(v.mz), up(v.E)}; }
__device__ __forceinline__ N2 dn(const N2& v) { return N2{dn(v.r), dn(v.mx), dn(v.mz), dn(v.E)}; }

// Per-step bookkeeping: the first sweep of a step publishes dt and time and
// clears the other max slot; the last one folds |u_a| + c of its output
// into that slot.
__device__ __forceinline__ void step_head(const Coef& c, Shared* sh, int slot, int first,
                                          double dt) {
  if (first && blockIdx.x == 0 && threadIdx.x < kMaxParts * 4) {
    if (threadIdx.x == 0) {
      sh->time += dt;
      sh->dt_last = dt;
    }
    sh->smax[slot ^ 1][threadIdx.x >> 2][threadIdx.x & 3] = 0ull;
  }
}

__device__ __forceinline__ void fold_max(const Coef& c, Shared* sh, int slot, double mx,
                                         double mz, double md, bool bad) {
  mx = wave_max(mx);
  mz = wave_max(mz);
  if (c.dt_rule) md = wave_min(md);
  unsigned long long anybad = __ballot(bad);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&sh->smax[slot ^ 1][max_part()][0], d2u(mx));
    atomicMax(&sh->smax[slot ^ 1][max_part()][2], d2u(mz));
    if (c.dt_rule) fold_rho_h2(sh, slot ^ 1, max_part(), md);
    if (anybad) atomicOr(&sh->flags, 1u);
  }
}

// izs: 1 on the uniform grid; 1/h_z of the row on a stretched one (the z
// slot then collects (|u_z| + c)/h_z, which dt divides into 1)
// h2: the row's diff_h2 (dt_rule = 1; md collects the minimum of rho h^2)
__device__ __forceinline__ void out_max(const Coef& c, const N2& o, double z, double izs,
                                        double h2, double& mx, double& mz, double& md,
                                        bool& bad, bool lane_out) {
  P2 q = prim2(c, o, z);
  double cs = sound(c, q.T);
  double sx = fabs(q.ux) + cs, sz = (fabs(q.uz) + cs) * izs;
  if (lane_out) {
    mx = fmax(mx, sx);
    mz = fmax(mz, sz);
    if (c.dt_rule) md = fmin(md, o.r * h2);
    if (!(o.r > 0.0) || !(q.T > 0.0) || !(sx < INFINITY) || !(sz < INFINITY)) bad = true;
  }
}

// ---------------------------------------------------------------------------
// L_z(tau): flux differences along the march, cross x-derivatives from the
// neighbouring lanes.

// Rows are prefetched kPF march steps ahead of their use (2; 4 was
// measured slower: its 20 extra registers cost more than the added slack).
#ifndef MTVD_PF
#define MTVD_PF 2
#endif
constexpr int kPF = MTVD_PF;
static_assert(kPF == 2 || kPF == 4, "prefetch ring period must divide the unroll");

struct Z2 {
  N2 pf[kPF];     // prefetched rows f+1 .. f+kPF, slot row % kPF
  double pz[kPF]; // their heights z_k, prefetched with them (a height loaded
                  // on use would make the wave wait for every load in flight)
  N2 x[4];      // X^n rows f-3..f, slot row & 3
  double zz[4]; // their heights
  P2 pn[4];     // primitives of X^n (p filled on use)
  double s[4];  // |u_z| + c of X^n
  double G[2];  // TVD coefficient of face row+1/2
  N2 Dp;        // G dX of the face below the next output row
  N2 F[2];      // predictor flux (forward inner derivatives), slot row & 1
  N2 xp[4];     // X^P
  P2 pp[4];     // primitives of X^P
  N2 FP[2];     // corrector flux (backward inner derivatives)
  double mx, mz, md;
  bool bad;
  // stretched grid only: metrics derived from the ring heights and carried
  // one march step (a table read per row would wait behind the row loads)
  double ihf1, ihf2;  // 1/h of faces f-3+1/2 and f-4+1/2
  double iw1;         // 1/w of row f-3
  double iwb, iwt;    // the two plate stencils' 1/(stencil applied to z)
};

// The stages of one march step f of L_z.  Ring slots: row f in S & 3,
// f-1 in (S+3) & 3, f-2 in (S+2) & 3, f-3 in (S+1) & 3; period-2 rings: row
// f (and f-2) in S & 1, f-1 in (S+1) & 1.
template <int S>
struct ZS {
  static constexpr int c0 = S & 3, c1 = (S + 3) & 3, c2 = (S + 2) & 3, c3 = (S + 1) & 3;
  static constexpr int c4 = S & 3;   // row f-4 (its slot is reused by row f)
  static constexpr int e0 = S & 1, e1 = (S + 1) & 1;
  static constexpr int q0 = S % kPF;   // prefetch slot of row f (and f+kPF)
};

// A: row f (prefetched kPF steps ago) and its primitives; prefetch row f+kPF.
//    Every step of the march runs this head, whether or not it computes:
//    the row index is clamped into [0, M], and no guard surrounds the
//    loads, because a guarded load has to be copied into the loop-carried
//    ring registers at the guard's end and the copy waits for the load.
//    Rows outside [first row, M] land in ring slots no stage reads.
//    The row is clamped to [flo, fhi], the rows the chunk's stages read:
//    the unrolled march prefetches past both ends of the chunk, and those
//    loads repeat a row just loaded, which the caches serve.
template <int S>
__device__ __forceinline__ void z2_load(const Coef& c, Z2& st, int f, int flo, int fhi,
                                        const Cols& L, const double* __restrict__ zr,
                                        const double* __restrict__ X) {
  using Z = ZS<S>;
  st.x[Z::c0] = st.pf[Z::q0];
  st.zz[Z::c0] = st.pz[Z::q0];
  const int fp = min(max(f + kPF, flo), fhi);
  st.pf[Z::q0] = load2(c, X, fp, L.col);
  st.pz[Z::q0] = zr[fp];
  st.pn[Z::c0] = prim2(c, st.x[Z::c0], st.zz[Z::c0]);
  st.s[Z::c0] = fabs(st.pn[Z::c0].uz) + sound(c, st.pn[Z::c0].T);
}

// B: predictor flux F_r of row r = f-2 (inner z forward; second-order
//    forward at the bottom plate when `wall`), central x cross-derivatives
//    On a stretched grid (STR) each difference is over the same difference
//    of the heights: face r+1/2, or the wall stencil applied to z.
template <int S, bool STR>
__device__ __forceinline__ void z2_pflux(const Coef& c, Z2& st, bool wall, double ihf) {
  using Z = ZS<S>;
  const P2& q0 = st.pn[Z::c2];
  const P2& q1 = st.pn[Z::c1];
  double dzux, dzuz, dzT;
  if (wall) {
    const P2& q2 = st.pn[Z::c0];
    double h2 = STR ? st.iwb : 0.5 * c.ihz;
    dzux = ((-3.0 * q0.ux + 4.0 * q1.ux) - q2.ux) * h2;
    dzuz = ((-3.0 * q0.uz + 4.0 * q1.uz) - q2.uz) * h2;
    dzT = ((-3.0 * q0.T + 4.0 * q1.T) - q2.T) * h2;
  } else {
    const double ih = STR ? ihf : c.ihz;
    dzux = (q1.ux - q0.ux) * ih;
    dzuz = (q1.uz - q0.uz) * ih;
    dzT = (q1.T - q0.T) * ih;
  }
  double dxux = (up(q0.ux) - dn(q0.ux)) * (0.5 * c.ihx);
  double dxuz = (up(q0.uz) - dn(q0.uz)) * (0.5 * c.ihx);
  P2 q = q0;
  q.p = c.a * st.x[Z::c2].r * q0.T;
  st.F[Z::e0] = flux_z2(c, st.x[Z::c2], q, dzux, dzuz, dzT, dxux, dxuz);
}

// C (interior rows): X^P_r = X_r - (tau/dz)(F_r - F_{r-1}) + tau S(X_r)
template <int S>
__device__ __forceinline__ void z2_pred(const Coef& c, Z2& st, double z, double tau, double lz) {
  using Z = ZS<S>;
  const N2& Fa = st.F[Z::e0];
  const N2& Fb = st.F[Z::e1];
  N2 v = st.x[Z::c2] - N2{lz * (Fa.r - Fb.r), lz * (Fa.mx - Fb.mx), lz * (Fa.mz - Fb.mz),
                          lz * (Fa.E - Fb.E)};
  v.mz = v.mz + tau * (-c.g * st.x[Z::c2].r);
  st.xp[Z::c2] = v;
  st.pp[Z::c2] = prim2(c, v, z);
}

// D: corrector flux F^P_r (inner z backward; second-order backward at the
//    top plate when `wall`), central x cross-derivatives of X^P
template <int S, bool STR>
__device__ __forceinline__ void z2_cflux(const Coef& c, Z2& st, bool wall) {
  using Z = ZS<S>;
  const P2& q0 = st.pp[Z::c2];
  const P2& qm = st.pp[Z::c3];
  double dzux, dzuz, dzT;
  if (wall) {
    const P2& qmm = st.pp[Z::c4];
    double h2 = STR ? st.iwt : 0.5 * c.ihz;
    dzux = ((3.0 * q0.ux - 4.0 * qm.ux) + qmm.ux) * h2;
    dzuz = ((3.0 * q0.uz - 4.0 * qm.uz) + qmm.uz) * h2;
    dzT = ((3.0 * q0.T - 4.0 * qm.T) + qmm.T) * h2;
  } else {
    const double ih = STR ? st.ihf1 : c.ihz;   // face r-1/2
    dzux = (q0.ux - qm.ux) * ih;
    dzuz = (q0.uz - qm.uz) * ih;
    dzT = (q0.T - qm.T) * ih;
  }
  double dxux = (up(q0.ux) - dn(q0.ux)) * (0.5 * c.ihx);
  double dxuz = (up(q0.uz) - dn(q0.uz)) * (0.5 * c.ihx);
  st.FP[Z::e0] = flux_z2(c, st.xp[Z::c2], q0, dzux, dzuz, dzT, dxux, dxuz);
}

// E (faces away from the plates): TVD coefficient of face r+1/2 from the
//    X^n ring
template <int S>
__device__ __forceinline__ double z2_tvd(const Coef& c, const Z2& st, double lz) {
  using Z = ZS<S>;
  N2 dm = st.x[Z::c2] - st.x[Z::c3];
  N2 d0 = st.x[Z::c1] - st.x[Z::c2];
  N2 dp = st.x[Z::c0] - st.x[Z::c1];
  double Co = lz * fmax(st.s[Z::c2], st.s[Z::c1]);
  return tvd_G(c, dot2(dm, d0), dot2(d0, dp), dot2(d0, d0), Co);
}

// F: corrector, average and TVD term of row o = f-3 (when `emit`); the face
//    o+1/2 term G dX is carried to the next row as its o-1/2 term
//    On a stretched grid G carries the face spacing (h G dX is the face's
//    dissipative flux) and the difference of the two face fluxes is taken
//    over the row's dual cell, as the flux differences are.
template <int S, bool FUSE, bool STR>
__device__ __forceinline__ void z2_out(const Coef& c, Z2& st, bool emit, int o, const Cols& L,
                                       double* __restrict__ Y, double tau, double lz) {
  using Z = ZS<S>;
  N2 d0 = st.x[Z::c2] - st.x[Z::c3];
  double G = st.G[Z::e1];
  N2 Dc{G * d0.r, G * d0.mx, G * d0.mz, G * d0.E};
  if (emit) {
    double iw = 1.0;
    if (STR) {
      iw = st.iw1;
      lz = tau * iw;
    }
    const N2& fp1 = st.FP[Z::e0];
    const N2& fp0 = st.FP[Z::e1];
    N2 xc = st.x[Z::c3] - N2{lz * (fp1.r - fp0.r), lz * (fp1.mx - fp0.mx),
                             lz * (fp1.mz - fp0.mz), lz * (fp1.E - fp0.E)};
    xc.mz = xc.mz + tau * (-c.g * st.xp[Z::c3].r);
    const N2& xp = st.xp[Z::c3];
    const N2& Dm = st.Dp;
    N2 out;
    if (STR) {
      out.r = 0.5 * (xp.r + xc.r) + (Dc.r - Dm.r) * iw;
      out.mx = 0.5 * (xp.mx + xc.mx) + (Dc.mx - Dm.mx) * iw;
      out.mz = 0.5 * (xp.mz + xc.mz) + (Dc.mz - Dm.mz) * iw;
      out.E = 0.5 * (xp.E + xc.E) + (Dc.E - Dm.E) * iw;
    } else {
      out.r = 0.5 * (xp.r + xc.r) + (Dc.r - Dm.r);
      out.mx = 0.5 * (xp.mx + xc.mx) + (Dc.mx - Dm.mx);
      out.mz = 0.5 * (xp.mz + xc.mz) + (Dc.mz - Dm.mz);
      out.E = 0.5 * (xp.E + xc.E) + (Dc.E - Dm.E);
    }
    if (FUSE)
      out_max(c, out, st.zz[Z::c3], STR ? fmax(st.ihf1, st.ihf2) : 1.0,
              c.dt_rule ? diff_h2(c, o) : 0.0, st.mx, st.mz, st.md, st.bad, L.out);
    if (L.out) store2(c, Y, o, L.col, out);
  }
  st.Dp = Dc;
}

// One march step: plates, chunk edges and the end of the grid are guarded.
template <int S, bool FUSE, bool STR>
__device__ __forceinline__ void z2_iter(const Coef& c, Z2& st, int f, int fs, int fe,
                                        int k0, int k1, const Cols& L,
                                        const double* __restrict__ zr,
                                        const double* __restrict__ X,
                                        double* __restrict__ Y, double tau, double lz) {
  using Z = ZS<S>;
  z2_load<S>(c, st, f, fs, min(c.M, k1 + 1), L, zr, X);
  if (f < fs || f > fe) return;
  const int M = c.M;
  const int r = f - 2;
  // stretched grid: face r+1/2 and dual cell of row r from the ring heights
  // (rows past a plate hold clamped heights; their values are never used)
  double hf = 0.0, ihf = 0.0, iw = 0.0;
  if (STR) {
    hf = st.zz[Z::c1] - st.zz[Z::c2];
    ihf = frcp(hf);
    iw = 2.0 * frcp(st.zz[Z::c1] - st.zz[Z::c3]);
  }
  if (r >= k0 - 2 && r >= 0 && r <= M - 1)
    z2_pflux<S, STR>(c, st, r == 0 && c.wall_order == 2, ihf);
  // C: plates: u = 0, T = T_plate, top density from the backward mass-flux
  //    difference
  if (r >= k0 - 1 && r >= 0 && r <= M) {
    if (r == 0) {
      double rho = st.x[Z::c2].r;
      st.xp[Z::c2] = N2{rho, 0.0, 0.0, rho * (c.cv * c.Tb + c.g * st.zz[Z::c2])};
      st.pp[Z::c2] = P2{0.0, 0.0, c.Tb, c.a * rho * c.Tb};
    } else if (r == M) {
      const double lt = STR ? tau * st.ihf1 : lz;   // face M-1/2
      double rho = st.x[Z::c2].r - lt * (st.x[Z::c2].mz - st.x[Z::c3].mz);
      st.xp[Z::c2] = N2{rho, 0.0, 0.0, rho * (c.cv * c.Tt + c.g * st.zz[Z::c2])};
      st.pp[Z::c2] = P2{0.0, 0.0, c.Tt, c.a * rho * c.Tt};
    } else {
      z2_pred<S>(c, st, st.zz[Z::c2], tau, STR ? tau * iw : lz);
    }
  }
  if (r >= k0 && r >= 1 && r <= M) z2_cflux<S, STR>(c, st, r == M && c.wall_order == 2);
  // E: zero on the two faces next to the plates (on a stretched grid the
  //    face's own spacing sets Co, and G carries that spacing)
  if (r >= k0 - 1 && r >= 0 && r <= M - 1) {
    double G = 0.0;
    if (c.tvd_on && r >= 1 && r <= M - 2) {
      if (STR)
        G = z2_tvd<S>(c, st, tau * ihf) * hf;
      else
        G = z2_tvd<S>(c, st, lz);
    }
    st.G[Z::e0] = G;
  }
  const int o = f - 3;
  if (o >= k0 - 1 && o >= 0 && o < k1 && o <= M - 1)
    z2_out<S, FUSE, STR>(c, st, o >= k0 && o >= 1, o, L, Y, tau, lz);
  if (o >= k0 && o < k1 && (o == 0 || o == M)) {
    N2 out;
    if (o == 0) {
      const double lb = STR ? tau * st.ihf1 : lz;   // face 1/2
      double rho = st.x[Z::c3].r - lb * (st.xp[Z::c2].mz - 0.0);
      out = N2{rho, 0.0, 0.0, rho * (c.cv * c.Tb + c.g * st.zz[Z::c3])};
    } else {
      double rho = st.xp[Z::c3].r;
      out = N2{rho, 0.0, 0.0, rho * (c.cv * c.Tt + c.g * st.zz[Z::c3])};
    }
    if (FUSE)
      out_max(c, out, st.zz[Z::c3], STR ? (o == 0 ? st.ihf1 : st.ihf2) : 1.0,
              c.dt_rule ? diff_h2(c, o) : 0.0, st.mx, st.mz, st.md, st.bad, L.out);
    if (L.out) store2(c, Y, o, L.col, out);
  }
  if (STR) {
    st.ihf2 = st.ihf1;
    st.ihf1 = ihf;
    st.iw1 = iw;
  }
}

// one wave's share of L_z: columns of `strip`, output rows of `chunk`
template <bool FUSE, bool STR>
__device__ __forceinline__ void z2_wave(const Coef& c, Shared* sh, const double* zr, int slot,
                                        double dt, const double* __restrict__ X,
                                        double* __restrict__ Y, int kc, int strip,
                                        int chunk, int lane) {
  const Cols L = lane_cols(c, strip, lane);
  const int k0 = chunk * kc;
  const int k1 = min(k0 + kc, c.nz);
  const double tau = 0.5 * dt;
  const double lz = tau * c.ihz;
  Z2 st;
  st.mx = 0.0;
  st.mz = 0.0;
  st.md = INFINITY;
  st.bad = false;
  st.Dp = N2{0.0, 0.0, 0.0, 0.0};
  st.ihf1 = st.ihf2 = st.iw1 = 0.0;
  st.iwb = st.iwt = 0.0;
  if (STR) {
    st.iwb = zmet(c, 0, kZM_IWALL);
    st.iwt = zmet(c, c.M, kZM_IWALL);
  }
  const int fs = max(0, k0 - 2);
  const int fe = k1 + 2;
  // the kPF steps before fs only load rows fs .. fs+kPF-1 (their heads);
  // the heads before them copy this defined, unused row
  for (int q = 0; q < kPF; ++q) {
    st.pf[q] = N2{1.0, 0.0, 0.0, 1.0};
    st.pz[q] = 0.0;
  }
  for (int fb = (fs - kPF) & ~3; fb <= fe; fb += 4) {
    z2_iter<0, FUSE, STR>(c, st, fb + 0, fs, fe, k0, k1, L, zr, X, Y, tau, lz);
    z2_iter<1, FUSE, STR>(c, st, fb + 1, fs, fe, k0, k1, L, zr, X, Y, tau, lz);
    z2_iter<2, FUSE, STR>(c, st, fb + 2, fs, fe, k0, k1, L, zr, X, Y, tau, lz);
    z2_iter<3, FUSE, STR>(c, st, fb + 3, fs, fe, k0, k1, L, zr, X, Y, tau, lz);
  }
  if (FUSE) fold_max(c, sh, slot, st.mx, st.mz, st.md, st.bad);
}

template <bool FUSE, bool STR>
__global__ __launch_bounds__(256) void sweep_z2d(Coef c, Shared* sh, const double* zr,
                                                 int slot, int first,
                                                 const double* __restrict__ X,
                                                 double* __restrict__ Y, int kc,
                                                 int nstrips, int nwaves) {
  const int lane = threadIdx.x & 63;
  // wave-uniform by construction; readfirstlane lets the compiler keep it scalar
  const int w = __builtin_amdgcn_readfirstlane(xcd_block() * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const double dt = step_dt<STR>(c, sh, slot);
  step_head(c, sh, slot, first, dt);
  if (w >= nwaves) return;
  z2_wave<FUSE, STR>(c, sh, zr, slot, dt, X, Y, kc, w % nstrips, w / nstrips, lane);
}

// ---------------------------------------------------------------------------
// L_x(tau): flux differences across lanes, cross z-derivatives from the
// march.  Plate rows are copied through.

struct X2 {
  N2 pf[kPF];    // as in Z2
  double pz[kPF];
  N2 x[4];
  double zz[4];
  P2 pn[4];      // p filled on use
  N2 xp[4];
  P2 pp[4];
  double mx, mz, md;
  bool bad;
  double icen1;  // stretched grid: 1/(z_k+1 - z_k-1) of row f-2, carried
};

// The stages of one march step f of L_x (ring slots as for L_z).
// the head of every step, as z2_load
template <int S>
__device__ __forceinline__ void x2_load(const Coef& c, X2& st, int f, int flo, int fhi,
                                        const Cols& L, const double* __restrict__ zr,
                                        const double* __restrict__ X) {
  using Z = ZS<S>;
  st.x[Z::c0] = st.pf[Z::q0];
  st.zz[Z::c0] = st.pz[Z::q0];
  const int fp = min(max(f + kPF, flo), fhi);
  st.pf[Z::q0] = load2(c, X, fp, L.col);
  st.pz[Z::q0] = zr[fp];
  st.pn[Z::c0] = prim2(c, st.x[Z::c0], st.zz[Z::c0]);
}

// predictor on interior row f-1: X^P_i = X_i - (tau/dx)(F_i - F_{i-1})
// icz: 1/(centred z span) of the row: dz/2 uniform, z_k+1 - z_k-1 stretched
template <int S>
__device__ __forceinline__ void x2_pred(const Coef& c, X2& st, double z, double lx, double icz) {
  using Z = ZS<S>;
  P2 q = st.pn[Z::c1];
  q.p = c.a * st.x[Z::c1].r * q.T;
  double dxux = (up(q.ux) - q.ux) * c.ihx;
  double dxuz = (up(q.uz) - q.uz) * c.ihx;
  double dxT = (up(q.T) - q.T) * c.ihx;
  double dzux = (st.pn[Z::c0].ux - st.pn[Z::c2].ux) * icz;
  double dzuz = (st.pn[Z::c0].uz - st.pn[Z::c2].uz) * icz;
  N2 Fi = flux_x2(c, st.x[Z::c1], q, dxux, dxuz, dxT, dzux, dzuz);
  N2 Fm = dn(Fi);
  N2 v = st.x[Z::c1] - N2{lx * (Fi.r - Fm.r), lx * (Fi.mx - Fm.mx), lx * (Fi.mz - Fm.mz),
                          lx * (Fi.E - Fm.E)};
  st.xp[Z::c1] = v;
  st.pp[Z::c1] = prim2(c, v, z);
}

// corrector, average and TVD term on interior row f-2
template <int S>
__device__ __forceinline__ N2 x2_corr(const Coef& c, const X2& st, double lx, double icz) {
  using Z = ZS<S>;
  const P2& q = st.pp[Z::c2];
  double dxux = (q.ux - dn(q.ux)) * c.ihx;
  double dxuz = (q.uz - dn(q.uz)) * c.ihx;
  double dxT = (q.T - dn(q.T)) * c.ihx;
  double dzux = (st.pp[Z::c1].ux - st.pp[Z::c3].ux) * icz;
  double dzuz = (st.pp[Z::c1].uz - st.pp[Z::c3].uz) * icz;
  N2 Fi = flux_x2(c, st.xp[Z::c2], q, dxux, dxuz, dxT, dzux, dzuz);
  N2 Fp = up(Fi);
  const N2& x0 = st.x[Z::c2];
  N2 xc = x0 - N2{lx * (Fp.r - Fi.r), lx * (Fp.mx - Fi.mx), lx * (Fp.mz - Fi.mz),
                  lx * (Fp.E - Fi.E)};
  // TVD: face i+1/2 belongs to lane i; its dX_{+3/2}.dX_{+1/2} product is
  // the dX_{-1/2}.dX_{+1/2} product of face i+3/2, one lane up
  N2 d0 = up(x0) - x0;
  double G = 0.0;
  if (c.tvd_on) {
    N2 dm = dn(d0);
    double a_m = dot2(dm, d0);
    double s0 = fabs(st.pn[Z::c2].ux) + sound(c, st.pn[Z::c2].T);
    double Co = lx * fmax(s0, up(s0));
    G = tvd_G(c, a_m, up(a_m), dot2(d0, d0), Co);
  }
  N2 D{G * d0.r, G * d0.mx, G * d0.mz, G * d0.E};
  N2 Dm = dn(D);
  const N2& xp = st.xp[Z::c2];
  N2 out;
  out.r = 0.5 * (xp.r + xc.r) + (D.r - Dm.r);
  out.mx = 0.5 * (xp.mx + xc.mx) + (D.mx - Dm.mx);
  out.mz = 0.5 * (xp.mz + xc.mz) + (D.mz - Dm.mz);
  out.E = 0.5 * (xp.E + xc.E) + (D.E - Dm.E);
  return out;
}

// One march step (plate rows are copied through).
template <int S, bool FUSE, bool STR>
__device__ __forceinline__ void x2_iter(const Coef& c, X2& st, int f, int fs, int fe,
                                        int k0, int k1, const Cols& L,
                                        const double* __restrict__ zr,
                                        const double* __restrict__ X,
                                        double* __restrict__ Y, double lx) {
  using Z = ZS<S>;
  x2_load<S>(c, st, f, fs, min(c.M, k1 + 1), L, zr, X);
  if (f < fs || f > fe) return;
  const int M = c.M;
  const int r1 = f - 1;
  // stretched grid: centred span of row r1 from the ring heights (rows past
  // a plate hold clamped heights; their values are never used)
  const double icen = STR ? frcp(st.zz[Z::c0] - st.zz[Z::c2]) : 0.5 * c.ihz;
  if (r1 >= k0 - 1 && r1 >= 0 && r1 <= M) {
    if (r1 == 0 || r1 == M) {
      st.xp[Z::c1] = st.x[Z::c1];
      st.pp[Z::c1] = st.pn[Z::c1];
    } else {
      x2_pred<S>(c, st, st.zz[Z::c1], lx, icen);
    }
  }
  const int r = f - 2;
  if (r >= k0 && r < k1) {
    N2 out = (r == 0 || r == M) ? st.x[Z::c2] : x2_corr<S>(c, st, lx, STR ? st.icen1 : icen);
    if (FUSE) {
      double izs = 1.0;
      if (STR) {   // 1/(narrowest face of row r); one face at a plate
        const double hu = st.zz[Z::c1] - st.zz[Z::c2], hd = st.zz[Z::c2] - st.zz[Z::c3];
        izs = frcp(r == 0 ? hu : r == M ? hd : fmin(hu, hd));
      }
      out_max(c, out, st.zz[Z::c2], izs, c.dt_rule ? diff_h2(c, r) : 0.0, st.mx, st.mz,
              st.md, st.bad, L.out);
    }
    if (L.out) store2(c, Y, r, L.col, out);
  }
  if (STR) st.icen1 = icen;
}

// one wave's share of L_x: columns of `strip`, output rows of `chunk`
template <bool FUSE, bool STR>
__device__ __forceinline__ void x2_wave(const Coef& c, Shared* sh, const double* zr, int slot,
                                        double dt, const double* __restrict__ X,
                                        double* __restrict__ Y, int kc, int strip,
                                        int chunk, int lane) {
  const Cols L = lane_cols(c, strip, lane);
  const int k0 = chunk * kc;
  const int k1 = min(k0 + kc, c.nz);
  const double lx = 0.5 * dt * c.ihx;
  X2 st;
  st.mx = 0.0;
  st.mz = 0.0;
  st.md = INFINITY;
  st.bad = false;
  st.icen1 = 0.0;
  const int fs = max(0, k0 - 2);
  const int fe = k1 + 1;
  // the kPF steps before fs only load rows fs .. fs+kPF-1 (their heads);
  // the heads before them copy this defined, unused row
  for (int q = 0; q < kPF; ++q) {
    st.pf[q] = N2{1.0, 0.0, 0.0, 1.0};
    st.pz[q] = 0.0;
  }
  for (int fb = (fs - kPF) & ~3; fb <= fe; fb += 4) {
    x2_iter<0, FUSE, STR>(c, st, fb + 0, fs, fe, k0, k1, L, zr, X, Y, lx);
    x2_iter<1, FUSE, STR>(c, st, fb + 1, fs, fe, k0, k1, L, zr, X, Y, lx);
    x2_iter<2, FUSE, STR>(c, st, fb + 2, fs, fe, k0, k1, L, zr, X, Y, lx);
    x2_iter<3, FUSE, STR>(c, st, fb + 3, fs, fe, k0, k1, L, zr, X, Y, lx);
  }
  if (FUSE) fold_max(c, sh, slot, st.mx, st.mz, st.md, st.bad);
}

template <bool FUSE, bool STR>
__global__ __launch_bounds__(256) void sweep_x2d(Coef c, Shared* sh, const double* zr,
                                                 int slot, int first,
                                                 const double* __restrict__ X,
                                                 double* __restrict__ Y, int kc,
                                                 int nstrips, int nwaves) {
  const int lane = threadIdx.x & 63;
  // wave-uniform by construction; readfirstlane lets the compiler keep it scalar
  const int w = __builtin_amdgcn_readfirstlane(xcd_block() * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const double dt = step_dt<STR>(c, sh, slot);
  step_head(c, sh, slot, first, dt);
  if (w >= nwaves) return;
  x2_wave<FUSE, STR>(c, sh, zr, slot, dt, X, Y, kc, w % nstrips, w / nstrips, lane);
}

// ---------------------------------------------------------------------------
// Many independent boxes in one launch: every wave takes one work item
// (box, strip, chunk, lead) and runs the same per-wave code on that box's
// constants, state, plate table and scalars.  The lead wave of a box does
// the box's per-step bookkeeping.

template <int AXIS, bool FUSE>
__global__ __launch_bounds__(256) void sweep_batch2d(const BoxDesc* __restrict__ boxes,
                                                     const int4* __restrict__ items,
                                                     int nitems, Shared* shs,
                                                     const double* zarena, int slot,
                                                     int first, const double* X,
                                                     double* Y) {
  const int lane = threadIdx.x & 63;
  // wave-uniform by construction; readfirstlane lets the compiler keep it scalar
  const int w = __builtin_amdgcn_readfirstlane(xcd_block() * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (w >= nitems) return;
  const int4 it = items[w];
  const BoxDesc* bd = boxes + it.x;
  const Coef c = bd->c;
  Shared* sh = shs + it.x;
  const double dt = step_dt(c, sh, slot);
  if (first && it.w) {
    if (lane == 0) {
      sh->time += dt;
      sh->dt_last = dt;
    }
    sh->smax[slot ^ 1][lane >> 2][lane & 3] = 0ull;   // 64 lanes, 16 x 4 entries
  }
  const double* zr = zarena + bd->zoff;
  if (AXIS == 2)
    z2_wave<FUSE, false>(c, sh, zr, slot, dt, X + bd->off, Y + bd->off, bd->kc_z, it.y, it.z,
                         lane);
  else
    x2_wave<FUSE, false>(c, sh, zr, slot, dt, X + bd->off, Y + bd->off, bd->kc_x, it.y, it.z,
                         lane);
}

// ---------------------------------------------------------------------------

int strips_2d(int nx) { return (nx + kStrip - 1) / kStrip; }

int wave_slots_2d(int axis, bool fuse) {
  int dev = 0, cus = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const void* fn;
  if (axis == 2)
    fn = fuse ? (const void*)sweep_z2d<true, false> : (const void*)sweep_z2d<false, false>;
  else
    fn = fuse ? (const void*)sweep_x2d<true, false> : (const void*)sweep_x2d<false, false>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, 0) != hipSuccess) return 0;
  // at most two waves per SIMD (two 4-wave blocks per CU): where a third
  // fits, longer marches for two still measured faster (fewer halo rows)
  return min(nb, 2) * 4 * cus;
}

hipError_t launch_batch_2d(int axis, const BoxDesc* boxes, const int4* items, int nitems,
                           Shared* shs, const double* zarena, int slot, int first, bool fuse,
                           const double* X, double* Y, hipStream_t s) {
  const int grid = (nitems + 3) / 4;
  if (axis == 2) {
    if (fuse)
      sweep_batch2d<2, true><<<grid, 256, 0, s>>>(boxes, items, nitems, shs, zarena, slot, first, X, Y);
    else
      sweep_batch2d<2, false><<<grid, 256, 0, s>>>(boxes, items, nitems, shs, zarena, slot, first, X, Y);
  } else {
    if (fuse)
      sweep_batch2d<0, true><<<grid, 256, 0, s>>>(boxes, items, nitems, shs, zarena, slot, first, X, Y);
    else
      sweep_batch2d<0, false><<<grid, 256, 0, s>>>(boxes, items, nitems, shs, zarena, slot, first, X, Y);
  }
  return hipGetLastError();
}

hipError_t launch_sweep_2d(int axis, const Coef& c, Shared* sh, const double* zr, int slot,
                           int first, bool fuse, const double* X, double* Y, int kc,
                           hipStream_t s) {
  const int nstrips = strips_2d(c.nx);
  const int nchunks = (c.nz + kc - 1) / kc;
  const int nwaves = nstrips * nchunks;
  const int block = 256;
  const int grid = (nwaves + 3) / 4;
#define MTVD_LAUNCH(K, F, T) K<F, T><<<grid, block, 0, s>>>(c, sh, zr, slot, first, X, Y, kc, nstrips, nwaves)
  const bool st = c.stretched != 0;
  if (axis == 2) {
    if (st) {
      if (fuse) MTVD_LAUNCH(sweep_z2d, true, true); else MTVD_LAUNCH(sweep_z2d, false, true);
    } else {
      if (fuse) MTVD_LAUNCH(sweep_z2d, true, false); else MTVD_LAUNCH(sweep_z2d, false, false);
    }
  } else {
    if (st) {
      if (fuse) MTVD_LAUNCH(sweep_x2d, true, true); else MTVD_LAUNCH(sweep_x2d, false, true);
    } else {
      if (fuse) MTVD_LAUNCH(sweep_x2d, true, false); else MTVD_LAUNCH(sweep_x2d, false, false);
    }
  }
#undef MTVD_LAUNCH
  return hipGetLastError();
}

}  // namespace mtvd
