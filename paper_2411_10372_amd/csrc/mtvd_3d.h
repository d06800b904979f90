// mtvd_3d.h -- fused predictor/corrector/TVD kernels of the directional
// operators L_x, L_y, L_z in 3D (Sec. 3.1 of arXiv:2411.10372), as
// templates; mtvd_3d_x.hip, mtvd_3d_y.hip and mtvd_3d_z.hip instantiate
// and launch one operator each (the L_z file without fused multiply-adds).
//
// Launch shape: a block of kNW = 8 waves.  Lanes run along x (60 output
// columns per wave plus two halo columns each side, exchanged with DPP wave
// shifts); each wave marches along one axis with its values in period-4
// register rings and rows prefetched two ahead; the 8 waves of a block sit
// at consecutive
// indices of the third axis, 4 of them produce output and 2 on each side
// are halo, and they exchange two scalars per row through LDS.
//   L_z: march z (flux direction, plates), waves along y (periodic)
//   L_y: march y (flux direction, periodic), waves along z (plate rows are
//        copied through; waves outside the plates idle)
//   L_x: flux across lanes, march z, waves along y
// Every kernel reads and writes each field of each node once (5 fields x 8 B
// in and out); halo re-reads hit in L2.
#pragma once

#include "mtvd_device.h"
#include "mtvd_launch.h"

namespace mtvd {

constexpr int kNW = 8;                  // waves per block
constexpr int kLW = 32;                 // lanes per plane row (x columns)
constexpr int kPPW = 64 / kLW;          // planes per wave
constexpr int kPB = kNW * kPPW;         // planes per block (2 halo each side)
constexpr int kPer = kPB - 4;           // output planes per block
constexpr int kStrip3 = kLW - 4;        // output columns per strip

struct N3 { double r, m[3], E; };
struct P3 { double u[3], T, p; };

__device__ __forceinline__ N3 sub3(const N3& a, const N3& b) {
  return N3{a.r - b.r, {a.m[0] - b.m[0], a.m[1] - b.m[1], a.m[2] - b.m[2]}, a.E - b.E};
}

__device__ __forceinline__ P3 prim3(const Coef& c, const N3& x, double z) {
  double ri = frcp(x.r);
  P3 q;
  q.u[0] = x.m[0] * ri;
  q.u[1] = x.m[1] * ri;
  q.u[2] = x.m[2] * ri;
  double ke = 0.5 * ((q.u[0] * q.u[0] + q.u[1] * q.u[1]) + q.u[2] * q.u[2]);
  q.T = (x.E * ri - ke - c.g * z) * c.icv;
  q.p = c.a * x.r * q.T;
  return q;
}

__device__ __forceinline__ double dot3(const N3& a, const N3& b) {
  return (((a.r * b.r + a.m[0] * b.m[0]) + a.m[1] * b.m[1]) + a.m[2] * b.m[2]) + a.E * b.E;
}

// Flux F_AL (Sec. 3.1) from the velocity gradient du[g][d] = d_d u_g and
// d_AL T; only the entries the flux uses are read: du[g][AL] (inner),
// du[AL][g] (cross) and the diagonal (divergence).
template <int AL>
__device__ __forceinline__ N3 flux3(const Coef& c, const N3& x, const P3& q,
                                    const double (&du)[3][3], double dT) {
  double div = (du[0][0] + du[1][1]) + du[2][2];
  double tau[3];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    if (g == AL)
      tau[g] = c.mu * ((du[AL][AL] + du[AL][AL]) + c.lam * div);
    else
      tau[g] = c.mu * (du[g][AL] + du[AL][g]);
  }
  const double ua = q.u[AL];
  N3 F;
  F.r = x.m[AL];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    double v = x.m[g] * ua - tau[g];
    if (g == AL) v = v + q.p;
    F.m[g] = v;
  }
  double work = (q.u[0] * tau[0] + q.u[1] * tau[1]) + q.u[2] * tau[2];
  F.E = (ua * (x.E + q.p) - c.K * dT) - work;
  return F;
}

// value of lane i+1 (shd) / lane i-1 (shu)
__device__ __forceinline__ double shd(double v) { return lane_from_above(v); }
__device__ __forceinline__ double shu(double v) { return lane_from_below(v); }
__device__ __forceinline__ N3 shd(const N3& v) {
  return N3{shd(v.r), {shd(v.m[0]), shd(v.m[1]), shd(v.m[2])}, shd(v.E)};
}
__device__ __forceinline__ N3 shu(const N3& v) {
  return N3{shu(v.r), {shu(v.m[0]), shu(v.m[1]), shu(v.m[2])}, shu(v.E)};
}

// A lane's place in the block: column x of its plane row (two halo columns
// each side) and plane p of the block (two halo planes each side); wave w
// holds planes kPPW w .. kPPW w + kPPW-1, so a plane row is kLW consecutive
// lanes and the lane shifts along x stay inside it for every lane whose
// result is kept.
struct Lane3 {
  int col;    // grid column
  int x, p;   // column in the plane row, plane in the block
  int role;   // 0: outer halo plane (X^n only), 1: inner halo plane (X^P), 2: output plane
  bool out;   // column of an output lane (the plane decides the rest)
};

__device__ __forceinline__ Lane3 lane3(const Coef& c, int strip, int w, int lane) {
  Lane3 r;
  r.x = lane % kLW;
  r.p = w * kPPW + lane / kLW;
  int i0 = strip * kStrip3;
  int i = i0 - 2 + r.x;
  int m = i % c.nx;
  r.col = (m < 0) ? m + c.nx : m;
  r.out = r.x >= 2 && r.x < kLW - 2 && (i0 + r.x - 2) < c.nx;
  r.role = (r.p == 0 || r.p == kPB - 1) ? 0 : ((r.p == 1 || r.p == kPB - 2) ? 1 : 2);
  return r;
}

// height of row k, z_k = k / M: the correctly rounded IEEE quotient, the
// same number as the plate table the library fills (and the oracle's), so
// computing it on use costs a division and no registers
__device__ __forceinline__ double zrow(int k, int M) { return (double)k / (double)M; }

__device__ __forceinline__ int wrap(int v, int n) {
  int m = v % n;
  return m < 0 ? m + n : m;
}

__device__ __forceinline__ N3 load3(const Coef& c, const double* __restrict__ X,
                                    long long n) {
  N3 v;
  v.r = X[n];
  v.m[0] = X[n + c.cnt];
  v.m[1] = X[n + 2 * c.cnt];
  v.m[2] = X[n + 3 * c.cnt];
  v.E = X[n + 4 * c.cnt];
  return v;
}

__device__ __forceinline__ void store3(const Coef& c, double* __restrict__ Y, long long n,
                                       const N3& v) {
  Y[n] = v.r;
  Y[n + c.cnt] = v.m[0];
  Y[n + 2 * c.cnt] = v.m[1];
  Y[n + 3 * c.cnt] = v.m[2];
  Y[n + 4 * c.cnt] = v.E;
}

// The same at node u + (this lane's node within a z plane), where u is the
// same for the whole wave and the lane's part comes as a byte offset below
// 4 GiB (the launcher checks 8 nx ny < 2^32): the field bases stay scalar
// and a lane's address costs one 32-bit register.
__device__ __forceinline__ const double& at_ob(const double* __restrict__ p, unsigned ob) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(p) + ob);
}
__device__ __forceinline__ N3 load3o(const Coef& c, const double* __restrict__ X, long long u,
                                     unsigned ob) {
  const double* b = X + u;
  N3 v;
  v.r = at_ob(b, ob);
  v.m[0] = at_ob(b + c.cnt, ob);
  v.m[1] = at_ob(b + 2 * c.cnt, ob);
  v.m[2] = at_ob(b + 3 * c.cnt, ob);
  v.E = at_ob(b + 4 * c.cnt, ob);
  return v;
}
__device__ __forceinline__ void store3o(const Coef& c, double* __restrict__ Y, long long u,
                                        unsigned ob, const N3& v) {
  char* b = reinterpret_cast<char*>(Y + u);
  const long long fs = c.cnt * (long long)sizeof(double);
  *reinterpret_cast<double*>(b + ob) = v.r;
  *reinterpret_cast<double*>(b + fs + ob) = v.m[0];
  *reinterpret_cast<double*>(b + 2 * fs + ob) = v.m[1];
  *reinterpret_cast<double*>(b + 3 * fs + ob) = v.m[2];
  *reinterpret_cast<double*>(b + 4 * fs + ob) = v.E;
}

// Two scalars of every lane to LDS, barrier, and their central differences
// across neighbouring planes (the block's edge planes take a zero
// difference; they are outer halo).  Each exchange array has two buffers that
// alternate with the parity of the march row: two exchanges in a row on the
// same array (at a chunk's first rows, at the top plate) then use different
// buffers, and the barrier of the second one orders every read of the first
// before the next write to its buffer, so a wave that runs ahead never
// overwrites a value a slower wave has yet to read.
__device__ __forceinline__ void exchange(double (&buf)[2][kPB * kLW], const Lane3& L,
                                         double a, double b, double ih2, double& da,
                                         double& db) {
  const int i = L.p * kLW + L.x;
  buf[0][i] = a;
  buf[1][i] = b;
  __syncthreads();
  const int im = (L.p > 0) ? i - kLW : i;
  const int ip = (L.p < kPB - 1) ? i + kLW : i;
  da = (buf[0][ip] - buf[0][im]) * ih2;
  db = (buf[1][ip] - buf[1][im]) * ih2;
}

struct Acc3 {
  double s[3];
  double md;   // min of rho h^2 (dt_rule = 1)
  bool bad;
};

// izs: 1 on the uniform grid; 1/h_z of the node on a stretched one (the z
// entry then collects (|u_z| + c)/h_z, which dt divides into 1)
// h2: the node's diff_h2 (dt_rule = 1)
// DIFF: also the minimum of rho h^2 (dt_rule = 1)
template <bool DIFF>
__device__ __forceinline__ void acc_out(const Coef& c, const N3& o, double z, double izs,
                                        double h2, Acc3& a, bool on) {
  P3 q = prim3(c, o, z);
  double cs = sound(c, q.T);
  double s0 = fabs(q.u[0]) + cs, s1 = fabs(q.u[1]) + cs, s2 = (fabs(q.u[2]) + cs) * izs;
  if (on) {
    a.s[0] = fmax(a.s[0], s0);
    a.s[1] = fmax(a.s[1], s1);
    a.s[2] = fmax(a.s[2], s2);
    if (DIFF) a.md = fmin(a.md, o.r * h2);
    if (!(o.r > 0.0) || !(q.T > 0.0) || !(s0 < INFINITY) || !(s1 < INFINITY) ||
        !(s2 < INFINITY))
      a.bad = true;
  }
}

template <bool DIFF>
__device__ __forceinline__ void fold3(Shared* sh, int slot, Acc3& a) {
  double m0 = wave_max(a.s[0]), m1 = wave_max(a.s[1]), m2 = wave_max(a.s[2]);
  const double md = DIFF ? wave_min(a.md) : 0.0;
  unsigned long long anybad = __ballot(a.bad);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&sh->smax[slot ^ 1][max_part()][0], d2u(m0));
    atomicMax(&sh->smax[slot ^ 1][max_part()][1], d2u(m1));
    atomicMax(&sh->smax[slot ^ 1][max_part()][2], d2u(m2));
    if (DIFF) fold_rho_h2(sh, slot ^ 1, max_part(), md);
    if (anybad) atomicOr(&sh->flags, 1u);
  }
}

__device__ __forceinline__ void head3(Shared* sh, int slot, int first, double dt) {
  if (first && blockIdx.x == 0 && threadIdx.x < kMaxParts * 4) {
    if (threadIdx.x == 0) {
      sh->time += dt;
      sh->dt_last = dt;
    }
    sh->smax[slot ^ 1][threadIdx.x >> 2][threadIdx.x & 3] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// L_z and L_y: flux along the march.  AX = 2: march z, waves along y;
// AX = 1: march y, waves along z.

struct MF {
  N3 pf[2];                // prefetched rows f+1, f+2 (slot row & 1)
  N3 x[4];                 // X^n rows f-3..f (slot row & 3)
  P3 pn[4];                // primitives of X^n (p filled on use)
  double s[4];             // |u_AX| + c of X^n
  double G[2];             // TVD coefficient of face row+1/2
  N3 Dp;                   // G dX of the face below the next output row
  N3 F[2];
  N3 xp[4];
  P3 pp[4];
  N3 FP[2];
  Acc3 acc;
  // stretched grid (L_z) only: the metrics derived from the heights (read
  // from LDS) carried one march step
  double ihf1, ihf2, iw1;  // 1/h of faces f-3+1/2, f-4+1/2; 1/w of row f-3
  double iwb, iwt;         // the plate stencils' 1/(stencil applied to z)
};

// Heights of the rows of a stretched grid for L_z, copied into LDS once per
// block: every wave of the block marches the same rows, and an LDS read waits
// only for LDS, not behind the rows in flight from HBM (a ring of prefetched
// heights in registers made these kernels spill).  The library accepts a
// stretched 3D grid up to this many rows.
constexpr int kZL3 = 2048;
__shared__ double zlds[kZL3];

// FO: 0 no fold; 1 fold max(|u_a| + c) of the output into the next step's
// slot; 2 also the minimum of rho h^2 (dt_rule = 1).
// PL: the launch's rows may touch a plate (L_z).  The rows between (first
// output row >= 4, last <= M-4: every stage then works on rows 2..M-4) run
// a copy compiled without the plate and wall code, whose registers fit
// without spilling.
// STR: a stretched z grid.  L_z takes every z spacing from the heights in
// LDS; L_y (waves along z) gets its wave's centred span and narrowest face
// in ihb2 and izw.
template <int AX, int S, int FO, bool PL, bool STR>
__device__ __forceinline__ void mf_iter(const Coef& c, MF& st, int f, int fs, int fe, int m0,
                                        int m1, const Lane3& L, unsigned lob, long long lnode,
                                        bool bval, bool bwall, bool owave,
                                        double (&xa)[2][2][kPB * kLW], double (&xb)[2][2][kPB * kLW],
                                        const double* __restrict__ zr,
                                        const double* __restrict__ X, double* __restrict__ Y,
                                        double tau, double lm, double zb, int flo, int fhi,
                                        double ihb2, double izw, double h2b) {
  constexpr int B = (AX == 2) ? 1 : 2;   // axis of the waves
  constexpr bool P = (AX == 2) && PL;    // plate rows possible in this chunk
  constexpr bool SZ = STR && AX == 2;    // stretched march along z
  const int M = c.M;
  const double ihm = (AX == 2) ? c.ihz : c.ihy;
  constexpr int c0 = S & 3, c1 = (S + 3) & 3, c2 = (S + 2) & 3, c3 = (S + 1) & 3, c4 = S & 3;
  constexpr int e0 = S & 1, e1 = (S + 1) & 1;
  const int role = L.role;
  // node of march row `row`: L_z the lane's column of z plane `row` (lane
  // part lob, a byte offset); L_y plane bidx, row `row` (lane part lnode)
  auto stnode = [&](int row, const N3& v) {
    if (AX == 2) store3o(c, Y, (long long)row * c.plane, lob, v);
    else store3(c, Y, (long long)wrap(row, c.ny) * c.nx + lnode, v);
  };
  // A (every step of the march, guarded by nothing): row f of X^n
  //    (prefetched two steps ago) and its primitives; prefetch row f+2 with
  //    its height; exchange across waves.  A guarded load would have to be
  //    copied into the loop-carried ring at the guard's end, and the copy
  //    waits for the load.  Row (L_z) and plane (waves outside the plates of
  //    L_y) indices are clamped into the grid; what such loads bring lands in
  //    ring slots no stage reads, and their exchanged values are zeroed.
  {
    st.x[c0] = st.pf[e0];
    const int fp = min(max(f + 2, flo), fhi);
    if (AX == 2) st.pf[e0] = load3o(c, X, (long long)fp * c.plane, lob);
    else st.pf[e0] = load3(c, X, (long long)wrap(fp, c.ny) * c.nx + lnode);
    st.pn[c0] = prim3(c, st.x[c0], SZ ? zlds[min(max(f, 0), M)] : (AX == 2) ? zrow(f, M) : zb);
    st.s[c0] = fabs(st.pn[c0].u[AX]) + sound(c, st.pn[c0].T);
  }
  if (f < fs || f > fe) return;
  // heights of rows f-2 and f-3 (L_z) or of the wave's plane (L_y)
  // (stretched L_z: rows past a plate read clamped heights; the values made
  // from them are never used)
  const double z_r = SZ ? zlds[min(max(f - 2, 0), M)] : (AX == 2) ? zrow(f - 2, M) : zb;
  const double z_o = SZ ? zlds[min(max(f - 3, 0), M)] : (AX == 2) ? zrow(f - 3, M) : zb;
  const int r = f - 2;
  // stretched L_z: face r+1/2 and dual cell of row r
  double hf = 0.0, ihf = 0.0, iw = 0.0;
  if (SZ) {
    const double z_1 = zlds[min(max(f - 1, 0), M)];
    hf = z_1 - z_r;
    ihf = frcp(hf);
    iw = 2.0 * frcp(z_1 - z_o);
  }
  const bool rin_F = P ? (r >= 0 && r <= M - 1) : true;
  // B: predictor flux F_r (inner derivatives forward along the march); the
  //    derivatives across the planes of row r first (every wave of the block
  //    takes part in the exchange: its condition is the same for all of them)
  double bb = 0.0, bm = 0.0;   // d_B u_B and d_B u_AX of X^n at row r
  if (r >= m0 - 2 && rin_F) {
    const double ub = bval ? st.pn[c2].u[B] : 0.0, um = bval ? st.pn[c2].u[AX] : 0.0;
    exchange(xa[S & 1], L, ub, um, ihb2, bb, bm);
  }
  if (r >= m0 - 2 && rin_F && role >= 1 && bval && !bwall) {
    P3 q0 = st.pn[c2];
    const P3& q1 = st.pn[c1];
    double du[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double dT;
    if (P && r == 0 && c.wall_order == 2) {
      const P3& q2 = st.pn[c0];
      double h2 = SZ ? st.iwb : 0.5 * ihm;
#pragma unroll
      for (int g = 0; g < 3; ++g) du[g][AX] = ((-3.0 * q0.u[g] + 4.0 * q1.u[g]) - q2.u[g]) * h2;
      dT = ((-3.0 * q0.T + 4.0 * q1.T) - q2.T) * h2;
    } else {
      const double ih = SZ ? ihf : ihm;
#pragma unroll
      for (int g = 0; g < 3; ++g) du[g][AX] = (q1.u[g] - q0.u[g]) * ih;
      dT = (q1.T - q0.T) * ih;
    }
    du[0][0] = (shd(q0.u[0]) - shu(q0.u[0])) * (0.5 * c.ihx);
    du[AX][0] = (shd(q0.u[AX]) - shu(q0.u[AX])) * (0.5 * c.ihx);
    du[B][B] = bb;
    du[AX][B] = bm;
    q0.p = c.a * st.x[c2].r * q0.T;
    st.F[e0] = flux3<AX>(c, st.x[c2], q0, du, dT);
  }
  // C: predictor X^P_r; exchange its velocities across the planes
  const bool rin_P = P ? (r >= 0 && r <= M) : true;
  double pb = 0.0, pm = 0.0;   // d_B u_B and d_B u_AX of X^P at row r
  if (r >= m0 - 1 && rin_P) {
    if (role >= 1 && bval) {
      if (bwall) {
        st.xp[c2] = st.x[c2];
        st.pp[c2] = st.pn[c2];
        st.pp[c2].p = c.a * st.x[c2].r * st.pn[c2].T;
      } else if (P && r == 0) {
        double rho = st.x[c2].r;
        st.xp[c2] = N3{rho, {0.0, 0.0, 0.0}, rho * (c.cv * c.Tb + c.g * z_r)};
        st.pp[c2] = P3{{0.0, 0.0, 0.0}, c.Tb, c.a * rho * c.Tb};
      } else if (P && r == M) {
        const double lt = SZ ? tau * st.ihf1 : lm;   // face M-1/2
        double rho = st.x[c2].r - lt * (st.x[c2].m[2] - st.x[c3].m[2]);
        st.xp[c2] = N3{rho, {0.0, 0.0, 0.0}, rho * (c.cv * c.Tt + c.g * z_r)};
        st.pp[c2] = P3{{0.0, 0.0, 0.0}, c.Tt, c.a * rho * c.Tt};
      } else {
        const N3& Fa = st.F[e0];
        const N3& Fb = st.F[e1];
        const N3& x0 = st.x[c2];
        const double lr = SZ ? tau * iw : lm;
        N3 v;
        v.r = x0.r - lr * (Fa.r - Fb.r);
#pragma unroll
        for (int g = 0; g < 3; ++g) v.m[g] = x0.m[g] - lr * (Fa.m[g] - Fb.m[g]);
        v.E = x0.E - lr * (Fa.E - Fb.E);
        if (AX == 2) v.m[2] = v.m[2] + tau * (-c.g * x0.r);
        st.xp[c2] = v;
        st.pp[c2] = prim3(c, v, z_r);
      }
    }
    double ub = (role >= 1 && bval) ? st.pp[c2].u[B] : 0.0;
    double um = (role >= 1 && bval) ? st.pp[c2].u[AX] : 0.0;
    exchange(xb[S & 1], L, ub, um, ihb2, pb, pm);
  }
  // D: corrector flux F^P_r (inner derivatives backward along the march)
  const bool rin_FP = P ? (r >= 1 && r <= M) : true;
  if (r >= m0 && rin_FP && role == 2 && bval && !bwall) {
    const P3& q0 = st.pp[c2];
    const P3& qm = st.pp[c3];
    double du[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double dT;
    if (P && r == M && c.wall_order == 2) {
      const P3& qmm = st.pp[c4];
      double h2 = SZ ? st.iwt : 0.5 * ihm;
#pragma unroll
      for (int g = 0; g < 3; ++g) du[g][AX] = ((3.0 * q0.u[g] - 4.0 * qm.u[g]) + qmm.u[g]) * h2;
      dT = ((3.0 * q0.T - 4.0 * qm.T) + qmm.T) * h2;
    } else {
      const double ih = SZ ? st.ihf1 : ihm;   // face r-1/2
#pragma unroll
      for (int g = 0; g < 3; ++g) du[g][AX] = (q0.u[g] - qm.u[g]) * ih;
      dT = (q0.T - qm.T) * ih;
    }
    du[0][0] = (shd(q0.u[0]) - shu(q0.u[0])) * (0.5 * c.ihx);
    du[AX][0] = (shd(q0.u[AX]) - shu(q0.u[AX])) * (0.5 * c.ihx);
    du[B][B] = pb;
    du[AX][B] = pm;
    st.FP[e0] = flux3<AX>(c, st.xp[c2], q0, du, dT);
  }
  // E: TVD coefficient of face r+1/2 along the march, jumps from the X ring
  const bool rin_G = P ? (r >= 0 && r <= M - 1) : true;
  if (r >= m0 - 1 && rin_G && role == 2 && bval && !bwall) {
    double G = 0.0;
    const bool active = P ? (r >= 1 && r <= M - 2) : true;
    if (c.tvd_on && active) {
      N3 dm = sub3(st.x[c2], st.x[c3]);
      N3 d0 = sub3(st.x[c1], st.x[c2]);
      N3 dp = sub3(st.x[c0], st.x[c1]);
      double Co = (SZ ? tau * ihf : lm) * fmax(st.s[c2], st.s[c1]);
      G = tvd_G(c, dot3(dm, d0), dot3(d0, dp), dot3(d0, d0), Co);
      if (SZ) G = G * hf;   // the face's dissipative flux carries its spacing
    }
    st.G[e0] = G;
  }
  // F: output row o = f-3; the face o+1/2 term G dX is carried to the next
  //    row as its o-1/2 term
  const int o = f - 3;
  const bool rin_O = P ? (o >= 0 && o <= M - 1) : true;
  if (o >= m0 - 1 && o < m1 && rin_O && owave && !bwall) {
    N3 d0 = sub3(st.x[c2], st.x[c3]);
    const double G = st.G[e1];
    N3 Dc{G * d0.r, {G * d0.m[0], G * d0.m[1], G * d0.m[2]}, G * d0.E};
    if (o >= m0 && (!P || o >= 1)) {
      const N3& fp1 = st.FP[e0];
      const N3& fp0 = st.FP[e1];
      const N3& x0 = st.x[c3];
      const N3& xp = st.xp[c3];
      const N3& Dm = st.Dp;
      const double lo = SZ ? tau * st.iw1 : lm;
      N3 xc;
      xc.r = x0.r - lo * (fp1.r - fp0.r);
#pragma unroll
      for (int g = 0; g < 3; ++g) xc.m[g] = x0.m[g] - lo * (fp1.m[g] - fp0.m[g]);
      xc.E = x0.E - lo * (fp1.E - fp0.E);
      if (AX == 2) xc.m[2] = xc.m[2] + tau * (-c.g * xp.r);
      N3 out;
      if (SZ) {   // face fluxes over the dual cell of row o
        const double iwo = st.iw1;
        out.r = 0.5 * (xp.r + xc.r) + (Dc.r - Dm.r) * iwo;
#pragma unroll
        for (int g = 0; g < 3; ++g)
          out.m[g] = 0.5 * (xp.m[g] + xc.m[g]) + (Dc.m[g] - Dm.m[g]) * iwo;
        out.E = 0.5 * (xp.E + xc.E) + (Dc.E - Dm.E) * iwo;
      } else {
        out.r = 0.5 * (xp.r + xc.r) + (Dc.r - Dm.r);
#pragma unroll
        for (int g = 0; g < 3; ++g) out.m[g] = 0.5 * (xp.m[g] + xc.m[g]) + (Dc.m[g] - Dm.m[g]);
        out.E = 0.5 * (xp.E + xc.E) + (Dc.E - Dm.E);
      }
      if (FO)
        acc_out<FO == 2>(c, out, z_o, SZ ? fmax(st.ihf1, st.ihf2) : izw,
                         FO == 2 ? ((AX == 2) ? diff_h2(c, o) : h2b) : 0.0, st.acc, L.out);
      if (L.out) stnode(o, out);
    }
    st.Dp = Dc;
  }
  if (o >= m0 && o < m1 && owave && (bwall || (P && (o == 0 || o == M)))) {
    N3 out;
    if (bwall) {
      out = st.x[c3];
    } else if (o == 0) {
      const double lb = SZ ? tau * st.ihf1 : lm;   // face 1/2
      double rho = st.x[c3].r - lb * (st.xp[c2].m[2] - 0.0);
      out = N3{rho, {0.0, 0.0, 0.0}, rho * (c.cv * c.Tb + c.g * z_o)};
    } else {
      double rho = st.xp[c3].r;
      out = N3{rho, {0.0, 0.0, 0.0}, rho * (c.cv * c.Tt + c.g * z_o)};
    }
    if (FO)
      acc_out<FO == 2>(c, out, z_o, SZ ? (bwall ? izw : o == 0 ? st.ihf1 : st.ihf2) : izw,
                       FO == 2 ? ((AX == 2) ? diff_h2(c, o) : h2b) : 0.0, st.acc, L.out);
    if (L.out) stnode(o, out);
  }
  if (SZ) {
    st.ihf2 = st.ihf1;
    st.ihf1 = ihf;
    st.iw1 = iw;
  }
}

template <int AX, int FO, bool PL, bool STR>
__global__ __launch_bounds__(64 * kNW) void sweep_mf3d(Coef c, Shared* sh, const double* zr,
                                                       int slot, int first,
                                                       const double* __restrict__ X,
                                                       double* __restrict__ Y, int kc,
                                                       int nstrips, int nbb, int row0,
                                                       int row_end) {
  __shared__ double xa[2][2][kPB * kLW];
  __shared__ double xb[2][2][kPB * kLW];
  constexpr int B = (AX == 2) ? 1 : 2;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const double dt = step_dt<STR>(c, sh, slot);
  head3(sh, slot, first, dt);
  int bid = xcd_block();
  const int strip = bid % nstrips;
  bid /= nstrips;
  const int bb = bid % nbb;
  const int chunk = bid / nbb;   // of this launch's rows [row0, row_end)
  const Lane3 L = lane3(c, strip, w, lane);
  const int nb_len = (B == 1) ? c.ny : c.nz;
  const int braw = bb * kPer - 2 + L.p;   // index of this lane's plane along B
  int bidx;
  bool bval, bwall;
  if (B == 1) {
    bidx = wrap(braw, c.ny);
    bval = true;
    bwall = false;
  } else {
    bidx = braw;
    bval = braw >= 0 && braw <= c.M;
    bwall = bval && (braw == 0 || braw == c.M);
  }
  const bool owave = L.role == 2 && braw >= 0 && braw < nb_len;
  const int m0 = row0 + chunk * kc;
  const int m1 = min(m0 + kc, row_end);
  const double tau = 0.5 * dt;
  const double lm = tau * ((AX == 2) ? c.ihz : c.ihy);
  MF st;
  st.acc.s[0] = st.acc.s[1] = st.acc.s[2] = 0.0;
  st.acc.md = INFINITY;
  st.acc.bad = false;
  st.Dp = N3{0.0, {0.0, 0.0, 0.0}, 0.0};
  const int fs = (AX == 2) ? max(0, m0 - 2) : m0 - 2;
  const int fe = m1 + 2;
  // rows the stages read: m0-2 .. m1+1 (in the plates for L_z); the head
  // loads clamped rows outside, which cache hits serve
  const int flo = (AX == 2) ? max(0, m0 - 2) : m0 - 2;
  const int fhi = (AX == 2) ? min(c.M, m1 + 1) : m1 + 1;
  // the plane this lane loads from (L_y: clamped into the plates) and its
  // height; the lane's part of its nodes' addresses
  const int bload = (AX == 1) ? min(max(bidx, 0), c.M) : bidx;
  const double zb = (AX == 1) ? zr[bload] : 0.0;
  const unsigned lob = (AX == 2) ? (unsigned)(bidx * c.nx + L.col) * 8u : 0u;
  const long long lnode = (AX == 1) ? (long long)bload * c.plane + L.col : 0;
  // L_y: h^2 of the lane's plane for the diffusion part of dt (dt_rule = 1)
  const double h2b = (AX == 1 && FO == 2) ? diff_h2(c, bload) : 0.0;
  // the centred span across the waves (y for L_z; z for L_y, which on a
  // stretched grid is the wave's plane's own) and, for L_y's dt entry, the
  // plane's narrowest face
  double ihb2 = 0.5 * ((B == 1) ? c.ihy : c.ihz), izw = 1.0;
  if (STR) {
    st.ihf1 = st.ihf2 = st.iw1 = 0.0;
    st.iwb = st.iwt = 0.0;
    if (AX == 2) {
      st.iwb = zmet(c, 0, kZM_IWALL);
      st.iwt = zmet(c, c.M, kZM_IWALL);
      for (int k = threadIdx.x; k <= c.M; k += blockDim.x) zlds[k] = zr[k];
      __syncthreads();
    } else {
      const double zu = zr[min(bload + 1, c.M)], zd = zr[max(bload - 1, 0)];
      if (bload >= 1 && bload <= c.M - 1) ihb2 = frcp(zu - zd);
      izw = frcp(bload == 0 ? zu - zb : bload == c.M ? zb - zd : fmin(zu - zb, zb - zd));
    }
  }
  // the steps fs-2 and fs-1 only load rows fs and fs+1 (their heads); the
  // heads before them copy this defined, unused row
  st.pf[0] = st.pf[1] = N3{1.0, {0.0, 0.0, 0.0}, 1.0};
  for (int fb = (fs - 2) & ~3; fb <= fe; fb += 4) {
    mf_iter<AX, 0, FO, PL, STR>(c, st, fb + 0, fs, fe, m0, m1, L, lob, lnode, bval, bwall, owave, xa, xb, zr, X, Y, tau, lm, zb, flo, fhi, ihb2, izw, h2b);
    mf_iter<AX, 1, FO, PL, STR>(c, st, fb + 1, fs, fe, m0, m1, L, lob, lnode, bval, bwall, owave, xa, xb, zr, X, Y, tau, lm, zb, flo, fhi, ihb2, izw, h2b);
    mf_iter<AX, 2, FO, PL, STR>(c, st, fb + 2, fs, fe, m0, m1, L, lob, lnode, bval, bwall, owave, xa, xb, zr, X, Y, tau, lm, zb, flo, fhi, ihb2, izw, h2b);
    mf_iter<AX, 3, FO, PL, STR>(c, st, fb + 3, fs, fe, m0, m1, L, lob, lnode, bval, bwall, owave, xa, xb, zr, X, Y, tau, lm, zb, flo, fhi, ihb2, izw, h2b);
  }
  if (FO) fold3<FO == 2>(sh, slot, st.acc);
}

// ---------------------------------------------------------------------------
// L_x: flux across lanes, march z, waves along y.

struct LF {
  N3 pf[2];                // prefetched rows f+1, f+2
  N3 x[4];
  P3 pn[4];
  double s[4];             // |u_x| + c of X^n
  double yx[4], yy[4];     // d_y u_x, d_y u_y of X^n
  N3 xp[4];
  P3 pp[4];
  double pyx[4], pyy[4];   // d_y u_x, d_y u_y of X^P
  Acc3 acc;
  double pz[2], zz[4];     // stretched grid: heights prefetched with their rows
  double icen1;            // stretched grid: 1/(z_k+1 - z_k-1) of row f-2
};

template <int S, int FO, bool STR>
__device__ __forceinline__ void lf_iter(const Coef& c, LF& st, int f, int fs, int fe, int k0,
                                        int k1, const Lane3& L, unsigned lob,
                                        bool owave, double (&xa)[2][2][kPB * kLW],
                                        double (&xb)[2][2][kPB * kLW],
                                        const double* __restrict__ zr,
                                        const double* __restrict__ X, double* __restrict__ Y,
                                        double lx, int flo, int fhi) {
  const int M = c.M;
  constexpr int c0 = S & 3, c1 = (S + 3) & 3, c2 = (S + 2) & 3, c3 = (S + 1) & 3;
  const int role = L.role;
  const double ihy2 = 0.5 * c.ihy;

  constexpr int e0 = S & 1;
  // every step, guarded by nothing (as in the march kernels of L_z, L_y)
  {
    st.x[c0] = st.pf[e0];
    if (STR) st.zz[c0] = st.pz[e0];
    const int fp = min(max(f + 2, flo), fhi);
    st.pf[e0] = load3o(c, X, (long long)fp * c.plane, lob);
    if (STR) st.pz[e0] = zr[fp];
    st.pn[c0] = prim3(c, st.x[c0], STR ? st.zz[c0] : zrow(f, M));
    st.s[c0] = fabs(st.pn[c0].u[0]) + sound(c, st.pn[c0].T);
    exchange(xa[S & 1], L, st.pn[c0].u[0], st.pn[c0].u[1], ihy2, st.yx[c0], st.yy[c0]);
  }
  if (f < fs || f > fe) return;
  // stretched grid: centred span of row f-1 from the ring heights (rows past
  // a plate hold clamped heights; their values are never used)
  const double icen = STR ? frcp(st.zz[c0] - st.zz[c2]) : 0.5 * c.ihz;
  // predictor on row f-1
  const int r1 = f - 1;
  if (r1 >= k0 - 1 && r1 >= 0 && r1 <= M) {
    if (role >= 1) {
      if (r1 == 0 || r1 == M) {
        st.xp[c1] = st.x[c1];
        st.pp[c1] = st.pn[c1];
      } else {
        P3 q = st.pn[c1];
        q.p = c.a * st.x[c1].r * q.T;
        double du[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int g = 0; g < 3; ++g) du[g][0] = (shd(q.u[g]) - q.u[g]) * c.ihx;
        double dT = (shd(q.T) - q.T) * c.ihx;
        du[0][1] = st.yx[c1];
        du[1][1] = st.yy[c1];
        du[0][2] = (st.pn[c0].u[0] - st.pn[c2].u[0]) * icen;
        du[2][2] = (st.pn[c0].u[2] - st.pn[c2].u[2]) * icen;
        N3 Fi = flux3<0>(c, st.x[c1], q, du, dT);
        N3 Fm = shu(Fi);
        const N3& x0 = st.x[c1];
        N3 v;
        v.r = x0.r - lx * (Fi.r - Fm.r);
#pragma unroll
        for (int g = 0; g < 3; ++g) v.m[g] = x0.m[g] - lx * (Fi.m[g] - Fm.m[g]);
        v.E = x0.E - lx * (Fi.E - Fm.E);
        st.xp[c1] = v;
        st.pp[c1] = prim3(c, v, STR ? st.zz[c1] : zrow(r1, M));
      }
    }
    double a = (role >= 1) ? st.pp[c1].u[0] : 0.0;
    double b = (role >= 1) ? st.pp[c1].u[1] : 0.0;
    exchange(xb[S & 1], L, a, b, ihy2, st.pyx[c1], st.pyy[c1]);
  }
  // corrector, average and TVD term on row f-2
  const int r = f - 2;
  if (r >= k0 && r < k1 && owave) {
    N3 out;
    if (r == 0 || r == M) {
      out = st.x[c2];
    } else {
      const P3& q = st.pp[c2];
      double du[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
      for (int g = 0; g < 3; ++g) du[g][0] = (q.u[g] - shu(q.u[g])) * c.ihx;
      double dT = (q.T - shu(q.T)) * c.ihx;
      du[0][1] = st.pyx[c2];
      du[1][1] = st.pyy[c2];
      const double icc = STR ? st.icen1 : icen;
      du[0][2] = (st.pp[c1].u[0] - st.pp[c3].u[0]) * icc;
      du[2][2] = (st.pp[c1].u[2] - st.pp[c3].u[2]) * icc;
      N3 Fi = flux3<0>(c, st.xp[c2], q, du, dT);
      N3 Fp = shd(Fi);
      const N3& x0 = st.x[c2];
      N3 xc;
      xc.r = x0.r - lx * (Fp.r - Fi.r);
#pragma unroll
      for (int g = 0; g < 3; ++g) xc.m[g] = x0.m[g] - lx * (Fp.m[g] - Fi.m[g]);
      xc.E = x0.E - lx * (Fp.E - Fi.E);
      N3 d0 = sub3(shd(x0), x0);
      double G = 0.0;
      if (c.tvd_on) {
        N3 dm = shu(d0);
        N3 dp = shd(d0);
        double Co = lx * fmax(st.s[c2], shd(st.s[c2]));
        G = tvd_G(c, dot3(dm, d0), dot3(d0, dp), dot3(d0, d0), Co);
      }
      N3 D{G * d0.r, {G * d0.m[0], G * d0.m[1], G * d0.m[2]}, G * d0.E};
      N3 Dm = shu(D);
      const N3& xp = st.xp[c2];
      out.r = 0.5 * (xp.r + xc.r) + (D.r - Dm.r);
#pragma unroll
      for (int g = 0; g < 3; ++g) out.m[g] = 0.5 * (xp.m[g] + xc.m[g]) + (D.m[g] - Dm.m[g]);
      out.E = 0.5 * (xp.E + xc.E) + (D.E - Dm.E);
    }
    if (FO) {
      double izs = 1.0;
      if (STR) {   // 1/(narrowest face of row r); one face at a plate
        const double hu = st.zz[c1] - st.zz[c2], hd = st.zz[c2] - st.zz[c3];
        izs = frcp(r == 0 ? hu : r == M ? hd : fmin(hu, hd));
      }
      acc_out<FO == 2>(c, out, STR ? st.zz[c2] : zrow(r, M), izs,
                       FO == 2 ? diff_h2(c, r) : 0.0, st.acc, L.out);
    }
    if (L.out) store3o(c, Y, (long long)r * c.plane, lob, out);
  }
  if (STR) st.icen1 = icen;
}

template <int FO, bool STR>
__global__ __launch_bounds__(64 * kNW) void sweep_lf3d(Coef c, Shared* sh, const double* zr,
                                                       int slot, int first,
                                                       const double* __restrict__ X,
                                                       double* __restrict__ Y, int kc,
                                                       int nstrips, int nbb) {
  __shared__ double xa[2][2][kPB * kLW];
  __shared__ double xb[2][2][kPB * kLW];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const double dt = step_dt<STR>(c, sh, slot);
  head3(sh, slot, first, dt);
  int bid = xcd_block();
  const int strip = bid % nstrips;
  bid /= nstrips;
  const int bb = bid % nbb;
  const int chunk = bid / nbb;
  const Lane3 L = lane3(c, strip, w, lane);
  const int jraw = bb * kPer - 2 + L.p;
  const int j = wrap(jraw, c.ny);
  const bool owave = L.role == 2 && jraw >= 0 && jraw < c.ny;
  const unsigned lob = (unsigned)(j * c.nx + L.col) * 8u;   // lane's part of its addresses
  const int k0 = chunk * kc;
  const int k1 = min(k0 + kc, c.nz);
  const double lx = 0.5 * dt * c.ihx;
  LF st;
  st.acc.s[0] = st.acc.s[1] = st.acc.s[2] = 0.0;
  st.acc.md = INFINITY;
  st.acc.bad = false;
  const int fs = max(0, k0 - 2);
  const int fe = k1 + 1;
  // rows the stages read (the head loads clamped rows outside, which cache
  // hits serve)
  const int flo = max(0, k0 - 2), fhi = min(c.M, k1 + 1);
  st.pf[0] = st.pf[1] = N3{1.0, {0.0, 0.0, 0.0}, 1.0};
  st.pz[0] = st.pz[1] = 0.0;
  st.icen1 = 0.0;
  for (int fb = (fs - 2) & ~3; fb <= fe; fb += 4) {
    lf_iter<0, FO, STR>(c, st, fb + 0, fs, fe, k0, k1, L, lob, owave, xa, xb, zr, X, Y, lx, flo, fhi);
    lf_iter<1, FO, STR>(c, st, fb + 1, fs, fe, k0, k1, L, lob, owave, xa, xb, zr, X, Y, lx, flo, fhi);
    lf_iter<2, FO, STR>(c, st, fb + 2, fs, fe, k0, k1, L, lob, owave, xa, xb, zr, X, Y, lx, flo, fhi);
    lf_iter<3, FO, STR>(c, st, fb + 3, fs, fe, k0, k1, L, lob, owave, xa, xb, zr, X, Y, lx, flo, fhi);
  }
  if (FO) fold3<FO == 2>(sh, slot, st.acc);
}

}  // namespace mtvd

namespace mtvd {

// one directional operator in 3D, per axis (mtvd_3d_x/y/z.hip); fo as FO
hipError_t launch_sweep_3d_x(const Coef& c, Shared* sh, const double* zr, int slot, int first,
                             int fo, const double* X, double* Y, int kc, hipStream_t s);
hipError_t launch_sweep_3d_y(const Coef& c, Shared* sh, const double* zr, int slot, int first,
                             int fo, const double* X, double* Y, int kc, hipStream_t s);
hipError_t launch_sweep_3d_z(const Coef& c, Shared* sh, const double* zr, int slot, int first,
                             int fo, const double* X, double* Y, int kc, hipStream_t s);

inline int strips_3d(int nx) { return (nx + kStrip3 - 1) / kStrip3; }

}  // namespace mtvd
