// mtvd_adjoint.h -- reverse mode (vector-Jacobian products) of one 2D
// directional operator L_a(tau) with tau fixed (frozen dt), stage by stage.
//
// The forward operator (Sec. 3.1 of arXiv:2411.10372) is taken as stages
// over whole arrays (primitives P of X; predictor fluxes F; X^P and its
// primitives P^P; corrector fluxes F^P; X^C; the TVD coefficient G of every
// face; the output).  Four passes take the cotangent of the output back to
// the cotangent of X and accumulate the cotangents of the diffusion
// coefficients mu and K (from which d/dRa follows): fw_all (P, |u|+c, X^P,
// P^P: forward values only, so it can run ahead of the cotangents), rv_tc
// (output, TVD faces and corrector), rv_pred (P^P -> X^P and the predictor)
// and rv_prim (P -> X).  Every pass is a function of one
// node that gathers what its neighbours contribute, recomputing the cheap
// neighbour values it needs instead of storing them, so no pass needs
// atomics.  fw_all runs as a kernel of its own; the three cotangent stages
// run fused over tiles (tile_tc, tile_pred, tile_prim: each stage's
// outputs stay in shared memory for the next), with the arithmetic of the
// per-node passes rv_tc, rv_pred and rv_prim, which state them over whole
// grids.  Limiter kinks take the branch the forward pass took.
//
// Layout: arrays of nf = 4 fields (or 4 primitive slots ux, uz, T, p) over
// nz x nx nodes, field-major, node n = k nx + i.
#pragma once

#ifndef MTVD_HD
#define MTVD_HD __host__ __device__
#endif

#include <math.h>

namespace mtvd {
namespace adj {

struct AC {                      // constants of one operator
  int nx, nz, M, axis;           // axis 0 = x, 2 = z
  long long cnt;
  double ihx, ihz, iha;          // 1/dx, 1/dz, 1/h along the axis
  double cv, icv, a, gam_a, g, mu, K, lam, Tb, Tt;
  double tau, lm;                // tau = dt/2, lm = tau/h_axis
  int wall_order, tvd_on, limiter_form;
};

// ---- indexing ---------------------------------------------------------------

MTVD_HD inline int wrapx(int i, int nx) { int m = i % nx; return m < 0 ? m + nx : m; }
MTVD_HD inline long long nid(const AC& c, int i, int k) { return (long long)k * c.nx + wrapx(i, c.nx); }
// neighbour of (i, k) along the operator's axis (d = +-1); plates bound z
MTVD_HD inline long long along(const AC& c, int i, int k, int d) {
  return c.axis == 0 ? nid(c, i + d, k) : nid(c, i, k + d);
}
MTVD_HD inline long long across(const AC& c, int i, int k, int d) {
  return c.axis == 0 ? nid(c, i, k + d) : nid(c, i + d, k);
}
MTVD_HD inline int pos(const AC& c, int i, int k) { return c.axis == 0 ? i : k; }

// Which nodes carry what (axis 0: rows 1..M-1 only; plate rows are copied).
MTVD_HD inline bool has_F(const AC& c, int i, int k) {      // predictor flux
  return c.axis == 0 ? (k >= 1 && k <= c.M - 1) : (k <= c.M - 1);
}
MTVD_HD inline bool has_FP(const AC& c, int i, int k) {     // corrector flux
  return c.axis == 0 ? (k >= 1 && k <= c.M - 1) : (k >= 1);
}
MTVD_HD inline bool interior(const AC& c, int k) { return k >= 1 && k <= c.M - 1; }
MTVD_HD inline bool has_D(const AC& c, int i, int k) {      // TVD face k+1/2 (or i+1/2)
  if (!c.tvd_on) return false;
  return c.axis == 0 ? (k >= 1 && k <= c.M - 1) : (k >= 1 && k <= c.M - 2);
}

MTVD_HD inline void ld4(const double* A, long long cnt, long long n, double v[4]) {
  for (int f = 0; f < 4; ++f) v[f] = A[f * cnt + n];
}
MTVD_HD inline void st4(double* A, long long cnt, long long n, const double v[4]) {
  for (int f = 0; f < 4; ++f) A[f * cnt + n] = v[f];
}

// ---- forward pieces -----------------------------------------------------------

// primitives (ux, uz, T, p) of a state node at height z
MTVD_HD inline void prim(const AC& c, const double x[4], double z, double q[4]) {
  double ri = 1.0 / x[0];
  q[0] = x[1] * ri;
  q[1] = x[2] * ri;
  double ke = 0.5 * (q[0] * q[0] + q[1] * q[1]);
  q[2] = (x[3] * ri - ke - c.g * z) * c.icv;
  q[3] = c.a * x[0] * q[2];
}

// flux along the axis from the state x, its primitives q and the
// derivatives d[0..4] = (D_a u_a, D_a u_c, D_a T, D_c u_a, D_c u_c), with u_a
// the velocity along the axis, u_c the other one, D_a the inner and D_c the
// central cross difference
MTVD_HD inline void flux(const AC& c, const double x[4], const double q[4], const double d[5],
                         double F[4]) {
  const int ia = c.axis == 0 ? 0 : 1, ic = 1 - ia;     // slots of u_a, u_c in q
  const double ma = x[1 + ia], mc = x[1 + ic], ua = q[ia], uc = q[ic], p = q[3];
  double div = d[0] + d[4];
  double taa = c.mu * ((d[0] + d[0]) + c.lam * div);
  double tca = c.mu * (d[1] + d[3]);
  F[0] = ma;
  F[1 + ia] = (ma * ua - taa) + p;
  F[1 + ic] = mc * ua - tca;
  F[3] = (ua * (x[3] + p) - c.K * d[2]) - (ua * taa + uc * tca);
}

// derivative inputs of the flux at node (i, k) from the primitive array Q
// (fwd = 1: inner forward difference, 0: backward), with the plate rule of
// the z operator
MTVD_HD inline void derivs(const AC& c, const double* Q, int i, int k, int fwd, double d[5]) {
  const long long cnt = c.cnt;
  const int ia = c.axis == 0 ? 0 : 1, ic = 1 - ia;
  const long long n = nid(c, i, k);
  double qa[3], q0[3];
  const int slots[3] = {ia, ic, 2};
  if (c.axis == 2 && fwd && k == 0 && c.wall_order == 2) {
    long long n1 = nid(c, i, 1), n2 = nid(c, i, 2);
    for (int s = 0; s < 3; ++s) {
      const double* A = Q + slots[s] * cnt;
      qa[s] = ((-3.0 * A[n] + 4.0 * A[n1]) - A[n2]) * (0.5 * c.iha);
    }
  } else if (c.axis == 2 && !fwd && k == c.M && c.wall_order == 2) {
    long long n1 = nid(c, i, c.M - 1), n2 = nid(c, i, c.M - 2);
    for (int s = 0; s < 3; ++s) {
      const double* A = Q + slots[s] * cnt;
      qa[s] = ((3.0 * A[n] - 4.0 * A[n1]) + A[n2]) * (0.5 * c.iha);
    }
  } else {
    long long m = along(c, i, k, fwd ? 1 : -1);
    for (int s = 0; s < 3; ++s) {
      const double* A = Q + slots[s] * cnt;
      q0[s] = A[n];
      qa[s] = fwd ? (A[m] - q0[s]) * c.iha : (q0[s] - A[m]) * c.iha;
    }
  }
  const double ihc2 = 0.5 * (c.axis == 0 ? c.ihz : c.ihx);
  long long cp = across(c, i, k, 1), cm = across(c, i, k, -1);
  d[0] = qa[0];
  d[1] = qa[1];
  d[2] = qa[2];
  d[3] = (Q[ia * cnt + cp] - Q[ia * cnt + cm]) * ihc2;
  d[4] = (Q[ic * cnt + cp] - Q[ic * cnt + cm]) * ihc2;
}

// ---- reverse pieces -------------------------------------------------------------

// Cotangents of the flux inputs: xb (state, added), qb (u_a, u_c, p slots
// of (ux, uz, T, p), added), db (the five derivative inputs, set), and the
// mu and K cotangents (added).
MTVD_HD inline void flux_vjp(const AC& c, const double x[4], const double q[4],
                             const double d[5], const double Fb[4], double xb[4],
                             double qb[4], double db[5], double* mub, double* Kb) {
  const int ia = c.axis == 0 ? 0 : 1, ic = 1 - ia;
  const double ma = x[1 + ia], mc = x[1 + ic], E = x[3], ua = q[ia], uc = q[ic], p = q[3];
  const double fr = Fb[0], fa = Fb[1 + ia], fc = Fb[1 + ic], fE = Fb[3];
  double div = d[0] + d[4];
  double taa = c.mu * ((d[0] + d[0]) + c.lam * div);
  double tca = c.mu * (d[1] + d[3]);
  xb[1 + ia] += fr + fa * ua;
  xb[1 + ic] += fc * ua;
  xb[3] += fE * ua;
  qb[ia] += fa * ma + fc * mc + fE * (E + p) - fE * taa;
  qb[ic] += -fE * tca;
  qb[3] += fa + fE * ua;
  double taab = -fa - fE * ua;
  double tcab = -fc - fE * uc;
  db[0] = c.mu * (2.0 + c.lam) * taab;
  db[4] = c.mu * c.lam * taab;
  db[1] = c.mu * tcab;
  db[3] = c.mu * tcab;
  db[2] = -c.K * fE;
  *mub += taab * ((d[0] + d[0]) + c.lam * div) + tcab * (d[1] + d[3]);
  *Kb += -fE * d[2];
}

// cotangent of the primitives (ux, uz, T, p) -> cotangent of the state
MTVD_HD inline void prim_vjp(const AC& c, const double x[4], double z, const double qb[4],
                             double xb[4]) {
  double ri = 1.0 / x[0];
  double ux = x[1] * ri, uz = x[2] * ri;
  double ke = 0.5 * (ux * ux + uz * uz);
  double T = (x[3] * ri - ke - c.g * z) * c.icv;
  double Tb = qb[2] + qb[3] * c.a * x[0];
  double rb = qb[3] * c.a * T;
  double eb = Tb * c.icv;
  double uxb = qb[0] - eb * ux, uzb = qb[1] - eb * uz;
  double rib = eb * x[3] + uxb * x[1] + uzb * x[2];
  xb[3] += eb * ri;
  xb[1] += uxb * ri;
  xb[2] += uzb * ri;
  xb[0] += rb - rib * ri * ri;
}

// TVD coefficient of a face and what its reverse needs
struct Face {
  double G, R, id, C, phi, Co, den;
  int arg;                       // 0: the max of Co taken at the lower node, 1: upper
  bool lin_phi, lin_C, live;
};

MTVD_HD inline double dot4(const double a[4], const double b[4]) {
  return ((a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]) + a[3] * b[3];
}

MTVD_HD inline Face face(const AC& c, const double dm[4], const double d0[4], const double dp[4],
                         double s0, double s1) {
  Face f;
  f.den = dot4(d0, d0);
  f.arg = s1 > s0 ? 1 : 0;
  f.Co = c.lm * (f.arg ? s1 : s0);
  f.live = f.den != 0.0;
  f.G = 0.0;
  f.R = f.id = f.C = f.phi = 0.0;
  f.lin_phi = f.lin_C = false;
  if (!f.live) return f;
  f.lin_C = f.Co <= 0.5;
  f.C = f.lin_C ? f.Co * (1.0 - f.Co) : 0.25;
  f.id = 1.0 / f.den;
  f.R = dot4(dm, d0) * f.id + dot4(d0, dp) * f.id;
  double t = 2.0 * f.R;
  f.lin_phi = t > 0.0 && t < 1.0;
  f.phi = t <= 0.0 ? 0.0 : (t >= 1.0 ? 1.0 : t);
  f.G = 0.5 * f.C * (1.0 - f.phi);
  return f;
}

// reverse of G = G(dm, d0, dp, s0, s1) for the printed limiter form, given
// Gb: adds to the jump cotangents and to the |u|+c cotangents of the two
// nodes (s0b lower, s1b upper)
MTVD_HD inline void face_vjp(const AC& c, const Face& f, const double dm[4], const double d0[4],
                             const double dp[4], double Gb, double dmb[4], double d0b[4],
                             double dpb[4], double* s0b, double* s1b) {
  if (!f.live) return;
  double Cb = Gb * 0.5 * (1.0 - f.phi);
  double phib = -Gb * 0.5 * f.C;
  double Rb = f.lin_phi ? 2.0 * phib : 0.0;
  double Cob = f.lin_C ? Cb * (1.0 - 2.0 * f.Co) : 0.0;
  double sb = Cob * c.lm;
  if (f.arg) *s1b += sb; else *s0b += sb;
  double amb = Rb * f.id, apb = Rb * f.id;
  double denb = -Rb * f.R * f.id;
  for (int q = 0; q < 4; ++q) {
    dmb[q] += amb * d0[q];
    d0b[q] += amb * dm[q] + apb * dp[q] + 2.0 * denb * d0[q];
    dpb[q] += apb * d0[q];
  }
}

// ---- the stages ---------------------------------------------------------------
// Arrays of one operator's reverse pass (4 x cnt unless noted):
//   X, P (primitives of X), S (1: |u_a| + c of X), XP, PP   forward values
//   Yb (output cotangent), Xb (input cotangent, the result)
//   XPb (X^P cotangent from the corrector), PPb, PB (primitive
//   cotangents), DPb, DB (5: derivative cotangents), SB (1: |u_a| + c
//   cotangent), MU, KB (1: per-node mu and K cotangents, accumulated over
//   every operator reversed until the caller clears them)
// The predictor fluxes, the X^C cotangent, the cotangents the TVD faces
// send to their jumps and the final X^P cotangent are not stored: the
// stages that need them recompute them for the few neighbours involved,
// with the same arithmetic.
struct Arr {
  const double *X, *zr;
  double *P, *S, *XP, *PP;
  const double* Yb;
  double *Xb, *XPb, *PPb, *PB, *DPb, *DB, *SB, *MU, *KB;
};

// primitives of X at a node
MTVD_HD inline void prim_node(const AC& c, const Arr& A, int i, int k, double q[4]) {
  double x[4];
  ld4(A.X, c.cnt, nid(c, i, k), x);
  prim(c, x, A.zr[k], q);
}

// derivative inputs of the predictor flux at (i, k) (forward inner
// differences, the bottom-plate rule of the z operator) from primitives
// recomputed from X: the same values derivs() takes from the stored P
MTVD_HD inline void derivs_x(const AC& c, const Arr& A, int i, int k, double d[5]) {
  const int ia = c.axis == 0 ? 0 : 1, ic = 1 - ia;
  const int slots[3] = {ia, ic, 2};
  double q0[4], qa[3];
  prim_node(c, A, i, k, q0);
  if (c.axis == 2 && k == 0 && c.wall_order == 2) {
    double q1[4], q2[4];
    prim_node(c, A, i, 1, q1);
    prim_node(c, A, i, 2, q2);
    for (int s = 0; s < 3; ++s)
      qa[s] = ((-3.0 * q0[slots[s]] + 4.0 * q1[slots[s]]) - q2[slots[s]]) * (0.5 * c.iha);
  } else {
    double qm[4];
    if (c.axis == 0) prim_node(c, A, i + 1, k, qm); else prim_node(c, A, i, k + 1, qm);
    for (int s = 0; s < 3; ++s) qa[s] = (qm[slots[s]] - q0[slots[s]]) * c.iha;
  }
  const double ihc2 = 0.5 * (c.axis == 0 ? c.ihz : c.ihx);
  double qp[4], qn[4];
  if (c.axis == 0) {
    prim_node(c, A, i, k + 1, qp);
    prim_node(c, A, i, k - 1, qn);
  } else {
    prim_node(c, A, i + 1, k, qp);
    prim_node(c, A, i - 1, k, qn);
  }
  d[0] = qa[0];
  d[1] = qa[1];
  d[2] = qa[2];
  d[3] = (qp[ia] - qn[ia]) * ihc2;
  d[4] = (qp[ic] - qn[ic]) * ihc2;
}

// predictor flux at (i, k) from X
MTVD_HD inline void flux_node(const AC& c, const Arr& A, int i, int k, double F[4]) {
  double x[4], q[4], d[5];
  ld4(A.X, c.cnt, nid(c, i, k), x);
  prim(c, x, A.zr[k], q);
  derivs_x(c, A, i, k, d);
  flux(c, x, q, d, F);
}

// forward: primitives and |u_a| + c of X; X^P and its primitives (plate
// rows as in the fused kernels), with the two predictor fluxes it needs
MTVD_HD inline void fw_all(const AC& c, const Arr& A, int i, int k) {
  long long n = nid(c, i, k);
  double x[4], v[4], q[4];
  ld4(A.X, c.cnt, n, x);
  prim(c, x, A.zr[k], q);
  st4(A.P, c.cnt, n, q);
  double ua = c.axis == 0 ? q[0] : q[1];
  A.S[n] = fabs(ua) + sqrt(c.gam_a * q[2]);
  if (c.axis == 0 && !interior(c, k)) {
    st4(A.XP, c.cnt, n, x);
    st4(A.PP, c.cnt, n, q);
    return;
  }
  if (c.axis == 2 && (k == 0 || k == c.M)) {
    double rho = x[0];
    double Tw = k == 0 ? c.Tb : c.Tt;
    if (k == c.M) rho = x[0] - c.lm * (x[2] - A.X[2 * c.cnt + nid(c, i, k - 1)]);
    v[0] = rho; v[1] = 0.0; v[2] = 0.0; v[3] = rho * (c.cv * Tw + c.g * A.zr[k]);
    q[0] = 0.0; q[1] = 0.0; q[2] = Tw; q[3] = c.a * rho * Tw;
    st4(A.XP, c.cnt, n, v);
    st4(A.PP, c.cnt, n, q);
    return;
  }
  double Fn[4], Fm[4];
  flux_node(c, A, i, k, Fn);
  if (c.axis == 0) flux_node(c, A, i - 1, k, Fm); else flux_node(c, A, i, k - 1, Fm);
  for (int f = 0; f < 4; ++f) v[f] = x[f] - c.lm * (Fn[f] - Fm[f]);
  if (c.axis == 2) v[2] = v[2] + c.tau * (-c.g * x[0]);
  prim(c, v, A.zr[k], q);
  st4(A.XP, c.cnt, n, v);
  st4(A.PP, c.cnt, n, q);
}

MTVD_HD inline void jump(const AC& c, const double* X, int i, int k, double d[4]) {
  // dX of the face between (i, k) and its upper neighbour along the axis
  long long n = nid(c, i, k), m = along(c, i, k, 1);
  for (int f = 0; f < 4; ++f) d[f] = X[f * c.cnt + m] - X[f * c.cnt + n];
}

// the output's cotangents of a node in row k, from its output cotangent yb
// (and, for row 1 of the z operator, y0: that of the plate node below it):
// the share of the input (plates that copy or close), of X^C and of X^P
MTVD_HD inline void out_cots(const AC& c, int k, const double yb[4], const double y0[4],
                             const double* zr, double xb[4], double xcb[4], double xpb[4]) {
  for (int q = 0; q < 4; ++q) xb[q] = xcb[q] = xpb[q] = 0.0;
  if (c.axis == 0) {
    if (interior(c, k)) {
      for (int q = 0; q < 4; ++q) xcb[q] = xpb[q] = 0.5 * yb[q];
    } else {
      for (int q = 0; q < 4; ++q) xb[q] = yb[q];    // plate rows are copied through
    }
    return;
  }
  if (k == 0) {                        // rho'_0 = rho_0 - lm m^P_z,1
    xb[0] = yb[0] + yb[3] * (c.cv * c.Tb + c.g * zr[0]);
  } else if (k == c.M) {               // rho'_M = rho^P_M
    xpb[0] = yb[0] + yb[3] * (c.cv * c.Tt + c.g * zr[c.M]);
  } else {
    for (int q = 0; q < 4; ++q) xcb[q] = xpb[q] = 0.5 * yb[q];
    if (k == 1) {                      // X^P_1 carries the bottom closure's m^P_z,1
      double r0b = y0[0] + y0[3] * (c.cv * c.Tb + c.g * zr[0]);
      xpb[2] += -c.lm * r0b;
    }
  }
}

// the reverse of one TVD face between two nodes along the axis, from the
// states x[0..3] of the four nodes around it (the face lies between x[1]
// and x[2]), |u|+c of its nodes (s0 lower, s1 upper) and their output
// cotangents (y0, y1): the cotangents it sends to its three jumps and to
// s0, s1
MTVD_HD inline void face_cot(const AC& c, const double (*x)[4], double s0, double s1,
                             const double y0[4], const double y1[4], double dmb[4],
                             double d0b[4], double dpb[4], double* s0b, double* s1b) {
  double dm[4], d0[4], dp[4];
  for (int q = 0; q < 4; ++q) {
    dm[q] = x[1][q] - x[0][q];
    d0[q] = x[2][q] - x[1][q];
    dp[q] = x[3][q] - x[2][q];
  }
  Face f = face(c, dm, d0, dp, s0, s1);
  // D_{n+1/2} enters Y_n with + and Y_{n+1} with -
  double Db[4];
  for (int q = 0; q < 4; ++q) Db[q] = y0[q] - y1[q];
  double Gb = dot4(Db, d0);
  for (int q = 0; q < 4; ++q) d0b[q] = f.G * Db[q];
  face_vjp(c, f, dm, d0, dp, Gb, dmb, d0b, dpb, s0b, s1b);
}

// What the first reverse stage yields at a node: the X cotangent so far,
// the X^P and P^P cotangents, the derivative-input cotangents of the
// corrector flux, the |u|+c cotangent and the node's mu and K cotangents.
struct TcOut {
  double xb[4], xpb[4], ppb[4], dpb[5], sb, mub, Kb;
};

// reverse of the output, the TVD faces and the corrector: the jump
// cotangents of the faces around (i, k) -> X; |u|+c cotangent of the node;
// X^C -> X; the corrector flux cotangent -> its inputs.  Reads only the
// forward values and the output cotangent, each value once, before any
// arithmetic: X on the seven nodes n-3..n+3 along the axis (the jumps of
// the faces n-2..n+1), |u|+c and the output cotangent on n-2..n+2, then
// X^P and P^P for the corrector flux.  Nodes beyond a plate read the node
// itself and are not used.
MTVD_HD inline void tc_node(const AC& c, const Arr& A, int i, int k, TcOut& o) {
  const long long n = nid(c, i, k);
  const long long cnt = c.cnt;
  const bool lo_ok = c.axis == 0 || k >= 1;        // a face below exists
  const bool hi_ok = c.axis == 0 || k <= c.M - 1;  // a face above exists
  const int di = c.axis == 0 ? 1 : 0, dk = c.axis == 0 ? 0 : 1;
  double x[7][4], s[5], yb[5][4];                  // index o+3 (x), o+2 (s, yb) for node n+o
  for (int o = -3; o <= 3; ++o) {
    const int kk = k + o * dk;
    const bool ok = c.axis == 0 || (kk >= 0 && kk <= c.M);
    const long long m = ok ? nid(c, i + o * di, kk) : n;
    for (int q = 0; q < 4; ++q) x[o + 3][q] = A.X[q * cnt + m];
    if (o >= -2 && o <= 2) {
      s[o + 2] = A.S[m];
      for (int q = 0; q < 4; ++q) yb[o + 2][q] = A.Yb[q * cnt + m];
    }
  }
  // faces (by lower node) n-2, n-1, n, n+1 along the axis: index f+2 for face n+f
  double am[4][4], a0[4][4], ap[4][4], s0[4], s1[4];
  for (int f = -2; f <= 1; ++f) {
    for (int q = 0; q < 4; ++q) am[f + 2][q] = a0[f + 2][q] = ap[f + 2][q] = 0.0;
    s0[f + 2] = s1[f + 2] = 0.0;
    const int kk = k + f * dk;
    const bool live = c.tvd_on && (c.axis == 0 ? (k >= 1 && k <= c.M - 1)
                                               : (kk >= 1 && kk <= c.M - 2));
    if (!live) continue;
    face_cot(c, x + f + 2, s[f + 2], s[f + 3],
             yb[f + 2], yb[f + 3], am[f + 2], a0[f + 2], ap[f + 2], &s0[f + 2], &s1[f + 2]);
  }
  double xb[4], xcb[4], xpb[4];
  out_cots(c, k, yb[2], yb[1], A.zr, xb, xcb, xpb);
  for (int q = 0; q < 4; ++q) {
    double own = 0.0, below = 0.0;
    if (hi_ok) {
      own = a0[2][q];                                                // face n
      if (c.axis == 0 || k + 1 <= c.M - 1) own += am[3][q];          // face n+1
      if (lo_ok) own += ap[1][q];                                    // face n-1
    }
    if (lo_ok) {
      below = a0[1][q];                                              // face n-1
      below += am[2][q];                                             // face n
      if (c.axis == 0 || k - 2 >= 0) below += ap[0][q];              // face n-2
    }
    xb[q] += below - own;
  }
  const double sb = s0[2] + (lo_ok ? s1[1] : 0.0);
  // X^C = X - lm (F^P_{n+1} - F^P_n) + tau S(X^P)
  for (int q = 0; q < 4; ++q) xb[q] += xcb[q];
  if (c.axis == 2 && interior(c, k)) xpb[0] += c.tau * (-c.g) * xcb[2];
  double qb[4] = {0, 0, 0, 0}, db[5] = {0, 0, 0, 0, 0};
  double mub = 0.0, Kb = 0.0;
  if (has_FP(c, i, k)) {
    double xcbm[4] = {0, 0, 0, 0};
    if (c.axis == 0 || k - 1 >= 1) {
      double t0[4], t1[4];
      out_cots(c, k - dk, yb[1], yb[0], A.zr, t0, xcbm, t1);
    }
    double Fb[4];
    for (int q = 0; q < 4; ++q) {
      double here = (c.axis == 0 || k <= c.M - 1) ? xcb[q] : 0.0;
      Fb[q] = c.lm * (here - xcbm[q]);
    }
    double xp[4], p4[4], d[5];
    ld4(A.XP, cnt, n, xp);
    ld4(A.PP, cnt, n, p4);
    derivs(c, A.PP, i, k, 0, d);
    flux_vjp(c, xp, p4, d, Fb, xpb, qb, db, &mub, &Kb);
  }
  for (int q = 0; q < 4; ++q) {
    o.xb[q] = xb[q];
    o.xpb[q] = xpb[q];
    o.ppb[q] = qb[q];
  }
  for (int q = 0; q < 5; ++q) o.dpb[q] = db[q];
  o.sb = sb;
  o.mub = mub;
  o.Kb = Kb;
}

// the first stage as a pass of its own: its outputs into the grid arrays
MTVD_HD inline void rv_tc(const AC& c, const Arr& A, int i, int k) {
  TcOut o;
  tc_node(c, A, i, k, o);
  const long long n = nid(c, i, k), cnt = c.cnt;
  const double mu0 = A.MU[n], K0 = A.KB[n];
  A.SB[n] = o.sb;
  st4(A.Xb, cnt, n, o.xb);
  st4(A.XPb, cnt, n, o.xpb);
  st4(A.PPb, cnt, n, o.ppb);
  for (int q = 0; q < 5; ++q) A.DPb[q * cnt + n] = o.dpb[q];
  A.MU[n] = mu0 + o.mub;
  A.KB[n] = K0 + o.Kb;
}

// Where the later stages read the outputs of the stages before them (the
// node's own and those of its neighbours): GridSrc takes them from the
// whole-grid arrays of a stage-per-kernel pass; a fused pass supplies the
// same accessors over on-chip copies.  xb is the X cotangent as the
// previous stage left it (the first stage's for the second, the second's
// for the third).
struct GridSrc {
  const AC& c;
  const Arr& A;
  MTVD_HD double xb(int i, int k, int q) const { return A.Xb[q * c.cnt + nid(c, i, k)]; }
  MTVD_HD double xpb(int i, int k, int q) const { return A.XPb[q * c.cnt + nid(c, i, k)]; }
  MTVD_HD double ppb(int i, int k, int q) const { return A.PPb[q * c.cnt + nid(c, i, k)]; }
  MTVD_HD double dpb(int i, int k, int s) const { return A.DPb[s * c.cnt + nid(c, i, k)]; }
  MTVD_HD double sb(int i, int k) const { return A.SB[nid(c, i, k)]; }
  MTVD_HD double pb(int i, int k, int q) const { return A.PB[q * c.cnt + nid(c, i, k)]; }
  MTVD_HD double db(int i, int k, int s) const { return A.DB[s * c.cnt + nid(c, i, k)]; }
};

// gather of a primitive array's cotangent from the derivative cotangents
// of the fluxes that read it (fwd = 1: forward inner differences of the
// predictor, 0: backward of the corrector) and from cross differences.
// D(i, k, s) gives derivative input s of the flux at (i, k).  Every
// candidate value is read first (rows clamped to the plates, so each read
// is of a node that exists) and added where its flux exists, by selects:
// the reads do not wait on the conditions.
template <class DF>
MTVD_HD inline void gather_prim(const AC& c, const DF& D, bool (*hasf)(const AC&, int, int),
                                int fwd, int i, int k, double qb[4]) {
  const int ia = c.axis == 0 ? 0 : 1, ic = 1 - ia;
  const int slots[3] = {ia, ic, 2};
  const double ih = c.iha;
  const bool z = c.axis == 2, w2 = c.wall_order == 2;
  const int di = c.axis == 0 ? 1 : 0, dk = c.axis == 0 ? 0 : 1;
  // inner: the flux at this node and the ones on the side that read it
  // (fwd: F_n reads q_n, q_{n+1}; corrector: F^P_n reads q_n, q_{n-1}), at
  // along offsets 0, e and 2e
  const int e = fwd ? -1 : 1;
  auto clampk = [&](int kk) { return kk < 0 ? 0 : (kk > c.M ? c.M : kk); };
  auto flux_at = [&](int d) -> bool {
    const int ii = i + d * di, kk = k + d * dk;
    if (z && (kk < 0 || kk > c.M)) return false;
    return hasf(c, ii, kk);
  };
  double Dv[3][3];                                 // [offset 0, e, 2e][s]
  for (int m = 0; m < 3; ++m)
    for (int s = 0; s < 3; ++s) Dv[m][s] = D(i + m * e * di, clampk(k + m * e * dk), s);
  const bool f0 = flux_at(0), f1 = flux_at(e);
  const bool f2 = z && w2 && k == (fwd ? 2 : c.M - 2) && flux_at(2 * e);
  // the plate closures (wall_order = 2): F_0 reads q_0, q_1, q_2 with
  // (-3, 4, -1) ih/2; F^P_M reads q_M, q_{M-1}, q_{M-2} with (3, -4, 1) ih/2
  const bool c0 = z && w2 && k == (fwd ? 0 : c.M), c1 = z && w2 && k == (fwd ? 1 : c.M - 1);
  for (int s = 0; s < 3; ++s) {
    double v = 0.0;
    if (fwd) {
      v = f0 ? v + (c0 ? -1.5 * ih * Dv[0][s] : -ih * Dv[0][s]) : v;
      v = f1 ? v + (c1 ? 2.0 * ih * Dv[1][s] : ih * Dv[1][s]) : v;
      v = f2 ? v + -0.5 * ih * Dv[2][s] : v;
    } else {
      v = f0 ? v + (c0 ? 1.5 * ih * Dv[0][s] : ih * Dv[0][s]) : v;
      v = f1 ? v + (c1 ? -2.0 * ih * Dv[1][s] : -ih * Dv[1][s]) : v;
      v = f2 ? v + 0.5 * ih * Dv[2][s] : v;
    }
    qb[slots[s]] += v;
  }
  // cross: the fluxes one step across read this node with +-1/(2h); this
  // node is the upper neighbour of the one at d = -1 (+), the lower of the
  // one at d = +1 (-)
  const double ihc2 = 0.5 * (c.axis == 0 ? c.ihz : c.ihx);
  for (int d = -1; d <= 1; d += 2) {
    const int ii = c.axis == 0 ? i : i + d, kk = c.axis == 0 ? k + d : k;
    const bool ok = (c.axis == 2 || (kk >= 0 && kk <= c.M)) && hasf(c, ii, clampk(kk));
    const double d3 = D(ii, clampk(kk), 3), d4 = D(ii, clampk(kk), 4);
    const double sg = d < 0 ? ihc2 : -ihc2;
    qb[ia] = ok ? qb[ia] + sg * d3 : qb[ia];
    qb[ic] = ok ? qb[ic] + sg * d4 : qb[ic];
  }
}

// The P^P cotangent of (i, k) (direct + gathered from the corrector fluxes
// that read it) taken back through the primitives.  Returns the kind of
// result in v: 0 the final X^P cotangent (v = 0 where X^P and P^P are
// constants, the bottom plate of L_z); 1 an addition to the X cotangent
// (plate rows that a horizontal operator copies: X^P = X, P^P = P); 2 the
// cotangent of the top plate's predicted density in v[0] (L_z, k = M).
template <class Src>
MTVD_HD inline int pp_back(const AC& c, const Arr& A, const Src& B, int i, int k, double v[4]) {
  long long n = nid(c, i, k);
  double qb[4];
  for (int q = 0; q < 4; ++q) qb[q] = B.ppb(i, k, q);
  gather_prim(c, [&](int ii, int kk, int s) { return B.dpb(ii, kk, s); }, has_FP, 0, i, k, qb);
  for (int q = 0; q < 4; ++q) v[q] = 0.0;
  if (c.axis == 0 && !interior(c, k)) {
    double x[4];
    ld4(A.X, c.cnt, n, x);
    prim_vjp(c, x, A.zr[k], qb, v);
    return 1;
  }
  if (c.axis == 2 && k == 0) return 0;
  for (int q = 0; q < 4; ++q) v[q] = B.xpb(i, k, q);
  if (c.axis == 2 && k == c.M) {
    // X^P_M = (r, 0, 0, r(cv Tt + g)), P^P_M = (0, 0, Tt, a r Tt)
    double r = v[0] + v[3] * (c.cv * c.Tt + c.g * A.zr[c.M]) + qb[3] * c.a * c.Tt;
    v[0] = r;
    v[1] = v[2] = v[3] = 0.0;
    return 2;
  }
  double x[4];
  ld4(A.XP, c.cnt, n, x);
  prim_vjp(c, x, A.zr[k], qb, v);
  return 0;
}

// What the second reverse stage yields at a node: the X cotangent so far,
// the primitive and derivative-input cotangents of the predictor flux, and
// the node's mu and K cotangents.
struct PredOut {
  double xb[4], pb[4], db[5], mub, Kb;
};

// reverse of the predictor: P^P and X^P cotangents of (i, k) and of the
// node above along the axis (pp_back), X^P -> X, and the predictor flux
// cotangent -> its inputs
template <class Src>
MTVD_HD inline void pred_node(const AC& c, const Arr& A, const Src& B, int i, int k, PredOut& o) {
  long long n = nid(c, i, k);
  double xb[4], v[4];
  for (int q = 0; q < 4; ++q) xb[q] = B.xb(i, k, q);
  const int kind = pp_back(c, A, B, i, k, v);
  if (kind == 1)
    for (int q = 0; q < 4; ++q) xb[q] += v[q];
  const bool in = interior(c, k);
  if (in) {
    for (int q = 0; q < 4; ++q) xb[q] += v[q];
    if (c.axis == 2) xb[0] += c.tau * (-c.g) * v[2];
  }
  if (c.axis == 2 && k == c.M) {           // r^P_M = rho_M - lm (m_z,M - m_z,M-1)
    xb[0] += v[0];
    xb[2] += -c.lm * v[0];
  }
  if (c.axis == 2 && k == c.M - 1) {
    double t[4];
    pp_back(c, A, B, i, c.M, t);
    xb[2] += c.lm * t[0];
  }
  double qb[4] = {0, 0, 0, 0}, db[5] = {0, 0, 0, 0, 0};
  double mub = 0.0, Kb = 0.0;
  if (has_F(c, i, k)) {
    double vu[4] = {0, 0, 0, 0};
    if (c.axis == 0 || k + 1 <= c.M - 1) {
      if (c.axis == 0) pp_back(c, A, B, i + 1, k, vu); else pp_back(c, A, B, i, k + 1, vu);
    }
    double Fb[4];
    for (int q = 0; q < 4; ++q) {
      double here = in ? v[q] : 0.0;
      Fb[q] = c.lm * (vu[q] - here);
    }
    double x[4], p4[4], d[5];
    ld4(A.X, c.cnt, n, x);
    ld4(A.P, c.cnt, n, p4);
    derivs(c, A.P, i, k, 1, d);
    flux_vjp(c, x, p4, d, Fb, xb, qb, db, &mub, &Kb);
  }
  for (int q = 0; q < 4; ++q) {
    o.xb[q] = xb[q];
    o.pb[q] = qb[q];
  }
  for (int q = 0; q < 5; ++q) o.db[q] = db[q];
  o.mub = mub;
  o.Kb = Kb;
}

MTVD_HD inline void rv_pred(const AC& c, const Arr& A, int i, int k) {
  PredOut o;
  pred_node(c, A, GridSrc{c, A}, i, k, o);
  const long long n = nid(c, i, k);
  st4(A.Xb, c.cnt, n, o.xb);
  st4(A.PB, c.cnt, n, o.pb);
  for (int q = 0; q < 5; ++q) A.DB[q * c.cnt + n] = o.db[q];
  A.MU[n] += o.mub;
  A.KB[n] += o.Kb;
}

// reverse of the primitives of X: the P cotangent (direct + gathered from
// the predictor fluxes + the TVD |u|+c) -> X; xb is the X cotangent the
// second stage left, returned complete
template <class Src>
MTVD_HD inline void prim_node(const AC& c, const Arr& A, const Src& B, int i, int k,
                              double xb[4]) {
  long long n = nid(c, i, k);
  double qb[4];
  for (int q = 0; q < 4; ++q) qb[q] = B.pb(i, k, q);
  gather_prim(c, [&](int ii, int kk, int s) { return B.db(ii, kk, s); }, has_F, 1, i, k, qb);
  const int ia = c.axis == 0 ? 0 : 1;
  double ua = A.P[ia * c.cnt + n], T = A.P[2 * c.cnt + n];
  double sb = B.sb(i, k);
  if (sb != 0.0) {
    qb[ia] += (ua > 0.0 ? 1.0 : (ua < 0.0 ? -1.0 : 0.0)) * sb;
    qb[2] += sb * c.gam_a / (2.0 * sqrt(c.gam_a * T));
  }
  double x[4];
  for (int q = 0; q < 4; ++q) xb[q] = B.xb(i, k, q);
  ld4(A.X, c.cnt, n, x);
  prim_vjp(c, x, A.zr[k], qb, xb);
}

MTVD_HD inline void rv_prim(const AC& c, const Arr& A, int i, int k) {
  double xb[4];
  prim_node(c, A, GridSrc{c, A}, i, k, xb);
  st4(A.Xb, c.cnt, nid(c, i, k), xb);
}

// ---- the three reverse stages of an operator in one pass ----------------------
// A block owns an output tile of kTA nodes along the axis by kTB across,
// starting at (a0, b0) (along, across).  The first stage runs on the
// kRA x kRB region from 2 nodes before the tile to 3 after it along the
// axis and 2 before to 2 after across it (what the second stage reads); the
// second on the region from 2 before to the tile's end along and 1 before
// to 1 after across (what the third reads); the third on the tile.  Each
// stage's outputs stay in the block's shared memory (field-major over the
// region; thread t computes region node t), so only the forward values,
// the output cotangent and the result pass through global memory.  The
// second stage's outputs are written over the first stage's X, X^P, P^P
// and derivative cotangents once every thread has read those (a barrier
// between tile_pred and tile_pred_put); the first stage's |u|+c, mu and K
// cotangents stay for the third.  Nodes beyond a plate are skipped; across the periodic x direction a region's
// nodes carry unwrapped indices (wrapped where global arrays are read).
// The stage arithmetic is that of rv_tc, rv_pred and rv_prim, so the
// result is bit for bit that of the three passes.
constexpr int kRA = 16, kRB = 16;                 // first-stage region
constexpr int kTA = kRA - 5, kTB = kRB - 4;       // output tile
constexpr int kPA = kTA + 2, kPB = kTB + 2;       // second-stage region
constexpr int kNT = kRA * kRB, kNP = kPA * kPB, kNO = kTA * kTB;
constexpr int kTcF = 20, kPrF = 15;               // doubles per node the stages keep
constexpr int kTileDoubles = kTcF * kNT;
static_assert(kPrF * kNP <= 17 * kNT, "second-stage outputs overlay the first stage's dead slots");

// index of region node (la, lb) (along, across offsets from the region's
// corner) in a region na along by nb across: consecutive indices run along
// x (along the axis for L_x, across it for L_z)
MTVD_HD inline int ridx(int axis, int la, int lb, int na, int nb) {
  return axis == 0 ? lb * na + la : la * nb + lb;
}
MTVD_HD inline int along_of(int axis, int i, int k) { return axis == 0 ? i : k; }
MTVD_HD inline int across_of(int axis, int i, int k) { return axis == 0 ? k : i; }

// the first stage's outputs held in shared memory (region corner at
// along a0 - 2, across b0 - 2)
struct TcTile {
  const AC& c;
  const double* L;
  int ca, cb;                                      // region corner
  MTVD_HD int at(int i, int k) const {
    return ridx(c.axis, along_of(c.axis, i, k) - ca, across_of(c.axis, i, k) - cb, kRA, kRB);
  }
  MTVD_HD double xb(int i, int k, int q) const { return L[q * kNT + at(i, k)]; }
  MTVD_HD double xpb(int i, int k, int q) const { return L[(4 + q) * kNT + at(i, k)]; }
  MTVD_HD double ppb(int i, int k, int q) const { return L[(8 + q) * kNT + at(i, k)]; }
  MTVD_HD double dpb(int i, int k, int s) const { return L[(12 + s) * kNT + at(i, k)]; }
  MTVD_HD double sb(int i, int k) const { return L[17 * kNT + at(i, k)]; }
};

// the second stage's outputs (region corner at along a0 - 2, across
// b0 - 1), and the first stage's |u|+c cotangent
struct PredTile {
  const AC& c;
  const double* L;
  int ca, cb;
  TcTile tc;
  MTVD_HD int at(int i, int k) const {
    return ridx(c.axis, along_of(c.axis, i, k) - ca, across_of(c.axis, i, k) - cb, kPA, kPB);
  }
  MTVD_HD double xb(int i, int k, int q) const { return L[q * kNP + at(i, k)]; }
  MTVD_HD double pb(int i, int k, int q) const { return L[(4 + q) * kNP + at(i, k)]; }
  MTVD_HD double db(int i, int k, int s) const { return L[(8 + s) * kNP + at(i, k)]; }
  MTVD_HD double sb(int i, int k) const { return tc.sb(i, k); }
};

// node (i, k) of region index t in a region na x nb with corner (ca, cb)
MTVD_HD inline void region_node(int axis, int t, int na, int nb, int ca, int cb, int* i, int* k) {
  const int la = axis == 0 ? t % na : t / nb, lb = axis == 0 ? t / na : t % nb;
  const int a = ca + la, b = cb + lb;
  *i = axis == 0 ? a : b;
  *k = axis == 0 ? b : a;
}

// first phase, thread t (< kNT): the first stage on region node t; L holds
// kTileDoubles doubles
MTVD_HD inline void tile_tc(const AC& c, const Arr& A, double* L, int a0, int b0, int t) {
  int i, k;
  region_node(c.axis, t, kRA, kRB, a0 - 2, b0 - 2, &i, &k);
  if (k < 0 || k > c.M) return;
  TcOut o;
  tc_node(c, A, i, k, o);
  for (int q = 0; q < 4; ++q) {
    L[q * kNT + t] = o.xb[q];
    L[(4 + q) * kNT + t] = o.xpb[q];
    L[(8 + q) * kNT + t] = o.ppb[q];
  }
  for (int q = 0; q < 5; ++q) L[(12 + q) * kNT + t] = o.dpb[q];
  L[17 * kNT + t] = o.sb;
  L[18 * kNT + t] = o.mub;
  L[19 * kNT + t] = o.Kb;
}

// second phase, thread t (< kNP): the second stage on region node t, into
// o; false for a node beyond a plate
MTVD_HD inline bool tile_pred(const AC& c, const Arr& A, const double* L, int a0, int b0, int t,
                              PredOut& o) {
  int i, k;
  region_node(c.axis, t, kPA, kPB, a0 - 2, b0 - 1, &i, &k);
  if (k < 0 || k > c.M) return false;
  pred_node(c, A, TcTile{c, L, a0 - 2, b0 - 2}, i, k, o);
  return true;
}

// its outputs into shared memory, over the first stage's dead slots (after
// a barrier that follows every thread's tile_pred)
MTVD_HD inline void tile_pred_put(double* L, int t, const PredOut& o) {
  for (int q = 0; q < 4; ++q) {
    L[q * kNP + t] = o.xb[q];
    L[(4 + q) * kNP + t] = o.pb[q];
  }
  for (int q = 0; q < 5; ++q) L[(8 + q) * kNP + t] = o.db[q];
  L[13 * kNP + t] = o.mub;
  L[14 * kNP + t] = o.Kb;
}

// The cotangent of the objective's plate Nusselt number at a state, added
// to the X cotangent xb of node (i, k) with state x: the mean of
// Nu(z=0) and Nu(z=1), Nu = -(dT/dz + D)/eps from one-sided second-order
// differences of the row means of T (rows 0, 1, 2 with weights -3, 4, -1
// and rows M-2, M-1, M with 1, -4, 3, over 2 dz), times the weight w of
// the state in the objective.  nu_a = w (-0.5/eps); a row that both plates
// read (nz = 5) takes the sum of its weights.
MTVD_HD inline void nu_cot(const AC& c, double nu_a, int k, const double x[4], double z,
                           double xb[4]) {
  const int rows[6] = {0, 1, 2, c.M - 2, c.M - 1, c.M};
  const double w[6] = {-3.0, 4.0, -1.0, 1.0, -4.0, 3.0};
  int r = 0;
  while (r < 6 && rows[r] != k) ++r;
  if (r == 6) return;
  double wr = w[r];
  for (int q = r + 1; q < 6; ++q)
    if (rows[q] == k) wr += w[q];
  // d Nu_mean / d T(i, k) = -(1/(2 eps)) wr (1/(2 dz)) / nx
  const double Tb = nu_a * wr * (0.5 * c.ihz) / (double)c.nx;
  const double qb[4] = {0.0, 0.0, Tb, 0.0};
  prim_vjp(c, x, z, qb, xb);
}

// third phase, thread t (< kNO): the X cotangent of an output node into
// A.Xb, and its mu and K cotangents added to A.MU and A.KB in the order of
// the separate passes.  nu_a != 0: the objective's cotangent at the
// operator's input state (nu_cot) is added to the result.
MTVD_HD inline void tile_prim(const AC& c, const Arr& A, const double* L, int a0, int b0, int t,
                              double nu_a = 0.0) {
  int i, k;
  region_node(c.axis, t, kTA, kTB, a0, b0, &i, &k);
  if (k > c.M || i >= c.nx) return;
  const TcTile tc{c, L, a0 - 2, b0 - 2};
  const PredTile pr{c, L, a0 - 2, b0 - 1, tc};
  double xb[4];
  prim_node(c, A, pr, i, k, xb);
  const long long n = nid(c, i, k);
  if (nu_a != 0.0) {
    double x[4];
    ld4(A.X, c.cnt, n, x);
    nu_cot(c, nu_a, k, x, A.zr[k], xb);
  }
  st4(A.Xb, c.cnt, n, xb);
  const int jt = tc.at(i, k), jp = pr.at(i, k);
  A.MU[n] = (A.MU[n] + L[18 * kNT + jt]) + pr.L[13 * kNP + jp];
  A.KB[n] = (A.KB[n] + L[19 * kNT + jt]) + pr.L[14 * kNP + jp];
}

}  // namespace adj
}  // namespace mtvd
