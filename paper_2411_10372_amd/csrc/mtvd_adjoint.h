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
// neighbour values it needs instead of storing them, so each pass is one
// kernel without atomics.  Limiter kinks take the branch the forward pass
// took.
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

// the output's cotangents at (i, k): the share of the input (plates that
// copy or close), of X^C and of X^P
MTVD_HD inline void out_cots(const AC& c, const Arr& A, int i, int k, double xb[4],
                             double xcb[4], double xpb[4]) {
  long long n = nid(c, i, k);
  double yb[4];
  ld4(A.Yb, c.cnt, n, yb);
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
    xb[0] = yb[0] + yb[3] * (c.cv * c.Tb + c.g * A.zr[0]);
  } else if (k == c.M) {               // rho'_M = rho^P_M
    xpb[0] = yb[0] + yb[3] * (c.cv * c.Tt + c.g * A.zr[c.M]);
  } else {
    for (int q = 0; q < 4; ++q) xcb[q] = xpb[q] = 0.5 * yb[q];
    if (k == 1) {                      // X^P_1 carries the bottom closure's m^P_z,1
      long long n0 = nid(c, i, 0);
      double r0b = A.Yb[n0] + A.Yb[3 * c.cnt + n0] * (c.cv * c.Tb + c.g * A.zr[0]);
      xpb[2] += -c.lm * r0b;
    }
  }
}

// the reverse of one TVD face (i, k)-(i, k)+1: the cotangents it sends to
// its three jumps and to |u|+c of its two nodes (zero where there is no face)
MTVD_HD inline void face_cot(const AC& c, const Arr& A, int i, int k, double dmb[4],
                             double d0b[4], double dpb[4], double* s0b, double* s1b) {
  for (int q = 0; q < 4; ++q) dmb[q] = d0b[q] = dpb[q] = 0.0;
  *s0b = *s1b = 0.0;
  if (!has_D(c, i, k)) return;
  long long n = nid(c, i, k);
  int im = c.axis == 0 ? i - 1 : i, km = c.axis == 0 ? k : k - 1;
  int ip = c.axis == 0 ? i + 1 : i, kp = c.axis == 0 ? k : k + 1;
  double dm[4], d0[4], dp[4];
  jump(c, A.X, im, km, dm);
  jump(c, A.X, i, k, d0);
  jump(c, A.X, ip, kp, dp);
  long long m1 = along(c, i, k, 1);
  Face f = face(c, dm, d0, dp, A.S[n], A.S[m1]);
  // D_{n+1/2} enters Y_n with + and Y_{n+1} with -
  double Db[4];
  for (int q = 0; q < 4; ++q) Db[q] = A.Yb[q * c.cnt + n] - A.Yb[q * c.cnt + m1];
  double Gb = dot4(Db, d0);
  for (int q = 0; q < 4; ++q) d0b[q] = f.G * Db[q];
  face_vjp(c, f, dm, d0, dp, Gb, dmb, d0b, dpb, s0b, s1b);
}

// reverse of the output, the TVD faces and the corrector: the jump
// cotangents of the faces around (i, k) -> X; |u|+c cotangent of the node;
// X^C -> X; the corrector flux cotangent -> its inputs
MTVD_HD inline void rv_tc(const AC& c, const Arr& A, int i, int k) {
  long long n = nid(c, i, k);
  const bool lo_ok = c.axis == 0 || k >= 1;        // a face below exists
  const bool hi_ok = c.axis == 0 || k <= c.M - 1;  // a face above exists
  // faces (by lower node) n-2, n-1, n, n+1 along the axis
  const int di = c.axis == 0 ? 1 : 0, dk = c.axis == 0 ? 0 : 1;
  double am[4][4], a0[4][4], ap[4][4], s0[4], s1[4];   // index f+2 for face n+f
  for (int f = -2; f <= 1; ++f) {
    const int kk = k + f * dk;
    if (c.axis == 2 && (kk < 0 || kk > c.M)) {
      for (int q = 0; q < 4; ++q) am[f + 2][q] = a0[f + 2][q] = ap[f + 2][q] = 0.0;
      s0[f + 2] = s1[f + 2] = 0.0;
      continue;
    }
    face_cot(c, A, i + f * di, kk, am[f + 2], a0[f + 2], ap[f + 2], &s0[f + 2], &s1[f + 2]);
  }
  double xb[4], xcb[4], xpb[4];
  out_cots(c, A, i, k, xb, xcb, xpb);
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
  A.SB[n] = s0[2] + (lo_ok ? s1[1] : 0.0);
  // X^C = X - lm (F^P_{n+1} - F^P_n) + tau S(X^P)
  for (int q = 0; q < 4; ++q) xb[q] += xcb[q];
  st4(A.Xb, c.cnt, n, xb);
  if (c.axis == 2 && interior(c, k)) xpb[0] += c.tau * (-c.g) * xcb[2];
  double qb[4] = {0, 0, 0, 0}, db[5] = {0, 0, 0, 0, 0};
  double mub = 0.0, Kb = 0.0;
  if (has_FP(c, i, k)) {
    double xcbm[4] = {0, 0, 0, 0};
    if (c.axis == 0 || k - 1 >= 1) {
      double t0[4], t1[4];
      if (c.axis == 0) out_cots(c, A, i - 1, k, t0, xcbm, t1);
      else out_cots(c, A, i, k - 1, t0, xcbm, t1);
    }
    double Fb[4];
    for (int q = 0; q < 4; ++q) {
      double here = (c.axis == 0 || k <= c.M - 1) ? xcb[q] : 0.0;
      Fb[q] = c.lm * (here - xcbm[q]);
    }
    double x[4], p4[4], d[5];
    ld4(A.XP, c.cnt, n, x);
    ld4(A.PP, c.cnt, n, p4);
    derivs(c, A.PP, i, k, 0, d);
    flux_vjp(c, x, p4, d, Fb, xpb, qb, db, &mub, &Kb);
  }
  st4(A.XPb, c.cnt, n, xpb);
  st4(A.PPb, c.cnt, n, qb);
  for (int q = 0; q < 5; ++q) A.DPb[q * c.cnt + n] = db[q];
  A.MU[n] += mub;
  A.KB[n] += Kb;
}

// gather of a primitive array's cotangent from the derivative cotangents
// of the fluxes that read it (fwd = 1: forward inner differences of the
// predictor, 0: backward of the corrector) and from cross differences
MTVD_HD inline void gather_prim(const AC& c, const double* D, bool (*hasf)(const AC&, int, int),
                                int fwd, int i, int k, double qb[4]) {
  const long long cnt = c.cnt;
  const int ia = c.axis == 0 ? 0 : 1, ic = 1 - ia;
  const int slots[3] = {ia, ic, 2};
  const double ih = c.iha;
  // inner: the flux at this node and the one on the side that reads it
  const int p0 = pos(c, i, k);
  auto flux_at = [&](int d) -> bool {
    int ii = c.axis == 0 ? i + d : i, kk = c.axis == 0 ? k : k + d;
    if (c.axis == 2 && (kk < 0 || kk > c.M)) return false;
    return hasf(c, ii, kk);
  };
  auto Dat = [&](int d, int s) -> double {
    int ii = c.axis == 0 ? i + d : i, kk = c.axis == 0 ? k : k + d;
    return D[s * cnt + nid(c, ii, kk)];
  };
  const bool z = c.axis == 2, w2 = c.wall_order == 2;
  for (int s = 0; s < 3; ++s) {
    double v = 0.0;
    if (fwd) {
      // F_n reads q_n (-ih) and q_{n+1} (+ih); F_0 of the z operator reads
      // q_0, q_1, q_2 with (-3, 4, -1) ih/2 when wall_order = 2
      if (flux_at(0)) v += (z && k == 0 && w2) ? -1.5 * ih * Dat(0, s) : -ih * Dat(0, s);
      if (flux_at(-1)) v += (z && k == 1 && w2) ? 2.0 * ih * Dat(-1, s) : ih * Dat(-1, s);
      if (z && w2 && k == 2 && flux_at(-2)) v += -0.5 * ih * Dat(-2, s);
    } else {
      // F^P_n reads q_n (+ih) and q_{n-1} (-ih); F^P_M of the z operator
      // reads q_M, q_{M-1}, q_{M-2} with (3, -4, 1) ih/2 when wall_order = 2
      if (flux_at(0)) v += (z && k == c.M && w2) ? 1.5 * ih * Dat(0, s) : ih * Dat(0, s);
      if (flux_at(1)) v += (z && k == c.M - 1 && w2) ? -2.0 * ih * Dat(1, s) : -ih * Dat(1, s);
      if (z && w2 && k == c.M - 2 && flux_at(2)) v += 0.5 * ih * Dat(2, s);
    }
    qb[slots[s]] += v;
  }
  (void)p0;
  // cross: the fluxes one step across read this node with +-1/(2h)
  const double ihc2 = 0.5 * (c.axis == 0 ? c.ihz : c.ihx);
  for (int d = -1; d <= 1; d += 2) {
    int ii = c.axis == 0 ? i : i + d, kk = c.axis == 0 ? k + d : k;
    if (c.axis == 0 && (kk < 0 || kk > c.M)) continue;
    if (!hasf(c, ii, kk)) continue;
    long long m = nid(c, ii, kk);
    // this node is the upper neighbour of m when d = -1 (+), lower when d = +1 (-)
    double sg = d < 0 ? ihc2 : -ihc2;
    qb[ia] += sg * D[3 * cnt + m];
    qb[ic] += sg * D[4 * cnt + m];
  }
}

// The P^P cotangent of (i, k) (direct + gathered from the corrector fluxes
// that read it) taken back through the primitives.  Returns the kind of
// result in v: 0 the final X^P cotangent (v = 0 where X^P and P^P are
// constants, the bottom plate of L_z); 1 an addition to the X cotangent
// (plate rows that a horizontal operator copies: X^P = X, P^P = P); 2 the
// cotangent of the top plate's predicted density in v[0] (L_z, k = M).
MTVD_HD inline int pp_back(const AC& c, const Arr& A, int i, int k, double v[4]) {
  long long n = nid(c, i, k);
  double qb[4];
  ld4(A.PPb, c.cnt, n, qb);
  gather_prim(c, A.DPb, has_FP, 0, i, k, qb);
  for (int q = 0; q < 4; ++q) v[q] = 0.0;
  if (c.axis == 0 && !interior(c, k)) {
    double x[4];
    ld4(A.X, c.cnt, n, x);
    prim_vjp(c, x, A.zr[k], qb, v);
    return 1;
  }
  if (c.axis == 2 && k == 0) return 0;
  ld4(A.XPb, c.cnt, n, v);
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

// reverse of the predictor: P^P and X^P cotangents of (i, k) and of the
// node above along the axis (pp_back), X^P -> X, and the predictor flux
// cotangent -> its inputs
MTVD_HD inline void rv_pred(const AC& c, const Arr& A, int i, int k) {
  long long n = nid(c, i, k);
  double xb[4], v[4];
  ld4(A.Xb, c.cnt, n, xb);
  const int kind = pp_back(c, A, i, k, v);
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
    pp_back(c, A, i, c.M, t);
    xb[2] += c.lm * t[0];
  }
  double qb[4] = {0, 0, 0, 0}, db[5] = {0, 0, 0, 0, 0};
  double mub = 0.0, Kb = 0.0;
  if (has_F(c, i, k)) {
    double vu[4] = {0, 0, 0, 0};
    if (c.axis == 0 || k + 1 <= c.M - 1) {
      if (c.axis == 0) pp_back(c, A, i + 1, k, vu); else pp_back(c, A, i, k + 1, vu);
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
  st4(A.Xb, c.cnt, n, xb);
  st4(A.PB, c.cnt, n, qb);
  for (int q = 0; q < 5; ++q) A.DB[q * c.cnt + n] = db[q];
  A.MU[n] += mub;
  A.KB[n] += Kb;
}

// reverse 5: P cotangent (direct + gathered + TVD |u|+c) -> X
MTVD_HD inline void rv_prim(const AC& c, const Arr& A, int i, int k) {
  long long n = nid(c, i, k);
  double qb[4];
  ld4(A.PB, c.cnt, n, qb);
  gather_prim(c, A.DB, has_F, 1, i, k, qb);
  const int ia = c.axis == 0 ? 0 : 1;
  double ua = A.P[ia * c.cnt + n], T = A.P[2 * c.cnt + n];
  double sb = A.SB[n];
  if (sb != 0.0) {
    qb[ia] += (ua > 0.0 ? 1.0 : (ua < 0.0 ? -1.0 : 0.0)) * sb;
    qb[2] += sb * c.gam_a / (2.0 * sqrt(c.gam_a * T));
  }
  double xb[4], x[4];
  ld4(A.Xb, c.cnt, n, xb);
  ld4(A.X, c.cnt, n, x);
  prim_vjp(c, x, A.zr[k], qb, xb);
  st4(A.Xb, c.cnt, n, xb);
}

}  // namespace adj
}  // namespace mtvd
