/*
 * mtvd_oracle.c -- plain CPU FP64 oracle of the MacCormack-TVD step.
 *
 * TEST INFRASTRUCTURE ONLY (see mtvd_oracle.h).  Slow on purpose: every stage
 * of the method is a separate loop over whole arrays, in the order the paper
 * states it, with no blocking or fusion.  Build with -ffp-contract=off and no
 * fast-math.
 *
 * Paper: Tiwari, Sharma & Verma, arXiv:2411.10372.
 *   Sec. 2, nondimensional equations (continuity/momentum/energy) and the
 *     definitions of p, E and tau_ij that follow them;
 *   Sec. 2, Nusselt numbers (bulk: volume_Nu; plates: mean_Nu);
 *   Sec. 3.1, conservative vector form (vector_eqn), fluxes F_alpha and
 *     sources S_alpha, split step (time_step), predictor, corrector,
 *     average plus TVD term, the TVD ratios r+-, G, phi and C.
 *
 * Where the paper is silent or garbled this file follows these readings:
 *   - corrector differences the predicted fluxes: F^P_{k+1} - F^P_k;
 *   - pressure enters the momentum row of its own direction (delta_{i,a} p);
 *   - tau_ij = mu*(d_j u_i + d_i u_j + lambda d_m u_m delta_ij) with
 *     lambda = bulk_coef (default -2/3);
 *   - derivatives inside F_alpha along alpha are one-sided opposite to the
 *     enclosing flux difference (forward in the predictor, backward in the
 *     corrector); cross derivatives are central; z-derivatives inside the
 *     two plate fluxes that the scheme uses (F_0 in the predictor, F^P_M in
 *     the corrector) are the second-order one-sided ones (forward at the
 *     bottom, backward at the top) when wall_order = 2, else the interior
 *     first differences;
 *   - plates: u = 0 and T = T_plate; plate density by a conservative half-
 *     cell update (bottom from the corrector flux, top from the predictor
 *     flux); no TVD flux on the two plate-adjacent faces; the x and y
 *     operators copy plate rows through;
 *   - TVD: both ratios of one face share the denominator |dX_{k+1/2}|^2; a
 *     face whose denominator is exactly 0 gets no TVD flux; Co of a face is
 *     (tau/h) max over its two nodes of (|u_a| + c) at level n;
 *   - dt = cfl * min over nodes and directions of h_a/(|u_a| + c);
 *   - the initial state: T = 1 - (eps+D) z, rho = T^(m-1) (hydrostatic for
 *     the unperturbed T), m = gamma D / ((gamma-1)(eps+D)), noise on
 *     interior T from SplitMix64.
 */
#include "mtvd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* constants of the nondimensional equations (Sec. 2)                        */

typedef struct {
  int ndim, nf, nx, ny, nz, M;
  int fR, fE, fm[3];         /* field slot of rho, E and rho*u_{x,y,z} */
  double h[3];               /* dx, dy, dz */
  double gamma, eps, D, Ra, Pr, aspect;
  double cv;                 /* 1/(gamma eps D): E = rho(u^2/2 + cv T + g z) */
  double a;                  /* (gamma-1)/(gamma eps D): p = a rho T */
  double g;                  /* gravity_scale/eps: momentum source -g rho */
  double mu;                 /* sqrt(Pr/Ra) (times diffusion_scale) */
  double K;                  /* 1/(eps D sqrt(Ra Pr)) (times diffusion_scale) */
  double lam;                /* bulk_coef */
  double Tb, Tt;             /* plate temperatures: 1 and 1-(eps+D) */
  double cfl;
  int limiter_form, tvd_on, pred_dir, sweep_order, wall_order;
} coefs;

static void make_coefs(const ora_params* p, coefs* c) {
  memset(c, 0, sizeof(*c));
  c->ndim = p->ndim;
  c->nf = p->ndim + 2;
  c->nx = p->nx;
  c->ny = (p->ndim == 3) ? p->ny : 1;
  c->nz = p->nz;
  c->M = p->nz - 1;
  c->fR = 0;
  c->fm[0] = 1;
  c->fm[1] = (p->ndim == 3) ? 2 : -1;
  c->fm[2] = (p->ndim == 3) ? 3 : 2;
  c->fE = c->nf - 1;
  c->h[0] = p->aspect / p->nx;
  c->h[1] = (p->ndim == 3) ? p->aspect / p->ny : 1.0;
  c->h[2] = 1.0 / (double)(p->nz - 1);
  c->gamma = p->gamma;
  c->eps = p->eps;
  c->D = p->D;
  c->Ra = p->Ra;
  c->Pr = p->Pr;
  c->aspect = p->aspect;
  c->cv = 1.0 / (p->gamma * p->eps * p->D);
  c->a = (p->gamma - 1.0) / (p->gamma * p->eps * p->D);
  c->g = p->gravity_scale / p->eps;
  c->mu = sqrt(p->Pr / p->Ra) * p->diffusion_scale;
  c->K = 1.0 / (p->eps * p->D * sqrt(p->Ra * p->Pr)) * p->diffusion_scale;
  c->lam = p->bulk_coef;
  c->Tb = 1.0;
  c->Tt = 1.0 - (p->eps + p->D);
  c->cfl = p->cfl;
  c->limiter_form = p->limiter_form;
  c->tvd_on = p->tvd_on;
  c->pred_dir = p->pred_dir;
  c->sweep_order = p->sweep_order;
  c->wall_order = p->wall_order;
}

static int check_params(const ora_params* p) {
  if (!p) return -1;
  if (p->ndim != 2 && p->ndim != 3) return -1;
  if (p->nx < 1 || p->nz < 3) return -1;
  if (p->ndim == 3 && p->ny < 1) return -1;
  if (!(p->gamma > 1.0) || !(p->eps > 0.0) || !(p->D > 0.0)) return -1;
  if (!(p->Ra > 0.0) || !(p->Pr > 0.0) || !(p->aspect > 0.0)) return -1;
  if (p->wall_order != 1 && p->wall_order != 2) return -1;
  return 0;
}

static void set_threads(const ora_params* p) {
#ifdef _OPENMP
  if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#else
  (void)p;
#endif
}

/* height of row k: z_k = k / M, so the plates sit exactly at 0 and 1 */
static double zrow(const coefs* c, int k) { return (double)k / (double)c->M; }

int ora_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

size_t ora_state_len(const ora_params* p) {
  size_t ny = (p->ndim == 3) ? (size_t)p->ny : 1;
  return (size_t)(p->ndim + 2) * (size_t)p->nz * ny * (size_t)p->nx;
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), counter form               */

uint64_t ora_splitmix64(uint64_t seed, uint64_t n) {
  uint64_t z = seed + n * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* initial state                                                             */

/* value of field f at global node (i, j, k) of the initial state */
static void init_node(const ora_params* p, const coefs* c, int i, int j,
                      int k, double* x /* nf values */) {
  double Delta = p->eps + p->D;                      /* (T_b - T_t) / d */
  double m = p->gamma * p->D / ((p->gamma - 1.0) * Delta);
  double expo = p->gravity_scale * m - 1.0;
  double z = zrow(c, k);
  double T0 = 1.0 - Delta * z;                       /* conduction profile */
  double rho = pow(T0, expo);                        /* hydrostatic for T0 */
  double T = T0;
  if (k > 0 && k < c->M && p->noise_amp != 0.0) {
    uint64_t lin = (uint64_t)i + (uint64_t)c->nx * ((uint64_t)j + (uint64_t)c->ny * (uint64_t)k);
    uint64_t r = ora_splitmix64(p->seed, lin + 1);
    double U = (double)(r >> 11) * 0x1.0p-53;        /* uniform in [0, 1) */
    T = T + p->noise_amp * (2.0 * U - 1.0);
  }
  for (int f = 0; f < c->nf; ++f) x[f] = 0.0;
  x[c->fR] = rho;
  x[c->fE] = rho * (c->cv * T + c->g * z);           /* u = 0 */
}

int ora_init(const ora_params* p, double* X) {
  if (check_params(p)) return -1;
  coefs c;
  make_coefs(p, &c);
  set_threads(p);
  size_t plane = (size_t)c.nx * c.ny, cnt = plane * c.nz;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < c.nz; ++k)
    for (int j = 0; j < c.ny; ++j)
      for (int i = 0; i < c.nx; ++i) {
        double x[5];
        init_node(p, &c, i, j, k, x);
        size_t n = (size_t)i + (size_t)c.nx * ((size_t)j + (size_t)c.ny * k);
        for (int f = 0; f < c.nf; ++f) X[f * cnt + n] = x[f];
      }
  (void)plane;
  return 0;
}

int ora_init_box(const ora_params* p, int i0, int j0, int bx, int by,
                 double* B) {
  if (check_params(p)) return -1;
  coefs c;
  make_coefs(p, &c);
  if (p->ndim == 2) by = 1;
  size_t cnt = (size_t)bx * by * c.nz;
  for (int k = 0; k < c.nz; ++k)
    for (int jb = 0; jb < by; ++jb)
      for (int ib = 0; ib < bx; ++ib) {
        int i = ((i0 + ib) % c.nx + c.nx) % c.nx;
        int j = (p->ndim == 3) ? ((j0 + jb) % c.ny + c.ny) % c.ny : 0;
        double x[5];
        init_node(p, &c, i, j, k, x);
        size_t n = (size_t)ib + (size_t)bx * ((size_t)jb + (size_t)by * k);
        for (int f = 0; f < c.nf; ++f) B[f * cnt + n] = x[f];
      }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* a box of nodes: bx x by columns, all nz rows, with its own strides        */

typedef struct {
  int bx, by, nz;
  ptrdiff_t s[3];   /* node strides along x, y, z */
  ptrdiff_t nn;     /* nodes in the box (field stride) */
} box;

static box make_box(int bx, int by, int nz) {
  box b;
  b.bx = bx;
  b.by = by;
  b.nz = nz;
  b.s[0] = 1;
  b.s[1] = bx;
  b.s[2] = (ptrdiff_t)bx * by;
  b.nn = (ptrdiff_t)bx * by * nz;
  return b;
}

/* primitive variables at every node (Sec. 2: E and p definitions):
 * u_a = (rho u_a)/rho, T = (E/rho - |u|^2/2 - g z)/cv, p = a rho T */
typedef struct {
  double *u[3], *T, *p;
} prims;

static void alloc_prims(const box* b, prims* q) {
  for (int d = 0; d < 3; ++d) q->u[d] = (double*)calloc((size_t)b->nn, sizeof(double));
  q->T = (double*)calloc((size_t)b->nn, sizeof(double));
  q->p = (double*)calloc((size_t)b->nn, sizeof(double));
}
static void free_prims(prims* q) {
  for (int d = 0; d < 3; ++d) free(q->u[d]);
  free(q->T);
  free(q->p);
}

static void primitives_at(const coefs* c, const box* b, const double* X,
                          prims* q, ptrdiff_t n) {
  int k = (int)(n / b->s[2]);
  double rho = X[c->fR * b->nn + n];
  double uu = 0.0;
  for (int d = 0; d < 3; ++d) {
    double u = (c->fm[d] >= 0) ? X[c->fm[d] * b->nn + n] / rho : 0.0;
    q->u[d][n] = u;
  }
  uu = (q->u[0][n] * q->u[0][n] + q->u[1][n] * q->u[1][n]) + q->u[2][n] * q->u[2][n];
  double e = X[c->fE * b->nn + n] / rho - 0.5 * uu - c->g * zrow(c, k);
  q->T[n] = e / c->cv;
  q->p[n] = c->a * rho * q->T[n];
}

static void primitives(const coefs* c, const box* b, const double* X,
                       prims* q) {
#pragma omp parallel for schedule(static)
  for (ptrdiff_t n = 0; n < b->nn; ++n) primitives_at(c, b, X, q, n);
}

/* finite differences of an array q along direction d at node n */
enum { DFWD, DBWD, DCEN, DW2F, DW2B };

static double deriv(const double* q, const box* b, const coefs* c,
                    ptrdiff_t n, int d, int mode) {
  ptrdiff_t s = b->s[d];
  double h = c->h[d];
  switch (mode) {
    case DFWD: return (q[n + s] - q[n]) / h;
    case DBWD: return (q[n] - q[n - s]) / h;
    case DCEN: return (q[n + s] - q[n - s]) / (2.0 * h);
    case DW2F: return ((-3.0 * q[n] + 4.0 * q[n + s]) - q[n + 2 * s]) / (2.0 * h);
    default:   return ((3.0 * q[n] - 4.0 * q[n - s]) + q[n - 2 * s]) / (2.0 * h);
  }
}

static int has_dir(const coefs* c, int d) { return d != 1 || c->ndim == 3; }

/* flux F_alpha at node n (Sec. 3.1, F_alpha; Sec. 2, tau_ij and the energy
 * equation), with the derivative along alpha taken in `mode` */
static void flux_at(const coefs* c, const box* b, const double* X,
                    const prims* q, int al, ptrdiff_t n, int mode,
                    double* F) {
  double dau[3] = {0, 0, 0};   /* d_alpha u_g */
  double dgua[3] = {0, 0, 0};  /* d_g u_alpha, g != alpha (central) */
  for (int g = 0; g < 3; ++g) {
    if (!has_dir(c, g)) continue;
    dau[g] = deriv(q->u[g], b, c, n, al, mode);
    if (g != al) dgua[g] = deriv(q->u[al], b, c, n, g, DCEN);
  }
  double div = 0.0;            /* d_m u_m */
  for (int m = 0; m < 3; ++m) {
    if (!has_dir(c, m)) continue;
    div += (m == al) ? dau[al] : deriv(q->u[m], b, c, n, m, DCEN);
  }
  double tau[3] = {0, 0, 0};   /* tau_{g alpha} */
  for (int g = 0; g < 3; ++g) {
    if (!has_dir(c, g)) continue;
    if (g == al)
      tau[g] = c->mu * ((dau[al] + dau[al]) + c->lam * div);
    else
      tau[g] = c->mu * (dau[g] + dgua[g]);
  }
  double dT = deriv(q->T, b, c, n, al, mode);
  double rho_ua = X[c->fm[al] * b->nn + n];
  double E = X[c->fE * b->nn + n];
  double p = q->p[n];
  double ua = q->u[al][n];
  F[c->fR] = rho_ua;
  for (int g = 0; g < 3; ++g) {
    if (!has_dir(c, g)) continue;
    double v = X[c->fm[g] * b->nn + n] * ua - tau[g];
    if (g == al) v = v + p;
    F[c->fm[g]] = v;
  }
  double work = 0.0;           /* sum_b u_b tau_{b alpha} */
  for (int g = 0; g < 3; ++g)
    if (has_dir(c, g)) work += q->u[g][n] * tau[g];
  F[c->fE] = (ua * (E + p) - c->K * dT) - work;
}

/* node ranges [lo, hi) per direction for one stage */
typedef struct { int lo[3], hi[3]; } range;

#define FOR_RANGE(b, r, n)                                               \
  for (int kk_ = (r).lo[2]; kk_ < (r).hi[2]; ++kk_)                      \
    for (int jj_ = (r).lo[1]; jj_ < (r).hi[1]; ++jj_)                    \
      for (int ii_ = (r).lo[0]; ii_ < (r).hi[0]; ++ii_)                  \
        for (ptrdiff_t n = ii_ + (b)->s[1] * jj_ + (b)->s[2] * kk_, once_ = 1; \
             once_; once_ = 0)

static range all_nodes(const box* b) {
  range r = {{0, 0, 0}, {b->bx, b->by, b->nz}};
  return r;
}

/* the ranges used below keep every stencil inside the box; x and y carry a
 * halo of two columns, z is always whole */
static void shrink(range* r, const coefs* c, int d, int lo, int hi) {
  if (!has_dir(c, d)) return;
  r->lo[d] += lo;
  r->hi[d] -= hi;
}

/* ------------------------------------------------------------------------ */
/* one directional predictor-corrector-TVD operator L_alpha(tau), Sec. 3.1   */

static void sweep_box(const coefs* c, const box* b, int al, double tau,
                      const double* X, double* Xo) {
  const int nf = c->nf;
  const int M = c->M;
  const double lam = tau / c->h[al];   /* (dt/2)/delta x_alpha */
  const int zdir = (al == 2);
  /* direction of the predictor flux difference: -1 backward (as printed) */
  const int sp = (zdir || c->pred_dir == 0) ? -1 : +1;
  const int inner_pred = (sp < 0) ? DFWD : DBWD;
  const int inner_corr = (sp < 0) ? DBWD : DFWD;
  const ptrdiff_t s = b->s[al];

  double* F = (double*)calloc((size_t)nf * b->nn, sizeof(double));
  double* XP = (double*)calloc((size_t)nf * b->nn, sizeof(double));
  double* FP = (double*)calloc((size_t)nf * b->nn, sizeof(double));
  double* XC = (double*)calloc((size_t)nf * b->nn, sizeof(double));
  double* Dl = (double*)calloc((size_t)nf * b->nn, sizeof(double)); /* D_{n+1/2} */
  double* cs = (double*)calloc((size_t)b->nn, sizeof(double));
  prims q, qP;
  alloc_prims(b, &q);
  alloc_prims(b, &qP);

  /* level-n primitives and sound speed c = sqrt(gamma p / rho) */
  primitives(c, b, X, &q);
  for (ptrdiff_t n = 0; n < b->nn; ++n)
    cs[n] = sqrt(c->gamma * q.p[n] / X[c->fR * b->nn + n]);

  /* ---- predictor fluxes F^(n) ---- */
  {
    range r = all_nodes(b);
    for (int d = 0; d < 3; ++d)
      if (d != al && d != 2) shrink(&r, c, d, 1, 1);
    if (zdir) {
      r.hi[2] = M;                         /* F_0 .. F_{M-1} */
    } else {
      r.lo[2] = 1; r.hi[2] = M;            /* interior rows */
      if (sp < 0) r.hi[al] -= 1; else r.lo[al] += 1;
    }
#pragma omp parallel for schedule(static)
    for (int kk = r.lo[2]; kk < r.hi[2]; ++kk) {
      range rr = r; rr.lo[2] = kk; rr.hi[2] = kk + 1;
      FOR_RANGE(b, rr, n) {
        double Fn[5];
        int mode = inner_pred;
        if (zdir && kk == 0 && c->wall_order == 2)
          mode = DW2F;                     /* second-order forward at the bottom */
        flux_at(c, b, X, &q, al, n, mode, Fn);
        for (int f = 0; f < nf; ++f) F[f * b->nn + n] = Fn[f];
      }
    }
  }

  /* ---- predictor X^P = X - lam (F_k - F_{k-1}) + tau S(X) ---- */
  {
    range r = all_nodes(b);
    for (int d = 0; d < 3; ++d)
      if (d != al && d != 2) shrink(&r, c, d, 1, 1);
    if (!zdir) shrink(&r, c, al, 1, 1);
    for (int kk = r.lo[2]; kk < r.hi[2]; ++kk) {
      range rr = r; rr.lo[2] = kk; rr.hi[2] = kk + 1;
      FOR_RANGE(b, rr, n) {
        if (!zdir && (kk == 0 || kk == M)) {
          /* plate rows are copied through by the horizontal operators */
          for (int f = 0; f < nf; ++f) XP[f * b->nn + n] = X[f * b->nn + n];
          continue;
        }
        if (zdir && (kk == 0 || kk == M)) {
          double rho;
          if (kk == 0) {
            rho = X[c->fR * b->nn + n];    /* not used by any later stage */
          } else {
            /* backward mass-flux difference at the top plate (m_z,M = 0) */
            rho = X[c->fR * b->nn + n] -
                  lam * (X[c->fm[2] * b->nn + n] - X[c->fm[2] * b->nn + n - s]);
          }
          double Tw = (kk == 0) ? c->Tb : c->Tt;
          for (int f = 0; f < nf; ++f) XP[f * b->nn + n] = 0.0;
          XP[c->fR * b->nn + n] = rho;
          XP[c->fE * b->nn + n] = rho * (c->cv * Tw + c->g * zrow(c, kk));
          continue;
        }
        ptrdiff_t np = (sp < 0) ? n : n + s;      /* F_{k}   (or F_{k+1}) */
        ptrdiff_t nm = (sp < 0) ? n - s : n;      /* F_{k-1} (or F_{k})   */
        for (int f = 0; f < nf; ++f) {
          double v = X[f * b->nn + n] - lam * (F[f * b->nn + np] - F[f * b->nn + nm]);
          if (zdir && f == c->fm[2]) v = v + tau * (-c->g * X[c->fR * b->nn + n]);
          XP[f * b->nn + n] = v;
        }
      }
    }
  }

  /* ---- predicted primitives and corrector fluxes F^P ---- */
  {
    range r = all_nodes(b);
    for (int d = 0; d < 3; ++d)
      if (d != al && d != 2) shrink(&r, c, d, 1, 1);
    if (!zdir) shrink(&r, c, al, 1, 1);
    FOR_RANGE(b, r, n) primitives_at(c, b, XP, &qP, n);
  }
  {
    range r = all_nodes(b);
    for (int d = 0; d < 3; ++d)
      if (d != al && d != 2) shrink(&r, c, d, 2, 2);
    if (zdir) {
      r.lo[2] = 1;                          /* F^P_1 .. F^P_M */
    } else {
      r.lo[2] = 1; r.hi[2] = M;
      if (sp < 0) { r.lo[al] += 2; r.hi[al] -= 1; }
      else        { r.lo[al] += 1; r.hi[al] -= 2; }
    }
#pragma omp parallel for schedule(static)
    for (int kk = r.lo[2]; kk < r.hi[2]; ++kk) {
      range rr = r; rr.lo[2] = kk; rr.hi[2] = kk + 1;
      FOR_RANGE(b, rr, n) {
        double Fn[5];
        int mode = inner_corr;
        if (zdir && kk == M && c->wall_order == 2)
          mode = DW2B;                     /* second-order backward at the top */
        flux_at(c, b, XP, &qP, al, n, mode, Fn);
        for (int f = 0; f < nf; ++f) FP[f * b->nn + n] = Fn[f];
      }
    }
  }

  /* ---- corrector X^C = X - lam (F^P_{k+1} - F^P_k) + tau S(X^P) ---- */
  range rout = all_nodes(b);
  for (int d = 0; d < 3; ++d)
    if (d != 2) shrink(&rout, c, d, 2, 2);
  if (!zdir) { rout.lo[2] = 1; rout.hi[2] = M; }
  {
    range r = rout;
    if (zdir) { r.lo[2] = 1; r.hi[2] = M; }
    FOR_RANGE(b, r, n) {
      ptrdiff_t np = (sp < 0) ? n + s : n;
      ptrdiff_t nm = (sp < 0) ? n : n - s;
      for (int f = 0; f < nf; ++f) {
        double v = X[f * b->nn + n] - lam * (FP[f * b->nn + np] - FP[f * b->nn + nm]);
        if (zdir && f == c->fm[2]) v = v + tau * (-c->g * XP[c->fR * b->nn + n]);
        XC[f * b->nn + n] = v;
      }
    }
  }

  /* ---- TVD flux on faces n+1/2 (Sec. 3.1: T, dX, r+-, G, phi, C) ---- */
  if (c->tvd_on) {
    range r = rout;
    /* faces n-1/2 and n+1/2 of every output node: face index n covers
     * (n, n+1), so faces from lo-1 to hi-1 */
    if (zdir) { r.lo[2] = 1; r.hi[2] = M - 1; }   /* faces 1/2 and M-1/2 stay 0 */
    else { r.lo[al] -= 1; }
    FOR_RANGE(b, r, n) {
      double dm[5], d0[5], dp[5];       /* dX_{n-1/2}, dX_{n+1/2}, dX_{n+3/2} */
      for (int f = 0; f < nf; ++f) {
        const double* x = X + f * b->nn;
        dm[f] = x[n] - x[n - s];
        d0[f] = x[n + s] - x[n];
        dp[f] = x[n + 2 * s] - x[n + s];
      }
      double a_m = 0.0, a_p = 0.0, den = 0.0;  /* dot products */
      for (int f = 0; f < nf; ++f) {
        a_m += dm[f] * d0[f];
        a_p += d0[f] * dp[f];
        den += d0[f] * d0[f];
      }
      double G = 0.0;
      if (den != 0.0) {
        double rplus = a_m / den;          /* r+_n     */
        double rminus = a_p / den;         /* r-_{n+1} */
        double sn = fabs(q.u[al][n]) + cs[n];
        double sn1 = fabs(q.u[al][n + s]) + cs[n + s];
        double Co = lam * (sn > sn1 ? sn : sn1);
        double C = (Co <= 0.5) ? Co * (1.0 - Co) : 0.25;
        if (c->limiter_form == 0) {
          double x = rplus + rminus;
          double phi = fmax(0.0, fmin(2.0 * x, 1.0));
          G = 0.5 * C * (1.0 - phi);
        } else {
          double phi1 = fmax(0.0, fmin(2.0 * rplus, 1.0));
          double phi2 = fmax(0.0, fmin(2.0 * rminus, 1.0));
          G = 0.5 * C * (1.0 - phi1) + 0.5 * C * (1.0 - phi2);
        }
      }
      for (int f = 0; f < nf; ++f) Dl[f * b->nn + n] = G * d0[f];
    }
  }

  /* ---- average + TVD:  X' = (X^P + X^C)/2 + D_{n+1/2} - D_{n-1/2} ---- */
  {
    range r = rout;
    if (zdir) { r.lo[2] = 1; r.hi[2] = M; }
    FOR_RANGE(b, r, n) {
      for (int f = 0; f < nf; ++f) {
        /* T = G dX_{n+1/2} - G dX_{n-1/2}, then the average plus T */
        double T = Dl[f * b->nn + n] - Dl[f * b->nn + n - s];
        Xo[f * b->nn + n] = 0.5 * (XP[f * b->nn + n] + XC[f * b->nn + n]) + T;
      }
    }
  }

  /* ---- plate rows ---- */
  {
    range r = rout;
    for (int kk = 0; kk <= M; kk += M) {
      r.lo[2] = kk; r.hi[2] = kk + 1;
      FOR_RANGE(b, r, n) {
        if (!zdir) {
          for (int f = 0; f < nf; ++f) Xo[f * b->nn + n] = X[f * b->nn + n];
          continue;
        }
        double rho, Tw;
        if (kk == 0) {
          /* bottom: half-cell update with the corrector mass flux
           * (m_z = 0 on the plate) */
          rho = X[c->fR * b->nn + n] - lam * (XP[c->fm[2] * b->nn + n + s] - 0.0);
          Tw = c->Tb;
        } else {
          /* top: the predicted density (backward mass-flux difference) */
          rho = XP[c->fR * b->nn + n];
          Tw = c->Tt;
        }
        for (int f = 0; f < nf; ++f) Xo[f * b->nn + n] = 0.0;
        Xo[c->fR * b->nn + n] = rho;
        Xo[c->fE * b->nn + n] = rho * (c->cv * Tw + c->g * zrow(c, kk));
      }
    }
  }

  free(F); free(XP); free(FP); free(XC); free(Dl); free(cs);
  free_prims(&q);
  free_prims(&qP);
}

int ora_sweep_box(const ora_params* p, int axis, double tau, int bx, int by,
                  const double* Bin, double* Bout) {
  if (check_params(p)) return -1;
  if (axis < 0 || axis > 2 || (axis == 1 && p->ndim != 3)) return -1;
  coefs c;
  make_coefs(p, &c);
  set_threads(p);
  if (p->ndim == 2) by = 1;
  if (bx < 5 || (p->ndim == 3 && by < 5)) return -1;
  box b = make_box(bx, by, c.nz);
  sweep_box(&c, &b, axis, tau, Bin, Bout);
  return 0;
}

/* whole periodic domain: pad two halo columns in x (and y), sweep, unpad */
int ora_sweep(const ora_params* p, int axis, double tau, const double* Xin,
              double* Xout) {
  if (check_params(p)) return -1;
  if (axis < 0 || axis > 2 || (axis == 1 && p->ndim != 3)) return -1;
  coefs c;
  make_coefs(p, &c);
  set_threads(p);
  int hy = (p->ndim == 3) ? 2 : 0;
  int bx = c.nx + 4, by = c.ny + 2 * hy;
  box b = make_box(bx, by, c.nz);
  size_t cnt = (size_t)c.nx * c.ny * c.nz;
  double* Bin = (double*)malloc(sizeof(double) * (size_t)c.nf * b.nn);
  double* Bout = (double*)calloc((size_t)c.nf * b.nn, sizeof(double));
  for (int f = 0; f < c.nf; ++f)
    for (int k = 0; k < c.nz; ++k)
      for (int jb = 0; jb < by; ++jb)
        for (int ib = 0; ib < bx; ++ib) {
          int i = ((ib - 2) % c.nx + c.nx) % c.nx;
          int j = ((jb - hy) % c.ny + c.ny) % c.ny;
          Bin[f * b.nn + ib + b.s[1] * jb + b.s[2] * k] =
              Xin[f * cnt + (size_t)i + (size_t)c.nx * ((size_t)j + (size_t)c.ny * k)];
        }
  sweep_box(&c, &b, axis, tau, Bin, Bout);
  for (int f = 0; f < c.nf; ++f)
    for (int k = 0; k < c.nz; ++k)
      for (int j = 0; j < c.ny; ++j)
        for (int i = 0; i < c.nx; ++i)
          Xout[f * cnt + (size_t)i + (size_t)c.nx * ((size_t)j + (size_t)c.ny * k)] =
              Bout[f * b.nn + (i + 2) + b.s[1] * (j + hy) + b.s[2] * k];
  free(Bin);
  free(Bout);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* time step                                                                 */

double ora_dt(const ora_params* p, const double* X) {
  if (check_params(p)) return -1.0;
  coefs c;
  make_coefs(p, &c);
  size_t cnt = (size_t)c.nx * c.ny * c.nz;
  double best = INFINITY;
  for (int k = 0; k < c.nz; ++k)
    for (int j = 0; j < c.ny; ++j)
      for (int i = 0; i < c.nx; ++i) {
        size_t n = (size_t)i + (size_t)c.nx * ((size_t)j + (size_t)c.ny * k);
        double rho = X[c.fR * cnt + n];
        double u[3] = {0, 0, 0};
        for (int d = 0; d < 3; ++d)
          if (c.fm[d] >= 0) u[d] = X[c.fm[d] * cnt + n] / rho;
        double uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
        double T = (X[c.fE * cnt + n] / rho - 0.5 * uu - c.g * zrow(&c, k)) / c.cv;
        double pr = c.a * rho * T;
        double cs = sqrt(c.gamma * pr / rho);
        for (int d = 0; d < 3; ++d) {
          if (!has_dir(&c, d)) continue;
          double v = c.h[d] / (fabs(u[d]) + cs);
          if (v < best) best = v;
        }
      }
  return c.cfl * best;
}

int ora_step(const ora_params* p, double* X, int nsteps, double* time,
             double* dt) {
  if (check_params(p)) return -1;
  coefs c;
  make_coefs(p, &c);
  size_t len = ora_state_len(p);
  double* Y = (double*)malloc(sizeof(double) * len);
  double frozen = (dt && *dt > 0.0) ? *dt : -1.0;
  if (p->dt_mode == 1 && frozen <= 0.0) frozen = ora_dt(p, X);
  /* X^{n+1} = L_x L_y L_z L_x L_y L_z X^n (Sec. 3.1, time_step), each L at
   * dt/2; in 2D L_y is absent.  sweep_order 1 mirrors the second half. */
  int order[6];
  int no = 0;
  if (p->ndim == 3) {
    int a[6] = {2, 1, 0, 2, 1, 0}, b[6] = {2, 1, 0, 0, 1, 2};
    for (int i = 0; i < 6; ++i) order[i] = p->sweep_order ? b[i] : a[i];
    no = 6;
  } else {
    int a[4] = {2, 0, 2, 0}, b[4] = {2, 0, 0, 2};
    for (int i = 0; i < 4; ++i) order[i] = p->sweep_order ? b[i] : a[i];
    no = 4;
  }
  double last = 0.0;
  for (int s = 0; s < nsteps; ++s) {
    double d = (p->dt_mode == 1) ? frozen : ora_dt(p, X);
    for (int o = 0; o < no; ++o) {
      ora_sweep(p, order[o], 0.5 * d, X, Y);
      memcpy(X, Y, sizeof(double) * len);
    }
    if (time) *time += d;
    last = d;
  }
  if (dt) *dt = (nsteps > 0) ? last : ((p->dt_mode == 1) ? frozen : ora_dt(p, X));
  free(Y);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* diagnostics (Sec. 2: volume_Nu, mean_Nu)                                  */

/* Neumaier compensated sum */
typedef struct { double s, c; } csum;
static void cadd(csum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double cval(const csum* a) { return a->s + a->c; }

int ora_diag(const ora_params* p, const double* X, ora_diag_t* d) {
  if (check_params(p)) return -1;
  coefs c;
  make_coefs(p, &c);
  set_threads(p);
  const int M = c.M;
  const size_t plane = (size_t)c.nx * c.ny, cnt = plane * c.nz;
  /* per-row sums: rho, rho|u|^2/2, E, rho u_z T_sa, rho u_z |u|^2, T */
  double* rs = (double*)calloc((size_t)c.nz * 6, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int k = 0; k < c.nz; ++k) {
    csum acc[6];
    memset(acc, 0, sizeof(acc));
    double z = zrow(&c, k);
    for (size_t t = 0; t < plane; ++t) {
      size_t n = t + plane * k;
      double rho = X[c.fR * cnt + n];
      double u[3] = {0, 0, 0};
      for (int q = 0; q < 3; ++q)
        if (c.fm[q] >= 0) u[q] = X[c.fm[q] * cnt + n] / rho;
      double uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
      double E = X[c.fE * cnt + n];
      double T = (E / rho - 0.5 * uu - c.g * z) / c.cv;
      double Tsa = T - (1.0 - c.D * z);      /* T minus adiabatic T_A */
      cadd(&acc[0], rho);
      cadd(&acc[1], 0.5 * rho * uu);
      cadd(&acc[2], E);
      cadd(&acc[3], rho * u[2] * Tsa);
      cadd(&acc[4], rho * u[2] * uu);
      cadd(&acc[5], T);
    }
    for (int q = 0; q < 6; ++q) rs[k * 6 + q] = cval(&acc[q]);
  }
  /* trapezoid weights in z, rectangle rule in the periodic directions */
  double dV = c.h[0] * c.h[2] * ((c.ndim == 3) ? c.h[1] : 1.0);
  double V = (c.ndim == 3) ? c.aspect * c.aspect : c.aspect;
  csum tot[5];
  memset(tot, 0, sizeof(tot));
  for (int k = 0; k <= M; ++k) {
    double w = (k == 0 || k == M) ? 0.5 : 1.0;
    for (int q = 0; q < 5; ++q) cadd(&tot[q], w * rs[k * 6 + q]);
  }
  d->mass = cval(&tot[0]) * dV;
  d->kinetic = cval(&tot[1]) * dV;
  d->total_energy = cval(&tot[2]) * dV;
  double sRP = sqrt(c.Ra * c.Pr);
  d->nu_conv = sRP / c.eps * (cval(&tot[3]) * dV / V);
  d->nu_kin = c.D * sRP / 2.0 * (cval(&tot[4]) * dV / V);
  d->nu_bulk = (1.0 + d->nu_conv) + d->nu_kin;
  int rows[6] = {0, 1, 2, M - 2, M - 1, M};
  for (int q = 0; q < 6; ++q) d->tmean[q] = rs[rows[q] * 6 + 5] / (double)plane;
  double dz = c.h[2];
  /* d<T_sa>/dz = d<T>/dz + D; second-order one-sided at each plate */
  double gb = ((-3.0 * d->tmean[0] + 4.0 * d->tmean[1]) - d->tmean[2]) / (2.0 * dz);
  double gt = ((3.0 * d->tmean[5] - 4.0 * d->tmean[4]) + d->tmean[3]) / (2.0 * dz);
  d->nu_bottom = -(gb + c.D) / c.eps;
  d->nu_top = -(gt + c.D) / c.eps;
  d->nu_mean = 0.5 * (d->nu_bottom + d->nu_top);
  free(rs);
  return 0;
}
