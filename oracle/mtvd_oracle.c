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
 *   - dt = cfl * min over nodes and directions of h_a/(|u_a| + c) (with
 *     dt_rule = 1 also of rho h^2 / kappa, the explicit diffusion limit);
 *   - the initial state: T = 1 - (eps+D) z, rho = T^(m-1) (hydrostatic for
 *     the unperturbed T), m = gamma D / ((gamma-1)(eps+D)), noise on
 *     interior T from SplitMix64.
 */
#include "mtvd_oracle.h"

#include <complex.h>
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
  double complex mu_cs, K_cs; /* mu and K of the complex-step mode */
  double Tb, Tt;             /* plate temperatures: 1 and 1-(eps+D) */
  double cfl;
  int limiter_form, tvd_on, pred_dir, sweep_order, wall_order;
  int stretched;             /* 1 on the tanh grid (stretch > 0) */
  double s, ths;             /* stretch s and tanh(s) */
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
  c->mu_cs = c->mu;
  c->K_cs = c->K;
  c->Tb = 1.0;
  c->Tt = 1.0 - (p->eps + p->D);
  c->cfl = p->cfl;
  c->limiter_form = p->limiter_form;
  c->tvd_on = p->tvd_on;
  c->pred_dir = p->pred_dir;
  c->sweep_order = p->sweep_order;
  c->wall_order = p->wall_order;
  c->stretched = p->stretch > 0.0;
  c->s = p->stretch;
  c->ths = c->stretched ? tanh(p->stretch) : 1.0;
}

static int check_params(const ora_params* p) {
  if (!p) return -1;
  if (p->ndim != 2 && p->ndim != 3) return -1;
  if (p->nx < 1 || p->nz < 3) return -1;
  if (p->ndim == 3 && p->ny < 1) return -1;
  if (!(p->gamma > 1.0) || !(p->eps > 0.0) || !(p->D > 0.0)) return -1;
  if (!(p->Ra > 0.0) || !(p->Pr > 0.0) || !(p->aspect > 0.0)) return -1;
  if (p->wall_order != 1 && p->wall_order != 2) return -1;
  if (!(p->stretch >= 0.0) || !(p->stretch <= 10.0)) return -1;
  if (p->dt_rule != 0 && p->dt_rule != 1) return -1;
  return 0;
}

static void set_threads(const ora_params* p) {
#ifdef _OPENMP
  if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#else
  (void)p;
#endif
}

/* height of row k: z_k = k / M on the uniform grid; on the tanh grid
 * z_k = (1 + tanh(s (2k - M)/M) / tanh s) / 2.  Both put the plates exactly
 * at 0 and 1 (tanh is odd, so the quotient is -1 and 1 at the ends). */
static double zrow(const coefs* c, int k) {
  if (!c->stretched) return (double)k / (double)c->M;
  double xi = (2.0 * (double)k - (double)c->M) / (double)c->M;
  return 0.5 * (1.0 + tanh(c->s * xi) / c->ths);
}

/* z spacing of face k+1/2 and the dual cell of row k (trapezoid weight in
 * units of length: (z_k+1 - z_k-1)/2 inside, half the face at a plate) */
static double zface(const coefs* c, int k) { return zrow(c, k + 1) - zrow(c, k); }
static double zdual(const coefs* c, int k) {
  if (k == 0) return 0.5 * zface(c, 0);
  if (k == c->M) return 0.5 * zface(c, c->M - 1);
  return 0.5 * (zrow(c, k + 1) - zrow(c, k - 1));
}

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

int ora_heights(const ora_params* p, double* z) {
  if (check_params(p)) return -1;
  coefs c;
  make_coefs(p, &c);
  for (int k = 0; k < c.nz; ++k) z[k] = zrow(&c, k);
  return 0;
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

/* finite differences of an array q along direction d at node n */
enum { DFWD, DBWD, DCEN, DW2F, DW2B };

static int has_dir(const coefs* c, int d) { return d != 1 || c->ndim == 3; }

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

/* the operator over double (the oracle) and over double complex (the
 * complex-step mode of the adjoint checks); see mtvd_oracle_sweep.inc */
#define R double
#define SFX(name) name
#define MU(c) ((c)->mu)
#define KK(c) ((c)->K)
#define RE(x) (x)
#define ABS(x) fabs(x)
#define SQRT(x) sqrt(x)
#define PHI(t) fmax(0.0, fmin((t), 1.0))
#include "mtvd_oracle_sweep.inc"
#undef R
#undef SFX
#undef MU
#undef KK
#undef RE
#undef ABS
#undef SQRT
#undef PHI

/* complex step: branches on real parts; |x| takes sign(0) = 0 */
static double complex cs_abs(double complex x) {
  return creal(x) > 0.0 ? x : (creal(x) < 0.0 ? -x : 0.0);
}
static double complex cs_phi(double complex t) {
  return creal(t) <= 0.0 ? 0.0 : (creal(t) >= 1.0 ? 1.0 : t);
}
#define R double complex
#define SFX(name) name##_cs
#define MU(c) ((c)->mu_cs)
#define KK(c) ((c)->K_cs)
#define RE(x) creal(x)
#define ABS(x) cs_abs(x)
#define SQRT(x) csqrt(x)
#define PHI(t) cs_phi(t)
#include "mtvd_oracle_sweep.inc"
#undef R
#undef SFX
#undef MU
#undef KK
#undef RE
#undef ABS
#undef SQRT
#undef PHI

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

int ora_sweep(const ora_params* p, int axis, double tau, const double* Xin,
              double* Xout) {
  if (check_params(p)) return -1;
  if (axis < 0 || axis > 2 || (axis == 1 && p->ndim != 3)) return -1;
  coefs c;
  make_coefs(p, &c);
  set_threads(p);
  sweep_periodic(&c, axis, tau, Xin, Xout);
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
          double h = c.h[d];
          if (d == 2 && c.stretched) {
            /* the narrower of the node's faces */
            h = (k == 0) ? zface(&c, 0) : (k == c.M) ? zface(&c, c.M - 1)
                : fmin(zface(&c, k - 1), zface(&c, k));
          }
          double v = h / (fabs(u[d]) + cs);
          if (v < best) best = v;
        }
        if (p->dt_rule == 1) {
          /* explicit diffusion limit: rho h^2 / kappa over the node's
           * smallest spacing */
          double hm = c.h[0];
          if (c.ndim == 3) hm = fmin(hm, c.h[1]);
          double hz = c.h[2];
          if (c.stretched)
            hz = (k == 0) ? zface(&c, 0) : (k == c.M) ? zface(&c, c.M - 1)
                 : fmin(zface(&c, k - 1), zface(&c, k));
          hm = fmin(hm, hz);
          double kappa = fmax(c.mu * (2.0 + fabs(c.lam)), c.K / c.cv);
          double v = (rho * (hm * hm)) / kappa;
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
    /* on the tanh grid the weights are the dual cells in units of dz */
    double w = c.stretched ? zdual(&c, k) / c.h[2] : (k == 0 || k == M) ? 0.5 : 1.0;
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
  /* d<T_sa>/dz = d<T>/dz + D; second-order one-sided at each plate (on the
   * tanh grid the same stencil applied to the heights is the divisor) */
  double db = 2.0 * dz, dt_ = 2.0 * dz;
  if (c.stretched) {
    db = (-3.0 * zrow(&c, 0) + 4.0 * zrow(&c, 1)) - zrow(&c, 2);
    dt_ = (3.0 * zrow(&c, M) - 4.0 * zrow(&c, M - 1)) + zrow(&c, M - 2);
  }
  double gb = ((-3.0 * d->tmean[0] + 4.0 * d->tmean[1]) - d->tmean[2]) / db;
  double gt = ((3.0 * d->tmean[5] - 4.0 * d->tmean[4]) + d->tmean[3]) / dt_;
  d->nu_bottom = -(gb + c.D) / c.eps;
  d->nu_top = -(gt + c.D) / c.eps;
  d->nu_mean = 0.5 * (d->nu_bottom + d->nu_top);
  free(rs);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* complex-step mode (checks of the adjoint)                                 */

/* Nu_mean (Sec. 2, mean_Nu) of a complex state: the row means of T on the
 * rows 0, 1, 2, M-2, M-1, M and the one-sided differences of ora_diag */
static double complex nu_mean_cs(const coefs* c, const double complex* X) {
  const int M = c->M;
  const size_t plane = (size_t)c->nx * c->ny, cnt = plane * c->nz;
  int rows[6] = {0, 1, 2, M - 2, M - 1, M};
  double complex tm[6];
  for (int q = 0; q < 6; ++q) {
    int k = rows[q];
    double z = zrow(c, k);
    double complex sum = 0.0;
    for (size_t t = 0; t < plane; ++t) {
      size_t n = t + plane * k;
      double complex rho = X[c->fR * cnt + n];
      double complex u[3] = {0, 0, 0};
      for (int d = 0; d < 3; ++d)
        if (c->fm[d] >= 0) u[d] = X[c->fm[d] * cnt + n] / rho;
      double complex uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
      sum += (X[c->fE * cnt + n] / rho - 0.5 * uu - c->g * z) / c->cv;
    }
    tm[q] = sum / (double)plane;
  }
  double dz = c->h[2];
  double db = 2.0 * dz, dt_ = 2.0 * dz;
  if (c->stretched) {
    db = (-3.0 * zrow(c, 0) + 4.0 * zrow(c, 1)) - zrow(c, 2);
    dt_ = (3.0 * zrow(c, M) - 4.0 * zrow(c, M - 1)) + zrow(c, M - 2);
  }
  double complex gb = ((-3.0 * tm[0] + 4.0 * tm[1]) - tm[2]) / db;
  double complex gt = ((3.0 * tm[5] - 4.0 * tm[4]) + tm[3]) / dt_;
  double complex nb = -(gb + c->D) / c->eps, nt = -(gt + c->D) / c->eps;
  return 0.5 * (nb + nt);
}

int ora_time_avg_nu_cs(const ora_params* p, const double* X0, const double* V, double h,
                       double dmu, double dK, int nsteps, double dt, double* J, double* dJ) {
  if (check_params(p)) return -1;
  if (nsteps < 1 || !(dt > 0.0) || !(h > 0.0)) return -1;
  coefs c;
  make_coefs(p, &c);
  set_threads(p);
  c.mu_cs = c.mu + (h * dmu) * I;
  c.K_cs = c.K + (h * dK) * I;
  size_t len = ora_state_len(p);
  double complex* X = (double complex*)malloc(sizeof(double complex) * len);
  double complex* Y = (double complex*)malloc(sizeof(double complex) * len);
  for (size_t n = 0; n < len; ++n) X[n] = X0[n] + (V ? (h * V[n]) * I : 0.0);
  int order[6], no;
  if (p->ndim == 3) {
    int a[6] = {2, 1, 0, 2, 1, 0}, b[6] = {2, 1, 0, 0, 1, 2};
    for (int i = 0; i < 6; ++i) order[i] = p->sweep_order ? b[i] : a[i];
    no = 6;
  } else {
    int a[4] = {2, 0, 2, 0}, b[4] = {2, 0, 0, 2};
    for (int i = 0; i < 4; ++i) order[i] = p->sweep_order ? b[i] : a[i];
    no = 4;
  }
  double complex acc = 0.0;
  for (int s = 0; s < nsteps; ++s) {
    for (int o = 0; o < no; ++o) {
      sweep_periodic_cs(&c, order[o], 0.5 * dt, X, Y);
      double complex* t = X; X = Y; Y = t;
    }
    acc += nu_mean_cs(&c, X);
  }
  *J = creal(acc) / nsteps;
  *dJ = cimag(acc) / nsteps / h;
  free(X);
  free(Y);
  return 0;
}
