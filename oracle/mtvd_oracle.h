/*
 * mtvd_oracle.h -- plain CPU FP64 oracle for one MacCormack-TVD time step of
 * the nondimensional compressible Navier-Stokes equations with gravity
 * (Tiwari, Sharma & Verma, arXiv:2411.10372, Sec. 2 and Sec. 3.1).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no source with the GPU path and includes none of
 * its headers.
 *
 * Layout of a state array: X[f][k][j][i], i (x) fastest, unpadded.
 *   fields f (2D): rho, rho*u_x, rho*u_z, E
 *   fields f (3D): rho, rho*u_x, rho*u_y, rho*u_z, E
 * x and y are periodic without a duplicated end point (dx = aspect/nx,
 * dy = aspect/ny); z has nz nodes with the plates on k = 0 and k = nz-1,
 * uniform (dz = 1/(nz-1)) or tanh-stretched (the stretch parameter).
 *
 * On a stretched grid every z difference divides by the same difference of
 * the node heights (forward (q_k+1 - q_k)/(z_k+1 - z_k), central over
 * z_k+1 - z_k-1, the one-sided plate stencils over the same stencil of
 * z), the flux differences of predictor and corrector divide by the dual
 * cell w_k = (z_k+1 - z_k-1)/2 (half the adjacent face at a plate), and
 * the TVD term is the difference of face fluxes h_k+1/2 G dX_k+1/2 divided
 * by w_k with the face Courant number tau |lambda| / h_k+1/2.  On the
 * uniform grid each of these is the printed scheme; the uniform code path
 * is kept as it was, so its results do not change.
 */
#ifndef MTVD_ORACLE_H
#define MTVD_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora_params {
  int32_t ndim;          /* 2 or 3 */
  int32_t nx, ny, nz;    /* ny = 1 in 2D; nz >= 3 */
  double aspect;         /* Gamma = L/d */
  double gamma, Pr, Ra, eps, D;
  double cfl;
  uint64_t seed;
  double noise_amp;      /* uniform +-noise_amp on interior T at init */
  int32_t dt_mode;       /* 0: dt from the state every step; 1: frozen */
  double bulk_coef;      /* lambda in tau_ij (the 2/3 term); -2/3 = Stokes */
  int32_t limiter_form;  /* 0: G(r+ + r-) as printed; 1: G(r+) + G(r-) */
  int32_t sweep_order;   /* 0: z,y,x,z,y,x as printed; 1: z,y,x,x,y,z */
  int32_t tvd_on;        /* 1 normally; 0 drops the TVD correction */
  double gravity_scale;  /* 1 normally; 0 switches gravity off */
  int32_t wall_order;    /* 2: z-derivatives inside the plate fluxes F_0 and
                            F^P_M are the second-order one-sided ones;
                            1: the same one-sided first differences as the
                            interior (compact) */
  /* knobs that exist only here, for the oracle's own pins */
  int32_t pred_dir;      /* 0: predictor uses backward flux differences (as
                            printed); 1: forward (periodic axes only) */
  double diffusion_scale;/* multiplies mu* and K*; 1 normally */
  int32_t nthreads;      /* OpenMP threads; 0 = runtime default */
  double stretch;        /* s of the tanh z grid (Sec. 3.1 grid): z_k =
                            (1 + tanh(s (2k/M - 1)) / tanh s) / 2; 0 gives
                            the uniform grid z_k = k/M */
  int32_t dt_rule;       /* 0: dt from the acoustic CFL condition alone;
                            1: also the explicit diffusion limit (ora_dt) */
} ora_params;

typedef struct ora_diag {
  double mass, kinetic, total_energy;
  double nu_bottom, nu_top, nu_mean, nu_bulk, nu_conv, nu_kin;
  double tmean[6];       /* <T>_A on rows 0, 1, 2, M-2, M-1, M */
} ora_diag_t;

/* OpenMP threads the oracle's parallel loops use */
int ora_threads(void);

/* number of doubles in one state array */
size_t ora_state_len(const ora_params* p);

/* n-th output (n >= 1) of the SplitMix64 generator started from `seed`
 * (Steele, Lea & Flood 2014): mix64(seed + n * 0x9E3779B97F4A7C15). */
uint64_t ora_splitmix64(uint64_t seed, uint64_t n);

/* the nz node heights z_k of the grid (uniform or tanh) */
int ora_heights(const ora_params* p, double* z);

/* initial state: conductive T, hydrostatic rho, seeded T noise, u = 0 */
int ora_init(const ora_params* p, double* X);

/* same values on a sub-box of bx x by columns starting at global (i0, j0),
 * wrapping periodically; all nz rows.  Layout B[f][k][j][i] of the box. */
int ora_init_box(const ora_params* p, int i0, int j0, int bx, int by,
                 double* B);

/* dt = cfl * min over nodes and directions of h_a / (|u_a| + c); with
 * dt_rule = 1 the minimum also runs over rho h^2 / kappa of every node, h
 * its smallest spacing (the narrowest z face on the tanh grid) and
 * kappa = max(mu (2 + |lambda|), K / c_v) the largest diffusivity times rho
 * (viscous with the bulk term, thermal), so that each directional operator
 * L(dt/2) has diffusion number kappa (dt/2) / (rho h^2) <= cfl/2 */
double ora_dt(const ora_params* p, const double* X);

/* one directional operator L_axis(tau) on the whole periodic domain;
 * axis 0 = x, 1 = y, 2 = z.  Xin and Xout must not alias. */
int ora_sweep(const ora_params* p, int axis, double tau, const double* Xin,
              double* Xout);

/* L_axis(tau) on a box of bx x by columns (all nz rows) whose outer two
 * columns in x (and in y for 3D) are halo: only columns 2..bx-3 (and rows
 * 2..by-3 in y) of Bout are written.  In 2D pass by = 1. */
int ora_sweep_box(const ora_params* p, int axis, double tau, int bx, int by,
                  const double* Bin, double* Bout);

/* nsteps full time steps in place.  *time is advanced.  *dt receives the
 * last dt used; with dt_mode = 1 a positive *dt on entry is used as the
 * frozen value (else it is computed from X on entry). */
int ora_step(const ora_params* p, double* X, int nsteps, double* time,
             double* dt);

int ora_diag(const ora_params* p, const double* X, ora_diag_t* d);

/* Complex-step mode (checks of the adjoint): N = nsteps steps with the fixed
 * dt from X0 + i h V (V may be NULL), mu + i h dmu and K + i h dK (mu and K
 * the viscosity and conductivity coefficients of the parameters), every
 * branch decided on real parts.  *J = (1/N) sum_{n=1..N} Nu_mean(X_n) of the
 * real part and *dJ = Im(...)/h, the derivative of J along (V, dmu, dK) on
 * the branches taken (Squire & Trapp, SIAM Review 40, 1998).  Returns -1 on
 * bad arguments. */
int ora_time_avg_nu_cs(const ora_params* p, const double* X0, const double* V, double h,
                       double dmu, double dK, int nsteps, double dt, double* J, double* dJ);

#ifdef __cplusplus
}
#endif
#endif
