/* Drives every entry point of the CPU oracle (oracle/mtvd_oracle.c) on tiny
 * grids, for a build with AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Every array is a heap block of exactly the length the oracle's contract
 * states (ora_state_len, the box sizes), so a read or write one element past
 * any field, row or box edge is reported by the sanitizer.  The grids are
 * the smallest the parameter checks accept (one column in x, three rows in
 * z, five-column boxes) and a few ragged ones, in 2D and 3D, with every
 * switch of the scheme (limiter form, sweep order, wall stencil, TVD on or
 * off, predictor direction, frozen dt).  Each result is also checked to be
 * finite, and each bad argument to be rejected.
 *
 * Exit status 0 and the last line "oracle sanitize driver ok" on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mtvd_oracle.h"

static int failures = 0;

#define CHECK(cond, ...)                        \
  do {                                          \
    if (!(cond)) {                              \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      fprintf(stderr, __VA_ARGS__);             \
      fputc('\n', stderr);                      \
      ++failures;                               \
    }                                           \
  } while (0)

static ora_params base(int ndim, int nx, int ny, int nz) {
  ora_params p;
  memset(&p, 0, sizeof p);
  p.ndim = ndim;
  p.nx = nx;
  p.ny = ndim == 3 ? ny : 1;
  p.nz = nz;
  p.aspect = 4.0;
  p.gamma = 1.4;
  p.Pr = 1.0;
  p.Ra = 1e5;
  p.eps = 0.1;
  p.D = 0.4;
  p.cfl = 0.5;
  p.seed = 5;
  p.noise_amp = 1e-2;
  p.dt_mode = 0;
  p.bulk_coef = -2.0 / 3.0;
  p.limiter_form = 0;
  p.sweep_order = 0;
  p.tvd_on = 1;
  p.gravity_scale = 1.0;
  p.wall_order = 2;
  p.pred_dir = 0;
  p.diffusion_scale = 1.0;
  p.nthreads = 1 + (nx % 3);  /* 1-3 OpenMP threads where built with OpenMP */
  p.stretch = 0.0;
  return p;
}

static double* alloc(size_t n) {
  double* a = (double*)malloc(n * sizeof(double));
  if (!a) {
    fprintf(stderr, "out of memory\n");
    exit(2);
  }
  return a;
}

static int all_finite(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

static void run_case(const ora_params* p, const char* label) {
  const size_t n = ora_state_len(p);
  double* X = alloc(n);
  double* Y = alloc(n);
  double* V = alloc(n);
  CHECK(ora_init(p, X) == 0, "%s: init", label);
  CHECK(all_finite(X, n), "%s: init not finite", label);

  const double dt = ora_dt(p, X);
  CHECK(dt > 0.0 && isfinite(dt), "%s: dt %g", label, dt);

  for (int axis = 0; axis < 3; ++axis) {
    if (axis == 1 && p->ndim != 3) {
      CHECK(ora_sweep(p, axis, dt, X, Y) == -1, "%s: y sweep in 2D accepted", label);
      continue;
    }
    CHECK(ora_sweep(p, axis, dt, X, Y) == 0, "%s: sweep %d", label, axis);
    CHECK(all_finite(Y, n), "%s: sweep %d not finite", label, axis);
  }

  memcpy(Y, X, n * sizeof(double));
  double t = 0.0, dt_used = 0.0;
  CHECK(ora_step(p, Y, 3, &t, &dt_used) == 0, "%s: step", label);
  CHECK(all_finite(Y, n) && t > 0.0 && dt_used > 0.0, "%s: step result", label);

  ora_diag_t d;
  CHECK(ora_diag(p, Y, &d) == 0, "%s: diag", label);
  CHECK(isfinite(d.nu_mean) && isfinite(d.mass) && isfinite(d.tmean[5]), "%s: diag values",
        label);

  for (size_t i = 0; i < n; ++i) V[i] = (double)((i * 7919u) % 13u) / 13.0 - 0.5;
  double J = 0.0, dJ = 0.0;
  CHECK(ora_time_avg_nu_cs(p, X, V, 1e-30, 0.3, -0.2, 2, dt, &J, &dJ) == 0, "%s: cs", label);
  CHECK(isfinite(J) && isfinite(dJ), "%s: cs values", label);
  CHECK(ora_time_avg_nu_cs(p, X, NULL, 1e-30, 1.0, 0.0, 1, dt, &J, &dJ) == 0, "%s: cs V=NULL",
        label);
  CHECK(ora_time_avg_nu_cs(p, X, V, 1e-30, 0.0, 0.0, 0, dt, &J, &dJ) == -1,
        "%s: cs nsteps=0 accepted", label);

  free(V);
  free(Y);
  free(X);
}

static void run_box(const ora_params* p, int i0, int j0, int bx, int by, const char* label) {
  const int byy = p->ndim == 3 ? by : 1;
  const size_t n = (size_t)(p->ndim + 2) * (size_t)p->nz * (size_t)byy * (size_t)bx;
  double* B = alloc(n);
  double* C = alloc(n);
  CHECK(ora_init_box(p, i0, j0, bx, byy, B) == 0, "%s: init_box", label);
  CHECK(all_finite(B, n), "%s: init_box not finite", label);
  const double tau = 1e-3;
  for (int axis = 0; axis < 3; ++axis) {
    if (axis == 1 && p->ndim != 3) continue;
    memcpy(C, B, n * sizeof(double));
    CHECK(ora_sweep_box(p, axis, tau, bx, byy, B, C) == 0, "%s: sweep_box %d", label, axis);
    CHECK(all_finite(C, n), "%s: sweep_box %d not finite", label, axis);
  }
  CHECK(ora_sweep_box(p, 0, tau, 4, byy, B, C) == -1, "%s: bx=4 accepted", label);
  free(C);
  free(B);
}

int main(void) {
  /* smallest accepted grids, ragged ones, and each switch of the scheme */
  struct {
    int ndim, nx, ny, nz;
  } grids[] = {
      {2, 1, 1, 3}, {2, 2, 1, 4}, {2, 7, 1, 5}, {2, 13, 1, 9},
      {3, 1, 1, 3}, {3, 3, 2, 4}, {3, 5, 7, 6},
  };
  char label[128];
  for (size_t g = 0; g < sizeof grids / sizeof grids[0]; ++g) {
    for (int variant = 0; variant < 7; ++variant) {
      ora_params p = base(grids[g].ndim, grids[g].nx, grids[g].ny, grids[g].nz);
      switch (variant) {
        case 1: p.limiter_form = 1; break;
        case 2: p.sweep_order = 1; p.wall_order = 1; break;
        case 3: p.tvd_on = 0; p.dt_mode = 1; break;
        case 4: p.pred_dir = 1; p.bulk_coef = 0.0; break;
        case 5: p.gravity_scale = 0.0; p.diffusion_scale = 0.0; break;
        case 6: p.stretch = 1.7; p.wall_order = 2; break;
        default: break;
      }
      snprintf(label, sizeof label, "%dD %dx%dx%d variant %d", p.ndim, p.nx, p.ny, p.nz,
               variant);
      run_case(&p, label);
    }
  }

  /* boxes: the minimum width, wrap-around starts, a ragged 3D box */
  ora_params p2 = base(2, 9, 1, 6);
  run_box(&p2, 0, 0, 5, 1, "2D box 5");
  run_box(&p2, 7, 0, 11, 1, "2D box wrap");
  p2.stretch = 2.0;
  run_box(&p2, 3, 0, 6, 1, "2D box stretched");
  ora_params p3 = base(3, 6, 5, 4);
  run_box(&p3, 0, 0, 5, 5, "3D box 5x5");
  run_box(&p3, 4, 3, 8, 6, "3D box wrap");

  /* bad parameters are rejected before any array is touched */
  ora_params bad = base(2, 8, 1, 2);
  double dummy[1] = {0.0};
  CHECK(ora_init(&bad, dummy) == -1, "nz=2 accepted");
  bad = base(4, 8, 1, 5);
  CHECK(ora_init(&bad, dummy) == -1, "ndim=4 accepted");
  bad = base(2, 8, 1, 5);
  bad.gamma = 1.0;
  CHECK(ora_dt(&bad, dummy) == -1.0, "gamma=1 accepted");
  bad = base(2, 8, 1, 5);
  bad.wall_order = 3;
  CHECK(ora_step(&bad, dummy, 1, dummy, dummy) == -1, "wall_order=3 accepted");
  CHECK(ora_init(NULL, dummy) == -1, "NULL params accepted");
  bad = base(2, 8, 1, 5);
  bad.stretch = -1.0;
  CHECK(ora_init(&bad, dummy) == -1, "stretch < 0 accepted");
  {
    ora_params g = base(2, 4, 1, 7);
    g.stretch = 1.5;
    double* z = alloc(7);
    CHECK(ora_heights(&g, z) == 0 && z[0] == 0.0 && z[6] == 1.0, "heights");
    free(z);
  }

  CHECK(ora_splitmix64(0, 1) == 0xE220A8397B1DCDAFULL, "splitmix64(0, 1)");

  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("oracle sanitize driver ok\n");
  return 0;
}
