// Drives the host-only entry points of the C ABI (include/mtvd.h) -- the
// ones that do no device work -- for a build of the library's host code
// with AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Every array handed to the library is a heap block of exactly the length
// the header states (MTVD_NUM_PROFILES * nz for a profile array, nz for a
// profile or an output row), so a read or write past its end is reported.
// Covered: default parameters, buffer sizes (single box, batch, adjoint),
// parameter validation in mtvd_create (every rejection returns before the
// first HIP call), the analysis scalars and profiles from a row-mean array,
// the boundary-layer thicknesses, and the error strings.
//
// Exit status 0 and the last line "host sanitize driver ok" on success.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "mtvd.h"

static int failures = 0;

#define CHECK(cond, ...)                                    \
  do {                                                      \
    if (!(cond)) {                                          \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                    \
      std::fputc('\n', stderr);                             \
      ++failures;                                           \
    }                                                       \
  } while (0)

static mtvd_params params(int ndim, int nx, int ny, int nz) {
  mtvd_params p;
  mtvd_default_params(&p);
  p.ndim = ndim;
  p.nx = nx;
  p.ny = ndim == 3 ? ny : 1;
  p.nz = nz;
  return p;
}

// exact-size heap copy, so the sanitizer sees the end of the block
static double* exact(const std::vector<double>& v) {
  double* a = static_cast<double*>(std::malloc(v.size() * sizeof(double)));
  std::memcpy(a, v.data(), v.size() * sizeof(double));
  return a;
}

static void sizes() {
  size_t sb = 0, wb = 0;
  mtvd_params p = params(2, 256, 1, 64);
  CHECK(mtvd_state_bytes(&p, &sb, &wb) == MTVD_OK, "state_bytes 2D");
  CHECK(sb == 4u * 64u * 256u * 8u && wb > 0 && wb % 256 == 0, "2D sizes %zu %zu", sb, wb);
  p = params(3, 16, 8, 9);
  CHECK(mtvd_state_bytes(&p, &sb, &wb) == MTVD_OK && sb == 5u * 9u * 8u * 16u * 8u, "3D sizes");
  p = params(2, 256, 1, 4);
  CHECK(mtvd_state_bytes(&p, &sb, &wb) == MTVD_EINVAL, "nz=4 accepted");
  CHECK(mtvd_state_bytes(nullptr, &sb, &wb) == MTVD_EINVAL, "NULL params accepted");

  // batch: exact-size array of boxes
  std::vector<mtvd_params> boxes = {params(2, 64, 1, 16), params(2, 40, 1, 9),
                                    params(2, 300, 1, 33)};
  mtvd_params* bx = static_cast<mtvd_params*>(std::malloc(boxes.size() * sizeof(mtvd_params)));
  std::memcpy(bx, boxes.data(), boxes.size() * sizeof(mtvd_params));
  CHECK(mtvd_batch_bytes(bx, (int32_t)boxes.size(), &sb, &wb) == MTVD_OK, "batch_bytes");
  CHECK(sb >= (64u * 16u + 40u * 9u + 300u * 33u) * 4u * 8u, "batch state bytes %zu", sb);
  CHECK(mtvd_batch_bytes(bx, 0, &sb, &wb) != MTVD_OK, "empty batch accepted");
  bx[2].dt_mode = 1;
  CHECK(mtvd_batch_bytes(bx, (int32_t)boxes.size(), &sb, &wb) == MTVD_EINVAL,
        "mixed dt_mode accepted");
  bx[2].dt_mode = bx[0].dt_mode;
  bx[1].ndim = 3;
  CHECK(mtvd_batch_bytes(bx, (int32_t)boxes.size(), &sb, &wb) == MTVD_EINVAL,
        "3D box accepted");
  mtvd_batch* batch = nullptr;
  CHECK(mtvd_batch_create(bx, (int32_t)boxes.size(), nullptr, &batch) == MTVD_EINVAL && !batch,
        "3D box accepted by create");
  std::free(bx);

  // stretched grid: sizes (the metric table is part of the workspace) and
  // the heights into an exact-size array
  p = params(2, 64, 1, 33);
  p.stretch = 1.5;
  size_t wb0 = 0;
  mtvd_params pu = params(2, 64, 1, 33);
  CHECK(mtvd_state_bytes(&pu, &sb, &wb0) == MTVD_OK, "uniform sizes");
  CHECK(mtvd_state_bytes(&p, &sb, &wb) == MTVD_OK && wb >= wb0 + 33u * 8u * 8u,
        "stretched workspace %zu vs %zu", wb, wb0);
  double* z = static_cast<double*>(std::malloc(33 * sizeof(double)));
  CHECK(mtvd_grid_heights(&p, z, 33) == MTVD_OK && z[0] == 0.0 && z[32] == 1.0, "heights");
  for (int k = 0; k < 32; ++k) CHECK(z[k + 1] > z[k], "heights not increasing at %d", k);
  CHECK(mtvd_grid_heights(&p, z, 32) == MTVD_ESIZE, "short heights array accepted");
  std::free(z);
  p.stretch = -1.0;
  CHECK(mtvd_state_bytes(&p, &sb, &wb) == MTVD_EINVAL, "negative stretch accepted");

  // adjoint workspace
  p = params(2, 64, 1, 16);
  CHECK(mtvd_adj_bytes(&p, 20, 5, &wb) == MTVD_OK && wb > 0, "adj_bytes");
  CHECK(mtvd_adj_bytes(&p, 0, 5, &wb) != MTVD_OK, "adj nsteps=0 accepted");
  CHECK(mtvd_adj_bytes(&p, 20, 0, &wb) != MTVD_OK, "adj every=0 accepted");
}

static void validation() {
  struct Bad {
    const char* what;
    int code;
    void (*edit)(mtvd_params*);
  } bad[] = {
      {"ndim 4", MTVD_EINVAL, [](mtvd_params* p) { p->ndim = 4; }},
      {"nz 4", MTVD_EINVAL, [](mtvd_params* p) { p->nz = 4; }},
      {"nx 0", MTVD_EINVAL, [](mtvd_params* p) { p->nx = 0; }},
      {"gamma 1", MTVD_EINVAL, [](mtvd_params* p) { p->gamma = 1.0; }},
      {"Ra < 0", MTVD_EINVAL, [](mtvd_params* p) { p->Ra = -1.0; }},
      {"Ra NaN", MTVD_EINVAL, [](mtvd_params* p) { p->Ra = std::nan(""); }},
      {"eps + D > 1", MTVD_EINVAL, [](mtvd_params* p) { p->eps = 0.6; p->D = 0.5; }},
      {"limiter 2", MTVD_EINVAL, [](mtvd_params* p) { p->limiter_form = 2; }},
      {"wall 3", MTVD_EINVAL, [](mtvd_params* p) { p->wall_order = 3; }},
      {"ny 2 in 2D", MTVD_EINVAL, [](mtvd_params* p) { p->ny = 2; }},
      {"cfl 1.5", MTVD_ESTABILITY, [](mtvd_params* p) { p->cfl = 1.5; }},
      {"cfl 0", MTVD_ESTABILITY, [](mtvd_params* p) { p->cfl = 0.0; }},
      {"diffusion number", MTVD_ESTABILITY,
       [](mtvd_params* p) { p->Ra = 1.0; p->nx = 4096; p->nz = 1024; }},
  };
  for (const Bad& b : bad) {
    mtvd_params p = params(2, 256, 1, 64);
    b.edit(&p);
    mtvd_ctx* ctx = reinterpret_cast<mtvd_ctx*>(&p);  // must be overwritten with NULL
    int rc = mtvd_create(&p, nullptr, &ctx);
    CHECK(rc == b.code && ctx == nullptr, "create %s: rc %d", b.what, rc);
  }
  mtvd_params p = params(2, 256, 1, 64);
  CHECK(mtvd_create(&p, nullptr, nullptr) == MTVD_EINVAL, "create NULL out accepted");
  mtvd_ctx* ctx = nullptr;
  CHECK(mtvd_create(nullptr, nullptr, &ctx) == MTVD_EINVAL && !ctx, "create NULL params");
}

static void analysis(int ndim, int nx, int ny, int nz) {
  mtvd_params p = params(ndim, nx, ny, nz);
  const int nq = MTVD_NUM_PROFILES;
  std::vector<double> v((size_t)nq * nz);
  for (int q = 0; q < nq; ++q)
    for (int k = 0; k < nz; ++k) {
      const double z = (double)k / (nz - 1);
      double x = 0.01 * std::sin(3.0 * z + q);
      if (q == 0) x = 1.0 - (p.eps + p.D) * z;          // <T>_A
      if (q == 1) x = std::pow(1.0 - p.D * z, 2.5);     // <rho>_A
      if (q == 2 || q == 4 || q == 5) x = x * x + 1e-4;  // squares
      v[(size_t)q * nz + k] = x;
    }
  double* prof = exact(v);
  double* tsa = static_cast<double*>(std::malloc(nz * sizeof(double)));
  double* drho = static_cast<double*>(std::malloc(nz * sizeof(double)));
  double* U = static_cast<double*>(std::malloc(nz * sizeof(double)));
  mtvd_analysis a;
  CHECK(mtvd_analysis_from_profiles(&p, prof, v.size(), &a, tsa, drho, U) == MTVD_OK,
        "analysis %dD nz %d", ndim, nz);
  CHECK(std::isfinite(a.Re) && std::isfinite(a.C) && std::isfinite(a.Fv), "analysis values");
  CHECK(std::fabs(tsa[nz - 1] + p.eps) < 1e-12 && std::fabs(tsa[0]) < 1e-15, "T_sa ends");
  for (int k = 0; k < nz; ++k) CHECK(U[k] >= 0.0 && std::isfinite(drho[k]), "row %d", k);
  CHECK(mtvd_analysis_from_profiles(&p, prof, v.size(), &a, nullptr, nullptr, nullptr) ==
            MTVD_OK,
        "analysis without rows");
  CHECK(mtvd_analysis_from_profiles(&p, prof, v.size() - 1, &a, tsa, drho, U) == MTVD_ESIZE,
        "short profile accepted");
  CHECK(mtvd_analysis_from_profiles(&p, nullptr, v.size(), &a, tsa, drho, U) == MTVD_EINVAL,
        "NULL profile accepted");

  // boundary layers of the conduction-like profile with steep ends
  std::vector<double> t(nz);
  for (int k = 0; k < nz; ++k) {
    const double z = (double)k / (nz - 1);
    t[k] = 1.0 - p.D * z - 0.1 * (1.0 - std::exp(-z / 0.05)) + 0.05 * (1.0 - std::exp(-(1.0 - z) / 0.05));
  }
  double* tm = exact(t);
  double lb = 0.0, lt = 0.0;
  CHECK(mtvd_bl_thickness(tm, nz, p.D, 0.1, &lb, &lt) == MTVD_OK, "bl_thickness");
  CHECK((lb == -1.0 || (lb > 0.0 && lb < 1.0)) && (lt == -1.0 || (lt > 0.0 && lt < 1.0)),
        "bl values %g %g", lb, lt);
  CHECK(mtvd_bl_thickness(tm, 2, p.D, 0.1, &lb, &lt) == MTVD_EINVAL, "nz=2 accepted");
  CHECK(mtvd_bl_thickness(tm, nz, -1.0, 0.1, &lb, &lt) == MTVD_EINVAL, "D<0 accepted");
  CHECK(mtvd_bl_thickness(tm, nz, p.D, -0.1, &lb, &lt) == MTVD_EINVAL, "rtol<0 accepted");
  std::free(tm);
  std::free(U);
  std::free(drho);
  std::free(tsa);
  std::free(prof);
}

int main() {
  sizes();
  validation();
  analysis(2, 64, 1, 5);
  analysis(2, 256, 1, 64);
  analysis(3, 16, 12, 9);
  for (int code = 1; code >= -8; --code) {
    const char* s = mtvd_strerror(code);
    CHECK(s != nullptr && std::strlen(s) > 0, "strerror %d", code);
  }
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("host sanitize driver ok\n");
  return 0;
}
