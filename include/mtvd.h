/*
 * mtvd.h -- C ABI of the MI355X (gfx950) MacCormack-TVD library.
 *
 * One explicit time step of the nondimensional, fully compressible
 * Navier-Stokes equations of an ideal gas under gravity (density, momentum,
 * total energy) in a box with periodic side walls and no-slip isothermal
 * plates, as defined by Tiwari, Sharma & Verma, arXiv:2411.10372:
 *   - equations, p, E and tau_ij:       Sec. 2 (nondimensional equations);
 *   - conservative vector form, fluxes: Sec. 3.1 (vector_eqn, F_alpha, S_alpha);
 *   - split step:                       Sec. 3.1 (time_step);
 *   - predictor / corrector / TVD:      Sec. 3.1 (the three update formulas
 *                                        and the definitions of T, r, G, phi, C);
 *   - Nusselt numbers:                  Sec. 2 (volume_Nu, mean_Nu).
 * Every step runs in HIP kernels on the caller's stream; the host only
 * launches.  FP64 throughout.
 *
 * State layout ("canonical"): one array of nf * nz * ny * nx doubles,
 * X[f][k][j][i], i fastest, no padding, with fields
 *   2D (nf = 4): rho, rho u_x, rho u_z, E
 *   3D (nf = 5): rho, rho u_x, rho u_y, rho u_z, E.
 * x and y are periodic (dx = aspect/nx, dy = aspect/ny, no repeated end
 * point); z has nz nodes with the bottom plate at k = 0 and the top plate
 * at k = nz-1 (dz = 1/(nz-1)).
 *
 * Ownership: the caller allocates and owns the two state buffers and the
 * workspace (device memory, 256-byte aligned, at least the sizes that
 * mtvd_state_bytes reports) and the stream.  The library owns only the
 * context.  A context is bound to one stream, is not thread-safe, and
 * keeps no pointer to host memory after a call returns.
 *
 * Errors: every function returns MTVD_OK (0) or a negative MTVD_E* code and
 * never aborts.  Asynchronous device errors (non-finite values, rho <= 0,
 * T <= 0) are latched in the workspace and reported by the next
 * synchronising call (mtvd_diagnostics, mtvd_get_state, mtvd_sync).
 */
#ifndef MTVD_H
#define MTVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MTVD_OK = 0,
  MTVD_EINVAL = -1,      /* bad parameters or argument */
  MTVD_ESIZE = -2,       /* buffer too small or misaligned, count mismatch */
  MTVD_ESTABILITY = -3,  /* cfl outside (0, 1] or diffusion number > 1/2 */
  MTVD_ESTATE = -4,      /* call out of order (no buffers / no state yet) */
  MTVD_ENONFINITE = -5,  /* device flag: NaN/Inf, rho <= 0 or T <= 0 seen */
  MTVD_EHIP = -6         /* HIP runtime error; text in mtvd_last_error */
};

/* Problem parameters.  Defaults (mtvd_default_params): the 2D 256x64 box,
 * gamma 1.4, Pr 1, Ra 1e6, eps 0.1, D 0.4, cfl 0.5, noise 1e-3, and the
 * readings listed with each knob. */
typedef struct mtvd_params {
  int32_t ndim;          /* 2 or 3 */
  int32_t nx, ny, nz;    /* ny = 1 in 2D; nz >= 5 (plates included) */
  double aspect;         /* Gamma = L/d */
  double gamma, Pr, Ra, eps, D;   /* Sec. 2 parameters; plates T = 1, 1-eps-D */
  double cfl;            /* dt = cfl * min_nodes,a h_a/(|u_a| + c) */
  uint64_t seed;         /* SplitMix64 seed of the initial T noise */
  double noise_amp;      /* uniform +-noise_amp on interior T at init */
  int32_t dt_mode;       /* 0: dt from the state at every step;
                            1: dt frozen at its value for the state given by
                            mtvd_init_state / mtvd_set_state */
  double bulk_coef;      /* lambda in tau_ij = mu(d_j u_i + d_i u_j +
                            lambda d_m u_m delta_ij); -2/3 (Stokes) by
                            default, +2/3 is the sign as printed */
  int32_t limiter_form;  /* 0: G(r+_k + r-_{k+1}) as printed (default);
                            1: G(r+_k) + G(r-_{k+1}) (Davis) */
  int32_t sweep_order;   /* 0: L_x L_y L_z L_x L_y L_z as printed (default);
                            1: L_z L_y L_x L_x L_y L_z (symmetric) */
  int32_t tvd_on;        /* 1 (default); 0 drops the TVD term */
  double gravity_scale;  /* 1 (default); 0 switches gravity off */
  int32_t wall_order;    /* 2 (default): z-derivatives inside the plate
                            fluxes are second-order one-sided; 1: interior
                            first differences */
  double stretch;        /* z grid (Sec. 3.1: tangent-hyperbolic in z):
                            0 (default) uniform, z_k = k/(nz-1); s in
                            (0, 10]: z_k = (1 + tanh(s (2k - M)/M)/tanh s)/2,
                            M = nz-1, nodes crowded at both plates.  Every z
                            difference then divides by the same difference
                            of the heights, the flux differences of
                            predictor and corrector by the dual cell
                            w_k = (z_k+1 - z_k-1)/2 (half the face at a
                            plate), and the TVD term is the difference of
                            the face fluxes h_k+1/2 G dX over w_k with the
                            face's own Courant number; dt takes the
                            narrowest face of each node, the diagnostics
                            weigh rows by w_k, and the analysis profiles
                            take every z derivative on the node heights.
                            Single boxes, 2D and 3D (3D: nz <= 2048);
                            MTVD_EINVAL in batches and for the adjoint. */
  int32_t dt_rule;       /* time-step rule (Sec. 3.1 gives none):
                            0 (default): dt = cfl min over nodes and
                            directions of h_a/(|u_a| + c), and mtvd_create
                            rejects a box whose initial diffusion number
                            exceeds 1/2 (MTVD_ESTABILITY);
                            1: the minimum also runs over rho h^2 / kappa of
                            every node, h its smallest spacing (on a
                            stretched grid the narrower z face next to it),
                            kappa = max(mu (2 + |lambda|), K/c_v), so that
                            every operator L(dt/2) keeps its diffusion
                            number at most cfl/2, and no box is rejected for
                            it */
} mtvd_params;

/* Diagnostics of the current state (Sec. 2: mass, kinetic energy, total
 * energy; Nu_{z=0}, Nu_{z=1} and their mean from <T>_A on the three rows next
 * to each plate with second-order one-sided differences; bulk Nu = 1 +
 * Nu_conv + Nu_K as volume averages; trapezoid weights in z). */
typedef struct mtvd_diag {
  int64_t step;          /* steps taken since init/set_state (+ given base) */
  double time;           /* simulated time */
  double dt;             /* dt of the next step */
  double mass, kinetic, total_energy;
  double nu_bottom, nu_top, nu_mean, nu_bulk, nu_conv, nu_kin;
  double tmean[6];       /* <T>_A on rows 0, 1, 2, nz-3, nz-2, nz-1 */
  int32_t flags;         /* latched device flags (bit 0: non-finite or
                            non-positive rho/T seen) */
} mtvd_diag;

/* Snapshot scalars of the analysis of Secs. 4-6 (and Re of Sec. 2), made on
 * the host from the row means of mtvd_profiles; volume means <.>_V use the
 * trapezoid rule in z over a box of height 1. */
typedef struct mtvd_analysis {
  double Re;             /* sqrt(Ra/Pr) sqrt(<|u|^2>_V) (Sec. 2, Eq. Re) */
  double C;              /* <rho u_z T_sa>_V / sqrt(<(rho u_z)^2>_V <T_sa^2>_V),
                            0 when either factor is 0 (Sec. 6.2, C(Ra)) */
  double Fn, Fp, Fb, Fv; /* <F>_V of the z-momentum terms (Sec. 6.1) */
  double u2, rho_uz_Tsa, rho_uz2, Tsa2;   /* <.>_V of the inputs above */
} mtvd_analysis;

/* Rows of the mtvd_profiles output, in order. */
#define MTVD_NUM_PROFILES 10
/* 0 T  1 rho  2 |u|^2  3 rho u_z T_sa  4 (rho u_z)^2  5 T_sa^2
   6 F_n = rho (u . grad) u_z   7 F_p = -dp/dz   8 F_b = rho g
   9 F_v = d_i tau_iz                                               */

typedef struct mtvd_ctx mtvd_ctx;

void mtvd_default_params(mtvd_params* p);

/* Host only, no device work: the nz node heights z_k of the grid these
 * parameters define (uniform, or the tanh grid of `stretch`; Sec. 3.1) into
 * z[0..nz-1] (count >= nz).  MTVD_EINVAL on bad parameters, MTVD_ESIZE if
 * count is too small. */
int mtvd_grid_heights(const mtvd_params* p, double* z, size_t count);

/* Bytes of one state buffer and of the workspace for these parameters. */
int mtvd_state_bytes(const mtvd_params* p, size_t* state_bytes,
                     size_t* workspace_bytes);

/* Validate parameters and create a context on `hip_stream` (a hipStream_t,
 * NULL = default stream) of the current device.  No device work.
 * Returns MTVD_EINVAL / MTVD_ESTABILITY on bad parameters. */
int mtvd_create(const mtvd_params* p, void* hip_stream, mtvd_ctx** out);

/* Attach caller-owned device memory: two state buffers (ping-pong) and the
 * workspace.  The pointers must be distinct, 256-byte aligned and at least
 * the sizes of mtvd_state_bytes (MTVD_ESIZE otherwise).  Buffer contents
 * are not read. */
int mtvd_bind(mtvd_ctx* c, double* buf_a, double* buf_b, void* workspace);

/* Write the initial state (conductive T = 1 - (eps+D) z, hydrostatic
 * rho = T^(m-1) with m = gamma D/((gamma-1)(eps+D)), u = 0, SplitMix64 noise
 * on interior T) into buffer a and compute its dt.  Time and step are reset
 * to 0.  Asynchronous. */
int mtvd_init_state(mtvd_ctx* c);

/* Advance nsteps >= 0 time steps of the split scheme (Sec. 3.1, time_step):
 * 2D L_x L_z L_x L_z, 3D L_x L_y L_z L_x L_y L_z (rightmost first), each
 * L_a(dt/2) a fused predictor/corrector/TVD kernel.  Asynchronous: no host
 * synchronisation, dt never leaves the device. */
int mtvd_step(mtvd_ctx* c, int32_t nsteps);

/* Apply one directional operator L_axis(dt/2) (axis 0 = x, 1 = y, 2 = z)
 * with dt computed from the current state; time and step are unchanged.
 * For per-operator checks.  Asynchronous. */
int mtvd_sweep(mtvd_ctx* c, int32_t axis);

/* Compute the diagnostics of the current state; synchronises the stream.
 * Returns MTVD_ENONFINITE (and still fills *out) if a device flag is set. */
int mtvd_diagnostics(mtvd_ctx* c, mtvd_diag* out);

/* Row means <.>_A (over the nx x ny nodes of each row k) of the ten node
 * quantities listed with MTVD_NUM_PROFILES, for the analysis of Secs. 4-6
 * (profiles T_sa(z), rho - rho_A(z), U(z), the correlation C(Ra), the
 * z-momentum balance F_n, F_p, F_b, F_v) and Re (Sec. 2).  Derivatives:
 * central second order along x, y and inside; second-order one-sided on
 * the plates ((-3, 4, -1)/(2 dz), (3, -4, 1)/(2 dz); second derivatives
 * (2, -5, 4, -1)/dz^2); on a stretched grid the same stencils on the node
 * heights (first derivatives over the same stencil of z; second derivatives
 * by the three-point formula inside and the cubic through the plate and
 * its three neighbours on a plate); F_v = mu (lap u_z + (1 + lambda) d_z
 * div u); F_b = rho g with g = gravity_scale/eps; T_sa = T - (1 - D z).
 * out: host array of count >= MTVD_NUM_PROFILES * nz doubles, written
 * quantity-major (out[q * nz + k]).  Device work on the context's stream,
 * then synchronises.  MTVD_ESTATE without a state, MTVD_ESIZE if count is
 * too small, MTVD_ENONFINITE if the device flag is set. */
int mtvd_profiles(mtvd_ctx* c, double* out, size_t count);

/* Host only, no device work: the snapshot scalars of a profile array
 * (count >= MTVD_NUM_PROFILES * p->nz) and, into each non-NULL array of
 * p->nz doubles, T_sa(z) = <T>_A - (1 - D z), rho(z) - rho_A(z) with
 * rho_A = (1 - D z)^(1/(gamma-1)), and U(z) = sqrt(<|u|^2>_A) (Sec. 5), at
 * the node heights of the grid p defines (volume means weigh the rows by
 * their dual cells on a stretched grid).
 * MTVD_EINVAL on bad arguments, MTVD_ESIZE if count is too small. */
int mtvd_analysis_from_profiles(const mtvd_params* p, const double* prof, size_t count,
                                mtvd_analysis* out, double* tsa_z, double* drho_z,
                                double* U_z);

/* Host only: thermal boundary-layer thicknesses of a (time-averaged)
 * profile tmean[k] = <T>_A(z_k), z_k = k/(nz-1) (Sec. 5: where the slope of
 * <T>_A meets the adiabatic gradient -D).  With slopes taken between
 * neighbouring rows, *lam_b is the height where, going up from z = 0, the
 * slope first rises to -(1 + rtol) D (linear interpolation between the
 * midpoints; half a cell if the first one already has), *lam_t the same
 * from z = 1 down, measured from the top; -1 where it never does.
 * MTVD_EINVAL on bad arguments (nz < 3, D <= 0, rtol < 0). */
int mtvd_bl_thickness(const double* tmean, int32_t nz, double D, double rtol, double* lam_b,
                      double* lam_t);

/* Host only: the same on a profile sampled at the increasing node heights
 * z[0..nz-1] (e.g. mtvd_grid_heights of a stretched grid): slopes over the
 * row spacings, at the midpoints of the rows.  MTVD_EINVAL also if z is
 * not increasing. */
int mtvd_bl_thickness_grid(const double* tmean, const double* z, int32_t nz, double D,
                           double rtol, double* lam_b, double* lam_t);

/* Copy the current state to host memory in the canonical layout; count
 * must equal nf*nz*ny*nx.  Synchronises. */
int mtvd_get_state(mtvd_ctx* c, double* host, size_t count);

/* Replace the current state by a host array in the canonical layout, set
 * time and step, recompute dt (and the frozen dt when dt_mode = 1), clear
 * the device flags.  Synchronises. */
int mtvd_set_state(mtvd_ctx* c, const double* host, size_t count, double time,
                   int64_t step);

/* Which bound buffer (0 = a, 1 = b) holds the current state. */
int mtvd_current(const mtvd_ctx* c, int32_t* which);

/* Wait for the context's stream and report latched device flags. */
int mtvd_sync(mtvd_ctx* c);

/* Rows per wave along the march for the sweep kernels (0 = library
 * default).  It changes the launch shape only: results are identical bit
 * for bit for any value >= 1. */
int mtvd_set_tiling(mtvd_ctx* c, int32_t rows_x, int32_t rows_z);

/* Per-launch timing of the sweep kernels with HIP events recorded on the
 * context's stream around each launch (for benchmarks).  enable != 0 starts
 * recording, 0 stops it.  mtvd_kernel_times synchronises, adds the elapsed
 * milliseconds and launch counts of the recorded launches to ms[axis] and
 * counts[axis] (axis 0 = L_x, 1 = L_y, 2 = L_z) and forgets them. */
int mtvd_set_timing(mtvd_ctx* c, int32_t enable);
int mtvd_kernel_times(mtvd_ctx* c, double ms[3], int64_t counts[3]);

int mtvd_destroy(mtvd_ctx* c);

const char* mtvd_strerror(int status);
const char* mtvd_last_error(const mtvd_ctx* c);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * time steps of mtvd_set_state + mtvd_step without a context or a
 * workspace.  buf_a holds the state (canonical layout, device memory);
 * buf_b is the second buffer of the ping-pong; both caller-owned, distinct,
 * 256-byte aligned, state-sized.  The dt of the state in buf_a is computed
 * first (time 0), then nsteps >= 0 steps run on hip_stream (NULL = default
 * stream) exactly as mtvd_step runs them, same kernels and launch shapes,
 * so the result equals that path's bit for bit; *which (host) tells which
 * buffer holds it (0 = a, 1 = b).  Asynchronous: no host synchronisation,
 * no allocation of any kind.  The scratch the steps need (the shared dt
 * maxima, time and flags, and the row heights) is a static device array of
 * MTVD_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends and
 * shared by every call on that GPU: it is cleared at the start of each
 * call, and calls that overlap on one GPU (other streams, other threads)
 * race.  Limits: uniform z grids (stretch = 0; MTVD_EINVAL otherwise) and
 * nz <= MTVD_NOALLOC_MAX_NZ (MTVD_ESIZE otherwise); other parameter errors
 * as mtvd_create.  Device flags (non-finite or non-positive values) are
 * not reported by this call.  MTVD_EHIP on a launch failure. */
#define MTVD_NOALLOC_MAX_NZ 8192
#define MTVD_NOALLOC_SCRATCH_BYTES (1280 + 8 * MTVD_NOALLOC_MAX_NZ)
int mtvd_step_noalloc(const mtvd_params* p, double* buf_a, double* buf_b, int32_t nsteps,
                      void* hip_stream, int32_t* which);

/* ---------------------------------------------------------------------------
 * Batches: many independent 2D boxes (each with its own grid, Ra, Pr, seed,
 * dt and time) advanced together.  Each directional operator of a step is
 * ONE launch covering every box (a device work list of (box, column strip,
 * row chunk) items); the launches of two steps are captured once into a
 * HIP graph and replayed, so a step costs one graph launch per two steps.
 * All boxes must be 2D and share dt_mode and sweep_order.  State buffers
 * hold the boxes one after another, each in the canonical layout, each
 * starting on a 256-byte boundary (mtvd_batch_offset gives the place).
 */
typedef struct mtvd_batch mtvd_batch;

int mtvd_batch_bytes(const mtvd_params* boxes, int32_t nbox, size_t* state_bytes,
                     size_t* workspace_bytes);
int mtvd_batch_create(const mtvd_params* boxes, int32_t nbox, void* hip_stream,
                      mtvd_batch** out);
/* Two state buffers (state_bytes each) and the workspace, as mtvd_bind. */
int mtvd_batch_bind(mtvd_batch* b, double* buf_a, double* buf_b, void* workspace);
/* Offset (in doubles) of box `box` inside a state buffer. */
int mtvd_batch_offset(const mtvd_batch* b, int32_t box, size_t* offset);
int mtvd_batch_init_state(mtvd_batch* b);
/* nsteps time steps of every box; pairs of steps replay the captured graph.
 * Asynchronous. */
int mtvd_batch_step(mtvd_batch* b, int32_t nsteps);
/* Diagnostics of one box (synchronises); see mtvd_diagnostics. */
int mtvd_batch_diagnostics(mtvd_batch* b, int32_t box, mtvd_diag* out);
int mtvd_batch_get_state(mtvd_batch* b, int32_t box, double* host, size_t count);
int mtvd_batch_set_state(mtvd_batch* b, int32_t box, const double* host, size_t count,
                         double time, int64_t step);
int mtvd_batch_current(const mtvd_batch* b, int32_t* which);
/* Rows per wave of one box's operators (0 = library default: for each
 * operator the smallest bound k >= 4 with which the whole launch -- every
 * box's column strips times its chunks of at most k rows -- fits the
 * device's resident waves in one round, each box's rows split into equal
 * chunks of at most k).  Results do not depend on it. */
int mtvd_batch_set_tiling(mtvd_batch* b, int32_t box, int32_t rows_x, int32_t rows_z);
/* Time trial steps of the whole batch for each distinct box size over the
 * candidate rows per wave (the default's and 4, 8, 16, 32, 64) for L_z and
 * then L_x, keep the fastest for every box of that size, and restore the
 * state, time and dt afterwards.
 * `scratch` is caller-owned device memory of at least state_bytes +
 * 2048 * nbox bytes.  Synchronises. */
int mtvd_batch_autotune(mtvd_batch* b, void* scratch, int32_t trial_steps);
int mtvd_batch_get_tiling(const mtvd_batch* b, int32_t box, int32_t* rows_x,
                          int32_t* rows_z);
int mtvd_batch_destroy(mtvd_batch* b);
const char* mtvd_batch_last_error(const mtvd_batch* b);

/* ---------------------------------------------------------------------------
 * Adjoint (reverse mode) of the time-averaged mean Nusselt number of a 2D
 * box with a frozen dt:
 *
 *   J(theta, Ra) = (1/N) sum_{n=1..N} Nu_mean(X_n),   X_n = S^n(X_0),
 *
 * with Nu_mean = (Nu(z=0) + Nu(z=1))/2 of the plates (Sec. 2, mean_Nu, from
 * the row means of T by one-sided second-order differences), S one step of
 * Sec. 3.1 (time_step) with the same dt for every step, and X_0(theta) the
 * conduction state of mtvd_init_state with T = T0 + theta on interior rows
 * (no noise).  Ra enters through mu = sqrt(Pr/Ra) and K = 1/(eps D
 * sqrt(Ra Pr)); dt and the initial density do not depend on theta or Ra.
 * The reverse of each directional operator is hand-written stage by stage;
 * at a kink of max/min/abs/phi it takes the branch the forward pass took.
 * Memory: checkpoints every `every` steps; for two intervals the operator
 * inputs (2 x 4 every states: the backward pass recomputes the next
 * interval on a second stream of its own, default priority, while it
 * reverses the current one); the forward values of two operators (2 x 13
 * doubles per node); two cotangent states and the mu and K accumulators
 * (mtvd_adj_bytes gives the total).
 * Restrictions: ndim = 2 and limiter_form = 0 (MTVD_EINVAL otherwise);
 * dt_mode is ignored (dt is always frozen).
 */
typedef struct mtvd_adj mtvd_adj;

/* Workspace bytes for N = nsteps >= 1 steps and checkpoints every
 * `every` >= 1 steps (clamped to nsteps). */
int mtvd_adj_bytes(const mtvd_params* p, int32_t nsteps, int32_t every,
                   size_t* workspace_bytes);
/* Validate and create (no device work; creates the second stream and its
 * events on the current device, MTVD_EHIP if that fails); stream as
 * mtvd_create. */
int mtvd_adj_create(const mtvd_params* p, int32_t nsteps, int32_t every, void* hip_stream,
                    mtvd_adj** out);
/* Attach a caller-owned, 256-byte aligned device workspace of at least
 * mtvd_adj_bytes bytes.  The workspace holds the checkpoints between
 * forward and backward. */
int mtvd_adj_bind(mtvd_adj* a, void* workspace);
/* Forward pass: X_0 from theta (device, nz*nx doubles in the canonical
 * node order; plate rows ignored; NULL = zero perturbation), N steps with
 * dt (> 0: that dt; 0: the CFL dt of X_0), J and the dt used to the host
 * (either pointer may be NULL).  Synchronises.  MTVD_ENONFINITE if J is not
 * finite. */
int mtvd_adj_forward(mtvd_adj* a, const double* theta, double dt, double* J, double* dt_used);
/* Backward pass of the latest forward pass for the cotangent Jbar: writes
 * Jbar dJ/dX_0 (device, 4 nz nx doubles, canonical layout), Jbar dJ/dtheta
 * (device, nz nx doubles, 0 on the plate rows) and Jbar dJ/dRa (host); any
 * of the three may be NULL.  May be called again for the same forward pass.
 * Synchronises. */
int mtvd_adj_backward(mtvd_adj* a, double Jbar, double* grad_x0, double* grad_theta,
                      double* grad_ra);
/* Jbar dJ/d(mu) and Jbar dJ/d(K) of the latest backward pass (host), mu and
 * K the viscosity and conductivity coefficients; d/dRa is made of these two
 * parts, d(mu)/dRa = -mu/(2 Ra) and d(K)/dRa = -K/(2 Ra).  MTVD_ESTATE before
 * a backward pass. */
int mtvd_adj_coef_grads(const mtvd_adj* a, double* grad_mu, double* grad_K);
int mtvd_adj_destroy(mtvd_adj* a);
const char* mtvd_adj_last_error(const mtvd_adj* a);

#ifdef __cplusplus
}
#endif
#endif
