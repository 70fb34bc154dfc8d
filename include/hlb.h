/*
 * hlb.h -- C ABI of the MI355X (gfx950) library for the hybrid free-energy
 * lattice Boltzmann method of Tiribocchi, Stella, Gonnella and Lamura,
 * "Hybrid lattice Boltzmann model for binary fluid mixtures"
 * (arXiv:0902.3921).
 *
 * One timestep t -> t+1 of a periodic lattice (D2Q9, or the D3Q19
 * three-dimensional generalisation) computes, from the state (f_t, phi_t):
 *   1. the force density F = -phi grad(mu), mu = a phi + b phi^3 - kappa lap phi
 *      (Sec. 2, Eqs. chempot and forza), with the derivatives taken by the
 *      3x3 stencils of Sec. 2.2 (Eqs. xstencil and laplstencil), parameters
 *      N and Q; by default in the expanded form
 *      F = -[(a phi + 3 b phi^3) grad phi - kappa phi grad(lap phi)] that the
 *      paper analyses in Sec. 3;
 *   2. the density n = sum f_i and the physical velocity
 *      n u* = sum f_i e_i + F/2 (Sec. 2.1, Eq. newvel);
 *   3. the BGK collision with the equilibrium of Eq. espdistrfunc at u* and
 *      the lattice forcing term of Eq. latticeforceterm, then streaming
 *      (Eq. forceevoleqn);
 *   4. m explicit finite-difference substeps of the convection-diffusion
 *      equation with Delta t_FD = Delta t_LB / m and u*_t held fixed: the
 *      advection half-step of Eqs. adv, centrdiff, backdiff and fordiff, then
 *      the diffusion step of Eq. diff (Sec. 2.3).
 *
 * Conventions shared by every entry point
 *   - Lattice units: Delta x = Delta t_LB = 1, c_s^2 = 1/3.
 *   - Sites are indexed idx = x + nx*(y + ny*z), x fastest; nz = 1 for D2Q9.
 *   - Host field arrays are double precision.  A scalar field holds ns =
 *     nx*ny*nz values; a vector field holds d*ns values, component-major
 *     ([component][idx]); populations hold q*ns values ([i][idx]).
 *   - Velocity order.  D2Q9: 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1)
 *     5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1).  D3Q19: 0:(0,0,0)
 *     1:(1,0,0) 2:(-1,0,0) 3:(0,1,0) 4:(0,-1,0) 5:(0,0,1) 6:(0,0,-1)
 *     7:(1,1,0) 8:(-1,-1,0) 9:(1,-1,0) 10:(-1,1,0) 11:(1,0,1) 12:(-1,0,-1)
 *     13:(1,0,-1) 14:(-1,0,1) 15:(0,1,1) 16:(0,-1,-1) 17:(0,1,-1) 18:(0,-1,1).
 *   - Populations are stored on the device as deviations g_i = f_i - w_i rho0
 *     in double (HLB_F64) or float (HLB_F32_SHIFTED) precision.
 *   - Device memory: the caller owns one workspace allocation of at least
 *     hlb_workspace_size() bytes, 256-byte aligned, that outlives the context.
 *     The library carves every device array out of it and allocates nothing.
 *   - Streams: all device work of a context is enqueued on the caller's HIP
 *     stream given at creation (a hipStream_t passed as void*, NULL for the
 *     default stream).  hlb_step returns without synchronising; calls that
 *     return host data synchronise the stream before returning.
 *   - Errors: every call returns an hlb_status and never aborts.
 *     hlb_last_error() describes the last failure of a context.  Argument
 *     checks happen on the host before any device work.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef HLB_H
#define HLB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hlb_ctx hlb_ctx;

typedef enum {
  HLB_OK = 0,
  HLB_EINVAL = -1,      /* invalid argument or parameter */
  HLB_ESHAPE = -2,      /* lattice size out of range, or workspace too small */
  HLB_EUNSTABLE = -3,   /* parameters violate the explicit-stability bound, or max|u*| >= c_s/2 */
  HLB_ENONFINITE = -4,  /* a non-finite value in the inputs or the state */
  HLB_EHIP = -5,        /* a HIP runtime call failed */
  HLB_ESTATE = -6       /* the context is in an error state (after HLB_ENONFINITE) */
} hlb_status;

typedef enum { HLB_D2Q9 = 0, HLB_D3Q19 = 1 } hlb_lattice;

typedef enum { HLB_F64 = 0, HLB_F32_SHIFTED = 1 } hlb_storage;

/* Model parameters (lattice units). */
typedef struct {
  double a, b, kappa;  /* free energy, Sec. 2 Eq. freenergy; b > 0, kappa >= 0 */
  double tau;          /* BGK relaxation time, Sec. 2.1 Eq. evoleqn; tau > 1/2 */
  double gamma;        /* mobility Gamma, Sec. 2 Eq. convdiffeqn; >= 0 */
  double N, Q;         /* force stencils, Sec. 2.2: 2D M = (1-2N)/4, R = (1-Q)/2;
                          3D M = (1-2N)/8, R = (1-Q)/4 (edge weights) */
  double cd_Q;         /* Laplacian parameter of the convection-diffusion step;
                          1 = the standard 5/7-point operator of Sec. 2.3 */
  int fd_substeps;     /* m = Delta t_LB / Delta t_FD (Sec. 2.3); 0 = the smallest m
                          with Gamma dt (kappa s^2 + a_eff s) <= 1.8, s the largest
                          |symbol| of the CH Laplacian, a_eff = -2a (a < 0) or
                          a + 3b (a >= 0) */
  int force_form;      /* 1 = expanded form (default), 0 = -phi grad_D(mu) */
  int advection;       /* 0 = the paper's non-conservative upwind step (default),
                          1 = conservative upwind face fluxes */
  int cd_model;        /* how phi is advanced: 0 = the finite differences of
                          Sec. 2.3 (default); 1 = the D2Q5 lattice Boltzmann
                          alternative that Sec. 2 names (D2Q9 contexts only):
                          populations h_i on c_0 = 0 and the four axis vectors,
                          weights 1/3 and 1/6, h_i^eq = w_i (Gamma_h mu +
                          phi c_i.u*) / c_s^2 (i > 0), h_0^eq = phi - sum of
                          the others, relaxation 1/tau_phi, Gamma_h =
                          Gamma / (tau_phi - 1/2), mu with the cd_Q Laplacian;
                          phi = sum h_i.  No substeps (fd_substeps 0 or 1), so
                          Gamma (kappa s^2 + a_eff s) <= 2 is required
                          (HLB_EUNSTABLE otherwise).  Fixed at creation: it sets
                          the workspace layout (hlb_workspace_size_params) */
  double g_ext[3];     /* uniform body acceleration: n*g_ext is added to F (Sec. 3) */
  double rho0;         /* reference density of the stored deviations; > 0 */
  double tau_phi;      /* relaxation time of the D2Q5 populations (cd_model 1);
                          0 = the smallest value >= 1 with Gamma_h (a_eff + kappa s)
                          <= 0.45, else > 1/2 */
} hlb_params;

/* Global diagnostics at the current time (all sums in double precision,
 * fixed summation order, so repeated calls give identical results). */
typedef struct {
  double mass;      /* sum n */
  double phi_sum;   /* sum phi */
  double kinetic;   /* sum n |u*|^2 / 2 */
  double umax;      /* max |u*| */
  double mom[3];    /* sum n u* */
  long long step;   /* timesteps taken since hlb_init_fields / hlb_set_state */
  int finite;       /* 1 if every population and phi is finite */
  int reserved;
} hlb_stats;

/* Fills p with a = -0.1, b = 0.1, kappa = 0.1, tau = 1, Gamma = 1, the paper's
 * optimal stencil N = 0.3, Q = 2.5 (Sec. 3, Table I), cd_Q = 1, m = 0
 * (automatic), expanded force, paper advection, the finite-difference
 * convection-diffusion model, g_ext = 0, rho0 = 1, tau_phi = 0. */
hlb_status hlb_params_default(hlb_params *p);

/* Checks p for lattice `lattice` without touching the device and writes the
 * number of convection-diffusion substeps m that a context would use.
 * Returns HLB_EINVAL for invalid values, HLB_EUNSTABLE if an explicit m
 * violates Gamma dt (kappa s^2 + a_eff s) <= 2. */
hlb_status hlb_check_params(int lattice, const hlb_params *p, int *m_out);

/* Bytes of device workspace a context of this lattice, storage and size
 * needs.  Sizes must be >= 1 (nz == 1 for D2Q9) with nx*ny*nz < 2^31;
 * otherwise HLB_ESHAPE.  Host only. */
hlb_status hlb_workspace_size(int lattice, int storage, int nx, int ny, int nz, size_t *bytes);

/* The same for a context created with parameters p (NULL: the defaults):
 * the D2Q5 convection-diffusion model (cd_model 1) adds two buffers of its
 * five populations.  Host only. */
hlb_status hlb_workspace_size_params(int lattice, int storage, int nx, int ny, int nz, const hlb_params *p,
                                     size_t *bytes);

/* Creates a context on the current HIP device.  `workspace` is a device
 * pointer to `bytes` bytes (>= hlb_workspace_size_params), `stream` a hipStream_t
 * or NULL.  The state is undefined until hlb_init_fields or hlb_set_state.
 * On failure *out is NULL. */
hlb_status hlb_create(hlb_ctx **out, int lattice, int storage, int nx, int ny, int nz,
                      const hlb_params *p, void *workspace, size_t bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): creates a
 * context exactly like hlb_create, but its workspace is a static device
 * array of the library of HLB_NOALLOC_MAX_BYTES bytes instead of caller
 * memory.  Allocates no device memory; each GPU the library runs on holds
 * its own array from the first call on it until the process ends.
 * Lattices whose hlb_workspace_size exceeds HLB_NOALLOC_MAX_BYTES (64 MiB:
 * e.g. D2Q9 up to 512 x 512 in float storage or 256 x 256 in double, D3Q19
 * up to 64^3 in float) are rejected with HLB_ESHAPE.  One such context per
 * device at a time: while one is alive, another hlb_create_noalloc on the
 * same device returns HLB_ESTATE; hlb_destroy frees the array again.  The
 * array keeps the last context's contents, which the next context never
 * reads before writing (initialise it with hlb_init_fields, hlb_set_state
 * or hlb_load).  Calls from several threads that overlap on one device's
 * array race, like any use of one context from several threads.  The
 * other calls of the context are the ones above, unchanged. */
#define HLB_NOALLOC_MAX_BYTES (64u << 20)
hlb_status hlb_create_noalloc(hlb_ctx **out, int lattice, int storage, int nx, int ny, int nz,
                              const hlb_params *p, void *stream);

/* Replaces the parameters between steps (revalidated as hlb_check_params). */
hlb_status hlb_set_params(hlb_ctx *ctx, const hlb_params *p);

/* Reads the parameters and the resolved m. */
hlb_status hlb_get_params(const hlb_ctx *ctx, hlb_params *p, int *m_out);

/* Sets phi and f_i = f_i^eq(n, u) (Eq. espdistrfunc) at every site from host
 * arrays phi[ns], n[ns], u[d*ns]; n or u may be NULL for n = 1, u = 0.
 * Resets the step counter.  HLB_ENONFINITE if any input is not finite or
 * n <= 0.  Synchronises the stream. */
hlb_status hlb_init_fields(hlb_ctx *ctx, const double *phi, const double *n, const double *u);

/* Sets the raw state: populations f[q*ns] (after streaming, before the
 * collision of the next step) and phi[ns], host double arrays.  Resets the
 * step counter.  Synchronises.  HLB_EINVAL with the D2Q5 model, whose state
 * also holds its populations (use hlb_init_fields or hlb_load). */
hlb_status hlb_set_state(hlb_ctx *ctx, const double *f, const double *phi);

/* Reads the raw state into host arrays f[q*ns] and phi[ns] (either may be
 * NULL).  Synchronises. */
hlb_status hlb_get_state(hlb_ctx *ctx, double *f, double *phi);

/* Enqueues nsteps >= 0 timesteps on the context's stream and returns. */
hlb_status hlb_step(hlb_ctx *ctx, long long nsteps);

/* Reads the fields at the current time into host arrays (any may be NULL):
 * n[ns] = sum f_i, u[d*ns] = u* of Eq. newvel, phi[ns], and mu[ns] =
 * a phi + b phi^3 - kappa lap_D phi with the force stencil (Eq. chempot).
 * Synchronises. */
hlb_status hlb_get_fields(hlb_ctx *ctx, double *n, double *u, double *phi, double *mu);

/* Computes the global diagnostics on the device and copies them to *out.
 * Returns HLB_ENONFINITE (and puts the context in the error state) if the
 * state holds a non-finite value, HLB_EUNSTABLE if max|u*| >= c_s/2 (the
 * low-Mach condition of Sec. 2.1); *out is filled in both cases.
 * Synchronises. */
hlb_status hlb_reduce(hlb_ctx *ctx, hlb_stats *out);

/* Bulk quantities of a drop for Laplace's law, Delta p = sigma / R in 2D and
 * 2 sigma / R in 3D, with sigma of Sec. 2, Eq. surftens.  Over the sites
 * whose minimum-image distance from centre (x, y[, z]; centre[2] is ignored
 * for D2Q9) is below r_in ("in") or above r_out ("out"), the means of the
 * bulk pressure of Eq. diagpress without its gradient terms,
 * p0 = n c_s^2 + a phi^2 / 2 + 3 b phi^4 / 4, of phi and of n = sum f_i;
 * dp = p_in - p_out; the sum of phi; and the equimolar radius: the volume
 * V = (sum phi - phi_out ns) / (phi_in - phi_out) of the phase of phi_in,
 * R = sqrt(V / pi) (2D) or (3 V / (4 pi))^(1/3) (3D).  Sums in double
 * precision on the device in a fixed order.  HLB_EINVAL unless
 * 0 <= r_in <= r_out and both regions hold a site.  Synchronises. */
typedef struct {
  double p_in, phi_in, n_in;
  double p_out, phi_out, n_out;
  double dp, phi_sum, radius;
  long long count_in, count_out;
} hlb_drop;
hlb_status hlb_drop_stats(hlb_ctx *ctx, const double centre[3], double r_in, double r_out, hlb_drop *out);

/* Runs nsteps timesteps like hlb_step, recording HIP events around every
 * kernel launch on the context's stream, synchronises, and writes the
 * summed kernel time in milliseconds per kernel class:
 *   ms[0] = force + collide-and-stream kernel, ms[1] = convection-diffusion
 *   kernels.  Intended for benchmarks; slower than hlb_step. */
hlb_status hlb_step_timed(hlb_ctx *ctx, long long nsteps, double ms[2]);

/* Execution plan of the convection-diffusion substeps (a performance
 * choice; every plan computes the same values up to rounding order):
 *   plan[0] kind: 0 = one tiled launch per substep (any lattice, any cd_Q);
 *                 1 = marching launches: in D2Q9 (cd_Q = 1 only) a launch
 *                     marches along y and runs plan[1] substeps; in D3Q19
 *                     (any cd_Q) a launch marches along z and runs one
 *                     substep;
 *                 2 = fused tiles (D2Q9, any cd_Q): a launch runs plan[1]
 *                     substeps (1, 2, 3 or 5) of plan[2] x plan[2] tiles
 *                     (16, 32, 48 or 64) in LDS, halo 3 per substep, when the
 *                     staged tile fits a CU's 160 KiB of LDS;
 *                 3 = fused tiles like kind 2 (edge 32, 48 or 64, plan[3]
 *                     = 512 or 1024 threads, 0 = 1024) in which every thread
 *                     keeps the same staged vectors in registers for the
 *                     whole launch (at most 3 per thread) and each site's
 *                     advection half-step is precomputed as five
 *                     coefficients;
 *   plan[1] fuse: substeps per launch, 1..5 (D2Q9), 1 (D3Q19);
 *   plan[2] bw:   D2Q9: columns per block, 64, 128 or 256 (256 with
 *                 HLB_F32_SHIFTED only), bw - 6*fuse >= 16;
 *                 D3Q19: threads per block, each owning two (x, y)
 *                 columns: 256 (16x32 columns), 512 (32x32) or 1024 (64x32,
 *                 HLB_F32_SHIFTED and cd_Q = 1 only);
 *   plan[3] seg:  kind 1: rows (D2Q9) or planes (D3Q19) per block, >= 1;
 *                 kind 2: threads per block, 256, 512 or 1024 (0 = 256);
 *                 kind 3: 512 or 1024 (0 = 1024).
 * hlb_create picks a plan from the lattice size; hlb_set_plan overrides it
 * (HLB_EINVAL if the plan cannot run this context).  hlb_set_params keeps a
 * user plan while it stays valid. */
hlb_status hlb_set_plan(hlb_ctx *ctx, const int plan[4]);
hlb_status hlb_get_plan(const hlb_ctx *ctx, int plan[4]);

/* Times the candidate plans on the current state, keeps the fastest and
 * writes its time per substep in microseconds to *best_us (may be NULL).
 * Each candidate runs as in a step: a collide-and-stream launch (which writes
 * the spare population buffer and u* of the current state), then all the
 * convection-diffusion substeps of a step from the current phi into scratch
 * buffers in the staging area; the collide-and-stream time is subtracted.
 * The state is unchanged.  Synchronises. */
hlb_status hlb_autotune(hlb_ctx *ctx, double *best_us);

/* Name of a device kernel as profiler traces print it (the full template
 * instantiation, without "void" and the argument list), for the context's
 * lattice, storage, parameters and plan: kernel_class 0 is the force +
 * collide-and-stream kernel, 1 the kernel of the first convection-diffusion
 * launch of a step (a fused plan may end a step with a launch of fewer
 * substeps, which is another instantiation).  The string is owned by the
 * context and valid until its next call; "" for an invalid argument. */
const char *hlb_kernel_name(const hlb_ctx *ctx, int kernel_class);

/* Average device time of the step's kernels, in microseconds, each measured
 * with one pair of HIP events around `reps` >= 1 repetitions on the
 * context's stream (after one untimed repetition of each):
 *   us[0] = one force + collide-and-stream launch (kernel class 0),
 *           repeated back to back;
 *   us[1] = the first convection-diffusion launch of a step (class 1),
 *           repeated back to back;
 *   us[2] = all convection-diffusion launches of one step, back to back;
 *   us[3] = all convection-diffusion launches of one step when each follows
 *           a collide-and-stream launch, as in a step: the time of `reps`
 *           such pairs minus that of us[0]'s launches.  Back-to-back
 *           launches of a kernel whose inputs fit the caches read them
 *           from there; us[3] includes the refetch after the
 *           collide-and-stream launch has streamed the populations.
 * The collide-and-stream launches read the current state and write only the
 * spare population buffer and u* (which then holds the current state's u*);
 * the substep launches read phi and u* and write scratch buffers in the
 * staging area.  The state and the step counter are unchanged.  For
 * benchmarks and profiles.  Synchronises. */
hlb_status hlb_time_kernels(hlb_ctx *ctx, int reps, double us[4]);

/* Checkpoints.  A timestep depends only on (f_t, phi_t) and the parameters
 * (Sec. 2: the force, u*, the collision and the substeps are all computed
 * from the state at time t), so a checkpoint holds a header (lattice,
 * storage, size, step counter, hlb_params, and the substep plan, because
 * plans agree only up to rounding order) and the state in its device
 * representation (populations as stored, then phi), and a run resumed in any
 * context of the same lattice, storage and size is bit-identical to an
 * uninterrupted one.
 *
 * hlb_checkpoint_size: bytes of a checkpoint of this context.
 * hlb_save: writes the checkpoint into the caller's host buffer (at least
 *   hlb_checkpoint_size bytes; HLB_EINVAL otherwise).  HLB_ESTATE after a
 *   non-finite state.  Synchronises.
 * hlb_load: restores a checkpoint of a context with the same lattice,
 *   storage and size (HLB_ESHAPE otherwise; HLB_EINVAL for a buffer that is
 *   not a checkpoint or is truncated), including the step counter, the
 *   parameters and the plan, and clears the error state.  Synchronises. */
hlb_status hlb_checkpoint_size(const hlb_ctx *ctx, size_t *bytes);
hlb_status hlb_save(hlb_ctx *ctx, void *host, size_t bytes);
hlb_status hlb_load(hlb_ctx *ctx, const void *host, size_t bytes);

/* Message of the context's last failure ("" if none); owned by the context,
 * valid until its next call.  ctx may be NULL for failures of hlb_create. */
const char *hlb_last_error(const hlb_ctx *ctx);

/* Destroys the context.  Does not free the workspace. */
hlb_status hlb_destroy(hlb_ctx *ctx);

/* Library version string. */
const char *hlb_version(void);

/* ------------------------------------------------------------------------
 * Batches of independent D2Q9 simulations.
 *
 * A batch advances nsim independent periodic D2Q9 simulations together, each
 * with its own lattice size nx[b] x ny[b] and its own hlb_params (so its own
 * tau, stencil weights N, Q, cd_Q, free-energy parameters, force form,
 * body force and number of substeps m_b).  Every simulation computes exactly
 * the timestep described at the top of this file (Sec. 2); the batch only
 * shares launches: a step is one force + collide-and-stream launch over the
 * tiles of all simulations, then max_b(m_b) substep launches, in which a
 * simulation that has done its m_b substeps copies phi through.  The
 * parameter sweeps of Sec. 3 (tau and the stencil pairs of Table I, the drop
 * radii of the Laplace test) are the intended use: many small lattices that
 * would each leave most of the device idle.
 *
 * Device storage: one caller-owned workspace of hlb_batch_workspace_size()
 * bytes (256-byte aligned) holds every simulation's arrays plus the tile
 * tables; nothing is allocated.  Steps are replayed from a HIP graph of two
 * steps built on the first call (the graph objects are host-side).  The
 * batch is not thread-safe.  Errors follow the conventions above;
 * hlb_batch_last_error(NULL) reports failures of hlb_batch_create.
 * ---------------------------------------------------------------------- */
typedef struct hlb_batch hlb_batch;

/* Bytes of device workspace for a batch of nsim simulations of sizes
 * nx[b] x ny[b] (host arrays of nsim ints).  HLB_ESHAPE if a size is < 1 or
 * nx*ny >= 2^31; HLB_EINVAL for nsim < 1 or NULL arguments. */
hlb_status hlb_batch_workspace_size(int storage, int nsim, const int *nx, const int *ny, size_t *bytes);

/* Creates a batch.  params: host array of nsim parameter sets, each checked
 * as by hlb_check_params (fd_substeps 0 selects m_b automatically).  The
 * workspace and stream follow the single-simulation conventions.  Copies the
 * per-simulation descriptors and tile tables to the device and synchronises.
 * Every simulation starts uninitialised: call hlb_batch_init_fields for each
 * before stepping. */
hlb_status hlb_batch_create(hlb_batch **out, int storage, int nsim, const int *nx, const int *ny,
                            const hlb_params *params, void *workspace, size_t bytes, void *stream);

/* Number of simulations, the largest m_b and (m_out, may be NULL, nsim ints)
 * the substeps of every simulation. */
hlb_status hlb_batch_info(const hlb_batch *b, int *nsim, int *max_m, int *m_out);

/* Equilibrium initial state of simulation sim, as hlb_init_fields: phi
 * (ns doubles), n (ns doubles, NULL = 1) and u (2*ns doubles, NULL = 0).
 * Does not change the batch step counter.  Synchronises. */
hlb_status hlb_batch_init_fields(hlb_batch *b, int sim, const double *phi, const double *n, const double *u);

/* Advances every simulation of the batch by nsteps timesteps.  Enqueues
 * work on the stream and returns without synchronising. */
hlb_status hlb_batch_step(hlb_batch *b, long long nsteps);

/* As hlb_batch_step, launched directly (no graph) with HIP events around
 * the kernels of each step: ms[0] receives the total milliseconds of the
 * collide-and-stream launches, ms[1] those of the substep launches.
 * Synchronises. */
hlb_status hlb_batch_step_timed(hlb_batch *b, long long nsteps, double ms[2]);

/* Tile shapes of the batch's launches.  plan[0] indexes the
 * collide-and-stream tiles {64x8, 32x8, 64x4, 32x16} (x by y sites).
 * plan[1] indexes the substep launches (Sec. 2.3's substeps):
 *   0-3   one substep per launch on tiles {64x8, 32x8, 64x16, 32x16};
 *   4     2 substeps fused in LDS on 32x32 tiles (HLB_F32_SHIFTED) or
 *         16x16 tiles (HLB_F64);
 *   5-11  a march along y of blocks of (columns, rows per segment) fusing
 *         f substeps, (f, columns, rows) = (1, 64, 32), (1, 64, 64),
 *         (1, 128, 32), (1, 128, 64), (1, 256, 32), (2, 128, 32),
 *         (2, 128, 64); the march needs cd_Q = 1 in every simulation (else
 *         HLB_EINVAL).
 * A step has ceil(max_b m_b / f) substep launches (f = 1 for 0-3); a
 * simulation with fewer substeps left than f in its last launch does only
 * those.  HLB_EINVAL out of range.  The state is kept.  Rebuilds the tile
 * tables and synchronises. */
hlb_status hlb_batch_set_plan(hlb_batch *b, const int plan[2]);

/* The current plan as plan = {lb index, substep index (the arguments of
 * hlb_batch_set_plan), lb_x, lb_y, substep kind (0 tiles, 1 fused tiles,
 * 2 march), substeps per launch, substep x, substep y}; for a march, x is
 * the block's columns and y its rows per segment. */
hlb_status hlb_batch_get_plan(const hlb_batch *b, int plan[8]);

/* Times every candidate of both launch classes on the current state (the
 * timed launches write only buffers that are not state between steps, so
 * the state is unchanged), keeps the fastest of each and writes their times
 * in microseconds to us[0] (one collide-and-stream launch) and us[1] (the
 * substep launches of one step); us may be NULL.  Synchronises. */
hlb_status hlb_batch_autotune(hlb_batch *b, double us[2]);

/* Moments of simulation sim, as hlb_get_fields (2D: u has 2*ns values).
 * Synchronises. */
hlb_status hlb_batch_get_fields(hlb_batch *b, int sim, double *n, double *u, double *phi, double *mu);

/* Global sums and maxima of simulation sim, as hlb_reduce (mom[2] = 0;
 * step is the batch's step counter).  HLB_ENONFINITE if the simulation's
 * state holds a non-finite value, HLB_EUNSTABLE if its max|u*| >= c_s/2.
 * Synchronises. */
hlb_status hlb_batch_reduce(hlb_batch *b, int sim, hlb_stats *out);

/* Message of the batch's last failure; b may be NULL for hlb_batch_create. */
const char *hlb_batch_last_error(const hlb_batch *b);

/* Destroys the batch and its graphs.  Does not free the workspace. */
hlb_status hlb_batch_destroy(hlb_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* HLB_H */
