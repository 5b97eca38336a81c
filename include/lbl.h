/*
 * lbl.h -- C ABI of the MI355X (gfx950) coupled lattice Boltzmann - Langevin
 * sweep for model H.
 *
 * One simulation advances a binary fluid on a periodic D2Q9, D3Q15 or D3Q19 lattice
 * by the hybrid scheme of Sumesh, Pagonabarraga & Adhikari (arXiv:1104.0078):
 *   - momentum: fluctuating lattice Boltzmann (FLBE, Sec. IV and App. B),
 *     multiple-relaxation-time collision with the force density
 *     F = -psi grad mu (or, as an option, the divergence of the stress of
 *     Eq. muf) and Landau-Lifshitz noise on every non-conserved mode;
 *   - order parameter psi: stochastic method of lines (SMOL, Sec. V) with the
 *     Landau chemical potential mu = A psi + B psi^3 - K lap psi (Sec. II.A),
 *     advection by the LB velocity, diffusion M lap mu and a conserved
 *     Langevin flux, in the finite-difference (Sec. V.A; noise from link
 *     fluxes, or built in Fourier space as the paper states it) or
 *     finite-volume (Sec. V.B) variant, integrated by Runge-Kutta with the
 *     noise held constant through the step.
 * Lattice units: dx = dt = 1, c_s^2 = 1/3 (Sec. VI).
 *
 * Conventions shared by every entry point:
 *   - Status codes: LBL_OK (0) or a negative lbl_status.  No C++ exception
 *     crosses this boundary.
 *   - Site index s = x + nx*(y + ny*z) with 0 <= x < nx etc.; 2-D lattices
 *     have nz = 1.
 *   - Populations are exchanged as "structure of arrays" FP64, element
 *     [i*N + s] for velocity i in the canonical order
 *       D2Q9 : 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1)
 *              7:(-1,-1) 8:(1,-1)
 *       D3Q15: 0:(0,0,0) 1:(1,0,0) 2:(-1,0,0) 3:(0,1,0) 4:(0,-1,0) 5:(0,0,1)
 *              6:(0,0,-1) 7:(1,1,1) 8:(-1,-1,-1) 9:(1,1,-1) 10:(-1,-1,1)
 *              11:(1,-1,1) 12:(-1,1,-1) 13:(-1,1,1) 14:(1,-1,-1)
 *       D3Q19: 0:(0,0,0) 1:(1,0,0) 2:(-1,0,0) 3:(0,1,0) 4:(0,-1,0) 5:(0,0,1)
 *              6:(0,0,-1) 7:(1,1,0) 8:(-1,-1,0) 9:(1,-1,0) 10:(-1,1,0)
 *              11:(1,0,1) 12:(-1,0,-1) 13:(1,0,-1) 14:(-1,0,1) 15:(0,1,1)
 *              16:(0,-1,-1) 17:(0,1,-1) 18:(0,-1,1)
 *     and they are the auxiliary distribution fbar of Eq. (barreln) after
 *     streaming, before collision, at the current step.
 *   - Vector fields are [alpha*N + s].
 *   - A simulation handle is not thread-safe; distinct handles are
 *     independent.  All device work of a handle is ordered on its stream.
 */
#ifndef LBL_H
#define LBL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBL_ABI_VERSION 5

typedef struct lbl_sim lbl_sim;

enum lbl_status {
  LBL_OK = 0,
  LBL_E_INVAL = -1,      /* invalid argument, parameter or combination */
  LBL_E_NOMEM = -2,      /* device memory could not be obtained */
  LBL_E_DEVICE = -3,     /* a HIP runtime call failed */
  LBL_E_NONFINITE = -4,  /* a conserved total became NaN or infinite */
  LBL_E_BUFSIZE = -5,    /* destination buffer smaller than the observable */
  LBL_E_UNSUPPORTED = -6 /* observable not available for this simulation */
};

enum lbl_lattice { LBL_D2Q9 = 9, LBL_D3Q15 = 15, LBL_D3Q19 = 19 };
enum lbl_smol { LBL_SMOL_FD = 0, LBL_SMOL_FV = 1 };
enum lbl_precision {
  LBL_FP64 = 0,   /* populations, psi and all arithmetic in FP64 */
  LBL_FP32DEV = 1 /* populations stored as FP32 deviations fbar - w_i rho,
                     psi in FP32, FP32 arithmetic; FP64 reductions */
};
enum lbl_coupling {
  LBL_FULL = 0,      /* the coupled model H step */
  LBL_SMOL_ONLY = 1, /* psi only, advected by the uniform u_imposed; fluid frozen
                        ("diffusion alone" runs of Sec. VI) */
  LBL_LB_ONLY = 2    /* fluctuating fluid only, no force, psi frozen */
};

/* Model H parameters (Sec. II) and numerical choices.
 *   rho   : mean density rho0 (also the density in the noise amplitudes);
 *   eta   : shear viscosity; the shear modes relax with
 *           omega_s = 1 / (1/2 + eta / (rho c_s^2)), which must lie in (0, 2);
 *   M     : mobility (Eq. advdiff);  a, b, kappa: A, B, K of Eqs. (Feng), (feng);
 *   kT    : temperature in energy units (>= 0);
 *   omega_bulk, omega_ghost : relaxation rates of the bulk stress mode and of
 *           every ghost mode, in (0, 2]; 1 projects them onto equilibrium;
 *   u_imposed: advecting velocity when coupling == LBL_SMOL_ONLY;
 *   rk_stages: 1 (Euler), 2 (Heun, default) or 4 (classical RK4);
 *   seed  : key of the Philox4x32-10 noise stream;
 *   sample_every: if > 0, the axis structure factors are accumulated on the
 *           device after every sample_every-th step (LBL_OBS_SK_AXES etc.),
 *           and the FP64 totals are checked for NaN/Inf at the same time (a
 *           failure surfaces as LBL_E_NONFINITE from the next lbl_observe). */
typedef struct lbl_params {
  int32_t lattice;   /* enum lbl_lattice */
  int32_t smol;      /* enum lbl_smol */
  int32_t precision; /* enum lbl_precision */
  int32_t coupling;  /* enum lbl_coupling */
  int32_t rk_stages;
  int32_t nx, ny, nz; /* each >= 4; nz == 1 for D2Q9; N = nx*ny*nz < 2^31 */
  double rho, eta, M, a, b, kappa, kT;
  double omega_bulk, omega_ghost;
  double u_imposed[3];
  uint64_t seed;
  int32_t sample_every;
  int32_t fd_noise;   /* enum lbl_fd_noise; LBL_FDNOISE_LINK unless smol == LBL_SMOL_FD */
  int32_t force_form; /* enum lbl_force_form */
  int32_t sample_full_k; /* 0 or 1: at every sample (sample_every > 0) also
                            accumulate the whole-zone spectrum LBL_OBS_SK_FULL */
  int32_t walls;      /* enum lbl_walls */
  int32_t reserved;   /* 0 */
  double u_wall[2][3]; /* velocities of the lower and upper wall (LBL_WALLS_LAST):
                          tangential, the component along the last axis is 0 */
} lbl_params;

/* Boundaries (the closing remark of Sec. V.B: the finite-volume SMOL admits
 * walls and shear boundaries):
 *  PERIODIC (default): every axis periodic;
 *  LAST: solid planar walls across the last axis (z in 3-D, y in 2-D), half a
 *    lattice spacing below layer 0 and above layer L-1, moving tangentially
 *    at u_wall[0] (lower) and u_wall[1] (upper).  The LB populations that
 *    would leave through a wall return to their site reversed (halfway
 *    bounce-back, with the term 2 w_i rho c_i.U / c_s^2 of a moving wall);
 *    the SMOL stencils drop every link that crosses a wall, so no order
 *    parameter flows through it and the fluctuation-dissipation balance of the
 *    noise is kept.  FV variant, force PSI_GRAD_MU; single simulations and
 *    pool requests (a pool batches requests with walls in groups of their
 *    own). */
enum lbl_walls { LBL_WALLS_PERIODIC = 0, LBL_WALLS_LAST = 1 };

/* Force density of the order parameter on the fluid (full coupling):
 *  PSI_GRAD_MU (default, the paper's discretisation, Sec. IV): F = -psi G mu
 *    with the variant's gradient G (FD central difference, FV Gamma).  Its
 *    lattice sum vanishes when B = 0 but not otherwise;
 *  STRESS: F_a = -sum_b G_b sigma_ab with sigma the stress of Eq. (muf),
 *    sigma_ab = K g_a g_b + delta_ab [A psi^2/2 + 3 B psi^4/4 - K psi L psi
 *    - K/2 |g|^2], g = G psi, L the Shinozaki-Oono Laplacian.  Equal to the
 *    default in the continuum (to second order in the lattice spacing); its
 *    lattice sum vanishes for any B, so momentum is conserved exactly.  Two
 *    extra per-site passes per step; single simulations only (a pool refuses
 *    such a request). */
enum lbl_force_form { LBL_FORCE_PSI_GRAD_MU = 0, LBL_FORCE_STRESS = 1 };

/* How the FD variant builds its conserved noise N^n (Sec. V.A), both with
 * covariance -2 kT M L_SO (Eq. etafdt):
 *  LINK (default): one Gaussian flux per undirected link of the
 *    Shinozaki-Oono stencil, amplitude sqrt(2 kT M lambda_l), N = the
 *    divergence of the fluxes; real space, in-kernel, no transform;
 *  FOURIER: the paper's own construction, N = F^-1[ sqrt(-2 kT M L(q)) F[w] ]
 *    with w(x) the white field of normal slot 0 (site x, step n, SMOL
 *    stream) and L(q) the stencil's symbol (Eq. solapft; its 2-D analogue);
 *    one real-to-complex and one complex-to-real hipFFT transform per step.
 *    Single simulations only (a pool refuses such a request); the FFT plans
 *    hold work memory of hipFFT's own beyond lbl_sim_bytes. */
enum lbl_fd_noise { LBL_FDNOISE_LINK = 0, LBL_FDNOISE_FOURIER = 1 };

enum lbl_init_kind {
  LBL_INIT_REST = 0,     /* fbar = equilibrium at (rho, boost_u); psi = psi_std * z */
  LBL_INIT_TANH_2IF = 1, /* as REST, plus two flat tanh interfaces (Eqs. tanh,
                            intthick) at L/4 and 3L/4 along the last axis;
                            needs a < 0 < b and kappa > 0 */
  LBL_INIT_USER = 2      /* fbar and psi copied from f0 and psi0 */
};

/* Initial state.  z is the normal of Philox slot 0, tag 2, step 0 at each
 * site.  f0 (Q*N FP64, canonical order) and psi0 (N FP64) are read during
 * lbl_create only; they are device pointers if user_on_device != 0.
 * step0 is the step counter of the initial state: the first lbl_step draws
 * the noise of counter step0, so a simulation created with USER from the
 * POP and PSI observables of another one at step n, with step0 = n,
 * continues it bitwise (resume).  0 <= step0 < 2^32 (the noise counter). */
typedef struct lbl_init {
  int32_t kind;
  int32_t user_on_device;
  double psi_std;
  double boost_u[3];
  const double *psi0;
  const double *f0;
  int64_t step0;
} lbl_init;

/* Device memory and stream injection.  If alloc is NULL the library uses
 * hipMalloc / hipFree.  alloc must return device memory valid on `stream`
 * (NULL on failure); free receives the same ctx and stream.  stream is a
 * hipStream_t (NULL selects the device's null stream). */
typedef void *(*lbl_alloc_fn)(void *ctx, size_t bytes, void *stream);
typedef void (*lbl_free_fn)(void *ctx, void *ptr, void *stream);
typedef struct lbl_env {
  int32_t device;
  int32_t reserved;
  void *stream;
  lbl_alloc_fn alloc;
  lbl_free_fn free;
  void *ctx;
} lbl_env;

/* Create a simulation: validates the parameters, allocates its device state
 * and writes the initial state (step 0) on env->stream.  On success *out owns
 * the state until lbl_destroy; on failure *out is NULL and nothing leaks.
 * Errors: LBL_E_INVAL (unknown enum, size out of range, omega outside (0,2),
 * kT < 0, TANH_2IF without a < 0 < b, missing USER pointers), LBL_E_NOMEM,
 * LBL_E_DEVICE. */
int lbl_create(const lbl_params *params, const lbl_init *init, const lbl_env *env,
               lbl_sim **out);

/* Enqueue nsteps coupled steps (Sec. VI: FLBE and SMOL marched alternately)
 * on the simulation's stream and return without waiting.  Step n draws the
 * noise of counter step n.  Within a step the SMOL noise is frozen over the
 * Runge-Kutta stages (Sec. V) and each stage advects with the velocity of
 * its own time level: u^n at t_n, the velocity of the streamed populations
 * (jbar^{n+1} + F^n/2)/rho^{n+1} at t_{n+1}, their mean at RK4 midpoints.  Errors of earlier asynchronous work (including
 * LBL_E_NONFINITE from the sampled totals) are reported by the next call that
 * synchronises (lbl_observe).  nsteps < 0 gives LBL_E_INVAL. */
int lbl_step(lbl_sim *sim, int64_t nsteps);

enum lbl_observable {
  LBL_OBS_PSI = 0,      /* N FP64: psi */
  LBL_OBS_RHO = 1,      /* N FP64: rho = sum_i fbar_i */
  LBL_OBS_U = 2,        /* d*N FP64: u = (sum_i fbar_i c_i + F/2)/rho, F the force
                           density of lbl_params.force_form (F = 0 for LB_ONLY).
                           LBL_E_UNSUPPORTED for SMOL_ONLY, which has no flow
                           field (its velocity is lbl_params.u_imposed) */
  LBL_OBS_POP = 3,      /* Q*N FP64: fbar, canonical order */
  LBL_OBS_TOTALS = 4,   /* 10 FP64: mass, Px, Py, Pz, Psi, then the L1 norms
                           sum|rho|, sum|jx|, sum|jy|, sum|jz|, sum|psi|,
                           with j = sum_i fbar_i c_i; reduced in FP64 */
  LBL_OBS_SK_AXES = 5,  /* d*Lmax FP64, Lmax = max(nx,ny,nz): mean over samples of
                           |sum_x psi e^{-i k x_alpha}|^2 / N at k = 2 pi m / L_alpha,
                           element [alpha*Lmax + m] (0 beyond L_alpha).  A sample
                           is taken after every sample_every-th step, on the new psi */
  LBL_OBS_UK_AXES = 6,  /* d*d*Lmax FP64: the same for each velocity component beta,
                           element [(alpha*d + beta)*Lmax + m]; the velocity sampled
                           is u^n, the one the sampled step computed (zero for
                           SMOL_ONLY, whose flow is imposed) */
  LBL_OBS_STEP = 7,     /* 1 int64: steps taken */
  LBL_OBS_NSAMPLES = 8, /* 1 int64: samples accumulated into SK/UK */
  LBL_OBS_PSIK_AXES = 9, /* 2*d*Lmax FP64: the current sum_x psi e^{-i k x_alpha} at
                           k = 2 pi m / L_alpha, element [(alpha*Lmax + m)*2 + {0: re, 1: im}] */
  LBL_OBS_SK2_AXES = 10, /* d*Lmax FP64: mean over samples of the square of each
                           SK_AXES sample (its variance is SK2 - SK^2) */
  LBL_OBS_UK2_AXES = 11, /* d*d*Lmax FP64: the same for UK_AXES */
  LBL_OBS_SK_FULL = 12,  /* nz*ny*(nx/2+1) FP64: mean over samples of
                            |sum_x psi e^{-i q.x}|^2 / N over the whole zone,
                            q = 2 pi (kx/nx, ky/ny, kz/nz), kx in [0, nx/2] (the
                            other half follows from S(-q) = S(q)), element
                            [kx + (nx/2+1)(ky + ny kz)]; one real-to-complex
                            hipFFT transform per sample.  Only with
                            lbl_params.sample_full_k: otherwise its size is 0 and
                            lbl_observe gives LBL_E_INVAL (Figs. test1b, test2a,
                            test2: the spectrum over wave-vector planes) */
  LBL_OBS_HEIGHTS = 13  /* 2*C FP64, C = nx*ny (3-D) or nx (2-D): heights of two
                           interfaces along the last axis (length L) per column
                           c = x + nx*y (3-D) or x (2-D): the zero crossing of
                           psi by linear interpolation between the two sites
                           that bracket it (Sec. VI.C), z + psi(z)/(psi(z) -
                           psi(z+1)) at the first z with psi(z) psi(z+1) <= 0 in
                           the window [L/8, 3L/8) (element [c], the interface
                           near L/4) or [5L/8, 7L/8) (element [C + c]); NaN
                           when the window holds none */
};

/* Copy an observable of the current state into dst (host memory, or device
 * memory if dst_is_device != 0).  Synchronises the simulation's stream first.
 * The caller owns dst.  Errors: LBL_E_INVAL (unknown `what`, NULL dst),
 * LBL_E_BUFSIZE (bytes too small), LBL_E_UNSUPPORTED, LBL_E_DEVICE, or a
 * deferred error of earlier steps. */
int lbl_observe(lbl_sim *sim, int what, void *dst, size_t bytes, int dst_is_device);

/* Size in bytes of an observable for this simulation (0 for unknown `what`,
 * and for LBL_OBS_SK_FULL without lbl_params.sample_full_k). */
size_t lbl_observable_bytes(const lbl_sim *sim, int what);

/* Release the simulation's device memory through the injected allocator
 * (after its stream has drained).  NULL is accepted. */
int lbl_destroy(lbl_sim *sim);

/* Per-kernel timing with HIP events recorded on the simulation's stream
 * around every kernel that lbl_step launches.  lbl_timing_enable(sim, 1)
 * clears the accumulators and starts recording; 0 stops.  lbl_timing_read
 * synchronises the stream and writes up to max_entries records (one per
 * kernel name, in first-launch order) and their count to *n_entries.
 * Errors: LBL_E_INVAL (NULL pointers), LBL_E_DEVICE. */
typedef struct lbl_kernel_time {
  char name[48];
  int64_t launches;
  double total_ms;
} lbl_kernel_time;
int lbl_timing_enable(lbl_sim *sim, int enable);
int lbl_timing_read(lbl_sim *sim, lbl_kernel_time *out, int max_entries, int *n_entries);

/* Launch schedule of one simulation.  It changes only speed, never results.
 * lb_width: sites along x per 256-thread block of the per-site LB kernels
 * (32, 64, 128 or 256; a block covers 256 / lb_width rows of one plane);
 * xcd_swizzle, bit 0: the LB blocks, bit 1: the SMOL tiles are ordered so
 * that each of the 8 XCDs sweeps one contiguous eighth of them (reads across
 * block edges then hit the same L2); zc: planes per block of the z-marching
 * kernels of a 3-D lattice, the stage, the preparation kernel and the velocity
 * pass that draws the noise alike (0 restores the library's
 * per-kernel defaults below, larger than nz is clamped; lbl_get_schedule
 * reports the stage's); overlap:
 * 1 runs the first Runge-Kutta stage on a second stream of the library's
 * own (default priority), concurrently with the velocity pass of the
 * streamed populations that only the later stages read (full coupling, 2 or
 * 4 stages); 2 draws the SMOL noise on that second stream, concurrently with
 * the LB passes (the noise depends on the counter alone), and joins it before
 * the first stage; 3 draws the SMOL noise inside the velocity pass, one
 * kernel on the SMOL tiles (z-marching in 3-D) on the stream, where a
 * velocity pass runs (full coupling, 2 or 4 stages) and the preparation
 * kernel would draw the noise (kT > 0; not the FD noise built in Fourier
 * space), and is 0 elsewhere; 0 runs everything on the simulation's stream,
 * the noise in the preparation kernel.  Default: the widest width up to 256
 * that fits nx, no swizzle, zc per kernel from its occupancy (the stage's
 * blocks fill the device's resident slots in one round, the preparation
 * kernel's and the velocity pass's in two; at least 8 planes), overlap 3.  The z-marching stress pass of force_form STRESS (FV, 3-D) keeps
 * its own default (two rounds) whatever zc is.  Errors: LBL_E_INVAL (NULL,
 * unsupported width, zc < 0, overlap not 0, 1, 2 or 3). */
typedef struct lbl_schedule {
  int32_t lb_width;
  int32_t xcd_swizzle;
  int32_t zc;
  int32_t overlap;
} lbl_schedule;
int lbl_set_schedule(lbl_sim *sim, const lbl_schedule *schedule);
int lbl_get_schedule(const lbl_sim *sim, lbl_schedule *out);

/* Diagnostics: the normals the sweep draws (the Gaussian noise of Secs. IV,
 * V and App. B, drawn from Philox4x32-10 with the Box-Muller map).  dst (host, n_sites * n_slots
 * FP64, [site][slot]) receives the normal of slot s (Philox block s/4, lane
 * s%4) of the counter (site0 + i, step, block, tag) under key seed, computed
 * on `device` with the transform of the given storage (LBL_FP64 or
 * LBL_FP32DEV).  Synchronous; allocates and frees its own device memory.
 * For tests of the generator against independent implementations.
 * Errors: LBL_E_INVAL (NULL dst, n_sites outside 1..2^24, n_slots outside
 * 1..64, unknown precision), LBL_E_NOMEM, LBL_E_DEVICE. */
int lbl_diag_normals(int32_t device, int32_t precision, uint64_t seed, uint32_t step,
                     uint32_t tag, uint32_t site0, int64_t n_sites, int32_t n_slots,
                     double *dst);

/* ------------------------------------------------------------------------
 * Pool: independent simulations batched on one device (the library's own
 * serving and ensemble layer, not the paper's).  Requests are admitted in
 * arrival order while their device memory fits the budget; every running
 * request of the same kind (storage, lattice, variant, stages, ghost rate)
 * advances together: each phase of a step is one launch over a work table of
 * (request, tile) items, and a tick of several steps is captured and replayed
 * as one graph.  A request's arithmetic, noise stream and results do not
 * depend on what else is resident.  Finished requests release their device
 * memory; their results stay until lbl_pool_release.
 * ------------------------------------------------------------------------ */
typedef struct lbl_pool lbl_pool;

enum lbl_request_state {
  LBL_REQ_QUEUED = 0,
  LBL_REQ_RUNNING = 1,
  LBL_REQ_DONE = 2,
  LBL_REQ_FAILED = 3 /* creation failed, or the final FP64 totals were not
                        finite (the request fails alone; no result) */
};

enum lbl_submit_flags {
  LBL_KEEP_PSI = 1 /* keep the final psi field as a result */
};

enum lbl_pool_result {
  LBL_RES_SK_AXES = 0, /* d*Lmax FP64: |sum_x psi e^{-i k x_alpha}|^2 / N of the final
                          state at k = 2 pi m / L_alpha, element [alpha*Lmax + m] */
  LBL_RES_TOTALS = 1,  /* 20 FP64: LBL_OBS_TOTALS at admission, then at completion */
  LBL_RES_TIMES = 2,   /* 3 FP64: submit, start, completion times in seconds of the
                          host's monotonic clock */
  LBL_RES_PSI = 3      /* N FP64: final psi (requests submitted with LBL_KEEP_PSI) */
};

typedef struct lbl_pool_info {
  uint64_t budget_bytes, used_bytes;
  int64_t queued, running, done, failed;
  int64_t ticks, site_updates; /* lattice-site updates executed so far */
} lbl_pool_info;

/* Create a pool with a device-memory budget.  env gives the device and the
 * allocator as for lbl_create; the pool runs all its work on a stream of its
 * own (default priority, created here) so that ticks can be captured as
 * graphs; env->stream is not used.  Errors: LBL_E_INVAL, LBL_E_DEVICE. */
int lbl_pool_create(uint64_t budget_bytes, const lbl_env *env, lbl_pool **out);

/* Queue one simulation of nsteps steps; never blocks.  *request receives its
 * id.  The parameters are validated now (LBL_E_INVAL); a request whose
 * device memory exceeds the whole budget gives LBL_E_NOMEM.  USER initial
 * states are copied at submission. */
int lbl_pool_submit(lbl_pool *pool, const lbl_params *params, const lbl_init *init,
                    int64_t nsteps, int32_t flags, int64_t *request);

/* One tick: admit what fits, advance every running request by up to
 * max_steps steps (each stops at its own step count), retire the finished
 * ones.  max_steps = 0 only admits (creating and initialising the admitted
 * requests and their work tables).  Synchronises the pool's stream.
 * *pending (may be NULL) receives the number of queued plus running requests
 * afterwards.  Errors: LBL_E_INVAL (NULL pool, max_steps < 0). */
int lbl_pool_run(lbl_pool *pool, int64_t max_steps, int64_t *pending);

/* State and completed steps of a request.  LBL_E_INVAL for an unknown id. */
int lbl_pool_poll(const lbl_pool *pool, int64_t request, int32_t *state, int64_t *steps_done);

/* Copy a result of a finished request into host memory dst.  Errors:
 * LBL_E_INVAL (unknown id or kind, not finished), LBL_E_BUFSIZE,
 * LBL_E_UNSUPPORTED (psi not kept). */
int lbl_pool_result(const lbl_pool *pool, int64_t request, int32_t what, void *dst,
                    size_t bytes);

/* Size in bytes of a result (0 if unknown). */
size_t lbl_pool_result_bytes(const lbl_pool *pool, int64_t request, int32_t what);

/* Forget a request: drops its results, or cancels it if queued or running
 * (freeing its device memory). */
int lbl_pool_release(lbl_pool *pool, int64_t request);

int lbl_pool_stats(const lbl_pool *pool, lbl_pool_info *out);

/* Work-table schedule of the batched launches (speed only, never results):
 * lb_width as for lbl_set_schedule (tiles of the LB work table);
 * xcd_swizzle != 0 gives each XCD a contiguous range of each work table, so
 * a request's neighbouring tiles share one L2; zc > 0 overrides the planes
 * per tile of the 3-D SMOL kernels (0: each request's own).  Takes effect at
 * the next lbl_pool_run; overlap must be 0.  Errors: LBL_E_INVAL. */
int lbl_pool_set_schedule(lbl_pool *pool, const lbl_schedule *schedule);
int lbl_pool_get_schedule(const lbl_pool *pool, lbl_schedule *out);

/* Device memory one simulation with these parameters needs (0 if invalid). */
uint64_t lbl_sim_bytes(const lbl_params *params);

/* Text of the pool's last error ("" if none). */
const char *lbl_pool_last_error(const lbl_pool *pool);

/* Release the pool, cancelling what is still queued or running. */
int lbl_pool_destroy(lbl_pool *pool);

/* ------------------------------------------------------------------------
 * Stepping without allocation.  For callers that cannot allocate device
 * memory: code under HIP graph capture, serving loops and harnesses that
 * forbid hipMalloc.
 *
 * lbl_step_static advances a state held by the caller by nsteps coupled
 * steps.  pop (Q*N FP64, the canonical order of the POP observable: fbar at
 * step step0) and psi (N FP64) are device memory of the current device; they
 * are read first and then overwritten with the state after nsteps steps.
 * The result is bit for bit that of lbl_create with an LBL_INIT_USER state
 * (pop, psi, step0) followed by lbl_step(nsteps) and the LBL_OBS_POP and
 * LBL_OBS_PSI observables.  Every other field of the step (the second
 * population buffer, stage inputs, velocities, chemical potential, noise)
 * lives in a workspace of LBL_STATIC_SCRATCH_BYTES bytes that the library
 * holds on each device until the process ends; the call allocates no device
 * memory and creates no stream, event or FFT plan.  Work is enqueued on
 * `stream` (a hipStream_t; NULL is the null stream) and the call returns
 * without waiting.  All calls on one device share its workspace, which keeps
 * the last call's contents: calls that overlap in time on one device race,
 * so order them on one stream.  The first call on a device resolves the
 * workspace's address (hipGetSymbolAddress); make it outside graph capture.
 * After that a call only enqueues kernels on `stream` (the workspace is
 * cleared by a kernel, not a memset), so it can be captured into a graph and
 * replayed; each replay repeats the captured step0 and nsteps.
 * Errors: LBL_E_INVAL (NULL pointers, nsteps < 0, invalid parameters as for
 * lbl_create, fd_noise = LBL_FDNOISE_FOURIER, sample_every or sample_full_k
 * not 0), LBL_E_NOMEM (the lattice's buffers, lbl_sim_bytes(params) plus
 * 256-byte alignment of each, exceed the workspace), LBL_E_DEVICE.  The
 * message of the last failure on this thread is lbl_last_error(NULL).
 */
#define LBL_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int lbl_step_static(const lbl_params *params, void *stream, int64_t step0, int64_t nsteps,
                    double *pop, double *psi);

/* Static text for a status code. */
const char *lbl_strerror(int status);

/* Text of the last error raised on this handle ("" if none).  With a NULL
 * handle: the last error of a failed lbl_create or lbl_step_static on this
 * thread. */
const char *lbl_last_error(const lbl_sim *sim);

/* LBL_ABI_VERSION of the loaded library. */
int lbl_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LBL_H */
