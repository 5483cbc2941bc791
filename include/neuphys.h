/*
 * neuphys.h -- C ABI of libneuphys.so: MI355X (gfx950) multigrid Poisson
 * solver and incompressible projection step after "Neural Physics"
 * (Chen, Heaney, Pain, arXiv 2402.17913).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers (hipMalloc'd memory, e.g. a torch
 *    tensor's data_ptr()) owned by the caller, unless a parameter says
 *    "host".  Layout: unpadded, contiguous, x fastest; a 2D field is
 *    [ny][nx], a 3D field [nz][ny][nx] (a torch tensor of shape (ny, nx) or
 *    (nz, ny, nx)).  Cell i along an axis has its centre at (i + 1/2) h.
 *  - Grids: ndim in {2, 3}, every axis the same size n, n a power of two,
 *    4 <= n <= 8192 in 2D, 4 <= n <= 1024 in 3D.  Anything else is
 *    NP_EINVAL and leaves every buffer untouched.
 *  - Boundary conditions are ghost values ("padding", Section 2.1):
 *    NP_BC_DIRICHLET0 sets the ghost to minus the adjacent interior value
 *    (zero on the boundary faces of the cell-centred grid); NP_BC_PERIODIC
 *    wraps; NP_BC_NEUMANN (explicit steps only) copies the adjacent value,
 *    a zero normal derivative.
 *  - Work is enqueued on opts->stream (a hipStream_t; NULL = the null
 *    stream).  Every call returns after its work on that stream is
 *    complete: convergence decisions need the residual norm on the host.
 *  - Errors are returned as np_status, never thrown; np_last_error() gives
 *    a message for the calling thread's last non-OK status.  Calls are
 *    thread-safe for distinct streams; the per-shape workspaces are cached
 *    inside the library and released by np_release_all().
 *  - The operator is A = -Lap_h, the paper's positive 5-point (2D) and
 *    7-point (3D) diffusion filters (Section 2.1 and Appendix A) with unit
 *    diffusivity: (A x)_c = (2d x_c - sum of the 2d face neighbours) / h^2.
 */
#ifndef NEUPHYS_H
#define NEUPHYS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NP_OK = 0,
    NP_EINVAL = -1,   /* bad argument; buffers untouched */
    NP_ENOCONV = -2,  /* tolerance not reached in max_cycles (or divergence); x holds the last iterate */
    NP_ENAN = -3,     /* a non-finite residual norm was seen; x holds the last iterate */
    NP_EHIP = -4,     /* HIP runtime error */
    NP_ENOMEM = -5    /* device allocation failed */
} np_status;

typedef enum { NP_BC_DIRICHLET0 = 0, NP_BC_PERIODIC = 1, NP_BC_NEUMANN = 2 } np_bc;

/* Storage precision of the smoothing and transfer steps.  NP_FP64: plain
 * FP64 V-cycles.  NP_FP32 / NP_BF16: mixed-precision iterative refinement --
 * FP64 residual and update, inner V-cycles storing fields in FP32 / BF16 with
 * FP32 arithmetic, FP64 coarsest solve. */
typedef enum { NP_FP64 = 0, NP_FP32 = 1, NP_BF16 = 2 } np_prec;

typedef struct {
    int ndim;       /* 2 or 3 */
    int64_t n[3];   /* n[0] = nx (fastest), n[1] = ny, n[2] = nz (ignored in 2D) */
} np_dims;

typedef struct {
    int nu1, nu2;         /* pre-/post-smoothing weighted-Jacobi sweeps per level (default 2, 2) */
    double omega;         /* Jacobi relaxation weight (default 2/3) */
    int max_cycles;       /* cap on V-cycles (FP64) or outer refinement steps (mixed), default 200 */
    int fixed_cycles;     /* > 0: run exactly this many cycles / outer steps and ignore tol */
    np_prec smooth_prec;  /* default NP_FP64 */
    int inner_cycles;     /* mixed only: V-cycles per refinement step; 0 = library default */
    int warm_start;       /* 0: x is zeroed first (the paper's zero initial estimate); 1: learned guess
                             (np_cnn_attach), judged against zero; 2: x is the initial guess */
    void *stream;         /* hipStream_t to run on; NULL = null stream */
    int cycle;            /* 0: V(nu1, nu2) (default); 1: the paper's sawtooth cycle (Section 2.2;
                             Appendix B): the residual restricted to the coarsest grid, then per
                             level from the coarsest up e = r/A_00 + P e_coarse and nu2 relaxed-
                             Jacobi steps with alpha = omega; FP64 only, nu1 must be 0 */
    int prolong;          /* sawtooth only: 0 linear (as the V-cycle), 1 the paper's copy of the
                             coarse value to its 2^d fine cells */
    int cnn_cgc;          /* learned coarse-grid correction (the hybrid of Sections 1 and 4; the
                             multigrid cycle as a U-Net, Appendix B): in the first cnn_cgc V-cycles
                             of an FP64 3D solve, the coarse problem on the attached network's grid
                             (np_cnn_attach) starts from the network's prediction for its
                             restricted residual instead of zero, kept only if it lowers that
                             level's energy-norm error (else zero, as without it); the cycle then
                             continues below and above as usual.  0 = off (default).  Requires
                             smooth_prec NP_FP64 and cycle 0; nothing happens without a network of
                             a grid the hierarchy has. */
} np_mg_opts;

typedef struct {
    int cycles;           /* V-cycles run (all precisions, inner cycles included) */
    int outer_iters;      /* refinement steps (mixed), = cycles for FP64 */
    int used_fallback;    /* warm_start = 1 only: 1 if no network fits or the guess was rejected */
    double rel_res;       /* final ||f - A x||_2 / ||f||_2 in FP64 (f mean-free when periodic) */
    double rho_est;       /* geometric mean residual reduction per cycle / outer step */
    double hist[256];     /* rel_res before each cycle / outer step and after the last */
    int cgc_accepted;     /* cnn_cgc > 0: cycles whose learned coarse-grid correction was kept */
} np_mg_stats;

/* Fills *opts with the defaults listed above. */
void np_default_opts(np_mg_opts *opts);

/*
 * Multigrid solve of A x = rhs (the implicit system of Section 2.2 and
 * Appendix B: residual, restriction by 2^d-cell averaging, Jacobi smoothing
 * dividing by the filter centre, prolongation, exact coarsest solve on the
 * 4^d grid, re-discretised operator with spacing 2^l h on level l).  Cycles
 * are V(nu1, nu2) cycles with cell-centred (bi/tri)linear prolongation.
 * rhs: device, read-only, FP64.  x: device, FP64, in/out (see warm_start).
 * Stops when ||rhs - A x||_2 / ||rhs||_2 <= tol, tested before each cycle
 * (or after opts->fixed_cycles cycles).  Periodic: rhs is made mean-free on
 * an internal copy and the mean-free solution is returned.  A zero rhs
 * returns x = 0, 0 cycles.  opts, stats: host, nullable.
 */
np_status mg_poisson_solve(np_dims dims, double h, np_bc bc, const double *rhs, double *x,
                           double tol, const np_mg_opts *opts, np_mg_stats *stats);

/*
 * mg_poisson_solve for callers that cannot allocate device memory (code
 * running under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same FP64 V-cycle solve, same arguments and results, but
 * every workspace buffer lives in one static 48 MiB device array of the
 * library (one copy per GPU, held until the process ends), so the call
 * allocates nothing and keeps no per-shape cache.  That holds every 2D grid up
 * to 1024^2 and every 3D grid up to 128^3, either boundary condition; larger
 * grids are NP_EINVAL with a message giving the bytes needed.  Only
 * opts->smooth_prec = NP_FP64, cycle = 0 and warm_start 0 or 2 are accepted
 * (NP_EINVAL otherwise).  Cycles are enqueued directly (no graph replay).
 * All calls on one GPU share its array and leave their contents in it: calls
 * that overlap in time on the same GPU (other host threads, other streams)
 * race and must be serialised by the caller.
 */
np_status mg_poisson_solve_noalloc(np_dims dims, double h, np_bc bc, const double *rhs, double *x,
                                   double tol, const np_mg_opts *opts, np_mg_stats *stats);

/*
 * One projection time step of the incompressible Navier-Stokes equations
 * (Section 2.4, the projection algorithm; momentum discretised as in
 * Sections 2.1 and 2.3 with sigma = 0) on a periodic staggered grid:
 * p at cell centres; u[k][j][i] on the x-face between cells i and i+1,
 * v on the y-face between rows j and j+1, w on the z-face.  Steps:
 * predictor q~ = q^n - dt F(q^n), corrector q* = q^n - dt F((q~ + q^n)/2)
 * with F(q) = (a . grad_c) q - nu Lap q + G p^n, a = u^n on the faces
 * (central differences); then A dp = -(1/dt) D q* solved by mg_poisson_solve
 * to tol; q = q* - dt G dp; p += dp.  The increment starts from zero
 * (opts->warm_start 0), the attached network's guess (1), or the previous
 * converged step's increment on the same grid size (2; zero when there is
 * none, e.g. the first step or after np_release_all).
 * u, v, p (and w in 3D; NULL in 2D): device, FP64, in/out.  h: cell size.
 * bc must be NP_BC_PERIODIC.  stats receive the pressure solve's numbers.
 */
np_status ns_projection_step(np_dims dims, double h, double *u, double *v, double *w, double *p,
                             double dt, double nu, np_bc bc, double tol, const np_mg_opts *opts,
                             np_mg_stats *stats);

/*
 * Many independent 2D Poisson solves of different sizes in one call (zero
 * Dirichlet only).  Problem p: dims[p] (n x n, n a power of two in
 * [4, 16384]), spacing h[p], right-hand side rhs[p] and solution x[p]
 * (device FP64 arrays; rhs, x, dims, h are host arrays of length nprob).
 * Each problem is solved by mixed-precision refinement: FP64 residual and
 * update, then V(nu1, nu2) cycles in opts->smooth_prec (NP_FP32, or NP_FP64)
 * on the rounded residual from a zero correction.  The cycles of all
 * problems run batched: levels are aligned from the coarsest (4x4) grid, so
 * every level launch covers all problems that have that level; levels at or
 * below 64x64 run in one workgroup per problem; refinement steps are
 * replayed from captured HIP graphs; convergence is decided per problem on
 * the device and converged problems drop out of later launches.  Each
 * problem stops at ||f - A x||_2/||f||_2 <= tol (or after opts->fixed_cycles
 * refinement steps).  opts->inner_cycles = 0 hands the settings to the
 * autotuner, which picks the cycles per refinement step (1..4), the sweeps
 * per level (nu1 = nu2 in 1..3, in place of the caller's) and the level
 * kernels' tiles (row-marching or one cell pair per thread; the workgroups a
 * row-marching launch aims for, which set its rows per group) by timing full
 * solves of this batch.  Its choice is cached for the process and in a JSON
 * file keyed by (GPU architecture, precision, omega, the multiset of sizes):
 * $NEUPHYS_TUNE_CACHE if set (empty: no file), else
 * $XDG_CACHE_HOME/neuphys/batched_autotune.json, else
 * $HOME/.cache/neuphys/batched_autotune.json; a cached entry skips the tuning.
 * Requires nu1 >= 1, nu1 + nu2 even, warm_start = 0.  stats: host array of
 * nprob or NULL; cycles = inner cycles run, outer_iters = refinement steps.
 */
np_status mg_poisson_solve_batched(int nprob, const np_dims *dims, const double *h, np_bc bc,
                                   const double *const *rhs, double *const *x, double tol,
                                   const np_mg_opts *opts, np_mg_stats *stats);

/* Inner cycles chosen by the last autotuning run on this thread and the
 * wall time it took (0, 0 if the last batched call did not tune). */
np_status np_last_autotune(int *inner_cycles, double *ms);

/* Settings the last batched solve on this thread ran with (host outputs,
 * each nullable): inner cycles per refinement step, sweeps nu1 and nu2, the
 * row-marching tiles (1) or one cell pair per thread (0), the workgroups a
 * row-marching launch aims for, and where they came from: 0 the caller
 * (inner_cycles > 0), 1 tuned by this call, 2 this process's cache, 3 the
 * cache file. */
np_status np_last_batched_settings(int *inner_cycles, int *nu1, int *nu2, int *row_marching, int *workgroups,
                                   int *source);

/*
 * One scalar advection-diffusion step, the second-order predictor-corrector
 * of Section 2.1 (the combined advection-diffusion filter applied to
 * (T~ + T^n)/2): T~ = T - dt R(T), T <- T - dt R((T~ + T)/2) with
 * R(T) = sum_e a_e (T[+e] - T[-e]) / (2h) - nu Lap T.  Unlike the solver,
 * any n >= 3 is accepted (all axes equal).  T: device FP64 in/out.
 * a: host array of ndim device pointers to collocated velocity fields, or
 * NULL for pure diffusion.  opts: only opts->stream is used.
 */
np_status np_ad_scalar_step(np_dims dims, double h, double *T, const double *const *a, double dt,
                            double nu, np_bc bc, const np_mg_opts *opts);

/*
 * The same predictor-corrector step with a choice of the paper's filter
 * families (Section 2.1 and Appendix A): scheme 0 central (as
 * np_ad_scalar_step); 1 first-order upwind advection, the value taken from
 * upstream (backward difference for a positive velocity component, forward
 * for a negative one; the printed upwind filter differences the other way)
 * with 5-/7-point diffusion; 2 the finite-element filters: 2D 9-point
 * advection (first difference averaged across the other axis with weights
 * 1, 4, 1 over 6) and diffusion (16 delta - (1,2,1)x(1,2,1), over 4 h^2); 3D
 * 27-point advection (weights (1,4,1)x(1,4,1)/36) and diffusion (88, -6, -3,
 * -2 on centre, faces, edges, corners, over 26 h^2).  bc may also be
 * NP_BC_NEUMANN: zero normal derivative by copying the adjacent value into
 * the padding (Section 2.4).  Arguments and errors as np_ad_scalar_step.
 */
np_status np_ad_explicit_step(np_dims dims, double h, double *T, const double *const *a, double dt, double nu,
                              np_bc bc, int scheme, const np_mg_opts *opts);

/* ---------------------------------------------------------------------- */
/* Implicit advection-diffusion (Section 2.2, the backward-Euler operator of
 * the advection-diffusion equation; its multigrid solve is the experiment of
 * Section 3.2).  One time step A T^{n+1} = T^n with
 *   A T = T + dt sum_e a_e D_e T + nu dt (2d T_c - sum of face neighbours) / h^2,
 * D_e the first difference along axis e: upwind (scheme 0: (T_c - T_{c-e})/h
 * for a_e >= 0, (T_{c+e} - T_c)/h for a_e < 0) or central (scheme 1:
 * (T_{c+e} - T_{c-e})/(2h)).  Constant coefficients; ghosts by the boundary
 * rule.  Coarser levels re-discretise with their own spacing, dt and a fixed. */
typedef struct {
    double dt;     /* time step, > 0 */
    double nu;     /* diffusivity, >= 0 */
    double a[3];   /* advection velocity along x, y, z (a[2] ignored in 2D) */
    int scheme;    /* 0 upwind, 1 central */
} np_ad_op;

/*
 * Multigrid solve of A x = rhs for the operator above, FP64.  opts as for
 * mg_poisson_solve: cycle 0 is V(nu1, nu2) with relaxed Jacobi dividing by
 * the filter centre A_00, linear prolongation and the exact (pivoted) solve on
 * the 4^d grid; cycle 1 is the paper's sawtooth (nu1 = 0, nu2 steps with
 * alpha = omega, prolong 0 linear / 1 copy).  smooth_prec must be NP_FP64 and
 * warm_start 0 (x zeroed: the paper's zero first estimate) or 2 (x is the
 * guess).  Stops when ||rhs - A x||_2 / ||rhs||_2 <= tol, tested before each
 * cycle, or after fixed_cycles; three successive increases end it with
 * NP_ENOCONV.  rhs, x: device FP64 n^d.  l1_change: host, nullable, 256
 * entries: entry k receives ||x_{k+1} - x_k||_1 over cycle k + 1 (the
 * convergence gauge of Section 3.2), zero past the last cycle.  opts, stats:
 * host, nullable.  A zero rhs returns x = 0, 0 cycles.
 */
np_status np_ad_implicit_solve(np_dims dims, double h, np_bc bc, const np_ad_op *op, const double *rhs, double *x,
                               double tol, const np_mg_opts *opts, np_mg_stats *stats, double *l1_change);

/* y = A x for the operator above (device FP64 n^d, y must not alias x);
 * synchronises the stream. */
np_status np_ad_apply(np_dims dims, double h, np_bc bc, const np_ad_op *op, const double *x, double *y,
                      void *stream);

/* Timing of the finest-level kernels of np_ad_implicit_solve on this grid
 * (the same kernels and launch shapes): `reps` back-to-back launches between
 * two events on the stream, *avg_ms their average.  kind 0: relaxed-Jacobi
 * sweep y = x + (2/3) (f - A x) / A_00; 1: residual restriction y = R (f - A x)
 * (y coarse, n/2 per axis); 2: prolongation and correction x += P y (y coarse;
 * f unused).  Device FP64 arrays; n >= 8. */
np_status np_ad_prof_level(np_dims dims, double h, np_bc bc, const np_ad_op *op, int kind, const double *f,
                           double *x, double *y, int reps, void *stream, double *avg_ms);

/*
 * The projection step with the paper's own discretisation choices (Section
 * 2.4: velocity components and pressure at the same cell centres; the
 * filter families of np_ad_explicit_step, scheme 0 central, 1 upwind
 * advection, 2 finite element), periodic: the momentum predictor-corrector
 * advected by the lagged velocity with the source -D p^n, A dp =
 * -(1/dt) sum_e D_e q*_e by the multigrid (A = -Lap_h, 5-/7-point), q = q* -
 * dt D dp, p += dp.  D is the scheme's first-derivative filter (finite
 * element for scheme 2, central otherwise).  The projection is approximate:
 * D.D differs from -A, so divergence modes the derivative filters cannot see
 * (the checkerboard) are not removed.  u, v, w, p: device FP64 n^d (w NULL in
 * 2D), in place; n a power of two.  opts and stats as mg_poisson_solve
 * (warm_start must be 0).
 */
np_status ns_collocated_step(np_dims dims, double h, double *u, double *v, double *w, double *p, double dt,
                             double nu, int scheme, double tol, const np_mg_opts *opts, np_mg_stats *stats);

/* div = sum_e D_e q_e with the first-derivative filter of ns_collocated_step's
 * scheme (finite element for 2, central otherwise), periodic; device FP64
 * n^d arrays (w NULL in 2D); synchronises the stream. */
np_status np_nsc_divergence(np_dims dims, double h, const double *u, const double *v, const double *w, int scheme,
                            double *div, void *stream);

/* ns_projection_step that also copies the pressure-correction right-hand
 * side -(1/dt) D q* and the increment dp it solved for into rhs_out and
 * dp_out (device FP64, n^d each; either may be NULL).  Used to generate
 * (rhs, dp) training pairs for the learned warm start. */
np_status ns_projection_step_io(np_dims dims, double h, double *u, double *v, double *w, double *p,
                                double dt, double nu, np_bc bc, double tol, const np_mg_opts *opts,
                                np_mg_stats *stats, double *rhs_out, double *dp_out);

/* ---------------------------------------------------------------------- */
/* Learned warm start (the hybrid of trained and fixed-weight networks the
 * paper motivates in Sections 1 and 4).  A periodic 3D U-Net on an n_in^3
 * grid: per level two 3x3x3 convolutions with ReLU (16 channels), 2x2x2
 * average between levels (the multigrid restriction filter), cell-centred
 * trilinear upsampling with additive skips, a final 16 -> 1 convolution.
 * Weights and activations are BF16, accumulation FP32 (MFMA implicit-GEMM
 * convolutions); master weights and Adam moments FP32.  Parameter vector:
 * per convolution in network order, W[27][16][16] (tap, out, in; tap =
 * (dz+1)*9 + (dy+1)*3 + (dx+1)) then b[16]; 4*levels - 1 convolutions.
 * All arrays below are device FP32 n_in^3 fields unless said otherwise. */
typedef struct np_cnn np_cnn;
/* n_in a power of two, n_in / 2^(levels-1) >= 16, n_in <= 512; weights zero
 * (np_cnn_init randomises them). */
np_status np_cnn_create(int n_in, int levels, np_cnn **out);
void np_cnn_destroy(np_cnn *net);
int64_t np_cnn_num_params(const np_cnn *net);
/* host float32 arrays of np_cnn_num_params entries; set also resets Adam. */
np_status np_cnn_set_params(np_cnn *net, const float *host, int64_t count);
np_status np_cnn_get_params(const np_cnn *net, float *host, int64_t count);
/* Gradient sums of the last np_cnn_gradients / np_cnn_train_step batch. */
np_status np_cnn_get_grads(const np_cnn *net, float *host, int64_t count);
np_status np_cnn_forward(np_cnn *net, const float *in, float *out, void *stream);
/* in, target: host arrays of `batch` device pointers.  Loss = sum over the
 * batch of mean((N(in) - target)^2); gradient sums stay in the network. */
np_status np_cnn_gradients(np_cnn *net, int batch, const float *const *in, const float *const *target,
                           double *loss, void *stream);
/* One Adam step (lr, beta 0.9/0.999, eps 1e-8) on the batch-mean gradient. */
np_status np_cnn_train_step(np_cnn *net, int batch, const float *const *in, const float *const *target,
                            float lr, double *loss, void *stream);
/* Training pair from a fine 3D grid: f and p (device FP64, dims) are
 * restricted by 2x2x2 averaging down to n_in^3 and divided by the rms of the
 * restricted f (*scale receives it); p, target may be NULL. */
np_status np_cnn_prepare(np_cnn *net, np_dims dims, const double *f, const double *p, float *in,
                         float *target, double *scale, void *stream);
/* Network used by warm_start = 1 (NULL detaches; 3D grids of at least n_in^3
 * only).  The solver restricts f to n_in^3, predicts, scales back, prolongates
 * to the fine grid and keeps the guess x0 only if its energy-norm error is
 * below that of zero, i.e. x0'A x0 - 2 f'x0 < 0 (else x = 0 and
 * stats.used_fallback = 1). */
np_status np_cnn_attach(np_cnn *net);
/* Re-initialises the weights: He-normal from a seeded host generator (fan-in
 * 27 for the first convolution, which reads channel 0 only; 27*16 for the
 * others; the output convolution writes channel 0 only at 0.1 times its
 * fan-in scale), zero biases, Adam state reset. */
np_status np_cnn_init(np_cnn *net, uint64_t seed);
/* Binary file: "NPCNN1\n", int32 levels, int32 n_in, int64 count, float32[count]. */
np_status np_cnn_save(const np_cnn *net, const char *path);
/* A network from a file written by np_cnn_save, as a caller-owned handle. */
np_status np_cnn_open(const char *path, np_cnn **out);
/* Loads weights_path into a library-owned network and attaches it, so that
 * warm_start = 1 uses it (replacing and freeing any network loaded before);
 * NULL detaches and frees it.  On error nothing changes. */
np_status np_cnn_load(const char *weights_path);
/* Trains a new network and writes it to weights_out (np_cnn_save format).
 * Pairs i = 0 .. npairs-1: rhs[i], p[i] are device FP64 cubes of dims[i]
 * (each a power of two >= n_in), a right-hand side and the solution it gives;
 * each is restricted to n_in^3 by 2^3 averaging and divided by the rms of the
 * restricted rhs (np_cnn_prepare), held on the device as FP32 for the whole
 * run (8 n_in^3 bytes per pair).  bc must be NP_BC_PERIODIC.  cfg_json: NULL
 * or a flat JSON object with any of "n_in" (128), "levels" (4), "epochs" (10),
 * "batch" (4), "lr" (5e-4), "seed" (0), "verbose" (0: nonzero prints each
 * finished epoch's loss and elapsed time to stderr); unknown keys are errors.  Seeded
 * initialisation (np_cnn_init), then per epoch a seeded shuffle and Adam steps
 * on minibatches (np_cnn_train_step).  epoch_loss: NULL or a host array of
 * "epochs" entries receiving each epoch's mean MSE.  Runs on the null stream
 * and returns when the file is written. */
np_status np_cnn_train(const np_dims *dims, np_bc bc, int npairs, const double *const *rhs,
                       const double *const *p, const char *cfg_json, const char *weights_out,
                       double *epoch_loss);

/* Message for the calling thread's last non-OK status ("" if none). */
const char *np_last_error(void);

/* Frees every cached workspace (level hierarchies, scratch) on every device. */
void np_release_all(void);

/* ---------------------------------------------------------------------- */
/* Single-operator entry points.  They run one step of the cycle on caller
 * buffers (device, FP64, layout as above) so each kernel can be checked on
 * its own; n is the size of the grid named first. */

/* y = A x (Section 2.1 diffusion filter, Appendix A 3D form). */
np_status np_op_apply(np_dims dims, double h, np_bc bc, const double *x, double *y, void *stream);
/* x_out = x_in + omega (f - A x_in) / A_00, A_00 = 2d/h^2 (Section 2.2, relaxed Jacobi;
 * Appendix B, division by the filter centre).  x_out must not alias x_in. */
np_status np_op_jacobi(np_dims dims, double h, np_bc bc, double omega, const double *f,
                       const double *x_in, double *x_out, void *stream);
/* fc = R (f - A x): residual then 2^d-cell average (Section 2.2 restriction;
 * Appendix B restriction recursion).  fc has n/2 cells per axis. */
np_status np_op_resid_restrict(np_dims dims, double h, np_bc bc, const double *f, const double *x,
                               double *fc, void *stream);
/* x += P ec, cell-centred (bi/tri)linear prolongation of the coarse error ec
 * (n/2 cells per axis) onto x (n cells per axis), coarse ghosts by bc. */
np_status np_op_prolong_add(np_dims dims, np_bc bc, const double *ec, double *x, void *stream);
/* One V(nu1, nu2) cycle x <- V(x, f) with the settings of opts (nullable; FP64 only). */
np_status np_op_vcycle(np_dims dims, double h, np_bc bc, const double *f, double *x,
                       const np_mg_opts *opts);
/* One step of a 3D level of n >= 32 cells per axis in storage precision prec,
 * with the kernels the V-cycle runs there (checks of the temporally blocked
 * kernels against the per-kernel path; Section 2.2 cycle steps).  Arrays are
 * device arrays of the precision (FP64 double, FP32 float, BF16 as uint16
 * bit patterns): f, x, xout fine (n^3), c coarse ((n/2)^3).  kind 0: x = two
 * weighted-Jacobi sweeps of A x = f from zero (omega 2/3); 1: c = R (f - A x);
 * 2: both in one pass, the block kernel of the small levels (x and c written);
 * 3: x <- sweep(sweep(x + P c)), the prolongation + first sweep kernel then a
 * sweep, xout used as the partner buffer; 4: xout = sweep(sweep(x + P c)) in
 * one pass, the block kernel (x unchanged); 5: the same on z-marching tiles,
 * the one-pass up-leg of levels from 128^3 to 1024^3; 6: xout =
 * sweep(sweep(x)) in one z-marching pass, the two pre-sweeps of those levels
 * from a nonzero iterate (c unused, may be NULL); 7: x = two sweeps from
 * zero and c = R (f - A x) in one z-marching pass, the zero-start down-leg of
 * those levels (xout unused, may be NULL); 8: xout = two sweeps of x and
 * c = R (f - A xout) in one z-marching pass, the down-leg of a nonzero iterate
 * (the cycle runs it in FP64 and FP32; knob "d2cpt" picks one or two cells per thread).  Kinds 5 to 8
 * need 128 <= n <= 1024.
 * Synchronises the stream. */
np_status np_op_level(np_dims dims, double h, np_bc bc, np_prec prec, int kind, const void *f, void *x, void *xout,
                      void *c, void *stream);
/* *out (host) = ||f - A x||_2 computed in FP64 by the library's reduction. */
np_status np_op_resid_norm(np_dims dims, double h, np_bc bc, const double *f, const double *x,
                           double *out, void *stream);

/* ---------------------------------------------------------------------- */
/* Kernel timing for the benchmark.  np_prof_enable(mask) starts bracketing
 * every finest-level launch of the selected kinds with HIP events on the
 * stream it is launched on (and disables graph replay meanwhile, so each
 * launch is seen); mask bits: 1 fused smoothing + residual + restriction,
 * 2 the same from a zero iterate, 4 fused prolongation + smoothing,
 * 8 Jacobi sweep, 16 residual + restriction, 32 prolongation + correction,
 * 64 FP64 update + residual of the mixed-precision refinement, 128 Jacobi
 * sweep from a zero iterate; 0 stops.  np_prof_read returns (host) the number
 * of bracketed launches since the last enable, the sum of their durations in
 * milliseconds and the algorithmic bytes they move (each field read once,
 * each output written once). */
void np_prof_enable(int mask);
np_status np_prof_read(int64_t *launches, double *total_ms, double *bytes);
/* Measurement hook: `reps` back-to-back launches of a level kernel the solver
 * runs on this grid and precision (same kernel and launch shape) between two
 * HIP events on `stream` (after one untimed launch); *avg_ms (host) = mean
 * duration per launch.  kind 0: the weighted-Jacobi sweep y = x + (2/3)
 * (f - A x) / A_00 (y fine, distinct from x); 1: residual and restriction
 * y = R (f - A x) (y coarse, n/2 per axis); 2: prolongation and correction
 * x += P y (y coarse; f unused).  f, x, y: device arrays of the precision
 * (FP64 double, FP32 float, BF16 as uint16 bit patterns); n >= 8. */
np_status np_prof_level(np_dims dims, double h, np_bc bc, np_prec prec, int kind, const void *f, void *x,
                        void *y, int reps, void *stream, double *avg_ms);

/* Tuning knobs (process-wide; used by the autotuner): "fused" (0/1: fused
 * level kernels for V(2,2)), "graphs" (0/1: replay cycles from HIP graphs),
 * "fmin2"/"fmin3" and "fmax2"/"fmax3" (smallest and largest level size
 * handled by fused kernels), "bz2"/"bz3"
 * (even number of planes per workgroup in fused kernels, 0 = automatic),
 * "inner_fp32"/"inner_bf16" (default inner cycles per refinement step),
 * "batch" (cycles enqueued before the first host read of the convergence
 * state), "sweep3" (0/1: z-marching smoothing, restriction, prolongation
 * and refinement kernels on 3D levels of n >= 128), "zero2" (0/1: the first
 * two sweeps from a zero iterate in one pass), "psweep" (0/1: prolongation + correction and the
 * first post-sweep in one pass: 2D levels above the tail, 3D levels of n >= 32), "ir_cpt" (1 or 2:
 * cells per thread of the 3D refinement kernel), "fuseb" (0/1: temporally blocked block kernels, 8^3 cells per workgroup, on 3D
 * levels from 32^3 to 2^"fbmax" cells per axis -- the down-leg from a zero iterate and the up-leg with two
 * post-sweeps, one pass each; default 1, fbmax 6; "fbnt" their threads per workgroup, 512 or 1024, default 1024), "sweep2z" (0/1: two sweeps in one z-marching pass on 3D
 * levels from 128^3 to 1024^3 -- the pre-sweeps of a nonzero iterate, with the convergence check, and the
 * up-leg with prolongation + correction; default 1), "down2z" (0/1: in FP64 and FP32, from 256^3, the
 * residual and the restriction in the down-leg's two-sweep pass too; default 1), "d2cpt" (1 or 2: that pass on
 * one cell per thread or two, default 2; FP32 takes it only with 2), "d2wg" (256, 512 or 1024: workgroups the
 * two-cell form aims for; default 0, which takes 256 in FP64 and 512 in FP32), "blk2" (0/1: 2D levels of
 * 128^2 .. 1024^2 take one block kernel per leg, both sweeps with the residual and restriction, or prolongation +
 * correction with both post-sweeps; default 1), "z2wg" (0/1: the 3D one-pass kernels that fit fewer than four
 * workgroups per CU -- the up-leg, FP64's zero-start down-leg -- take planes for 512 workgroups, not 1024
 * (the FP64 up-leg for 256); default 1), "greps" (1, 2, 4 or 8: the most cycles, or refinement steps, one replayed graph holds;
 * default 8), "tailck" (0/1: a cycle's convergence check run by the one-workgroup kernel of its coarse levels
 * rather than by a launch of its own; default 1), "zbar" (1 or 2: barriers per plane step of the 3D zero-start
 * down-leg pass, default 1), "batched_graphs", "batched_autotune" and "batched_rm" (0/1 for the
 * batched solver; batched_rm: row-marching level kernels above the one-workgroup depths),
 * "batched_wg" (workgroups a row-marching batched launch aims for, 64 .. 2^20, default 4096; the
 * caller's setting when the autotuner does not run), "zmarch_explicit" (0/1: z-marching tiles for the 3D explicit, collocated and staggered
 * momentum steps, n >= 32,
 * and row-marching tiles for the 2D explicit step, n >= 1024 a multiple of 256), "mom_rows" (4 or 8: tile rows
 * of the staggered corrector stage on those tiles, default 4), "mom_ring" (2 or 3: planes per field in the staggered
 * stages' LDS rings; 2 keeps the own column's out-of-ring z-neighbours in registers; default 2),
 * "zc3" (planes per workgroup of the 3D z-marching solver kernels: 0 automatic, else a power of two
 * from 2 to 64; it also sets the one-pass two-sweep kernels' planes), "conv3z" (z-marching tiles for the network's convolutions: 0 off, 1 automatic planes per workgroup, else
 * a power of two from 2 to 64 planes), "wgrad_mfma" (0/1: the network's weight gradients on the matrix
 * cores).  Returns NP_EINVAL for an unknown key or value.  Changing a knob
 * drops cached graphs.  np_get_tuning returns the value, -1 if unknown. */
np_status np_set_tuning(const char *key, int value);
int np_get_tuning(const char *key);

#ifdef __cplusplus
}
#endif

#endif /* NEUPHYS_H */
