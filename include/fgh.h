/*
 * fgh.h -- C-ABI of libfgh: Fourier-Galerkin FFT homogenization on AMD MI355X (gfx950).
 *
 * Method: Mishra, Vondrejc, Zeman, "A comparative study on low-memory iterative solvers for
 * FFT-based homogenization of periodic media" (arXiv 1508.02045).
 *
 * Problem (Sec. 2, eq:homog_form): given a periodic field of symmetric positive-definite
 * d x d coefficients A(x) on the unit cell, with c_A |v|^2 <= v.A(x)v <= C_A |v|^2 (eq:A), and a
 * macroscopic gradient E, find the curl-free zero-mean fluctuation e minimising the energy
 * (A(E+e), E+e); the minimum is (A_H E, E).  Discretised by trigonometric polynomials of odd
 * order N (Sec. 2.1), with the trapezoidal rule on the N grid (GaNi, eq:GaNi) or with exact
 * integration on the double grid 2N-1 (Ga, eq:Ga, eq:Ga_eval), it becomes the linear system
 * C x = b with C = G A, b = -G A E (eq:linsys), solved by Richardson, conjugate gradients,
 * Chebyshev or Eyre-Milton iterations (Sec. 3, Algorithms 1-4).
 *
 * Conventions shared by every entry point
 *  - d is 2 or 3.  N[a] >= 3 and odd for every axis a (Sec. 2.1: N_alpha odd).
 *  - The integration grid is N (GaNi) or M = 2N-1 (Ga).  Its points are C-ordered, the last
 *    axis contiguous; array index i on an axis of n points stands for the grid point x = m/n
 *    with m = i if 2i < n else i - n (Sec. 2.1: grid points x_N^m = m/N), so the origin is
 *    index 0.
 *  - A vector field is double[d][grid] (structure of arrays).
 *  - Inner products and norms are (a,b)_2 = (1/|grid|) sum_points a.b (Notation paragraph);
 *    the norm of a constant field E is the Euclidean |E|.
 *  - Device pointers are HIP device memory on the current device.  The library allocates
 *    nothing: the caller provides one device workspace per plan (size from
 *    fgh_plan_workspace) and keeps it, A and the field buffers alive until
 *    fgh_plan_destroy.  All work is enqueued on the plan's stream.
 *  - Errors are returned as fgh_status codes; nothing aborts and no exception crosses the ABI.
 *  - A plan is not thread-safe; distinct plans may be used from distinct threads.
 */
#ifndef FGH_H
#define FGH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fgh_plan_s* fgh_plan;

typedef enum {
    FGH_OK = 0,
    FGH_E_INVALID = 1,        /* bad argument: d, even or < 3 N, tolerance outside (0,1), NULL */
    FGH_E_NOT_SPD = 2,        /* some A(x) has lambda_min <= 0, or c_A > C_A given */
    FGH_E_UNSUPPORTED = 3,    /* Eyre-Milton with exact integration (Sec. 3.4, Table 1) */
    FGH_E_WORKSPACE = 4,      /* workspace NULL or smaller than fgh_plan_workspace reports */
    FGH_E_NO_CONVERGENCE = 5, /* iteration cap reached; outputs hold the last iterate */
    FGH_E_DIVERGED = 6,       /* non-finite values or a step norm above 1e12 |E| */
    FGH_E_DEVICE = 7,         /* a HIP runtime call failed */
    FGH_E_CANCELLED = 8       /* served request discarded by fgh_server_destroy before admission */
} fgh_status;

typedef enum {
    FGH_GANI = 0, /* Galerkin with numerical (trapezoidal) integration on the N grid, eq:GaNi */
    FGH_GA = 1    /* Galerkin with exact integration on the 2N-1 double grid, eq:Ga_eval     */
} fgh_rule;

typedef enum {
    FGH_RICHARDSON = 0,  /* Algorithm 1, omega = 2/(c_A + C_A)            */
    FGH_CG = 1,          /* Algorithm 2                                    */
    FGH_CHEBYSHEV = 2,   /* Algorithm 3 on the interval [c_A, C_A]         */
    FGH_EYRE_MILTON = 3  /* Algorithm 4, omega = sqrt(c_A C_A); GaNi only  */
} fgh_solver;

typedef enum {
    FGH_FP64 = 0,        /* every step in double precision                                   */
    FGH_FP32_REFINED = 1 /* FFTs, projection and A(x) multiply in single precision inside a
                            double-precision defect-correction loop; residuals, reductions
                            and A_H in double precision                                      */
} fgh_precision;

typedef enum {
    FGH_A_SYM = 0,   /* per point packed symmetric d x d: double[ncoef][N grid], ncoef = 3 (2D:
                        a00 a01 a11) or 6 (3D: a00 a01 a02 a11 a12 a22)                        */
    FGH_A_ISO = 1,   /* per point isotropic scalar a: A(x) = a(x) I, double[N grid]          */
    FGH_A_PHASE = 2  /* uint8 phase index per point on the N grid plus a host table of
                        n_phases packed symmetric matrices (double[n_phases][ncoef])         */
} fgh_akind;

typedef struct {
    int32_t iters;             /* loop bodies executed, each with exactly one operator apply
                                  (FP32_REFINED: inner FP32 bodies summed over outer steps)   */
    int32_t outer_iters;       /* FP32_REFINED: defect-correction steps; FP64: 0              */
    int32_t fp64_applies;      /* double-precision operator applications performed            */
    int32_t status;            /* fgh_status of this load                                    */
    double rel_res_recursive;  /* the stopping-test quantity at exit (see fgh_solve)         */
    double rel_res_true;       /* ||b - C x||_2 / ||b||_2 recomputed at exit (0 if b = 0)      */
    double c_A, C_A;           /* spectral bounds used                                       */
    double seconds;            /* wall time of this load's solve                             */
} fgh_stats;

/* Size in bytes of the device workspace a plan with these parameters needs (and its required
 * alignment is 256 bytes).  N, rule, precision and the coefficient kind determine it; solver
 * state for every solver is included.  Returns FGH_E_INVALID for bad d or N. */
fgh_status fgh_plan_workspace(int d, const int32_t* N, fgh_rule rule, fgh_precision precision,
                              fgh_akind a_kind, size_t* bytes);

/* Create a plan (Sec. 2.2-2.3): validates the input, derives c_A and C_A (eq:A) from A unless
 * both are given (> 0), builds the operator's coefficients on the device -- A itself for GaNi
 * (eq:GaNi), the double-grid coefficients A_{2N-1} of the pixel-wise constant field for Ga
 * (eq:Ga_exact_integration, assembled from the exact pixel Fourier coefficients) -- and lays
 * out every buffer inside `workspace`.
 *   A        device pointer, layout per a_kind on the N grid (NULL for FGH_A_PHASE).
 *   phase    device uint8 [N grid] for FGH_A_PHASE, else NULL; values < n_phases.
 *   phase_table  host double[n_phases][ncoef] for FGH_A_PHASE, else NULL; 1 <= n_phases <= 16.
 *   c_A, C_A spectral bounds to use; if either is <= 0 both are derived from A.
 *   stream   hipStream_t to enqueue on (NULL = default stream).
 * Blocks until set-up is complete.  Errors: FGH_E_INVALID, FGH_E_NOT_SPD, FGH_E_WORKSPACE,
 * FGH_E_DEVICE.  On error *out is NULL. */
fgh_status fgh_plan_create(fgh_plan* out, int d, const int32_t* N, fgh_rule rule,
                           fgh_precision precision, fgh_akind a_kind, const void* A,
                           const uint8_t* phase, const double* phase_table, int n_phases,
                           double c_A, double C_A, void* workspace, size_t workspace_bytes,
                           void* stream);

/* Release the plan's host state (the workspace stays the caller's). NULL is ignored. */
void fgh_plan_destroy(fgh_plan plan);

/* Number of points of the plan's integration grid (|N| for GaNi, |2N-1| for Ga). */
int64_t fgh_plan_grid_points(fgh_plan plan);

/* Spectral bounds the plan uses (eq:A). */
fgh_status fgh_plan_bounds(fgh_plan plan, double* c_A, double* C_A);

/* y = C x = G A x in double precision (eq:linsys; G as in eq:discrete_proj, band-limited to
 * Z_N on the double grid for Ga).  x and y: device double[d][grid] of the integration grid;
 * they must not overlap.  Asynchronous on the plan's stream. */
fgh_status fgh_apply(fgh_plan plan, const double* x, double* y);

/* Same operator in single precision: x, y device float[d][grid] (the FP32 path of
 * FGH_FP32_REFINED plans; FGH_E_UNSUPPORTED for FGH_FP64 plans). */
fgh_status fgh_apply_f32(fgh_plan plan, const float* x, float* y);

/* The operator of fgh_apply without a plan and without any device allocation, for callers that
 * cannot allocate: code being captured into a HIP graph, tight serving loops, harnesses that
 * forbid hipMalloc.  y = G A x in double precision on the N grid (GaNi), for the coefficients
 * given as in fgh_plan_create (A device, or phase device + phase_table host, n_phases <= 16;
 * phase values must be below n_phases and are not checked).  x, y: device double[d][N grid], not
 * overlapping; the caller owns them.  The passes' intermediate buffers (twiddle tables computed on
 * the device, two half-spectrum buffers, partial sums) live in a 64 MiB array of device memory
 * that the library holds on each GPU it runs on until the process ends: grids whose buffers do
 * not fit it (about 111^3 and above in 3D; 2D up to beyond 1000^2) are rejected with
 * FGH_E_WORKSPACE.  Every call on one GPU uses that GPU's array, so calls that overlap in time on
 * one GPU (other streams, other threads) race and must be serialised by the caller; nothing in the
 * array needs to start at zero.  Static tile choices (no plan-time timing).  Asynchronous on
 * `stream` (NULL: the default stream).  Errors: FGH_E_INVALID, FGH_E_WORKSPACE, FGH_E_DEVICE. */
fgh_status fgh_apply_noalloc(int d, const int32_t* N, fgh_akind a_kind, const void* A, const uint8_t* phase,
                             const double* phase_table, int n_phases, const double* x, double* y,
                             void* stream);

/* Write the double-grid coefficients A_{2N-1} of a Ga plan (eq:Ga_exact_integration) to device
 * double[ncoef_op][M grid], where ncoef_op is 1 for FGH_A_ISO / FGH_A_PHASE (A_{2N-1} is a
 * scalar field times I) and 3 or 6 packed symmetric entries for FGH_A_SYM.  FGH_E_INVALID for
 * GaNi plans.  Blocks. */
fgh_status fgh_ga_coefficients(fgh_plan plan, double* out);

/* Solve C e = b for nrhs loads E (host double[nrhs][d]), each independently (Algorithms 1-4):
 *   Richardson: x0 = 0, stop when ||x_m - x_{m-1}||_2 <= tol |E|.
 *   CG, Chebyshev: x0 = 0, stop when ||r_m||_2 <= tol ||b||_2 (recursive residual); if
 *     ||b||_2 <= 1e-12 ||A E||_2 the load is taken as b = 0 and returns e = 0, iters = 0.
 *   Eyre-Milton: x0 = E, x_m = (A + wI)^{-1}[F^{-1}(I - 2G^)F (A - wI) x_{m-1} + 2wE], stop
 *     when ||x_m - x_{m-1}||_2 <= tol |E|; the returned fluctuation is x_m - E.
 * e: device double[nrhs][d][grid] output.  tol in (0,1).  max_iter >= 1 caps loop bodies
 * (inner bodies per outer step for FGH_FP32_REFINED).  stats: host fgh_stats[nrhs] or NULL.
 * FGH_FP32_REFINED: outer FP64 residual r = b - C x, inner FP32 solve of C delta = r to the
 * relative tolerance max(tol_abs/||r||, 1e-4) by the same solver, then x += G delta in FP64;
 * stops on the true FP64 residual ||b - C x|| <= tol ||b|| (CG, Chebyshev), on the FP64 step
 * Richardson would take next, w ||b - C x|| <= tol |E| (Richardson; that step is taken, so the
 * test is Algorithm 1's own), or on the outer step norm (Eyre-Milton).  rel_res_recursive is then
 * the stopping-test quantity of the last outer step.  Blocks until done.  Returns the worst load
 * status. */
fgh_status fgh_solve(fgh_plan plan, fgh_solver solver, const double* E, int nrhs, double tol,
                     int max_iter, double* e, fgh_stats* stats);

/* Same as fgh_solve with the iteration count fixed: exactly `iters` loop bodies per load, the
 * stopping test skipped (iterate-matched comparisons).  FGH_FP64 plans only. */
fgh_status fgh_solve_fixed(fgh_plan plan, fgh_solver solver, const double* E, int nrhs,
                           int iters, double* e, fgh_stats* stats);

/* Several independent solves of one shape at once (serving; not a method of the paper): plans[k]
 * (distinct, same d, N, rule and precision) each solve C e = b for the load E[k] (host
 * double[n][d]) to tol[k] with `solver`, as fgh_solve on that plan with nrhs = 1 would; e[k]:
 * device double[d][grid] output of plan k.  For FGH_FP32_REFINED plans of a size-specialised
 * grid (45, 63, 81, 125, 135, 243 along every axis) with conjugate gradients or Eyre-Milton and
 * n >= 2, the inner FP32 loop bodies of up to 8 members run in shared launches (one launch per pass for all
 * of them, one grid row per member) while each member's outer FP64 steps stay its own; a
 * member's iterates, counts and results are bitwise those of fgh_solve on its plan alone.  Other
 * combinations solve the members one after another.  retire (may be NULL) is called as
 * retire(user, k) on the calling thread as soon as member k's e[k] and stats[k] are final, before
 * the others have finished; plan k is back on its own stream then, and for k >= 1 it and its
 * buffers are no longer used by this call (the callback may release them).  Plan 0 hosts the
 * shared stream and must stay alive until the call returns.  All work runs on plans[0]'s internal
 * stream after every member's stream has drained; blocks until done; the captured loop graph of
 * any member may be replaced.  stats: host fgh_stats[n] or NULL.  Returns the
 * worst member status; FGH_E_INVALID for mismatched, repeated or NULL plans, n outside [1, 64]
 * or a tolerance outside (0, 1). */
typedef void (*fgh_retire_fn)(void* user, int member);
fgh_status fgh_solve_batch(fgh_plan* plans, int n, fgh_solver solver, const double* E, const double* tol,
                           int max_iter, double* const* e, fgh_stats* stats, fgh_retire_fn retire,
                           void* user);

/* Effective quantities from solved fluctuations (eq:ev_bounds), accumulated in double:
 *   bilinear  host double[nrhs][nrhs] (may be NULL): B[i][j] = (A(E_j + e_j), E_i + e_i)_2;
 *             with the d unit loads this is A_H (eq:ev_bounds_Ga / eq:GaNi).
 *   flux      host double[nrhs][d] (may be NULL): <A(E_j + e_j)>, the flux column of load j.
 * E: host double[nrhs][d]; e: device double[nrhs][d][grid] as written by fgh_solve.
 * Sums run over the integration grid (the double grid for Ga).  Blocks. */
fgh_status fgh_effective(fgh_plan plan, const double* E, int nrhs, const double* e,
                         double* bilinear, double* flux);

/* Loop history of later fgh_solve / fgh_solve_fixed calls on an FGH_FP64 plan (Sec. 4.2 residual
 * histories; Sec. 4.3, eq:guar_upper_bound_m, the energy of each iterate; Sec. 4.4 the
 * non-conformity).  For load j and loop body m (m = 0: the initial iterate) the entry at
 * j * capacity + (m mod capacity) of each array given receives
 *   res_hist     the stopping-test quantity relative to its scale: ||r_m|| / ||b|| (CG,
 *                Chebyshev; 1 at m = 0, 0 for a load taken as b = 0) or ||x_m - x_{m-1}|| / |E|
 *                (Richardson, Eyre-Milton; 1 at m = 0);
 *   energy_hist  U_E(x_m) = (A(E + e_m), E + e_m)_2 on the integration grid (for Eyre-Milton the
 *                whole iterate x_m in place of E + e_m); with `ga` set (a Ga plan on the same N,
 *                this plan GaNi) instead the guaranteed bound of the iterate,
 *                (A_{2N-1}(E + R G_N e_m), E + R G_N e_m) on the double grid (eq:ev_bounds_GaNi),
 *                which costs about two more operator applications per body.  For the conforming
 *                solvers U_E(x_m) - U_E(x*) is the squared energy-norm error of Sec. 4.5;
 *   nonconf_hist ||G e_m - e_m||_2 with e_m the fluctuation (x_m - E for Eyre-Milton; G removes
 *                the mean, so this is ||G x_m + E - x_m||), the non-conformity of Sec. 4.4 (G with
 *                the band of the plan's rule);
 *   mean_hist    |<e_m>|, the mean-value part of the orthogonal split of the non-conformity; the
 *                zero-mean part is sqrt(nonconf^2 - mean^2).  These two cost one more operator
 *                application per body, and `scratch` (device double[d][grid], the integration
 *                grid) to hold G e_m; FGH_E_INVALID without it.
 * Arrays: device double[nrhs][capacity], any of them NULL; all NULL (with ga NULL) turns
 * recording off.  The arrays and `ga` must stay alive while recording is on; the Ga plan's
 * spectrum and two FP64 vectors are overwritten.  Entries for m beyond the last body are left
 * untouched; the stats' iters tell how many are valid.  FGH_E_UNSUPPORTED for FGH_FP32_REFINED
 * plans, FGH_E_INVALID for capacity < 1 or mismatched plans. */
fgh_status fgh_plan_set_history(fgh_plan plan, double* res_hist, double* energy_hist, double* nonconf_hist,
                                double* mean_hist, double* scratch, int capacity, fgh_plan ga);

/* Guaranteed upper bound of the GaNi solution (Sec. 2.3, eq:ev_bounds_GaNi; Sec. 4.3): the GaNi
 * fluctuation e_N is read as a trigonometric polynomial, so its prolongation R e_N to the double
 * grid 2N-1 (interpolate on N, evaluate on 2N-1) is conforming and the exactly integrated energy
 *   bound = (A_{2N-1}(E + R e_N), E + R e_N)_{2N-1}
 * bounds (A_H E, E) from above (eq:bounds).
 * gani: a GaNi plan; ga: a Ga plan on the same N and microstructure (it supplies A_{2N-1} and is
 * used as scratch: its spectrum and one FP64 vector are overwritten).  E: host double[d];
 * e: device double[d][N grid] (e.g. from fgh_solve on `gani`).  bound: host double.  Waits for
 * the GaNi plan's stream, runs on the Ga plan's stream and blocks.  FGH_E_INVALID when the
 * rules, d or N do not match. */
fgh_status fgh_gani_bound(fgh_plan gani, fgh_plan ga, const double* E, const double* e,
                          double* bound);

/* Adaptive spectral bounds: an extension of this library, not a method of the paper.  The paper's
 * Richardson, Chebyshev and Eyre-Milton take their parameters from the pointwise bounds c_A, C_A
 * of eq:A (Algorithms 1, 3, 4); its closing outlook (Sec. 5) names a more robust Chebyshev method
 * as further work but gives no estimate.  This entry point estimates the spectrum of C from the CG
 * coefficients (the Lanczos connection of CG), for use with fgh_plan_set_bounds.  Runs up to `iters` bodies of Algorithm 2 in
 * double precision on C e = b, b = -G A E (eq:linsys), from e = 0.  The CG coefficients alpha_k,
 * beta_k = ||r_{k+1}||^2 / ||r_k||^2 define the Lanczos matrix T_m of C on the Krylov space
 * K_m(C, b):
 *   T[0][0] = 1/alpha_0,  T[k][k] = 1/alpha_k + beta_{k-1}/alpha_{k-1},  T[k][k+1] = sqrt(beta_k)/alpha_k,
 * whose eigenvalues (Ritz values) lie inside the spectrum of C on compatible fields, itself
 * inside [c_A, C_A] (eq:A).  lo and hi receive the smallest and largest Ritz value (Sturm
 * bisection on the host); they approach the extreme eigenvalues from inside as m grows.
 *   E      host double[d] load (b must be nonzero: FGH_E_INVALID for a homogeneous medium).
 *   iters  1 .. 4096 CG bodies; fewer are taken when ||r_m|| <= 1e-14 ||b|| (K_m invariant).
 *   e      device double[d][grid]: receives the CG iterate after the last body taken.
 *   tri    host double[2 * iters] or NULL: T's diagonal in [0, m), its off-diagonal in
 *          [iters, iters + m - 1); the rest zero.
 *   steps  host int or NULL: m, the bodies taken.
 * Synchronises once per body.  Overwrites the plan's CG vectors.  The plan's own bounds are not
 * changed: see fgh_plan_set_bounds.  FGH_E_NOT_SPD if (C b, b) <= 0. */
fgh_status fgh_estimate_bounds(fgh_plan plan, const double* E, int iters, double* e, double* tri,
                               int* steps, double* lo, double* hi);

/* Replace the spectral bounds a plan's Richardson, Chebyshev and Eyre-Milton use (Algorithms 1,
 * 3 and 4: omega = 2/(c_A + C_A), the interval [c_A, C_A], omega = sqrt(c_A C_A)); e.g. estimates
 * from fgh_estimate_bounds, widened by a margin since Ritz values lie inside the spectrum.
 * Chebyshev still converges for eigenvalues outside [c_A, C_A] as long as all lie in
 * (0, c_A + C_A).  Eyre-Milton contracts with (A - w I)(A + w I)^{-1} pointwise, so its rate is
 * set by the pointwise eigenvalues of A, and bounds narrower than those can slow it down.
 * Waits for the plan's stream.  FGH_E_INVALID unless 0 < c_A <= C_A < inf. */
fgh_status fgh_plan_set_bounds(fgh_plan plan, double c_A, double C_A);

/* Per-pass device timing (profiling aid, off by default).  `enable` is a bit mask of launch kinds
 * -- bit 0 first (A multiply + forward transform of the last axis), bit 1 forward strided axis,
 * bit 2 middle (transform of axis 0 with the Fourier multiplier), bit 3 inverse strided axis,
 * bit 4 last (inverse transform of the last axis + solver epilogue; in fused loops also the next
 * body's first pass), bit 5 CG update (r -= alpha q, (r, r), and x += alpha p unless the next
 * body's first pass applies it), bit 6 single-workgroup
 * loop reductions; 0 turns timing off.  Every launch of a selected kind is bracketed by HIP events
 * on the stream it runs on and its duration accumulated; solver loops then run without graph
 * replay.  Enabling resets the counters. */
fgh_status fgh_plan_set_profiling(fgh_plan plan, int enable);

/* Accumulated milliseconds and launch counts per launch kind (arrays of 7) over the launches that
 * did work: solver-loop launches issued after the device-side stopping test has fired return at
 * once, and launches shorter than 30 % of their kind's median are left out.  Times are those of
 * the dispatches themselves (start and stop events attached to the launch).  Synchronises. */
fgh_status fgh_plan_read_profile(fgh_plan plan, double* ms, int64_t* launches);

/* ------------------------------------------------------------------------------------------
 * Serving.  Solves of mixed d, N, rule, contrast, solver and tolerance are submitted as they
 * arrive and run by a pool of worker slots, each with its own HIP stream; the fields and solver
 * state of an admitted request stay in HBM until it retires.  A request is admitted (FIFO) once
 * its footprint -- plan workspace, fluctuation field on the integration grid (the 2N-1 grid for
 * Ga), phase map -- fits into the free part of the caller's device pool; concurrently running
 * requests overlap on the device.  A slot that admits a request whose shape shares launches
 * (FP32_REFINED CG or Eyre-Milton on a size-specialised grid of at most 262144 points, see
 * fgh_solve_batch) also admits up to 7 queued requests of the same size class (d, N, rule,
 * precision, solver, max_iter) whose predicted work is within a factor 2 of its own (sqrt(C_A /
 * c_A) log(2 / tol); C_A / c_A from the request or its phase table; a group runs until its
 * slowest member is done) and that fit the pool, and solves them together; each retires --
 * result posted, pool memory freed -- as soon as its own solve has finished.  Each request's arithmetic is that of fgh_solve on its own plan,
 * so its result does not depend on what else is in flight (bitwise).  The coefficients of a request are a
 * phase map (host uint8, copied at submission) and a phase table, as for FGH_A_PHASE.
 * ------------------------------------------------------------------------------------------ */
typedef struct fgh_server_s* fgh_server;

typedef struct {
    int32_t d;
    int32_t N[3];
    int32_t rule;          /* fgh_rule */
    int32_t precision;     /* fgh_precision */
    int32_t solver;        /* fgh_solver */
    int32_t max_iter;
    double tol;
    double E[3];
    const uint8_t* phase;  /* host [N grid], copied by fgh_server_submit */
    const double* phase_table; /* host [n_phases][ncoef], copied */
    int32_t n_phases;
    int32_t pad;
    double c_A, C_A;       /* <= 0: derived from the phases present */
} fgh_request;

typedef struct {
    int64_t id;
    int32_t status;        /* fgh_status of the solve */
    int32_t iters, outer_iters, pad;
    double energy;         /* (A(E + e), E + e)_2 */
    double flux[3];        /* <A(E + e)> */
    double rel_res_true;
    double t_submit, t_admit, t_done;  /* seconds since fgh_server_create */
    double solve_seconds;
} fgh_result;

/* Pool bytes a request holds while admitted. */
fgh_status fgh_request_footprint(const fgh_request* request, size_t* bytes);

/* Create a server over the device pool [pool, pool + pool_bytes) (256-byte aligned, caller-owned,
 * on device `device`) with max_active worker slots (1..16). */
fgh_status fgh_server_create(fgh_server* out, void* pool, size_t pool_bytes, int max_active, int device);

/* Queue a request (thread-safe, non-blocking).  FGH_E_WORKSPACE if it can never fit the pool,
 * FGH_E_UNSUPPORTED for Eyre-Milton with Ga, FGH_E_INVALID for bad fields. */
fgh_status fgh_server_submit(fgh_server server, const fgh_request* request, int64_t* id);

/* FGH_OK and the result if request `id` has finished (the result is then released: a later poll or
 * wait on the same id returns FGH_E_INVALID), FGH_E_NO_CONVERGENCE while it is pending,
 * FGH_E_INVALID for an id that was never issued or whose result was already returned. */
fgh_status fgh_server_poll(fgh_server server, int64_t id, fgh_result* out);

/* Block until request `id` has finished and return its result (released as by fgh_server_poll).
 * FGH_E_INVALID at once for an id that was never issued or whose result was already returned
 * (also when another thread takes the same result first). */
fgh_status fgh_server_wait(fgh_server server, int64_t id, fgh_result* out);

/* Block until every submitted request has finished. */
fgh_status fgh_server_drain(fgh_server server);

/* Server clock, peak pool bytes in use and peak number of concurrently active requests. */
fgh_status fgh_server_stats(fgh_server server, double* now_seconds, size_t* peak_pool_bytes, int* peak_active);

/* Size-class batching: the largest group of requests admitted together and the number of groups
 * (a request admitted alone counts as a group of one). */
fgh_status fgh_server_batch_stats(fgh_server server, int* peak_batch, int64_t* batches);

/* Stop the workers after the requests already admitted; requests still queued are discarded: their
 * result has status FGH_E_CANCELLED, and threads blocked in fgh_server_wait on them return it.
 * Returns once those threads have left; no other call on the server may start after this one. */
void fgh_server_destroy(fgh_server server);

const char* fgh_status_string(fgh_status status);

#ifdef __cplusplus
}
#endif

#endif /* FGH_H */
