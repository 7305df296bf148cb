/*
 * wc.h -- C ABI of the MI355X (gfx950) block omega-circulant solver library.
 *
 * The library solves the all-at-once theta-method optimality system of the
 * parabolic tracking problem of Fung & Hon, "Block omega-circulant
 * preconditioners for parabolic optimal control problems":
 *
 *   min 1/2 ||y - g||^2 + gamma/2 ||u||^2  s.t.  y_t - div(a grad y) = f + u,
 *   y = 0 on the boundary, y(0) = y0                     (Section 1, eqn:heat)
 *
 * discretised with the theta-method in time (theta = 1 backward Euler,
 * theta = 1/2 Crank-Nicolson) and conservative finite differences in space
 * (M = I, K = -L_h), on the unit interval or square with h = 1/(M+1),
 * tau = T/n (Section 1, eqn:main_system_before).  The unknown of the
 * transformed systems is x = [sqrt(gamma) y_tilde; p_tilde] (eqn:main_system).
 *
 * Methods (Section 4 naming):
 *   WC_MINRES_ABS_PS : MINRES on A (eqn:matrix_A) with |P_S| (eqn:matrix_P)
 *   WC_MINRES_PMS    : MINRES on A with P_MS (eqn:matrix_P_MS)
 *   WC_GMRES_PS      : right-preconditioned GMRES(restart) on A_hat
 *                      (eqn:matrix_A_hat) with P_S (eqn:matrix_P_GMRES)
 *
 * Conventions shared by every entry point:
 *  - Array arguments are DEVICE pointers to FP64 data owned by the caller
 *    (the library never frees them).  Host pointers are named *_host.
 *  - Space-time arrays are time major: element (k, s) at k*m + s, with the
 *    spatial index s = x2*M + x1 (x1 fastest), m = M^dims.
 *  - A "system vector" has 2*n*m doubles: block row 1 then block row 2, each
 *    an (n, m) time-major array (time slices 1..n).
 *  - Work is enqueued on the plan's HIP stream (hipStream_t passed as void*;
 *    NULL = the default stream).  wc_rhs, wc_matvec, wc_pc_apply and
 *    wc_recover are asynchronous; wc_krylov and wc_solve return after the
 *    solve has finished (they synchronise the plan's stream).
 *  - Every call returns a wc_status and never aborts.  Arguments are checked
 *    before any launch.  A plan is not thread safe: calls on one plan must
 *    be serialised by the caller.
 */
#ifndef WC_H_
#define WC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WC_OK = 0,
  WC_E_ARG = 1,          /* invalid argument (sizes, theta, gamma, NULL pointer, ...) */
  WC_E_SINGULAR_S2 = 2,  /* S_n^(2) singular and s2_remedy == 0 (remark in Section 1) */
  WC_E_NOMEM = 3,        /* device allocation failed */
  WC_E_MAXIT = 4,        /* maxit reached; the last iterate is still written */
  WC_E_BREAKDOWN = 5,    /* Krylov breakdown (non-positive preconditioned norm) */
  WC_E_NONFINITE = 6,    /* NaN/Inf met in a Krylov scalar */
  WC_E_CANCELLED = 7,    /* request cancelled (server) */
  WC_E_ADMISSION = 8,    /* request larger than the server's memory budget */
  WC_E_UNSUPPORTED = 9,  /* valid problem outside what the GPU path implements */
  WC_E_HIP = 10,         /* a HIP runtime call failed */
  WC_E_INTERNAL = 11
} wc_status;

typedef enum { WC_MINRES_ABS_PS = 0, WC_MINRES_PMS = 1, WC_GMRES_PS = 2 } wc_method;

/* Arithmetic of the preconditioner apply.  The Krylov recurrence, inner
 * products, the all-at-once matvec and all tables are FP64 in both modes. */
typedef enum { WC_FP64 = 0, WC_MIXED = 1 } wc_precision;

/* Spatial discretisation (Section 1: mass M_m and stiffness K_m).  WC_FD: finite
 * differences, M_m = I, K_m = -L_h (any a).  WC_FEM: continuous linear (1D) / bilinear (2D)
 * elements on the same grid with a == 1, consistent mass M_m and stiffness K_m; the system
 * is solved after the change of variables of eqn:main_system, whose spatial operator is
 * M_m^{-1/2} K_m M_m^{-1/2}.  Both matrices are diagonal in the orthonormal sine basis U
 * (U M1 U = diag(h/3 (2 + cos(j pi h))), U K1 U = diag(2/h (1 - cos(j pi h)))), so a
 * WC_FEM plan works in sine coordinates: the system vectors of wc_rhs (its output),
 * wc_matvec, wc_pc_apply, wc_krylov and wc_recover (its input) are (I (x) U) times the
 * physical ones, the preconditioner apply is its time transform, the per-mode solves and
 * the inverse time transform, and wc_rhs / wc_recover transform the data and the solution
 * (f, g, y0 in and y, p, u out stay physical nodal values). */
typedef enum { WC_FD = 0, WC_FEM = 1 } wc_disc;

/* Boundary data (Section 1: homogeneous Dirichlet; Section 4, Example 3: homogeneous
 * Neumann).  WC_NEUMANN: finite differences with constant a (= kappa), on M nodes per
 * dimension that include both boundary nodes (x_j = j h, h = 1/(M-1), m = M^dims);
 * Neumann data by mirrored ghost nodes, so K_m is not symmetric and the same K_m sits
 * in the state and adjoint block rows: the system is solved by GMRES-P_S only.  K_m is
 * diagonalised by the cosine matrix C[j][k] = cos(j k pi/(M-1)), not orthogonal, with
 * C^{-1} = (2/(M-1)) W C W (W the trapezoidal weights); the preconditioner's spatial
 * step applies C^{-1} and C as dense transforms along x1 and x2 (any M from 2 to 1024). */
typedef enum { WC_DIRICHLET = 0, WC_NEUMANN = 1 } wc_bc;

/* The discrete problem (Section 1 and the Section 4 protocol). */
typedef struct {
  int dims;           /* 1 or 2 */
  int M;              /* interior points per dimension; h = 1/(M+1); m = M^dims */
  int n;              /* time steps; tau = T/n */
  double T;           /* final time, > 0 */
  double theta;       /* 1/2 <= theta <= 1 (Section 1) */
  double gamma;       /* regularisation, > 0 */
  double zeta;        /* omega = exp(i zeta); the paper's experiments use pi */
  double s2_remedy;   /* value replacing a zero eigenvalue of S_n^(2); 0 => error */
  const double *a_face_host;  /* HOST pointer or NULL (a == 1).  Diffusion
                         coefficient at cell-face midpoints: 1D M+1 values at
                         (i+1/2)h; 2D faces normal to x1 as an (M, M+1) array
                         [x2 node][x1 face] followed by faces normal to x2 as
                         an (M+1, M) array [x2 face][x1 node].  Copied at plan
                         creation. */
  int disc;           /* wc_disc (0 = finite differences); WC_FEM needs a_face_host NULL
                         and no low-rank form */
  int bc;             /* wc_bc (0 = Dirichlet) */
  double kappa;       /* constant a (K_m scaled by kappa) when a_face_host is NULL; 0 is
                         read as 1; must be 0 or 1 with a_face_host */
} wc_problem;

typedef struct {
  int method;         /* wc_method */
  int precision;      /* wc_precision */
  double tol;         /* stop when ||b - A x||_2 / ||b||_2 <= tol (true residual) */
  int maxit;          /* total Krylov iteration cap */
  int restart;        /* GMRES restart length (1..32) */
  int flexible;       /* GMRES: store preconditioned basis (forced on for WC_MIXED) */
  int mg_max_cycles;  /* multigrid V-cycles per spatial solve (variable a) */
  double mg_tol;      /* multigrid relative residual target (variable a); 0 = exactly
                         mg_max_cycles cycles */
  int graphs;         /* 1: replay each Krylov iteration's launches from a captured
                         hipGraph (cached per plan; not while profiling, and for
                         variable a only with mg_tol = 0) */
  int lowrank;        /* GMRES-P_S with a = 1, FP64: run the Arnoldi process in the
                         compact coordinates given by the GMRES proposition (Sec. 3):
                         Ahat - P_S acts only in time and has rank one per block row,
                         so every Krylov vector is c r0_perp + [g (x) s1; r (x) s2].
                         Same iterates; the basis takes (restart+1)(1+2m) doubles and
                         each step is one preconditioner apply whose last pass
                         contracts over time.  WC_E_ARG with any other method,
                         precision or a variable coefficient. */
} wc_opts;

typedef struct {
  int status;         /* wc_status of the solve */
  int iters;          /* Krylov iterations */
  int restarts;       /* GMRES cycles / MINRES true-residual restarts */
  double relres;      /* explicit ||b - A x||_2 / ||b||_2 at exit (FP64) */
  double relres_est;  /* recurrence estimate at exit */
  double ms;          /* wall time of the Krylov solve */
  int mg_cycles_max;  /* largest V-cycle count of any spatial solve (variable a) */
  int reorth;         /* GMRES: iterations that needed a second Gram-Schmidt pass */
} wc_info;

typedef struct wc_plan wc_plan;

/* Human-readable name of a status code (static string). */
const char *wc_status_str(int status);

/* Defaults: GMRES_PS, FP64, tol 1e-8, maxit 500, restart 30, flexible 0,
 * mg_max_cycles 30, mg_tol 1e-10, graphs 1, lowrank 0. */
void wc_opts_default(wc_opts *opts);

/* Device bytes a plan for (problem, opts) allocates (tables, spectral
 * workspaces, Krylov vectors).  Returns 0 if the arguments are invalid. */
size_t wc_plan_footprint_bytes(const wc_problem *prob, const wc_opts *opts);

/* Validate, build the FP64 eigenvalue / twiddle tables (Section 1 remark on
 * S_n^(2) and Section 3.4), upload them, allocate workspaces.  *out is set to
 * NULL on failure.  stream: hipStream_t or NULL.  WC_FEM problems need the
 * preconditioner's coverage (zeta == pi, n and M+1 powers of two in [4, 1024]),
 * else WC_E_UNSUPPORTED. */
wc_status wc_plan_create(const wc_problem *prob, const wc_opts *opts, void *stream,
                         wc_plan **out);
wc_status wc_plan_destroy(wc_plan *plan);
/* Re-point a plan at another problem of the same shape without allocating: same
 * dims, M, n, method, precision, restart, flexible, lowrank, disc and bc, a_face_host
 * given iff it was at creation, and the same preconditioner path (the FFT path or the
 * general path) (WC_E_ARG otherwise).  theta, gamma, T, zeta, s2_remedy, kappa, the
 * coefficient values and the remaining options may change; every table is rebuilt.
 * Synchronises the plan's stream first.  On an error other than WC_E_ARG the plan
 * refuses solves until a retarget succeeds. */
wc_status wc_plan_retarget(wc_plan *plan, const wc_problem *prob, const wc_opts *opts);
/* Later calls of the plan run on stream; the old stream is synchronised first. */
wc_status wc_plan_set_stream(wc_plan *plan, void *stream);
/* Times the preconditioner apply (reps applies per candidate, after one warm-up)
 * for every time-pass choice and, in 2D with a = 1, every x2-pass choice (the values
 * of wc_plan_set_tiles), keeps the fastest pair in the plan and reports it (ts, tx may
 * be NULL).  Uses the plan's Krylov vectors as scratch: call it between solves.
 * Synchronous. */
wc_status wc_plan_autotune(wc_plan *plan, int reps, int *ts, int *tx);
/* Sets the preconditioner's kernel choices directly (e.g. to reuse a choice autotuned on
 * another plan): ts for the time passes (4, 8, 16: tiles of that many spatial columns
 * with both block rows packed in one complex sequence; -8, -16, -32: tiles of 8, 16 or 32
 * columns of one block row, each transformed as an n/2-point sequence, n >= 64; -32 runs
 * as -16 where its tile exceeds the CU's LDS, FP64 at n = 1024), tx for the
 * 2D x2 pass (4, 8, 16: tiles of that many x1 columns; -4, -8: x1 passes that write a
 * transposed copy in tiles of 4 or 8 rows and an x2 pass on its contiguous rows, M+1 >=
 * 128); 0 = default.  WC_E_ARG for other values.  Synchronises the plan's stream. */
wc_status wc_plan_set_tiles(wc_plan *plan, int ts, int tx);

/* Right-hand side of the transformed system (Section 1: f_tilde, g_tilde
 * with M = I; eqn:main_system / eqn:main_system_nonsym).
 * f, g: (n+1)*m samples at time levels 0..n; y0: m values; b: 2*n*m out.
 * MINRES methods get b = [g_tilde; sqrt(gamma) f_tilde], GMRES gets
 * [sqrt(gamma) f_tilde; g_tilde]. */
wc_status wc_rhs(wc_plan *plan, const double *f, const double *g, const double *y0,
                 double *b);

/* y = A x (MINRES methods) or y = A_hat x (GMRES), x and y of 2*n*m doubles,
 * distinct buffers (eqn:matrix_A, eqn:matrix_A_hat; time factor
 * B_n = (B^(2))^{-1} B^(1) applied by its two-term recurrences). */
wc_status wc_matvec(wc_plan *plan, const double *x, double *y);

/* w = P^{-1} v for the plan's preconditioner (|P_S|, P_MS or P_S) by the
 * three-step procedure of Section 3.4: omega-scaled time FFT, independent
 * spatial problems per frequency, inverse transform.  v, w: 2*n*m doubles,
 * may alias.  Arithmetic in FP64 or FP32 per opts.precision.
 * Paths: zeta == pi with n and M+1 powers of two in [4, 1024] (Dirichlet; Neumann: n a
 * power of two, any M) run the FFT path (half spectrum, sine transforms, multigrid for
 * variable a).  Other n <= 1024, M <= 1024 or zeta with constant-coefficient finite
 * differences run the general path: the time step as a dense product over all n
 * frequencies, dense spatial steps, and the real part of P^{-1} v (for zeta not in
 * {0, pi} P_S is complex; the real part is the preconditioner of the real system).  In
 * 2D with Dirichlet data, n a power of two in [4, 1024] and M+1 one in [128, 1024], the
 * general path takes n-point FFTs over all n frequencies and the FFT path's sine passes
 * instead of the dense products (same result to rounding).
 * Variable a and finite elements need the FFT path (WC_E_UNSUPPORTED otherwise). */
wc_status wc_pc_apply(wc_plan *plan, const double *v, double *w);

/* Recover y (levels 1..n), p (levels 0..n-1), each n*m doubles, from
 * x = [sqrt(gamma) B^(2) y; (B^(2))^T p] (eqn:main_system).  u (optional,
 * may be NULL) receives p/gamma, the control (u = p/gamma, eqn:heat_2). */
wc_status wc_recover(wc_plan *plan, const double *x, double *y, double *p, double *u);

/* Solve the transformed system for right-hand side b (2*n*m) into x (2*n*m,
 * overwritten; zero initial guess).  Synchronous.  info may be NULL. */
wc_status wc_krylov(wc_plan *plan, const double *b, double *x, wc_info *info);

/* Whole path: wc_rhs, wc_krylov, wc_recover.  y, p: n*m each; u optional.
 * Synchronous.  Returns the solve status (WC_E_MAXIT still writes y, p). */
wc_status wc_solve(wc_plan *plan, const double *f, const double *g, const double *y0,
                   double *y, double *p, double *u, wc_info *info);

/* ---- per-kernel timing (tracing) --------------------------------------------
 * wc_profile(plan, 1) clears and starts recording a hipEvent pair around every
 * kernel the plan launches on its stream; wc_profile(plan, 0) stops.
 * wc_profile_read synchronises the stream, folds the recorded pairs into one
 * entry per kernel family (launch count, summed duration) and writes at most
 * `max` entries to `out` (host memory); returns the number of entries, or -1
 * on error.  Recording adds no synchronisation to the solve.  `bytes` is the
 * summed algorithmic HBM traffic of the family's launches: the bytes each
 * launch must read and write at minimum (operands once, results once). */
typedef struct {
  char name[32];
  int launches;
  double total_ms;
  double bytes;
} wc_kernel_stat;

wc_status wc_profile(wc_plan *plan, int enable);
int wc_profile_read(wc_plan *plan, wc_kernel_stat *out, int max);

/* ---- serving ------------------------------------------------------------------
 * A server runs submitted requests on the device current at wc_server_create:
 *  - GMRES(k)-P_S requests in the standard form (lowrank 0) on 2D grids with a == 1,
 *    zeta == pi and n, M+1 in {64, 128, 256, 512} are continuously batched: one
 *    batcher thread advances every active solve by one Krylov step per round, with the
 *    preconditioner of all of them applied in one launch per pass (the batched applies
 *    below); queued requests join at the next round boundary (up to 32 active) and a
 *    solve leaves in the round it converges;
 *  - every other request runs a whole solve (wc_solve) on one of the worker threads,
 *    each with its own HIP stream, so requests of different sizes share the GPU at
 *    kernel granularity.
 *
 * Admission by HBM footprint: a request needs wc_plan_footprint_bytes(prob,
 * opts) of device memory for its plan; requests start in submission order while
 * the plans of running requests plus the idle plan cache fit in hbm_budget
 * bytes (idle plans are freed first when room is needed).  A request whose own
 * footprint exceeds the budget is refused at submission (WC_E_ADMISSION).
 * Plans are kept after a request and reused, through wc_plan_retarget, for a
 * later request of the same shape (no device allocation then).
 *
 * f, g, y0, y, p, u are device pointers as for wc_solve; the caller keeps them
 * valid and untouched until the request is done, and makes sure the inputs are
 * complete (e.g. synchronises its stream) before submitting.  The problem
 * struct and a_face_host are copied at submission.  Results are bitwise those
 * of the same wc_solve run alone: the kernels' reductions have a fixed order. */
typedef struct wc_server wc_server;

/* max_concurrency: worker threads (1..64).  hbm_budget: bytes (0 = 90% of the
 * device memory free at creation). */
wc_status wc_server_create(size_t hbm_budget, int max_concurrency, wc_server **out);
/* Waits for running requests, cancels queued ones, frees every plan.  No other
 * call on the server may be in progress or follow. */
wc_status wc_server_destroy(wc_server *srv);
wc_status wc_server_submit(wc_server *srv, const wc_problem *prob, const wc_opts *opts,
                           const double *f, const double *g, const double *y0, double *y,
                           double *p, double *u, uint64_t *ticket);
/* *done = 1 once the request finished (then info, if not NULL, holds its wc_info,
 * whose status field is the solve's wc_status).  Returns WC_E_ARG for an unknown
 * ticket. */
wc_status wc_server_poll(wc_server *srv, uint64_t ticket, int *done, wc_info *info);
/* Blocks until the request is done; like wc_server_poll otherwise.  queue_ms:
 * submission to start; total_ms: submission to completion (host clock); either
 * may be NULL.  The ticket is released by this call. */
wc_status wc_server_wait(wc_server *srv, uint64_t ticket, wc_info *info, double *queue_ms,
                         double *total_ms);
/* Removes a request that has not started (its status becomes WC_E_CANCELLED);
 * returns WC_E_ARG if it is unknown or already running or done. */
wc_status wc_server_cancel(wc_server *srv, uint64_t ticket);
/* Device bytes the server holds in plans (running plus idle). */
size_t wc_server_bytes_in_use(wc_server *srv);
/* Continuous batching statistics: requests served by the batcher so far and the largest
 * number of solves active in one of its rounds (either pointer may be NULL). */
wc_status wc_server_stats(wc_server *srv, uint64_t *batched, int *max_active);

/* ---- batches: many right-hand sides and instances in one launch per pass ---------
 * The preconditioner apply of the three-step decomposition (time transform, spatial
 * sine transforms with the per-mode 2x2 solves, inverse transforms; Section 3 and the
 * P_S / |P_S| / P_MS applies of Section 4) for up to 32 instances at once: each pass
 * is one kernel launch over the work units of every instance (per precision class,
 * FP64 or mixed), whatever their grid M and steps n.  Many right-hand sides of one
 * problem are several plans of that problem.
 *
 * wc_batch_create: plans[0..count) (1 <= count <= 32), distinct plans, each 2D finite
 * differences with a == 1 (a_face NULL), n and M+1 in {64, 128, 256, 512}; otherwise WC_E_ARG (null,
 * repeated plan, count out of range) or WC_E_UNSUPPORTED.  The batch borrows the plans
 * (their spectral workspaces and tables): they must outlive it and must not be
 * retargeted while it exists.  Every call runs on the plans' stream, which must be the
 * same for all of them at the time of the call (else WC_E_ARG).
 *
 * wc_batch_pc_apply: w[i] = P_i^{-1} v[i] (device pointers, 2*n_i*m_i doubles each,
 * v[i] != w[i]); stream-ordered and asynchronous, results equal to wc_pc_apply's for
 * each plan.
 *
 * wc_batch_solve: wc_solve for every instance (f, g, y0, y, p arrays of device
 * pointers, one per plan, sizes as for wc_solve) by GMRES(k)-P_S in the standard
 * form (each plan's method must be WC_GMRES_PS, lowrank 0 and disc WC_FD, else
 * WC_E_UNSUPPORTED),
 * advanced in lockstep: each round applies the preconditioner of every instance still
 * iterating in one batched apply and synchronises the host once.  Each instance keeps
 * its own tolerance, restart length, precision and iteration count, and stops on its
 * own true residual.  infos[count] (may be NULL) receives each instance's wc_info;
 * ms is the wall time of the whole batch.  Synchronous.  Returns WC_OK when every
 * instance converged, else the first failure (WC_E_MAXIT if that is the only one);
 * WC_E_MAXIT still writes y, p. */
typedef struct wc_batch wc_batch;
wc_status wc_batch_create(wc_plan *const *plans, int count, wc_batch **out);
wc_status wc_batch_destroy(wc_batch *batch);
wc_status wc_batch_pc_apply(wc_batch *batch, const double *const *v, double *const *w);
wc_status wc_batch_solve(wc_batch *batch, const double *const *f, const double *const *g,
                         const double *const *y0, double *const *y, double *const *p,
                         wc_info *infos);

/* ---- preconditioner apply that allocates nothing ---------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): w = P^{-1} v as wc_pc_apply computes
 * it, with no plan.  The tables and the spectral workspace live in a static device array
 * of wc_pc_apply_noalloc_limit() bytes (256 MiB) that each device the library runs on
 * holds until the process ends; the tables are rebuilt on the device at every call.
 * No hipMalloc, hipFree or other allocating routine is called.
 *
 * prob: as for wc_plan_create (a_face_host must be NULL: a == 1; disc WC_FD); method: wc_method;
 * precision: wc_precision; v, w: device pointers, 2*n*m doubles each (may alias);
 * stream: hipStream_t or NULL.  Asynchronous, stream-ordered.
 * Errors: WC_E_ARG for invalid arguments or a problem whose tables plus spectral array
 * (n*m complex of the precision) exceed the limit; WC_E_UNSUPPORTED where wc_pc_apply's
 * GPU path does not apply (variable a, zeta != pi, n or M+1 not a power of two in
 * [4, 1024]) and for WC_FEM; WC_E_SINGULAR_S2 as for wc_plan_create.
 * Every call on a device shares that device's array and keeps the last call's contents:
 * calls that overlap on one GPU (different streams, or host threads without ordering)
 * race and must be serialised by the caller. */
wc_status wc_pc_apply_noalloc(const wc_problem *prob, int method, int precision,
                              const double *v, double *w, void *stream);
size_t wc_pc_apply_noalloc_limit(void);

/* Library build identification (static string). */
const char *wc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* WC_H_ */
