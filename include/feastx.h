/*
 * feastx -- dense Hermitian FEAST eigensolver on AMD MI355X (gfx950).
 *
 * Finds the eigenpairs (lambda, x) of A x = lambda B x inside a search
 * interval [Emin, Emax] for a dense real symmetric or complex Hermitian A and
 * a symmetric/Hermitian positive definite B (B = NULL: standard problem,
 * B = I).  Method: the FEAST subspace iteration of the FEAST v3.0 user guide,
 * section "The FEAST Algorithm" -- at each Gauss-Legendre node z_j of the
 * half contour around the interval, factor z_j B - A and solve it against
 * the M0 right-hand sides B X; accumulate Q = sum_j w_j Y_j; Rayleigh-Ritz
 * on Q (Q^H A Q, Q^H B Q, reduced eigenproblem, residuals); repeat.
 *
 * Conventions shared by every entry point:
 *   - Matrices are column-major (Fortran order) with full storage, as the
 *     guide's dense interfaces (section "Matrix storage", UPLO = 'F').
 *   - Complex numbers are interleaved {double re, im} (feast_z).
 *   - The return value is `info` with the codes of the guide's Table
 *     "tab_info": 0 success; 1 no eigenvalue in the interval; 2 no
 *     convergence within maxloop; 3 subspace too small (M0 <= M); 4 only the
 *     subspace Q was returned (mode 1); 5 only the stochastic estimate of
 *     the eigenvalue count was returned (mode 2); 200 bad interval; 201 bad M0;
 *     202 bad N; 100+i bad option i (fpm numbering: 102 ne, 103 tol,
 *     104 maxloop, 105 x0, 106 conv, 110 keep_factors, 114 mode, 140
 *     precision, 141 refine); -1 device allocation failed; -2 the factorisation
 *     of a shifted matrix failed (zero or non-finite pivot); -3 the reduced
 *     eigenproblem failed (B not positive definite); -4 other GPU runtime
 *     error; -(100+i) argument i is invalid (e.g. a NULL pointer).
 *     No exception crosses the interface.
 *   - Outputs E, X, res are valid for info in {0, 2, 3} (for info 5 see
 *     feast_opts.mode).  Their first M
 *     entries are the eigenpairs inside [Emin, Emax], ascending; then the
 *     remaining Ritz pairs outside the interval, ascending; spurious pairs
 *     (inside the interval but with residual > 0.1) come last with res = -1
 *     (Table "tab_common", remark on E, X and res).
 *   - Each host thread has its own context for the single-problem entry
 *     points: device workspace (factors, subspaces) and streams, created at
 *     the thread's first call, kept between its calls and freed by
 *     feast_release() from that thread.  Threads may call concurrently; the
 *     batched entry points and the server run their own executor.  The
 *     library never frees caller memory.
 */
#ifndef FEASTX_H
#define FEASTX_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double re, im;
} feast_z;

/* Options; the fpm(i) of the guide's Table "tab_fpm" each field stands for
 * is given in brackets. */
typedef struct {
    int ne;           /* [fpm(2)] Gauss-Legendre nodes on the half contour, >= 1; default 8 */
    int maxloop;      /* [fpm(4)] refinement loops after the first, >= 0; default 20 */
    int conv;         /* [fpm(6)] 1: max residual < tol (default); 0: trace change < tol */
    int x0;           /* [fpm(5)] 1: X holds the start subspace on entry; 0: seeded random start */
    int keep_factors; /* [fpm(10)] 1: factor once, keep the factors resident (default); 0: refactor every loop */
    int precision;    /* 0: FP64 (complex128 factors and solves, default);
                         1: mixed (complex64 factors and solves on FP32 matrix cores,
                            FP64 residual correction; everything else FP64) */
    int refine;       /* must be 0 (the mixed path uses the FP64 residual-correction form from
                         the second loop on); any other value returns info 141 */
    int mode;         /* [fpm(14)] 0: normal; 1: return Q after one contour in X (info 4);
                         2: stochastic estimate of the number of eigenvalues in the interval
                         (section "Stochastic estimate", info 5): one contour pass over the M0
                         probe columns of X (the caller's with x0 = 1, else random +-1 entries
                         drawn from seed); sample c is N Re(x_c^H q_c) / (x_c^H x_c) with q_c the
                         filtered probe; res[c] returns the running average of samples 0..c, M
                         the nearest integer to res[M0-1] (at least 0), X the filtered probes,
                         E zeros.  A small M0 (about 10) and Ne (about 3) suffice. */
    int verbose;      /* [fpm(1)] 1: print one line per loop to stderr */
    double tol;       /* [fpm(3)] convergence tolerance, > 0; default 1e-12 */
    unsigned long long seed; /* seed of the random start subspace (x0 = 0) */
    int integration;  /* [fpm(16)] half-contour rule: 0 Gauss-Legendre (default), 1 trapezoidal;
                         2 (Zolotarev) is not in this build: info 116 */
    int ellipse;      /* [fpm(18)] contour ellipse, vertical over horizontal semi-axis in percent:
                         100 circle (default), 50 flat, 200 tall; >= 1, else info 118 */
    const feast_z *Zne; /* expert mode (the guide's Zne, Wne arguments): ne custom half-contour nodes */
    const feast_z *Wne; /* and weights, both or neither (else info -113); read during the call (the
                           server copies them at submit); integration and ellipse are then unused */
    /* non-Hermitian FEAST (feast_gsolve_*) only: */
    int ne_full;          /* [fpm(8)] nodes of the full contour, 1..256 (default 16), else info 108 */
    int integration_full; /* [fpm(17)] 0: Gauss-Legendre, 1: trapezoidal (default); else info 117 */
    int angle;            /* [fpm(19)] rotation of the ellipse in degrees, -180..180 (default 0), else
                             info 119 */
} feast_opts;

/* Per-stage timings of the most recent solve (milliseconds, from HIP events
 * on the solve's stream) and the algorithmic work behind them. */
typedef struct {
    double t_total, t_shift, t_factor, t_solve, t_accum, t_rr, t_reduced, t_resid;
    double t_lu_gemm;        /* with feast_set_timing(1): time inside the complex matrix-product
                                launches of one precision: complex128 for FP64 and for mixed solves
                                with at least half of their nodes in complex128 (fp64_nodes >=
                                ne / 2), else complex64: LU trailing updates, triangular-solve
                                updates and, for complex128 in complex pencils, the loop's other
                                complex128 products (Rayleigh-Ritz, Ritz vectors) */
    double lu_gemm_flops;    /* algorithmic real flops of those launches (8 per complex multiply-add) */
    long long lu_gemm_launches;
    double factor_flops;     /* ne * (8/3) N^3 */
    double solve_flops;      /* 8 N^2 M0 per node per triangular pair, all loops */
    int loops;               /* FEAST loops executed (loop + 1) */
    int m0_final;            /* subspace size at exit */
    int eig_calls;           /* reduced Hermitian eigensolves */
    int eig_sweeps;          /* Jacobi sweeps summed over those calls */
    double t_lu_update;      /* with feast_set_timing(1): the part of t_lu_gemm issued by the shifted
                                LU itself (its trailing and panel-column updates) */
    double lu_update_flops;  /* algorithmic real flops of those launches */
    long long lu_update_launches;
    int fp64_nodes;          /* mixed precision: contour nodes factored and solved in complex128 */
} feast_stats;

/* Defaults of the guide's feastinit (Table "tab_fpm"), with keep_factors = 1. */
void feast_default_opts(feast_opts *opts);

/* ---- minimal form: host arrays, defaults except Ne and tol, random start.
 * A, B: N x N (B may be NULL).  E[M0], res[M0], X[N*M0] allocated by the caller. */
int feast_solve_d(int N, const double *A, const double *B, double Emin, double Emax, int M0, int Ne,
                  double tol, double *E, double *X, int *M, double *res);
int feast_solve_z(int N, const feast_z *A, const feast_z *B, double Emin, double Emax, int M0, int Ne,
                  double tol, double *E, feast_z *X, int *M, double *res);

/* ---- full form, host arrays.  M0 is in/out: on exit the subspace size kept
 * (directions with B-norm below 1e-14 of the largest are dropped; the
 * guide's "new suitable M0").  loop: index of the last FEAST loop (0-based).
 * epsout: relative trace change of the last loop (1 at loop 0). */
int feast_solve_d_ex(int N, const double *A, int lda, const double *B, int ldb, double Emin, double Emax,
                     int *M0, const feast_opts *opts, double *E, double *X, int ldx, int *M, double *res,
                     int *loop, double *epsout);
int feast_solve_z_ex(int N, const feast_z *A, int lda, const feast_z *B, int ldb, double Emin,
                     double Emax, int *M0, const feast_opts *opts, double *E, feast_z *X, int ldx, int *M,
                     double *res, int *loop, double *epsout);

/* ---- device form: A, B, X are device pointers (HBM), E/res/M/loop/epsout
 * are host pointers.  `stream` is a hipStream_t (NULL: the library's own
 * stream); the call returns after the solve has finished on it. */
int feast_solve_d_dev(int N, const double *dA, int lda, const double *dB, int ldb, double Emin,
                      double Emax, int *M0, const feast_opts *opts, double *E, double *dX, int ldx, int *M,
                      double *res, int *loop, double *epsout, void *stream);
int feast_solve_z_dev(int N, const feast_z *dA, int lda, const feast_z *dB, int ldb, double Emin,
                      double Emax, int *M0, const feast_opts *opts, double *E, feast_z *dX, int ldx,
                      int *M, double *res, int *loop, double *epsout, void *stream);

/* ---- no-allocation form of feast_solve_d_dev, for callers that cannot
 * allocate device memory during the call (code running under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The same
 * arguments, results and info codes as feast_solve_d_dev, but every device
 * buffer of the solve comes from a static scratch array of
 * FEASTX_NOALLOC_SCRATCH_BYTES on each device (held from the library's load
 * until the process ends) and the call allocates nothing: no hipMalloc,
 * hipFree, pinned host memory, stream or event.
 *   Limit: a problem whose workspace (Ne factors and their solve form, solve
 *   panels, subspace blocks) exceeds the scratch returns -1 at once with a
 *   message on stderr, before any GPU work: with Ne = 8, N up to about 700 in
 *   mixed precision and about 512 in FP64 for M0 of a few dozen.
 *   Scratch contents persist between calls: the solve initialises every
 *   buffer it reads.  Calls on one device share its scratch and take turns
 *   (a lock per device); work the caller queues on `stream` after the call
 *   may overlap nothing of it, because the call returns after the solve has
 *   finished.  The stream may be NULL (the null stream).  The stage timers of
 *   feast_stats stay 0. */
#define FEASTX_NOALLOC_SCRATCH_BYTES (128ull << 20)
int feast_solve_d_dev_noalloc(int N, const double *dA, int lda, const double *dB, int ldb, double Emin,
                              double Emax, int *M0, const feast_opts *opts, double *E, double *dX, int ldx,
                              int *M, double *res, int *loop, double *epsout, void *stream);

/* ---- non-Hermitian FEAST (guide: the variant for non-Hermitian pencils,
 * with dual subspaces Q and Q-hat for the right and left eigenvectors, a full
 * contour around a two-dimensional search region, Table "tab_fpm" fpm(8),
 * fpm(17), fpm(18), fpm(19), Table "tab_common" for E, X, res):
 *   A, B general (B = NULL: identity), complex (_z) or real (_d, solved in
 *   complex arithmetic); host arrays, column-major.
 *   Region: the ellipse centred at Emid with horizontal semi-axis r > 0,
 *   vertical semi-axis r fpm(18)/100, turned by fpm(19) degrees
 *   counter-clockwise.
 *   E[M0] (complex out): the first M are the eigenvalues inside the region,
 *   then the other Ritz values, spurious ones last; each group by increasing
 *   real part, then imaginary part.
 *   X (N x 2 M0, leading dimension ldx >= N, complex): on entry the right and
 *   then the left start subspaces if opts.x0 = 1; on exit the right
 *   eigenvectors in columns 0..M0-1 and the left eigenvectors in columns
 *   M0..2 M0-1, in the order of E, each of unit 2-norm.
 *   res[2 M0]: right residuals ||A x - lambda B x||_1 / (alpha ||B x||_1),
 *   then left residuals ||A^H y - conj(lambda) B^H y||_1 / (alpha ||B^H y||_1),
 *   alpha = |Emid| + r; spurious pairs (inside, with a residual above 0.1 from
 *   the second loop on) have -1.
 *   Convergence (fpm(6) = 1): both residuals of every pair inside below tol.
 *   opts.precision: 0 FP64; 1 mixed (complex64 factors and solves, and
 *   from the second loop on they act only on the FP64 right and left Ritz
 *   residuals; everything else FP64).  Normal mode only (opts.mode != 0:
 *   info 114); opts.ne, integration and custom nodes are not used.
 *   info as for feast_solve_*, plus 108 (ne_full), 117 (integration_full),
 *   119 (angle), 200 (r <= 0 or not finite). */
int feast_gsolve_z(int N, const feast_z *A, int lda, const feast_z *B, int ldb, feast_z Emid, double r, int *M0,
                   const feast_opts *opts, feast_z *E, feast_z *X, int ldx, int *M, double *res, int *loop,
                   double *epsout);
int feast_gsolve_d(int N, const double *A, int lda, const double *B, int ldb, feast_z Emid, double r, int *M0,
                   const feast_opts *opts, feast_z *E, feast_z *X, int ldx, int *M, double *res, int *loop,
                   double *epsout);
/* The same on device arrays (complex; a real pencil is passed with zero
 * imaginary parts): dA, dB (or NULL), dX (N x 2 M0, start subspaces on entry
 * if opts.x0 = 1, eigenvectors on exit) in HBM, column-major with leading
 * dimensions lda, ldb, ldx >= N; E, res, M, loop, epsout on the host.  Runs
 * on `stream` (a hipStream_t; NULL: the library's own) and returns when the
 * results are ready. */
int feast_gsolve_z_dev(int N, const feast_z *dA, int lda, const feast_z *dB, int ldb, feast_z Emid, double r,
                       int *M0, const feast_opts *opts, feast_z *E, feast_z *dX, int ldx, int *M, double *res,
                       int *loop, double *epsout, void *stream);

/* ---- batched: many independent problems in one call (the guide's first
 * level of parallelism, independent search intervals / problems).  Each job
 * carries its problem and receives its outputs; `opts` is shared (opts.x0 =
 * 1: every job's X holds its start subspace).  device = 1: A, B, X are device
 * arrays; 0: host arrays.  Up to `concurrency` problems (0: 4, at most 8)
 * run at once, each on its own stream and device workspace, so their kernels
 * overlap on the GPU; every job runs the same kernels as a single solve and
 * gets the result it would get alone.  Returns 0 when every job ran (its
 * status in job.info), or an argument error (-101 njobs, -102 jobs, -104
 * device). */
typedef struct {
    int n;                  /* order N */
    const void *A;          /* double (real symmetric) or feast_z (Hermitian), N x N */
    int lda;
    const void *B;          /* NULL: B = I */
    int ldb;
    double emin, emax;
    int m0;                 /* subspace size */
    void *X;                /* N x M0: start subspace (opts.x0 = 1) on entry, eigenvectors on exit */
    int ldx;
    double *E, *res;        /* M0 entries each */
    /* outputs */
    int info, M, m0_out, loop;
    double epsout;
    double ms;              /* wall time from submission to completion */
} feast_job;
int feast_solve_batched_d(int njobs, feast_job *jobs, const feast_opts *opts, int device, int concurrency);
int feast_solve_batched_z(int njobs, feast_job *jobs, const feast_opts *opts, int device, int concurrency);

/* ---- spectrum slicing (section "Multiple search intervals and FEAST-MPI":
 * neighbouring search intervals without overlap, each an independent FEAST
 * run; here one batched job on one GPU).  Slice s is the closed interval
 * [bounds[s], bounds[s+1]] of the pencil (A, B); bounds has nslices + 1
 * ascending entries.  A and B are staged on the device once and every slice
 * reads them (device = 0: A, B and the slices' X are host arrays; 1: device
 * arrays).  slices[s] carries m0 (with auto_m0: the most that slice may
 * use), X (N x m0, leading dimension ldx; the start subspace if opts.x0 = 1),
 * E and res (m0 entries each, host); the call sets its n, A, lda, B, ldb,
 * emin and emax and fills info, M, m0_out, loop, epsout and ms as
 * feast_solve_batched does.
 * auto_m0 = 1: every slice first runs the stochastic count estimate (mode 2,
 * 16 probes, Ne = 3) and then solves with M0 = min(m0, max(8, ceil(1.5
 * estimate + 4))); a slice that ends with info 3 (M0 too small) runs again
 * with twice its M0, up to its m0.  With auto_m0 the start subspaces are the
 * library's random ones (opts.x0 is ignored).
 * An eigenvalue exactly on a shared bound belongs to both neighbours and is
 * reported by both.  Returns 0 when every slice ran (its status in
 * slices[s].info), else: 200 bounds not ascending, 201 a slice's m0 outside
 * [1, N], 202 N < 1, -102 A NULL, -103 lda < N, -105 ldb < N, -106
 * nslices < 1, -107 bounds NULL, -108 slices NULL or a slice's X, E, res
 * NULL or ldx < N, -110 device not 0 or 1; -1 staging allocation failed; -4
 * other HIP error.  Slices run concurrently as in feast_solve_batched. */
int feast_solve_slices_d(int N, const double *A, int lda, const double *B, int ldb, int nslices,
                         const double *bounds, feast_job *slices, const feast_opts *opts, int device, int concurrency,
                         int auto_m0);
int feast_solve_slices_z(int N, const feast_z *A, int lda, const feast_z *B, int ldb, int nslices,
                         const double *bounds, feast_job *slices, const feast_opts *opts, int device, int concurrency,
                         int auto_m0);

/* ---- serving: a request loop that admits eigenproblems of mixed size while
 * others run.  A request is admitted when a slot is free and its device
 * footprint (factors + subspaces + staged inputs) fits next to the running
 * ones within hbm_budget_gb (the oldest request first); admitted requests
 * run concurrently on separate streams with their factors and subspaces
 * resident on the device for all their FEAST loops.  Results are those of
 * the same request solved alone.  The request's host arrays A, B (and X0)
 * must stay valid until the request completes. */
typedef struct feast_server feast_server;
typedef struct {
    int slots;              /* concurrent requests on the device (0: 4, at most 8) */
    double hbm_budget_gb;   /* admission limit (0: 64 GB) */
} feast_server_cfg;
typedef struct {
    int hermitian;          /* 0: real symmetric (double), 1: complex Hermitian (feast_z) */
    int n;
    const void *A;
    int lda;
    const void *B;          /* NULL: B = I */
    int ldb;
    double emin, emax;
    int m0;
    const void *X0;         /* NULL: seeded random start (opts.seed) */
    int ldx;
    feast_opts opts;        /* opts.x0 is set from X0 */
} feast_request;
typedef struct {
    int info, M, m0, loop;
    double epsout;
    double *E, *res;        /* caller buffers of M0 entries, filled if not NULL */
    void *X;                /* caller buffer N x M0 (leading dimension ldx), filled if not NULL */
    int ldx;
    double queue_ms, run_ms, latency_ms;   /* submit->start, start->end, submit->end */
} feast_result;
feast_server *feast_server_create(const feast_server_cfg *cfg);   /* NULL on failure */
/* 0 on success (id set), else the request's argument/info error code */
int feast_server_submit(feast_server *srv, const feast_request *req, unsigned long long *id);
/* 0: done and out filled (the request is then forgotten); 1: still pending;
 * -102: unknown id */
int feast_server_poll(feast_server *srv, unsigned long long id, feast_result *out);
int feast_server_wait(feast_server *srv, unsigned long long id, feast_result *out);
/* finishes the queued requests, then frees everything */
void feast_server_destroy(feast_server *srv);

/* ---- tools (host only, no GPU), with the guide's arguments.
 * Half-contour nodes and weights (tool "[cz]feast_contour"; section "Defining
 * a search contour"): with c = (Emin + Emax)/2, r = (Emax - Emin)/2 and
 * a = fpm18 / 100, the contour is z(theta) = c + r cos(theta) + i a r sin(theta),
 * and the filter rho(lambda) = (1 / 2 pi i) contour-integral dz / (z - lambda)
 * taken over its upper half (doubled real part) at fpm2 nodes:
 *   fpm16 = 0: theta_j = (pi/2)(1 - x_j), dtheta_j = (pi/2) omega_j,
 *              (x_j, omega_j) Gauss-Legendre on [-1, 1];
 *   fpm16 = 1: theta_j = pi (fpm2 - j - 1/2) / fpm2, dtheta_j = pi / fpm2;
 *   z_j = z(theta_j), w_j = (dtheta_j / pi)(a r cos(theta_j) + i r sin(theta_j)).
 * Nodes come in increasing real part.  Returns 0, 102 (fpm2 < 1), 116
 * (fpm16), 118 (fpm18 < 1), 200 (Emin >= Emax), -105/-106 (NULL output). */
int feast_contour(double Emin, double Emax, int fpm2, int fpm16, int fpm18, feast_z *Zne, feast_z *Wne);
/* Filter rho(lambda) = Re sum_j w_j / (z_j - lambda) at the m points eig
 * (tool "[sd]feast_rational"); the same codes, -108 for a NULL eig or f. */
int feast_rational(double Emin, double Emax, int fpm2, int fpm16, int fpm18, const double *eig, int m, double *f);
/* The same filter for custom nodes and weights (tool "[sd]feast_rationalx"). */
int feast_rationalx(const feast_z *Zne, const feast_z *Wne, int fpm2, const double *eig, int m, double *f);

/* Statistics of the calling thread's last solve; 0 on success. */
int feast_last_stats(feast_stats *stats);
/* Enable (1) or disable (0) per-launch HIP-event timing of the complex
 * matrix-product kernel in each solve's factor precision (reported in
 * feast_stats). */
void feast_set_timing(int on);

/* ---- tile autotuner (spec batching: tile shapes chosen on the device).
 * The complex products (LU updates, triangular-solve updates, Rayleigh-Ritz)
 * have FEAST_TILE_VARIANTS tile shapes per precision; which one runs is read
 * from a process-wide table indexed by precision (0 complex64, 1 complex128)
 * and depth class (0: depth <= 64, the LU's panel-by-panel updates and the
 * Cholesky updates; 1: deeper, the LU's 128-deep block updates, the solve
 * updates and the Rayleigh-Ritz products).  Variant 0 is the default.
 * Every variant accumulates each output over the depth in the same order, so
 * the table changes times, never results. */
#define FEAST_TILE_VARIANTS 3
typedef struct {
    int choice[2][2];        /* [precision][class] -> variant, 0 .. FEAST_TILE_VARIANTS - 1 */
    double tflops[2][2][FEAST_TILE_VARIANTS]; /* feast_autotune: measured rate of each variant
                                (8 flops per complex multiply-add); 0 when not measured */
} feast_tiles;
/* Time every variant on the current device on the shapes of a solve of order
 * n with m0 right-hand sides and ne contour nodes (capped at n = 4096 and
 * ne = 8 to bound the scratch; class 0: one depth-64 trailing update of
 * n - 64 rows and columns; class 1: one depth-128 trailing update of n - 128
 * rows and columns together with one depth-256 solve update with m0 columns;
 * batch ne), install the fastest per precision and class in the table (a
 * variant replaces the
 * default only when at least 5 % faster), and return both in *out (may be
 * NULL).  Allocates and frees its own device scratch (up to about 2.2 GB).
 * Not to be called while solves run on other threads.  Returns 0, 202 (n < 64),
 * 201 (m0 < 1), 102 (ne < 1), -1 (device allocation failed), -4 (HIP error). */
int feast_autotune(int n, int m0, int ne, feast_tiles *out);
/* The current table (tflops zero). */
void feast_get_tiles(feast_tiles *out);

/* ---- the factorisation's launch schedule (host logic only; no device call).
 * The shifted LU of every contour node (the factorisation step of the FEAST
 * loop, "The FEAST Algorithm") is issued as a fixed list of steps that
 * depends only on n, on whether a second (panel) stream is used and on the
 * form.  form: -1 the schedule the library runs for this n (see
 * feast_set_lu_form), 0 panels in pairs (depth-64
 * trailing products), 1 panels in blocks of four (depth-128 trailing
 * products).  This writes the first min(cap, count) steps into ops
 * (FEAST_LU_OP_INTS ints each, caller-owned; ops may be NULL) and returns
 * the count, or -1 for n < 1 or another form.  Step layout: kind (0 panel factorisation of columns k..k+nbw-1,
 * 1 row interchanges / U rows, 2 trailing product, 3 event record, 4 stream
 * wait), side (1: the panel stream), k, nbw, c0, c1, c2, c3 (kind 1: the
 * column ranges [c0, c1) and [c2, c3); kind 2: rows [c0, c1), columns
 * [c2, c3)), kc0, kc1 (kind 1: rows of the earlier panels' correction;
 * kind 2: the product's depth range), mode (kind 1: 1 interchanges, 2 U
 * rows, 4 correction), list (the move list written or read).  For tests
 * that replay the schedule on the host. */
#define FEAST_LU_OP_INTS 12
int feast_lu_schedule(int n, int side, int form, int *ops, int cap);
/* The schedule every later factorisation uses: -1 (the default) pairs below
 * n = 6144 and blocks from there, 0 pairs, 1 blocks.  Both factor with
 * partial pivoting and give the same factors up to rounding; the choice is
 * one of speed (blocks: deeper trailing products; pairs: a shorter panel
 * chain).  Returns 0, or -1 for another value (nothing changed).  Not to be
 * changed while solves run on other threads. */
int feast_set_lu_form(int form);
/* The current setting (-1, 0 or 1). */
int feast_get_lu_form(void);
/* Install a table (choices only); 0, or -101 for NULL / an out-of-range entry. */
int feast_set_tiles(const feast_tiles *tiles);
/* Free the calling thread's context (device workspace and streams). */
void feast_release(void);
/* Library version string. */
const char *feast_version(void);

#ifdef __cplusplus
}
#endif
#endif
