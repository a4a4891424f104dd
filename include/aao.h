/*
 * aao.h -- C ABI of the all-at-once parallel-in-time solver for gfx950 (MI355X).
 *
 * The library solves the monolithic ("all-at-once") time-stepping system
 *     A U = b,   A block lower-triangular Toeplitz, U = [u_1; ...; u_ell]
 * of Goddard & Wathen, "A note on parallel preconditioning for all-at-once
 * evolutionary PDEs" (arXiv 1810.00615), Sec. 2, by GMRES preconditioned with the
 * block circulant C of McDonald, Pestana & Wathen (eq. standardheatprecon,
 * eq. wavepreconditioner), applied through its Fourier diagonalisation
 * (Sec. 3, eq. precon2para).
 *
 * Discretisation (Sec. 2): 1D, Omega = [0,1], n interior nodes of a uniform P1
 * mesh (h = 1/(n+1)), M = (h/6) tridiag(1,4,1), K = (1/h) tridiag(-1,2,-1), a
 * diffusivity / wave-speed factor kappa multiplying K, ell time steps of size tau.
 *   AAO_HEAT_IE  implicit Euler, eq. timestepproblem1 / monolithicheat:
 *                A_0 = M + tau kappa K, A_1 = -M            (s = 1)
 *   AAO_WAVE_BD2 two-step backward difference, system C_BD2:
 *                A_0 = M + tau^2 kappa K, A_1 = -2M, A_2 = M (s = 2)
 *   AAO_WAVE_BD4 four-step backward difference, eq. BD4 and system C_BD4:
 *                A_0 = 2M + tau^2 kappa K, A_1 = -5M, A_2 = 4M, A_3 = -M from the
 *                third row on; start-up rows B u_1 and C u_1 + B u_2 (B = M +
 *                tau^2 kappa K, C = -2M); the circulant R_BD4 wraps A_0..A_3
 *   AAO_WAVE_CD  central differences, eq. CenDiffDisc and system C_CD: two-sided,
 *                M u_{k-1} + (tau^2 kappa K - 2M) u_k + M u_{k+1} (no u_{ell+1});
 *                the circulant R_CD has the real, indefinite symbol
 *                tau^2 kappa K - 4 sin^2(pi j / ell) M, whose blocks can be nearly
 *                singular (the shifted solves do not pivot)
 * (The paper prints the heat block as K + tau M; implicit Euler on
 * M u' = -K u gives M + tau K, which is what is built.)
 *
 * Conventions for every entry point:
 *   - Vectors of the monolithic system are caller-owned DEVICE pointers to
 *     ell*n contiguous doubles, row-major ell x n: row k holds time level k+1,
 *     the n spatial nodes contiguous.  Per-node vectors (u0, v0, gradients) are
 *     device pointers to n doubles.  Arrays marked "host" are host memory.
 *   - Operations are enqueued on the context's stream (aao_set_stream; default:
 *     the null stream).  apply_* return without synchronising; gmres /
 *     adjoint_solve / grad synchronise the stream before they return.
 *   - Input and output vectors must not overlap (AAO_ERR_ARG otherwise).
 *   - A negative status is an error and leaves outputs unspecified.  The context
 *     stays usable after every error except AAO_ERR_HIP.  No C++ exception
 *     crosses this interface.
 *   - A context is not thread-safe; distinct contexts may be used from distinct
 *     threads on distinct streams.
 *
 * The library reads no environment variables: every option is an argument or a
 * flag of this interface.
 */
#ifndef AAO_H
#define AAO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aao_ctx_s *aao_ctx;

typedef enum {
    AAO_OK = 0,
    AAO_NOT_CONVERGED = 1,  /* maxit reached: x holds the last iterate, info filled */
    AAO_ERR_ARG = -1,       /* bad size, step, pointer, aliasing or option        */
    AAO_ERR_ALLOC = -2,     /* device allocation failed                            */
    AAO_ERR_HIP = -3,       /* HIP runtime error (context unusable afterwards)     */
    AAO_ERR_NUMERIC = -4,   /* non-finite residual / breakdown of a shifted solve  */
    AAO_ERR_STATE = -5,     /* call out of order (e.g. steps set for BD2)          */
    AAO_ERR_UNSUPPORTED = -6
} aao_status;

enum { AAO_HEAT_IE = 0, AAO_WAVE_BD2 = 1, AAO_WAVE_BD4 = 2, AAO_WAVE_CD = 3 };

/* Precision of the preconditioner apply inside GMRES (aao_set_precision).  In every
 * mode the outer flexible GMRES (matvec, residual, Arnoldi, update) stays double.
 *   AAO_PREC_FP64      FFTs, spectra and shifted solves in double.
 *   AAO_PREC_MIXED     FFTs and spectra in single precision, shifted solves in
 *                      double arithmetic on single-precision spectra.
 *   AAO_PREC_FP32      as MIXED with the shifted solves in single precision too.
 *   AAO_PREC_MIXED_IN  single precision on the input side only: the forward FFT and
 *                      the spectrum it writes; the shifted solves (double arithmetic),
 *                      their output spectrum and the inverse FFT in double.  A
 *                      rounding error d of the input side reaches the preconditioned
 *                      residual as A C^{-1} d ~ d (C^{-1} A is the identity plus a
 *                      low-rank term), so it costs no accuracy; one of the output side
 *                      is multiplied by ||A|| ||C^{-1} r|| / ||r||, which is what makes
 *                      AAO_PREC_MIXED need more GMRES iterations. */
enum { AAO_PREC_FP64 = 0, AAO_PREC_MIXED = 1, AAO_PREC_FP32 = 2, AAO_PREC_MIXED_IN = 3 };

typedef struct {
    int iters;              /* preconditioner applies (GMRES iterations)          */
    int restarts;           /* completed restart cycles                            */
    int converged;          /* 1 if the true relative residual <= tol              */
    double rel_resid_est;   /* last least-squares estimate |g_{j+1}| / ||b||      */
    double rel_resid_true;  /* ||b - A x|| / ||b|| recomputed in FP64 at the end   */
} aao_info;

/* Create a context for n >= 1 interior nodes, ell >= 1 steps of size tau > 0
 * (tau is the step of the Toeplitz matrix and of the circulant; the mean step
 * when variable steps are set), scheme AAO_HEAT_IE, AAO_WAVE_BD2, AAO_WAVE_BD4 or
 * AAO_WAVE_CD.  kappa = 1.
 * Allocates the device tables on the current HIP device.  Sec. 2. */
aao_status aao_create(int64_t n, int64_t ell, double tau, int scheme, aao_ctx *out);

/* Create a context on the unit square [0,1]^2: bilinear (Q1) elements on a uniform
 * grid of nx x ny interior nodes (hx = 1/(nx+1), hy = 1/(ny+1)), zero Dirichlet data,
 *     M2 = My (x) Mx,   K2 = Ky (x) Mx + My (x) Kx
 * (Mx, Kx, My, Ky the 1D matrices above along each axis), and the time structure of
 * `scheme` unchanged: blocks a_m M2 + b_m kappa K2.  The paper works in one space
 * dimension; Sec. 3 and Sec. 5 note that beyond it the blocks of the middle factor of
 * eq. precon2para stop being tridiagonal.  Here they are reduced to tridiagonal ones
 * by the orthonormal sine transform along y, which diagonalises My and Ky: per
 * frequency j and sine mode q the x-tridiagonal (alpha_j my_q + beta_j kappa ky_q) Mx
 * + beta_j kappa my_q Kx, solved like the 1D blocks.
 * A time level is ny x nx doubles, x fastest (node (ix, iy) at iy nx + ix); a
 * monolithic vector is ell levels (ell nx ny doubles), per-node vectors nx ny
 * doubles.  Requires ny + 1 a power of two (ny <= 2047), 1 <= nx <= 16384,
 * 1 <= ell <= 65535; AAO_ERR_UNSUPPORTED otherwise.
 * Supported on such a context: aao_set_stream, aao_set_kappa, aao_set_precision,
 * aao_build_rhs (M2 in place of M, K2 of K), aao_apply_A, aao_apply_Pinv (order
 * 0), aao_gmres, aao_gmres_ex, aao_adjoint_solve, aao_set_timing*, aao_get_timing*,
 * aao_tune, aao_get_config, aao_set_config, aao_config_shape (the shifted solves'
 * shapes apply to rows of nx unknowns).  aao_set_steps, aao_set_neumann_order (q >
 * 0), aao_project_sine, aao_grad and aao_grad_checkpointed return
 * AAO_ERR_UNSUPPORTED.
 * aao_gmres, aao_gmres_ex and aao_adjoint_solve iterate in sine coordinates along y
 * (the sine transform is orthonormal and its own inverse, so the steps and residual
 * norms are those of the nodal system): the right-hand side is transformed into one
 * more vector of the context (allocated on the first solve), the iterate in place on
 * entry and exit; x holds nodal values when the call returns, also after a failure. */
aao_status aao_create_2d(int64_t nx, int64_t ny, int64_t ell, double tau, int scheme,
                         aao_ctx *out);

/* Free every device buffer of the context.  NULL is accepted. */
aao_status aao_destroy(aao_ctx ctx);

/* Stream on which every later call of this context is enqueued (a hipStream_t;
 * NULL = the null stream). */
aao_status aao_set_stream(aao_ctx ctx, void *hip_stream);

/* Multiply K by kappa > 0 in every block (heat diffusivity, squared wave speed). */
aao_status aao_set_kappa(aao_ctx ctx, double kappa);

/* Variable steps tau_1..tau_ell (host array of ell positive doubles), heat only:
 * the matrix B of eq. nonuniformmonolithicheat with A_0^k = M + tau_k kappa K.
 * aao_apply_A and aao_gmres then use B, and aao_apply_Pinv with order q >= 1
 * applies the truncated Neumann series of eq. preconapprox1 for
 * Q = C + blockdiag((tau_k - tau) kappa K).  NULL restores uniform steps.
 * AAO_ERR_STATE for the wave scheme. */
aao_status aao_set_steps(aao_ctx ctx, const double *tau_k);

/* AAO_PREC_FP64 (default), AAO_PREC_MIXED, AAO_PREC_FP32 or AAO_PREC_MIXED_IN (which
 * allocates its single-precision input spectrum on first selection). */
aao_status aao_set_precision(aao_ctx ctx, int prec);

/* Initial data as a sine series s(x) = sum_m amps[m] sin(modes[m] pi x) (host
 * arrays of J entries, modes >= 1): writes the L2 projection u0 = M^{-1} f onto
 * the P1 space (device, n doubles), f_i = int s phi_i.  The initial state
 * "is a projection of the initial data" (Sec. 2, after eq. timestepproblem1). */
aao_status aao_project_sine(aao_ctx ctx, int J, const int *modes, const double *amps,
                            double *u0);

/* Right-hand side b (device, ell x n) from u0 (device, n) and, for BD2, the
 * initial velocity v0 (device, n, or NULL for v0 = 0):
 *   heat: b_1 = M u0 (eq. monolithicheat), other rows 0;
 *   BD2:  b_1 = A_0 (u0 + tau v0), b_2 = -M u0, other rows 0 (system C_BD2,
 *         with the start-up row u_1 = u0 + tau v0);
 *   BD4:  b_1 = B (u0 + tau v0), b_2 = -M u0, b_3 = M u0 (system C_BD4);
 *   CD:   b_1 = -M u0 (system C_CD; the scheme has no initial velocity: v0 must be
 *         NULL, AAO_ERR_ARG otherwise). */
aao_status aao_build_rhs(aao_ctx ctx, const double *u0, const double *v0, double *b);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1); with variable steps, B
 * or B^T.  x, y: device, ell x n.  Sec. 2, eq. monolithicheat / C_BD2. */
aao_status aao_apply_A(aao_ctx ctx, const double *x, double *y, int transpose);

/* z = C^{-1} r (transpose = 0) or C^{-T} r (transpose = 1) through
 * eq. precon2para: FFT along time, one complex shifted tridiagonal solve per
 * frequency, inverse FFT.  neumann_order q >= 1 (variable steps set) applies
 * sum_{m=0}^{q} (-C^{-1} E)^m C^{-1} r (eq. preconapprox1 with i = q + 1 terms),
 * evaluated as z_0 = C^{-1} r, z_m = C^{-1}(r - E z_{m-1}); with uniform steps
 * every order equals order 0.  Uses the context precision.  r, z: device,
 * ell x n, must not overlap. */
aao_status aao_apply_Pinv(aao_ctx ctx, const double *r, double *z, int neumann_order,
                          int transpose);

/* z = C^{-1} r (transpose = 0) or C^{-T} r as aao_apply_Pinv with neumann_order 0,
 * for callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): no context, and no allocation by
 * this call.  The twiddles, the symbol and partition tables and the half spectrum
 * live in one static device array of 64 MiB per GPU, held until the process ends:
 * 16 ell + 64 H + 2 H (3 CW + 8) w_a + H lds w_s (+ 8 H lds for AAO_PREC_MIXED_IN)
 * bytes, each term rounded up to 256, with H = ell/2 + 1, lds = n rounded up to 16,
 * CW the chunk width of the default shifted-solve shape for n (at most 8 up to
 * n = 4096), w_a = 16 (8 for AAO_PREC_FP32) and w_s = 8 for AAO_PREC_MIXED and
 * AAO_PREC_FP32, else 16; e.g. n = 2047, ell = 2048 needs at most 34.8 MB in FP64.  Sizes beyond it, ell not a power of two in [2, 16384] or n > 16384:
 * AAO_ERR_UNSUPPORTED; bad values or overlapping r, z: AAO_ERR_ARG.  kappa > 0 as in
 * aao_set_kappa; scheme and prec as in aao_create / aao_set_precision; r, z device,
 * ell x n; stream a hipStream_t (NULL = null stream).  The call is asynchronous and
 * leaves its result in z only; every call on one GPU shares that GPU's array, so
 * calls that overlap in time on one GPU (other streams, other threads) race, and
 * must be ordered by the caller.  The first call on a GPU looks the array up
 * (hipGetSymbolAddress); make that call outside any stream capture. */
aao_status aao_apply_Pinv_noalloc(int64_t n, int64_t ell, double tau, double kappa, int scheme,
                                  int prec, const double *r, double *z, int transpose,
                                  void *stream);

/* Restarted right-preconditioned flexible GMRES(restart) for A x = b (device
 * vectors; x holds the initial guess on entry -- pass zeros for x0 = 0 -- and
 * the solution on return), preconditioner aao_apply_Pinv(neumann_order =
 * aao_set_neumann_order, default 0).  Arnoldi is classical Gram-Schmidt with
 * one re-orthogonalisation (CGS2) in FP64.  Stops when the least-squares
 * estimate |g_{j+1}| / ||b|| <= tol, then confirms with the true residual
 * ||b - A x|| / ||b|| and restarts if it is above tol.  At most maxit
 * preconditioner applies.  Returns AAO_OK, AAO_NOT_CONVERGED (x = last iterate)
 * or an error; info (host, may be NULL) is filled in either of the first two
 * cases.  GMRES: Saad & Schultz, cited in Sec. 1. */
aao_status aao_gmres(aao_ctx ctx, const double *b, double *x, int restart, double tol,
                     int maxit, aao_info *info);

/* aao_gmres with flags:
 *   AAO_GMRES_ZERO_GUESS   x0 = 0 whatever x holds on entry (x is only written; the
 *                          first basis vector is b itself, so the initial residual
 *                          costs no matvec);
 *   AAO_GMRES_TRANSPOSE    solve A^T x = b with C^{-T} (as aao_adjoint_solve);
 *   AAO_GMRES_CGS2_CLASSIC three-pass CGS2 (project, re-project, update + norm) instead
 *                          of the re-orthogonalisation deferred by one step (the same
 *                          Hessenberg columns up to rounding; a comparison path);
 *   AAO_GMRES_EARLY_CHECK  check the Hessenberg column before the update pass at every
 *                          step, not only where the residual history predicts
 *                          convergence (exercises the path where that check fails).
 * The early check forms the last column entry from |w|^2 - |h|^2, which loses relative
 * accuracy once that difference falls below about 1e-8 |w|^2; when it skips the update
 * pass, rel_resid_est comes from that column.  Convergence is always decided by the
 * true residual (rel_resid_true).  Unknown bits: AAO_ERR_ARG. */
enum {
    AAO_GMRES_ZERO_GUESS = 1,
    AAO_GMRES_TRANSPOSE = 2,
    AAO_GMRES_CGS2_CLASSIC = 4,
    AAO_GMRES_EARLY_CHECK = 8
};
aao_status aao_gmres_ex(aao_ctx ctx, const double *b, double *x, int restart, double tol,
                        int maxit, int flags, aao_info *info);

/* Neumann order used by aao_gmres and aao_adjoint_solve (default 0). */
aao_status aao_set_neumann_order(aao_ctx ctx, int q);

/* Adjoint solve A^T lam = g: the transpose of the monolithic matrix of Sec. 2
 * (eq. monolithicheat, system C_BD2; block upper-triangular, A^T = J A J with J the
 * reversal of the time levels, every block being symmetric), by the same GMRES
 * preconditioned with C^{-T}.  C^T is the block circulant of the same blocks wrapped
 * the other way; its Fourier diagonalisation (eq. precon2para) has the conjugated
 * symbol, so C^{-T} costs what C^{-1} costs.  g, lam: device, ell x n; lam holds the
 * initial guess on entry.  Same return convention as aao_gmres. */
aao_status aao_adjoint_solve(aao_ctx ctx, const double *g, double *lam, int restart,
                             double tol, int maxit, aao_info *info);

/* Gradient reductions for L(U) with A(kappa) U = b(u0, v0, kappa) (the monolithic
 * system and right-hand side of Sec. 2, eq. monolithicheat / system C_BD2, whose
 * blocks are linear in kappa), given the forward solution U and the adjoint lam
 * (A^T lam = dL/dU), all device:
 *   g_u0    (device, n)   = (db/du0)^T lam   heat: M lam_1;
 *                                            BD2: A_0 lam_1 - M lam_2;
 *                                            BD4: B lam_1 - M lam_2 + M lam_3;
 *                                            CD: -M lam_1
 *   g_v0    (device, n or NULL) = (db/dv0)^T lam  (BD2: tau A_0 lam_1; BD4:
 *           tau B lam_1; heat, CD: 0)
 *   g_kappa (host scalar, may be NULL) = lam^T db/dkappa - lam^T (dA/dkappa) U,
 *           (dA/dkappa U)_k = sum_m b_m^{(k)} K u_{k-m}.
 * u0 and v0 are needed only for the BD2 / BD4 kappa term (NULL allowed otherwise). */
aao_status aao_grad(aao_ctx ctx, const double *u0, const double *v0, const double *U,
                    const double *lam, double *g_u0, double *g_v0, double *g_kappa);

/* Gradient with the forward trajectory checkpointed over time (heat scheme; the
 * trajectory is the sequential solution of eq. timestepproblem1 that the monolithic
 * system of eq. monolithicheat packages):
 * Uck (device) holds rows stride-1, 2*stride-1, ... of U (floor(ell/stride) rows
 * of n doubles; may be NULL when stride >= ell).  The levels in between are
 * recomputed by sequential implicit Euler steps (eq. timestepproblem1) from the
 * nearest earlier checkpoint (or u0), one workgroup per segment, while the kappa
 * reduction of aao_grad runs, so U is never stored whole: memory O(n ell/stride).
 * g_u0 (device, n) = M lam_1; g_kappa (host, may be NULL); U_out (device ell x n,
 * may be NULL) receives the recomputed trajectory.  AAO_ERR_UNSUPPORTED for BD2. */
aao_status aao_grad_checkpointed(aao_ctx ctx, const double *u0, const double *Uck, int stride,
                                 const double *lam, double *g_u0, double *g_kappa,
                                 double *U_out);

/* Per-kernel timing, for measurement.  aao_set_timing_mask(ctx, mask) clears the
 * accumulators and brackets every later launch of the kernel classes whose bit
 * (1 << AAO_K_...) is set with a pair of HIP events on the context stream;
 * aao_set_timing(ctx, e) sets all bits (e != 0) or none.  aao_get_timing[_ex]
 * synchronises the stream and returns the summed duration (ms), the launch count
 * and (bytes may be NULL) the summed algorithmic bytes of one class: every operand
 * counted once per launch (ell x n FP64 vectors 8 n ell bytes, half spectra
 * (ell/2 + 1) n complex entries of 16 or 8 bytes). */
enum {
    AAO_K_FFT_FWD = 0,          /* time-axis transform, real -> half spectrum     */
    AAO_K_SHIFTED_SOLVE = 1,    /* complex shifted tridiagonal solves             */
    AAO_K_FFT_INV = 2,          /* half spectrum -> real                          */
    AAO_K_MATVEC = 3,           /* block-Toeplitz matvec / residual               */
    AAO_K_CGS_DOT = 4,          /* Gram-Schmidt: projections                      */
    AAO_K_CGS_UPDATE_DOT = 5,   /* Gram-Schmidt: update + re-projections          */
    AAO_K_CGS_UPDATE_NORM = 6,  /* Gram-Schmidt: update + norm                    */
    AAO_K_AXPY = 7,             /* solution update x += Z y                       */
    AAO_K_ARNOLDI_UPDATE = 8,   /* Arnoldi update, delayed re-orthogonalisation   */
    AAO_K_SINE_Y = 9,           /* sine transform along y (unit-square contexts)  */
    AAO_NUM_KERNELS = 10
};
aao_status aao_set_timing(aao_ctx ctx, int enable);
aao_status aao_get_timing(aao_ctx ctx, int kernel, double *total_ms, int64_t *count);
aao_status aao_set_timing_mask(aao_ctx ctx, unsigned mask);
aao_status aao_get_timing_ex(aao_ctx ctx, int kernel, double *total_ms, int64_t *count,
                             double *bytes);

/* Launch shapes of the three kernels of the preconditioner apply (Sec. 3: forward
 * time transform, shifted solves, inverse transform) and of the block-Toeplitz
 * matvec (Sec. 2), and their autotuner.
 * Shape codes:
 *   AAO_CFG_FFT_FWD / AAO_CFG_FFT_INV: 16 v + log2 W, W = columns per workgroup,
 *     v = 0: min(ell/2, 16) points per thread (radix-16 stages), v = 1: 8 points per
 *     thread (radix-8 stages, ell = 1024..8192);
 *   AAO_CFG_SHIFTED_SOLVE: index of a (chunk CW, threads NT, LDS staging) triple;
 *     a staged shape passes the row through LDS half a row at a time;
 *   AAO_CFG_MATVEC: 3 v + r, R = 4 << r time levels per thread, v = 1 for DPP
 *     cross-lane moves, v = 0 for ds_bpermute.
 * -1 means the built-in default.  Shapes are kept per precision mode.
 * aao_tune times every admissible shape of each kernel `reps` times on the context
 * stream with HIP events (on scratch data; the context's vectors are untouched) and
 * keeps the fastest for the current precision mode; it synchronises the stream.
 * Results are cached per process by (device, kernel, precision, n, ell); once
 * aao_set_tune_cache has named a file, results are also read from and appended to it,
 * one line "kernel precision n ell code microseconds" (on a unit-square context n is
 * recorded as -(ny 2^20 + nx), and the matvec has a single shape).
 * aao_set_config rejects a code that does not fit (n, ell) with AAO_ERR_ARG.
 * aao_config_shape decodes a code: FFT -> {points per thread, W, 0}; solve -> {CW,
 * NT, staged}; matvec -> {R, DPP, 0}. */
typedef enum {
    AAO_CFG_FFT_FWD = 0,
    AAO_CFG_SHIFTED_SOLVE = 1,
    AAO_CFG_FFT_INV = 2,
    AAO_CFG_MATVEC = 3,
    AAO_NUM_CFG = 4
} aao_cfg_kind;
aao_status aao_tune(aao_ctx ctx, int reps);
/* Process-wide file of tuned launch shapes (host string, copied; NULL or "" = none). */
aao_status aao_set_tune_cache(const char *path);
aao_status aao_get_config(aao_ctx ctx, int kind, int *code);
aao_status aao_set_config(aao_ctx ctx, int kind, int code);
aao_status aao_config_shape(aao_ctx ctx, int kind, int code, int shape[3]);

/* ------------------------------------------------------------------ batch
 * Many independent problems of uneven size advanced together: every phase of an
 * Arnoldi step is one launch over a work table spanning all problems, converged
 * problems are masked out on the device, and the launch sequence of a group of
 * Arnoldi steps (AAO_BCFG_GRAPH_SPAN, up to a whole restart cycle) is captured once
 * into a hipGraph and replayed.  Batch vectors
 * concatenate the ell_p x n_p arrays of the problems at the offsets returned by
 * aao_batch_offsets (aligned to 64 elements); per-node vectors (u0)
 * concatenate the n_p-vectors without gaps.  The transform along time uses
 * Bluestein's chirp-z form for any ell_p (power-of-two convolution length
 * M_p >= 2 ell_p - 1), so ell_p need not be smooth.  Limits: 1 <= n_p <= 4096,
 * 2 <= ell_p <= 2048.  The batch owns its own HIP stream.
 * Member p is the system A_p U_p = b_p of Sec. 2 (eq. monolithicheat, or system
 * C_BD2) with its own n_p, ell_p, tau_p and kappa_p, preconditioned by its circulant
 * C_p applied as in Sec. 3 (eq. precon2para); the members share no data. */
typedef struct aao_batch_s *aao_batch;

/* count problems; n, ell, kappa: host arrays of count entries; tau: host array or
 * NULL (tau_p = 1/ell_p); scheme as aao_create; prec as aao_set_precision
 * (AAO_PREC_MIXED: single-precision transforms/spectra, FP64 solves and outer
 * GMRES). */
aao_status aao_batch_create(int count, const int64_t *n, const int64_t *ell, const double *tau,
                            const double *kappa, int scheme, int prec, aao_batch *out);
aao_status aao_batch_destroy(aao_batch b);
/* offsets (host, count entries, may be NULL) and total length of a batch vector */
aao_status aao_batch_offsets(aao_batch b, int64_t *offsets, int64_t *total);
/* hipGraph replay of the Arnoldi steps on (1, default) or off (0, eager launches) */
aao_status aao_batch_set_graph(aao_batch b, int enable);
/* Launch shapes of a batch and their tuner.
 *   AAO_BCFG_SLAB        elements per slab of the Gram-Schmidt, update and solution
 *                        passes (a power of two in [256, 65536]; default 4096)
 *   AAO_BCFG_MATVEC_ROWS time levels per matvec tile (2, 4 or 8; default 4)
 *   AAO_BCFG_GRAPH_SPAN  Arnoldi steps per captured graph (1..63), or 0 for the rest of
 *                        the restart cycle: one graph launch per cycle, the host reads
 *                        the number of active problems once per graph.  Steps after
 *                        every problem converged run fully masked, so the results do
 *                        not depend on the span (default 1)
 * aao_batch_tune times the candidates of each shape on the batch's own sizes (reps
 * launches of the slab passes and of the matvec on scratch data; with a right-hand
 * side bvec (device batch vector, may be NULL: span not tuned), reps zero-guess
 * FGMRES(restart) solves of it for each span) and keeps the fastest; results are
 * cached per process and in the aao_set_tune_cache file. */
enum { AAO_BCFG_SLAB = 0, AAO_BCFG_MATVEC_ROWS = 1, AAO_BCFG_GRAPH_SPAN = 2, AAO_NUM_BCFG = 3 };
aao_status aao_batch_get_config(aao_batch b, int kind, int *value);
aao_status aao_batch_set_config(aao_batch b, int kind, int value);
aao_status aao_batch_tune(aao_batch b, const double *bvec, int restart, double tol, int maxit,
                          int reps);
/* u0 (device, sum n_p) = L2 projections of sum_q amps[p*J + q] sin(modes[q] pi x) */
aao_status aao_batch_project_sine(aao_batch b, int J, const int *modes, const double *amps,
                                  double *u0);
/* batch right-hand side from the concatenated u0 (heat: b_1 = M u0 per problem,
 * eq. monolithicheat) */
aao_status aao_batch_build_rhs(aao_batch b, const double *u0, double *bvec);
/* y_p = A_p x_p (A_p^T x_p if transpose) for every member (Sec. 2); x, y device batch
 * vectors, must not overlap */
aao_status aao_batch_apply_A(aao_batch b, const double *x, double *y, int transpose);
/* z_p = C_p^{-1} r_p (C_p^{-T} r_p if transpose) for every member through
 * eq. precon2para: transform along time, shifted tridiagonal solves per frequency,
 * inverse transform, in the batch precision */
aao_status aao_batch_apply_Pinv(aao_batch b, const double *r, double *z, int transpose);
/* FGMRES(restart) on every problem to tol (true relative residual per problem), the
 * preconditioned GMRES of Sec. 4 in its right-preconditioned flexible form, CGS2
 * Arnoldi; x: initial guess in, solutions out; infos: host array of count entries or
 * NULL.  AAO_OK when every problem converged, AAO_NOT_CONVERGED otherwise. */
aao_status aao_batch_gmres(aao_batch b, const double *bvec, double *x, int restart, double tol,
                           int maxit, aao_info *infos);
/* aao_batch_gmres with flags (the AAO_GMRES_* bits of aao_gmres_ex):
 * AAO_GMRES_ZERO_GUESS -- x0 = 0 for every problem whatever x holds (the members'
 * ranges of x are only written, the alignment padding between them not at all; the
 * first cycle starts from b itself, with no residual matvec);
 * AAO_GMRES_TRANSPOSE -- solve A_p^T x_p = b_p with C_p^{-T};
 * AAO_GMRES_CGS2_CLASSIC -- three-pass CGS2.  Captured step graphs are rebuilt when
 * the orientation, the CGS2 form, restart, tol or maxit change.  Other bits:
 * AAO_ERR_ARG. */
aao_status aao_batch_gmres_ex(aao_batch b, const double *bvec, double *x, int restart,
                              double tol, int maxit, int flags, aao_info *infos);
const char *aao_batch_last_error(aao_batch b);

/* Text of a status code (static storage). */
const char *aao_status_string(aao_status st);

/* Last error detail recorded on this context (static per context; "" if none). */
const char *aao_last_error(aao_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* AAO_H */
