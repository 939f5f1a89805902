/*
 * sadi.h -- C ABI of the MI355X (gfx950) implementation of the splitting-ADI
 * (S-ADI) time stepping of Sun & Sun, "Splitting ADI scheme for fractional
 * Laplacian wave equations" (arXiv 2312.06206).
 *
 * Problem (section "Introduction"): d^2u/dt^2 = -kappa (-Delta)^{alpha/2} u + g(u) on
 * Omega = (a,b)^2, u = 0 outside Omega, u(0) = phi1, u_t(0) = phi2, 1 < alpha < 2.
 * Grid (section "Construction of S-ADI scheme"): N interior nodes per direction,
 * h = (b-a)/(N+1), x_i = a + i h; tau is the time step.
 *
 * One step (section "Fast implementation based on GS formula", delta form):
 *   (1 + tau^2 kappa/2 delta_x)(1 + tau^2 kappa/2 delta_y) Uhat = B,
 *   B = -tau^2 kappa L_h u^n + tau^2 g(u^n)                        (n >= 1)
 *   B = tau phi2 - tau^2/2 kappa L_h u^0 + tau^2/2 g(u^0)          (n = 0)
 *   u^{n+1} = 2 u^n - u^{n-1} + Uhat  (n >= 1),   u^1 = u^0 + Uhat  (n = 0)
 * with L_h applied by a block-circulant embedding and 2D FFT, and the two line
 * sweeps H^-1 (H = I + kappa tau^2/(2 h^alpha) T(a_0..a_{N-1})) by the
 * Gohberg-Semencul formula (Proposition 1, Algorithm 1).
 *
 * Conventions for every grid array argument:
 *   - DEVICE pointer to float64, owned by the caller, N*N elements, contiguous;
 *   - element (x_i, y_j), 1 <= i,j <= N, is stored at index (j-1)*N + (i-1)
 *     (x fastest: the paper's column-stacking vec(U));
 *   - arrays must not overlap unless an entry point says so.
 * Calls after setup are asynchronous on the context's stream (default: the null
 * stream), allocate nothing and do not synchronise; device faults surface as
 * SADI_E_DEVICE at a later call or synchronisation.  A context is not
 * thread-safe; any number of contexts may coexist.  The library never aborts:
 * every failure is a status plus a message from sadi_last_error().
 *
 * Supported sizes: 15 <= N <= 4095.  The line transforms have length M, the smallest power
 * of two >= N + 1 (the block-circulant embedding of L_h has size 2M).  The line solves
 * apply the Gohberg-Semencul formula to H_M = I + beta T(a_0..a_{M-1}) and correct to
 * H_N^-1 through the Schur complement, H_N^-1 v = w[0:N] - F w[N:M] with w = H_M^-1 [v; 0]
 * and F = -H_N^-1 H_M[0:N, N:M]: a rank-one correction when N + 1 = M (the fast case),
 * rank M - N otherwise.  In the time step a correction of rank above 3 is applied to all
 * lines at once by one matrix-core product per sweep (the library's own kernel, on the
 * context stream).  The float32 line solves need N + 1 = M.
 */
#ifndef SADI_H
#define SADI_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sadi_ctx sadi_ctx;

typedef enum {
  SADI_OK = 0,
  SADI_E_INVALID = -1,     /* bad argument (range, NULL, size) */
  SADI_E_NOMEM = -2,       /* device or host allocation failed */
  SADI_E_DEVICE = -3,      /* HIP runtime error (launch, copy, earlier async fault) */
  SADI_E_UNSUPPORTED = -4, /* valid problem the library does not handle (N outside [15, 4095], ...) */
  SADI_E_STATE = -5        /* NULL or destroyed context */
} sadi_status;

/* Nonlinearity g(u). */
typedef enum {
  SADI_G_ZERO = 0,
  SADI_G_NEG_SIN = 1,    /* -sin u   (sine-Gordon, the paper's first example) */
  SADI_G_NEG_CUBE = 2,   /* -u^3     (Klein-Gordon, the paper's second example) */
  SADI_G_NEG_LINEAR = 3  /* -m u     (m = g_param) */
} sadi_g_kind;

/* Arithmetic of the Gohberg-Semencul line solves (state, right-hand side and
 * BTTB product are always float64). */
typedef enum {
  SADI_FP64 = 0,         /* float64 transforms */
  SADI_FP32_REFINE = 1,  /* float32 transforms + one float64 residual correction per line */
  SADI_FP32 = 2          /* float32 transforms only (error about 1e-7 relative) */
} sadi_precision;

/* Create a context for (alpha, kappa, N, tau, Omega = (domain[0], domain[1])^2).
 * Validates 1 < alpha < 2, kappa > 0, tau > 0, domain[1] > domain[0] (all finite).
 * Computes the 1D coefficients a_k (closed form, section 2; host, extended precision),
 * the 2D coefficients a_ij of L_h (Fourier coefficients of the symbol by a quadrature of
 * its subordination integral: Bessel node rows from a per-device table, two matrix-core
 * products on the device, an exact low-order corner from the host), the generating vector
 * H_M^-1 e_1 of the size-M line matrix and its circulant / skew-circulant eigenvalues
 * (Proposition 1; on the device in double-double arithmetic when N + 1 = M, else on the
 * host in extended precision with the rank-(M - N) correction), and the eigenvalues of
 * the block-circulant embedding of L_h (device).  Allocates the device workspaces in one
 * block.  Uses the current HIP device; the device work runs on streams of its own.
 * Host-synchronous.  Defaults: g = -sin u, float64.  domain: host pointer to 2 doubles.
 * *out receives the context (NULL on error). */
sadi_status sadi_setup(double alpha, double kappa, int n, double tau, const double* domain, sadi_ctx** out);

/* Same, with caller-supplied coefficient tables instead of the computed ones
 * (host pointers): a1 holds a_0..a_N (N+1 values), a2 holds a_ij for
 * 0 <= i,j < N at a2[j*N + i].  alpha only enters through h^alpha here, and
 * alpha = 2 is accepted (classical 3-point / 5-point operators). */
sadi_status sadi_setup_with_coeffs(double alpha, double kappa, int n, double tau, const double* domain,
                                   const double* a1, const double* a2, sadi_ctx** out);

/* Select g and the line-solve arithmetic (takes effect at the next call).  With
 * SADI_FP32_REFINE every line solve is x0 = GS32(v), r = v - H x0 in float64 (product with
 * H through a 2(N+1)-point circulant embedding), x = x0 + GS32(r); SADI_FP32 stops at x0.
 * Both apply to sadi_first_step / sadi_step / sadi_run and sadi_toeplitz_solve. */
sadi_status sadi_set_options(sadi_ctx* ctx, sadi_g_kind g, double g_param, sadi_precision prec);

/* Run subsequent calls on this HIP stream (a hipStream_t, e.g. torch's current
 * stream); NULL selects the null stream.  The stream must outlive its use. */
sadi_status sadi_set_stream(sadi_ctx* ctx, void* hip_stream);

/* Start-up step n = 0 (scheme (ADI scheme initial)): u1 <- u^1 from u^0 = phi1 and
 * u_t(0) = phi2.  phi1, phi2, u1: device grid arrays; u1 must not alias phi1/phi2. */
sadi_status sadi_first_step(sadi_ctx* ctx, const double* phi1, const double* phi2, double* u1);

/* One step n >= 1 (scheme (ADI scheme)): on entry u_prev = u^{n-1}, u_cur = u^n;
 * on exit u_prev = u^{n+1} (u_cur unchanged). */
sadi_status sadi_step(sadi_ctx* ctx, double* u_prev, const double* u_cur);

/* Allocation-free form of sadi_step, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, result and stream as sadi_step; allocates nothing (no hipMalloc, no library
 * call that allocates, no timing events).  The step's work space -- the half spectrum and
 * the x-sweep result, 16 (N+1)(M+8) + 8 (N+1) M bytes -- lives in a static device array of
 * 32 MiB instead of the context's buffers.  Each GPU that loads the library holds its own
 * array until the process ends; its address is looked up at sadi_setup with the context's
 * device current.  Limits: the work space must fit (N <= 1023) and M - N <= 3
 * (SADI_E_UNSUPPORTED otherwise, with the sizes in the message); the context's device must
 * be current (SADI_E_INVALID).  All calls on one GPU share the array and it keeps the last
 * call's contents (every step writes what it reads, nothing needs clearing): calls that
 * overlap in time on one GPU -- other streams, contexts or threads -- race and give wrong
 * results. */
sadi_status sadi_step_noalloc(sadi_ctx* ctx, double* u_prev, const double* u_cur);

/* nsteps >= 0 steps n >= 1.  On entry (u_prev, u_cur) = (u^{n-1}, u^n); on exit
 * (u_prev, u_cur) = (u^{n+nsteps-1}, u^{n+nsteps}).  Unless the correction rank M - N
 * exceeds 3, the steps alternate between the grid and its transpose (the scheme is
 * symmetric in x and y), in every precision: the state is copied into the context's own
 * arrays (in pairs of rows, u^{n-1} transposed) before the first step and back after the
 * last, and u_prev is read only there.  Above rank 3 both arrays are work space while the
 * calls run.  The result matches nsteps calls of sadi_step to rounding. */
sadi_status sadi_run(sadi_ctx* ctx, double* u_prev, double* u_cur, int nsteps);

/* In place, lines[r*ld + i] <- (H^-1 v_r)_i for r < nlines, i < N, where v_r is
 * line r and H = I + kappa tau^2/(2 h^alpha) T(a_0..a_{N-1}) (Proposition 1 /
 * Algorithm 1).  lines: device float64 pointer; ld >= N. */
sadi_status sadi_toeplitz_solve(sadi_ctx* ctx, double* lines, int nlines, int ld);

/* out <- L_h u (the discrete fractional Laplacian, section 2), device grid arrays,
 * no aliasing. */
sadi_status sadi_apply_lh(sadi_ctx* ctx, const double* u, double* out);

/* Per-kernel timing (observability).  When enabled, sadi_first_step / sadi_step /
 * sadi_run record HIP events on the context's stream between the kernels of every
 * step (one event before the first kernel and one after each kernel), so each
 * kernel's device time is the difference of consecutive events.  Enabling resets
 * the accumulators; events are created on demand (at most 8192 steps are kept).
 * sadi_get_kernel_times synchronises the stream and writes, for the four parts
 * of a step -- 0 row forward transforms, 1 column convolution, 2 row inverse
 * transforms + right-hand side + x-line solves, 3 y-line solves + update --
 * the summed milliseconds (ms[4]) and the number of steps timed (count[4]).  In a
 * float64 sadi_run the y-line kernel also does the next step's row transforms (on the
 * transposed grid), so part 0 holds time only for the run's first step. */
sadi_status sadi_set_kernel_timing(sadi_ctx* ctx, int enable);
sadi_status sadi_get_kernel_times(sadi_ctx* ctx, double* ms, long long* count);

/* The context's Gohberg-Semencul tables (Proposition 1, Algorithm 1) copied to host memory:
 * lam_s, lam_c (M complex values each, as 2M doubles re/im) and the correction f ((M - N) x N
 * values; f[k] = c[M-1-k] / c[0] when N + 1 = M).  Any pointer may be NULL.  When N + 1 = M
 * they were formed on the device (double-double Levinson-Durbin recursion for
 * c = H_M^-1 e_1, then direct DFTs); sadi_host_line_tables gives the host's own.
 * Host-synchronous. */
sadi_status sadi_get_line_tables(const sadi_ctx* ctx, double* lam_s, double* lam_c, double* f);

/* Sizes of the context: N, M = N+1, and device bytes held (any pointer may be NULL). */
sadi_status sadi_get_info(const sadi_ctx* ctx, int* n, int* m, long long* device_bytes);

/* Free the context and its device memory (synchronises its stream).  NULL is a no-op. */
sadi_status sadi_destroy(sadi_ctx* ctx);

/* Message of the last failing call on this thread ("" if none). */
const char* sadi_last_error(void);

/* ---- host-only helpers (no GPU needed) ------------------------------------
 * The host setup mathematics, exposed for testing and for callers that want
 * the tables.  All pointers are HOST pointers. */

/* a_k, k = 0..count-1, of the 1D fractional centred difference (closed form of
 * section 2, evaluated by its Gamma-ratio recurrence in extended precision). */
sadi_status sadi_host_riesz_coeffs(double alpha, int count, double* out);

/* a_ij, 0 <= i,j < n, of L_h (out[j*n + i]); Fourier coefficients of
 * (4 sin^2(eta/2) + 4 sin^2(xi/2))^{alpha/2}, computed through the subordination
 * integral s^beta = beta/Gamma(1-beta) int_0^inf (1 - e^{-ts}) t^{-1-beta} dt. */
sadi_status sadi_host_laplacian_coeffs(double alpha, int n, double* out);

/* c = H_M^-1 e_1 of the bordered line matrix (M = n+1 unknowns, Levinson-Durbin in
 * extended precision); out has n+1 entries. */
sadi_status sadi_host_line_generator(double alpha, double kappa, int n, double tau, const double* domain,
                                     double* out);

/* The same tables computed on the host (extended-precision Levinson-Durbin recursion and
 * FFTs), for the problem sadi_setup would build: lam_s, lam_c: 2M doubles each; f: (M - N) N
 * doubles.  Host pointers. */
sadi_status sadi_host_line_tables(double alpha, double kappa, int n, double tau, const double* domain,
                                  double* lam_s, double* lam_c, double* f);

/* Node rows of the quadrature that gives a_ij (the subordination integral above, on
 * nodes t_q equally spaced in log t): *nodes receives their number, x (if not NULL) the
 * arguments x_q = 2 t_q, and rows (if not NULL, nodes x nrows values) e^{-x_q} I_k(x_q) at
 * rows[q * nrows + k] for k < nrows <= 4096.  fp64 = 0: the host's extended-precision (long
 * double) recurrence; fp64 = 1: the double-double float64 recurrence that builds the table
 * on the GPU, run here on the host (the two are compared in the tests).  Host pointers. */
sadi_status sadi_host_quadrature_rows(int nrows, int fp64, int* nodes, double* x, double* rows);

/* Reverse-mode (adjoint) step, for gradients of a scalar J(u^K) with respect to phi1 and
 * kappa through the delta form above.  With J_n = H^-1 (-c kappa L_h + c diag g'(u^n)) H^-1
 * the Jacobian of the increment (c = tau^2, or tau^2/2 for the start-up step; H, L_h
 * symmetric, so J_n^T has the same form with the sweeps applied first):
 *   mode 0 (step n >= 1):  a_cur = 2 a_next - a_next2 + J_n^T a_next,
 *   mode 1 (start-up n=0): a_cur =   a_next - a_next2 + J_0^T a_next   (= dJ/dphi1),
 * where a_next = dJ/du^{n+1}, a_next2 = dJ/du^{n+2} (NULL: zero), both totals.  dkappa
 * (device pointer to one double) is incremented by <a_next, d u^{n+1} / d kappa> at fixed
 * u^n, u^{n-1}: -c <L_h z, u^n> - (2 <a, U> - <H_x^-1 a, U> - <H_y^-1 a, U>) / kappa with
 * z = H^-1 a H^-1 and U = u^{n+1} - u^n - (u^n - u^{n-1}) (mode 1: u^1 - u^0); the sweep terms
 * use d H^-1 / d kappa = -H^-1 (H - I) H^-1 / kappa.  u_prev = u^{n-1} (unused for mode 1),
 * u_cur = u^n, u_next = u^{n+1}: device grids as above; a_cur must not alias the other
 * arguments.  float64 contexts only (SADI_E_UNSUPPORTED otherwise).  Uses the context's
 * workspaces; asynchronous on the context stream. */
sadi_status sadi_adjoint_step(sadi_ctx* c, int mode, const double* u_prev, const double* u_cur,
                              const double* u_next, const double* a_next, const double* a_next2, double* a_cur,
                              double* dkappa);

/* ---------------------------------------------------------------------------------
 * Batches: many independent problems of the same scheme (same tau, domain and g = -sin u,
 * FP64), each with its own N, alpha and kappa, advanced together.  Instances with equal N
 * form a group; every phase of a step (the passes of the delta form above) is one launch
 * over all instances of a group, or one launch over several groups (see
 * sadi_batch_set_schedule).  The two line sweeps of a group take one of three
 * paths:
 *   SADI_PATH_FFT_GS       the Gohberg-Semencul line solves (Proposition 1, Algorithm 1);
 *   SADI_PATH_DENSE        X = H^-1 B H^-1 as two batched FP64 matrix products with the
 *                          explicit inverse (H is fixed for the whole run, section "Fast
 *                          implementation based on GS formula"), computed once at creation
 *                          by the line solve on the identity;
 *   SADI_PATH_DENSE_MIXED  the same products with FP32 operands on the FP32 matrix cores,
 *                          then one FP64 residual R = B - H Y H (two FP64 products with H)
 *                          and the FP32 correction Y + H^-1 R H^-1: about FP64 accuracy
 *                          (the FP32 error squared), the state and B staying FP64.
 * sadi_batch_tune times them and keeps the fastest per group.  Multi-step runs can be
 * replayed from a captured HIP graph.  The batch works on its own HIP stream (see
 * sadi_batch_synchronize); the caller must have finished writing the bound arrays
 * before a call and must synchronise before reading them. */
typedef struct sadi_batch sadi_batch;

typedef enum { SADI_PATH_FFT_GS = 0, SADI_PATH_DENSE = 1, SADI_PATH_DENSE_MIXED = 2 } sadi_line_path;

/* count instances; n, alpha, kappa: host arrays of count entries (each validated as in
 * sadi_setup); tau and domain (host, 2 doubles) are shared.  Groups with N <= dense_max_n
 * may take the two dense paths; their explicit inverses (N*N doubles per instance) and,
 * for SADI_PATH_DENSE_MIXED, the FP32 copies and H itself (N*N floats and doubles) are
 * built when a dense path is first timed (sadi_batch_tune) or chosen (sadi_batch_set_path).
 * Host-synchronous; allocates everything the batch needs.  The instances are set up on
 * concurrent host threads; the line tables of all of them (N + 1 a power of two) are then
 * built in one pair of launches.  All groups start on SADI_PATH_FFT_GS. */
sadi_status sadi_batch_create(int count, const int* n, const double* alpha, const double* kappa, double tau,
                              const double* domain, int dense_max_n, sadi_batch** out);

/* Bind the state: host arrays of count DEVICE pointers, each an N_i*N_i float64 grid in
 * the layout above (caller-owned).  u_prev[i] holds u^{n-1} (or phi1 before the start-up
 * step), u_cur[i] holds u^n.  phi2 (may be NULL unless sadi_batch_first_step is used):
 * start-up velocities.  Host-synchronous (uploads the instance descriptors). */
sadi_status sadi_batch_bind(sadi_batch* b, double* const* u_prev, double* const* u_cur, const double* const* phi2);

/* Start-up step of every instance (delta form, n = 0): u_cur <- u^1 from u_prev = phi1. */
sadi_status sadi_batch_first_step(sadi_batch* b);

/* nsteps steps n >= 1 of every instance, in place: on return u_prev, u_cur hold
 * u^{n+nsteps-1}, u^{n+nsteps}.  Asynchronous on the batch stream; no allocation (the
 * first call with graphs enabled captures and instantiates the graph).  The arrays are
 * work space while the call runs: groups on the FFT path alternate between the grid and
 * its transpose from step to step, as sadi_run does. */
sadi_status sadi_batch_run(sadi_batch* b, int nsteps);

/* enable != 0: sadi_batch_run replays two steps at a time from a captured HIP graph. */
sadi_status sadi_batch_set_graph(sadi_batch* b, int enable);

/* Force the line-sweep path of the group with this N (SADI_E_UNSUPPORTED for the dense
 * paths above dense_max_n). */
sadi_status sadi_batch_set_path(sadi_batch* b, int n, int path);

/* Schedule of the step's launches: 1 (default) -- the groups on SADI_PATH_FFT_GS with
 * M <= 2048 share one launch per phase (column convolution, row pass with the x-sweep,
 * y-sweep with the next row transform), each workgroup taking its instance and block from a
 * device work list ordered so that an instance stays on one XCD and the XCDs get equal work;
 * other groups (SADI_PATH_DENSE, M = 4096) are launched on their own; 0 -- every group is
 * launched on its own. */
sadi_status sadi_batch_set_schedule(sadi_batch* b, int schedule);
/* The current schedule and the tuned milliseconds per step of schedules 0 and 1 (-1: not
 * timed).  Any pointer may be NULL. */
sadi_status sadi_batch_get_schedule(const sadi_batch* b, int* schedule, double* ms_groups, double* ms_lists);

/* Autotuner: for every group, time `steps` steps of each available path on zero scratch
 * state (the bound state is not touched) -- the dense paths with both tile shapes of their
 * products (64 x 64 and 32 x 32 blocks of the result per workgroup) -- and keep the fastest;
 * then time the whole step under both schedules with those paths and keep the faster
 * schedule.  Host-synchronous. */
sadi_status sadi_batch_tune(sadi_batch* b, int steps);

/* Group `index` (0 <= index < groups): its N, member count, current path, the tuned
 * milliseconds per step of each path (-1 if not timed) and the tile of the products of the
 * current dense path (SADI_PATH_DENSE's when on the FFT path; 64 or 32, 0: chosen by the
 * number of tiles).  Any output pointer may be NULL. */
sadi_status sadi_batch_get_group(const sadi_batch* b, int index, int* n, int* members, int* path, double* ms_fft,
                                 double* ms_dense, double* ms_dense_mixed, int* dense_tile);

/* Instance and group counts, device bytes held by the batch. */
sadi_status sadi_batch_get_info(const sadi_batch* b, int* count, int* groups, long long* bytes);

/* Wait for all work queued on the batch stream. */
sadi_status sadi_batch_synchronize(sadi_batch* b);

sadi_status sadi_batch_destroy(sadi_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* SADI_H */
