/*
 * adr.h -- C ABI of the MI355X (gfx950) ILU(0)-preconditioned BiCGSTAB solver
 * for the 2-D steady advection-diffusion problem of Datta & Carrasco Heres,
 * arXiv:1308.5215:
 *
 *     eps (u_xx + u_yy) + a(x,y) u_x + b(x,y) u_y = f   on [0,X] x [0,Y],
 *     a = 1 + x^2,  b = X exp(-y),                      (Section 2, eq. (1))
 *
 * with Dirichlet data on x = 0 and y = 0 and either Dirichlet or Neumann data
 * on x = X and y = Y, taken from the manufactured solution
 * u = exp(-x/X) (1 - exp(-y/Y)) y (Sections 2-3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid.   nx * ny interior unknowns; unknown (i, j), 0 <= i < nx, 0 <= j < ny,
 *         lives at x = (i+1) dx, y = (j+1) dy, dx = X/(nx+1), dy = Y/(ny+1),
 *         and is stored at k = j*nx + i (x fastest; the lexicographic order of
 *         the paper's assembly).  nx = m-1, ny = n-1 for the paper's m, n
 *         intervals.
 * Vectors. FP64, length nx*ny, in that order.  "_dev" pointers are device
 *         pointers on the current HIP device; "_host" pointers are host
 *         memory.  The caller owns every pointer it passes; the library
 *         copies what it keeps and never frees caller memory.
 * Streams. Every call is issued on the stream given to adr_assemble (NULL =
 *         the default stream) and has completed on return.
 * Errors.  Negative adr_status values are call errors (nothing or only part
 *         of the work was done: check adr_last_error()); non-negative values
 *         are outcomes.  Argument errors are detected before any device work.
 * Threads. A problem handle must not be used by two threads at once.
 */
#ifndef ADR_H
#define ADR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ADR_OK = 0,
  ADR_ERR_ARG = -1,       /* invalid argument (see adr_last_error)          */
  ADR_ERR_NOMEM = -2,     /* device allocation failed                       */
  ADR_ERR_DEVICE = -3,    /* HIP runtime error or device-side fault report  */
  ADR_ERR_STATE = -4,     /* call out of order (e.g. solve before ilu0)     */
  ADR_MAXIT = 1,          /* maxit passes done without convergence          */
  ADR_BREAKDOWN_RHO = 2,  /* rho = r^.r = 0 at the start of a pass          */
  ADR_OMEGA_ZERO = 3,     /* omega = 0 (the method's own stop)              */
  ADR_ZERO_PIVOT = 4,     /* ILU(0) met a zero or non-finite pivot          */
  ADR_NONFINITE = 5,      /* a scalar of the iteration became Inf or NaN    */
  ADR_INACCURATE = 6      /* the recursively updated residual passed the
                             stopping test but the true residual b - A x did
                             not, and the restarts allowed are used up        */
} adr_status;

typedef enum {
  ADR_UPWIND = 0,   /* the paper's "hybrid" scheme: centred second differences,
                       backward first differences (Section 4)                */
  ADR_CENTERED = 1  /* centred first and second differences (Section 4)     */
} adr_scheme;

typedef enum {
  ADR_BC_DIRICHLET = 0,  /* Dirichlet on all four sides                     */
  ADR_BC_NEUMANN_XY = 1  /* Dirichlet on x = 0, y = 0; Neumann on x = X and
                            y = Y, closed by the one-sided difference of the
                            paper's Neumann assembly routines               */
} adr_bc;

typedef enum {
  ADR_FP64 = 0,          /* factors and sweeps in FP64                      */
  ADR_FP32_FACTORS = 1,  /* ILU(0) factors stored in FP32, sweep arithmetic
                            in FP64                                          */
  ADR_FP32_SWEEPS = 2    /* ILU(0) factors stored in FP32 and the triangular
                            sweeps computed in FP32; SpMV, inner products,
                            scalars and the stopping test stay FP64         */
} adr_precision;

typedef struct adr_problem adr_problem;   /* opaque, library-owned */

typedef struct {
  int32_t status;       /* adr_status of the solve                               */
  int32_t iters;        /* loop passes started; a half-step exit counts         */
  int32_t hist_len;     /* valid entries in hist_l2 / hist_max                  */
  int32_t half_step;    /* 1 if the solve ended on the ||s|| test               */
  double bnorm;         /* ||b||_2                                               */
  double true_relres;   /* ||b - A x||_2 / ||b||_2 recomputed at exit            */
  double solve_ms;      /* device time of the iteration (events on the stream)  */
  int32_t restarts;     /* restarts from the current iterate (see the solve)    */
  int32_t pad;
} adr_solve_info;

/* ---------------------------------------------------------------------------
 * adr_assemble -- Section 4 discretisation into five diagonals.
 *
 * Builds, on the device, S (k-nx), W (k-1), C (k), E (k+1), N (k+nx) and the
 * right-hand side of every interior equation multiplied by dx^2 dy^2:
 *   upwind:   S = eps dx^2 - b dx^2 dy,        W = eps dy^2 - a dx dy^2,
 *             C = -2 eps (dx^2 + dy^2) + a dx dy^2 + b dx^2 dy,
 *             E = eps dy^2,                   N = eps dx^2;
 *   centered: S = eps dx^2 - b dx^2 dy / 2,    W = eps dy^2 - a dx dy^2 / 2,
 *             C = -2 eps (dx^2 + dy^2),
 *             E = eps dy^2 + a dx dy^2 / 2,   N = eps dx^2 + b dx^2 dy / 2;
 *   rhs = f dx^2 dy^2 minus boundary couplings times boundary data; Neumann:
 *   C += E (x = X edge), C += N (y = Y edge), rhs -= E dx g_x, rhs -= N dy g_y.
 * Couplings to boundary nodes are stored as 0.
 * f is the manufactured forcing of Section 3; if field_dev != NULL (nx*ny
 * FP64 values), f = f_man + amp * max|f_man| * field (max over interior
 * nodes), the forcing perturbation of a random-field workload.
 * eps, X, Y > 0; nx, ny >= 1; nx*ny <= 2^31 - 1.
 * stream: a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream) or NULL.
 * On success *out receives a new problem handle (free with adr_destroy).
 * ------------------------------------------------------------------------- */
adr_status adr_assemble(double eps, double X, double Y, int32_t nx, int32_t ny,
                        int32_t scheme, int32_t bc,
                        const double *field_dev, double amp,
                        void *stream, adr_problem **out);

/* ---------------------------------------------------------------------------
 * adr_ilu0 -- ILU(0) of Section 5.1 (Saad): the incomplete LU factorisation
 * whose sparsity pattern is that of A.  For the five-point matrix the factor
 * L is unit lower with lw at (k,k-1) and ls at (k,k-nx), U = diag(d) + the
 * E, N diagonals of A, and the pivots follow
 *     d_k = C_k - lw_k E_{k-1} - ls_k N_{k-nx},
 *     lw_k = W_k / d_{k-1},  ls_k = S_k / d_{k-nx}
 * (computed as invd = 1/d, lw = W*invd_{k-1}, ls = S*invd_{k-nx},
 *  d = fma(-ls, N_{k-nx}, fma(-lw, E_{k-1}, C))), swept over anti-diagonals.
 * precision selects the storage/arithmetic of the sweeps that apply M^{-1}
 * (adr_precision).  Returns ADR_ZERO_PIVOT if some pivot is 0 or not finite;
 * then *bad_index (if not NULL) receives the first such k in lexicographic
 * order and the problem cannot be solved.  Otherwise *bad_index = -1.
 * ------------------------------------------------------------------------- */
adr_status adr_ilu0(adr_problem *p, int32_t precision, int64_t *bad_index);

/* ---------------------------------------------------------------------------
 * adr_bicgstab_solve -- right-preconditioned BiCGSTAB of Section 5.2 with
 * M = L U from adr_ilu0.
 *   r0 = b - A x0, r^ = r0; per pass i: rho = r^.r (ADR_BREAKDOWN_RHO if 0);
 *   p = r (i = 1) or r + beta (p - omega v), beta = (rho_i/rho_{i-1})(alpha/omega);
 *   p^ = M^{-1} p; v = A p^; alpha = rho / r^.v; s = r - alpha v;
 *   if ||s||_2 < tol ||b||_2: x += alpha p^ and stop (half step);
 *   z = M^{-1} s; t = A z; omega = t.s / t.t; x += alpha p^ + omega z;
 *   r = s - omega t; stop if ||r||_2 < tol ||b||_2; stop if omega = 0.
 * Inner products are double-double accumulations rounded once to FP64, so the
 * result does not depend on the summation order.  If ||r0|| already passes
 * the test no pass is made; b = 0 gives x = 0.
 * True residual: the tests above read the recursively updated residual, which
 * can drift from b - A x (the paper does not address this).  A solve is
 * reported ADR_OK only if ||b - A x||_2 < tol ||b||_2 too: when the recursion
 * converges the next pass slot recomputes e = b - A x; if e passes, the solve
 * stops OK; otherwise, with passes left and fewer than max_restarts restarts
 * made (adr_set_max_restarts, default 8), the method restarts from the
 * current x as from an initial guess (r = r^ = p = e, and that slot is the
 * first pass of the restart); with no pass left the status is ADR_MAXIT,
 * with no restart left ADR_INACCURATE.
 * x0_dev: initial guess (device, nx*ny) or NULL for zero.
 * x_dev:  output (device, nx*ny); may equal x0_dev.
 * hist_l2_host, hist_max_host: NULL or host arrays of maxit+1 entries:
 *   entry 0 = ||r0||, entry i = ||r_i|| after pass i (the recursively updated
 *   residual), or ||s|| at a half-step exit; 2-norm and max-norm.
 * info: optional summary.  tol >= 0, maxit >= 0.
 * Returns the solve status (ADR_OK, ADR_MAXIT, ADR_BREAKDOWN_RHO,
 * ADR_OMEGA_ZERO, ADR_NONFINITE, ADR_INACCURATE) or a call error; x_dev holds
 * the last iterate in every outcome.
 * ------------------------------------------------------------------------- */
adr_status adr_bicgstab_solve(adr_problem *p, double tol, int32_t maxit,
                              const double *x0_dev, double *x_dev,
                              double *hist_l2_host, double *hist_max_host,
                              adr_solve_info *info);

/* Restarts allowed by the true-residual confirmation of a solve (above):
 * n >= 0 restarts (default 8), or -1 to accept the recursive residual's test
 * alone, as the algorithm of Section 5.2 and the appendix's solver do.
 * ADR_ERR_ARG for n < -1. */
adr_status adr_set_max_restarts(adr_problem *p, int32_t n);

/* ---------------------------------------------------------------------------
 * adr_assemble_data -- Section 4 assembly from the caller's problem data, as
 * the paper's assembly routines take it (forcing f and the boundary data of
 * the four sides), with the paper's input rule: each item is either absent
 * (NULL pointer, length 0: the manufactured value of Sections 2-3), a single
 * value used at every node (length 1), or one value per node (length nx*ny
 * for f, ny for the x-sides, nx for the y-sides); any other length is
 * ADR_ERR_ARG.
 *   f     forcing at the interior nodes (k = j*nx + i);
 *   u_x0  u(0, y_j);   u_xX  u(X, y_j), or du/dx(X, y_j) with ADR_BC_NEUMANN_XY;
 *   u_y0  u(x_i, 0);   u_yY  u(x_i, Y), or du/dy(x_i, Y) with ADR_BC_NEUMANN_XY.
 * f_on_device = 1: f is device memory (length nx*ny only); the edge arrays
 * are host memory.  Everything else is as adr_assemble (stencils, the
 * Neumann closure, errors, the handle).
 * ------------------------------------------------------------------------- */
typedef struct {
  const double *f;    int64_t f_len;
  const double *u_x0; int64_t u_x0_len;
  const double *u_xX; int64_t u_xX_len;
  const double *u_y0; int64_t u_y0_len;
  const double *u_yY; int64_t u_yY_len;
  int32_t f_on_device;
  int32_t pad;
} adr_problem_data;

adr_status adr_assemble_data(double eps, double X, double Y, int32_t nx, int32_t ny,
                             int32_t scheme, int32_t bc, const adr_problem_data *data,
                             void *stream, adr_problem **out);

/* ---------------------------------------------------------------------------
 * adr_max_error -- the discretisation error of a solution (Sections 6.1-6.8):
 * max over all (nx+2) x (ny+2) grid nodes of |U - u_exact|, with
 * u_exact = exp(-x/X) (1 - exp(-y/Y)) y and U the solution x_dev at the
 * interior nodes, the exact u on Dirichlet sides, and on the Neumann sides
 * of ADR_BC_NEUMANN_XY the one-sided closure U(X, y) = U(x_nx, y) + dx g_x(y),
 * U(x, Y) = U(x, y_ny) + dy g_y(x) (corner from the x-direction), as the
 * paper's Neumann drivers reconstruct them.  Meaningful for the manufactured
 * problem.  x_dev: a (batched) device vector; err_host: one double per
 * instance.
 * ------------------------------------------------------------------------- */
adr_status adr_max_error(adr_problem *p, const double *x_dev, double *err_host);

/* ---------------------------------------------------------------------------
 * adr_classify -- what an instance's discretisation looks like before it is
 * solved (Section 6.3, mesh Reynolds number; the Neumann failures noted in
 * Section 6.1).  Host-only, no device work.
 *   pe_x, pe_y   cell Peclet numbers max_i a_i dx / eps, max_j b_j dy / eps;
 *   g_y          X (1 - exp(-Y)) / eps, the integral of b / eps over y: the
 *                Neumann-closed operator grows like exp(g_y);
 *   neg_offdiag  couplings between interior unknowns that are negative;
 *   nonneg_diag  unknowns whose diagonal C is >= 0 (sign change: ILU(0)
 *                pivots can pass through zero);
 *   expect_fail  1 if the solve is not expected to reach
 *                ||b - A x|| < tol ||b||: Neumann data with g_y > ln(tol/u),
 *                u = 2^-53 (the true residual cannot fall below about
 *                u exp(g_y)); a diagonal that changes sign inside the grid;
 *                or the upwind scheme (downwind for eq. (1)) with a negative
 *                diagonal and a cell Peclet number above 2 (Section 6.3).
 * ------------------------------------------------------------------------- */
typedef struct {
  double pe_x, pe_y, g_y;
  int64_t neg_offdiag, nonneg_diag;
  int32_t expect_fail;
  int32_t pad;
} adr_instance_class;

adr_status adr_classify(double eps, double X, double Y, int32_t nx, int32_t ny, int32_t scheme,
                        int32_t bc, double tol, adr_instance_class *out);

/* Release every device resource of the problem (NULL is a no-op). */
void adr_destroy(adr_problem *p);

/* ---------------------------------------------------------------------------
 * Batches: many independent instances (each its own eps, X, Y, nx, ny,
 * scheme, bc) held in one problem and advanced together by the same kernel
 * launches -- one launch per step of the method covers every instance, so
 * small grids share the GPU and the wavefront latency of one instance is
 * hidden behind the others.  Instance k occupies elements
 * [offset[k], offset[k+1]) of every batched vector (adr_batch_layout), in the
 * per-instance order described above.  A single-instance problem is a batch
 * of one; the single-instance calls above accept only count == 1.
 * ------------------------------------------------------------------------- */

/* Section 4 assembly of `count` instances (arrays of `count` entries; the
 * argument rules of adr_assemble apply to each).  field_dev: NULL or a
 * batched device vector added to each instance's manufactured forcing with
 * amplitude amp * max|f_man| of that instance. */
adr_status adr_batch_assemble(int32_t count, const double *eps, const double *X, const double *Y,
                              const int32_t *nx, const int32_t *ny, const int32_t *scheme,
                              const int32_t *bc, const double *field_dev, double amp,
                              void *stream, adr_problem **out);

/* The same from each instance's own problem data (adr_assemble_data);
 * data: `count` records, or NULL for the manufactured problems. */
adr_status adr_batch_assemble_data(int32_t count, const double *eps, const double *X, const double *Y,
                                   const int32_t *nx, const int32_t *ny, const int32_t *scheme,
                                   const int32_t *bc, const adr_problem_data *data,
                                   void *stream, adr_problem **out);

/* Number of instances and their offsets (count + 1 entries; the last is the
 * total length of a batched vector).  Either output may be NULL. */
adr_status adr_batch_layout(const adr_problem *p, int32_t *count, int64_t *offsets);

/* ILU(0) of every instance (Section 5.1), one launch for the batch.
 * bad_index: NULL or `count` entries (-1, or the first zero pivot). */
adr_status adr_batch_ilu0(adr_problem *p, int32_t precision, int64_t *bad_index);

/* BiCGSTAB (Section 5.2) on every instance with the same tol and maxit; each
 * instance stops on its own tests and is skipped by later launches.
 * x0_dev / x_dev: batched device vectors (x0 may be NULL).
 * hist_l2, hist_max: NULL or count*(maxit+1) host doubles, instance-major.
 * info: NULL or `count` records (solve_ms is the batch's time).
 * Returns ADR_OK if every instance reached the tolerance, else the status of
 * the first instance that did not, or a call error. */
adr_status adr_batch_solve(adr_problem *p, double tol, int32_t maxit, const double *x0_dev,
                           double *x_dev, double *hist_l2, double *hist_max, adr_solve_info *info);

/* Sweep-schedule autotuner: times M^{-1} on the problem's right-hand sides
 * for every supported schedule -- 16-row strips, and 32-row strips with one
 * workgroup per CU (deep LDS ring) or two (compact ring) -- keeps the fastest
 * and returns its strip height (and the time of one application in ms).
 * Needs adr_ilu0 / adr_batch_ilu0 first; results do not depend on the choice. */
adr_status adr_autotune(adr_problem *p, int32_t *rows_chosen, double *ms_per_apply);

/* ---------------------------------------------------------------------------
 * Inspection and single-step entry points (the same kernels the solve uses).
 * ------------------------------------------------------------------------- */

/* Copy the assembled diagonals and rhs to host arrays of nx*ny entries
 * (any may be NULL). */
adr_status adr_get_dia(const adr_problem *p, double *S, double *W, double *C,
                       double *E, double *N, double *rhs);

/* Replace the assembled diagonals and rhs from host arrays (all six
 * required); invalidates the factorisation. */
adr_status adr_set_dia(adr_problem *p, const double *S, const double *W,
                       const double *C, const double *E, const double *N,
                       const double *rhs);

/* Copy the FP64 factors (lw, ls, invd; any may be NULL) to host arrays. */
adr_status adr_get_factors(const adr_problem *p, double *lw, double *ls, double *invd);

/* v = A x (device vectors), the five-point product with out-of-grid
 * neighbours contributing 0: fma(N,x_n, fma(E,x_e, fma(W,x_w, fma(S,x_s, C x)))). */
adr_status adr_spmv(adr_problem *p, const double *x_dev, double *v_dev);

/* z = M^{-1} q = U^{-1} L^{-1} q with the current factors (device vectors):
 *   y_k = fma(-ls, y_{k-nx}, fma(-lw, y_{k-1}, q_k)),
 *   z_k = fma(-N, z_{k+nx}, fma(-E, z_{k+1}, y_k)) * invd_k. */
adr_status adr_precond(adr_problem *p, const double *q_dev, double *z_dev);

/* The two halves of adr_precond, one wavefront kernel each:
 * adr_lsolve: y = L^{-1} q;  adr_usolve: z = U^{-1} y  (device vectors). */
adr_status adr_lsolve(adr_problem *p, const double *q_dev, double *y_dev);
adr_status adr_usolve(adr_problem *p, const double *y_dev, double *z_dev);

/* Double-double inner product of two device vectors of length n, rounded to
 * FP64, written to *out (host). */
adr_status adr_dot(const double *x_dev, const double *y_dev, int64_t n, void *stream,
                   double *out);

/* Streaming copy dst[k] = src[k], k < n (device vectors, stream as in
 * adr_dot): a plain HBM-bound kernel, the practical bandwidth reference for
 * the roofline figures.  Asynchronous: the copy is enqueued on `stream` and
 * ordered with the caller's other work there (time it with events on that
 * stream). */
adr_status adr_stream_copy(const double *src_dev, double *dst_dev, int64_t n, void *stream);

/* ---------------------------------------------------------------------------
 * adr_dot_noalloc -- adr_dot for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  The same double-double inner product and the same result
 * bits, but its per-block partial sums live in a fixed library-owned device
 * array (2048 entries of 16 bytes, 32 KiB, on each GPU the library runs on,
 * held until the process ends) instead of memory allocated per call, and the
 * result goes to device memory.  No hipMalloc or hipFree is made.
 * x_dev, y_dev: n doubles each; out_dev: one double of device memory.
 * 0 <= n <= 2^31 - 1 (at most 2048 partial sums), else ADR_ERR_ARG.
 * Asynchronous: queued on `stream`, the result is in out_dev when the stream
 * reaches it.  Calls on one GPU share the array: calls that overlap (other
 * streams, other host threads) race on it and must be serialised.
 * ------------------------------------------------------------------------- */
adr_status adr_dot_noalloc(const double *x_dev, const double *y_dev, int64_t n, void *stream,
                           double *out_dev);

/* Bytes of device memory the problem holds (after ilu0 / solve buffers). */
size_t adr_device_bytes(const adr_problem *p);

/* Sweep geometry: rows per strip (R = 16 or 32) for the wavefront kernels,
 * or 0 for the default (32, also the height a new problem starts with).
 * Also returns 32-row strips to the automatic ring choice (the compact ring
 * while the strips fit one per CU or once they exceed 1.5 per CU -- 384 on
 * 256 CUs -- the deep ring in between).  Results do not depend on it.  For
 * tuning and tests. */
adr_status adr_set_sweep_rows(adr_problem *p, int32_t rows);

/* Ring of the 32-row sweeps: -1 automatic (the default), 0 one workgroup per
 * CU with a deep LDS ring, 1 a four-slot ring small enough for two per CU
 * (with three loader waves instead of five where the strips fit one per CU;
 * used where a tile holds at most three arrays: the L sweeps and the
 * table-driven U sweep; the U sweep reading the diagonals keeps the deep
 * ring).  Results do not depend on it.  ADR_ERR_ARG for another mode.  For
 * tuning and tests. */
adr_status adr_set_sweep_ring(adr_problem *p, int32_t mode);

/* The ring the 32-row sweeps use now: 0 deep, 1 compact. */
int32_t adr_sweep_ring(const adr_problem *p);

/* Stencil tables.  The off-diagonals of the operator of Section 4 are
 * separable: W and E depend only on the column, S and N only on the row
 * (a = a(x), b = b(y), couplings to boundary nodes zero).  After
 * adr_assemble / adr_batch_assemble / adr_set_dia the library copies them into
 * per-instance column and row tables and checks every point against them bit
 * for bit; when all match, the iteration reads the tables instead of the
 * four off-diagonals (the stencil products then read the diagonal C only, the
 * FP64 L sweep forms lw = W invd_w and ls = S invd_s from invd as the
 * factorisation does, and the U sweep takes E and N from the tables), which
 * changes no result bit.  adr_use_stencil_tables(p, 0) makes the iteration
 * read the full diagonals; 1 (the default) allows the tables.
 * adr_stencil_tables returns 1 if the next solve reads the tables, 0 if it
 * reads the diagonals (also for p == NULL). */
adr_status adr_use_stencil_tables(adr_problem *p, int32_t enable);
int32_t adr_stencil_tables(const adr_problem *p);

/* Device time in ms of the kernels of the last adr_spmv, adr_precond,
 * adr_lsolve or adr_usolve call on p: HIP events recorded on the problem's
 * stream right before the first and after the last launch of the call, so
 * the host's turnaround between calls is not included.  0 before any such
 * call or for p == NULL. */
double adr_last_call_ms(const adr_problem *p);

/* Caller-provided workspace.  By default the library allocates its device
 * memory itself.  A caller that owns the device memory (e.g. a PyTorch
 * tensor) can instead hand it the buffers created after assembly: the
 * wavefront hand-off memory, the ILU(0) factors, the nine iteration vectors
 * and the per-instance solve states.
 * adr_workspace_bytes: bytes these need for factors of `precision`
 * (adr_precision); 0 for p == NULL or an unknown precision.
 * adr_bind_workspace: dev_ptr (device memory on the problem's device, 256-byte
 * aligned) of `bytes` >= adr_workspace_bytes(p, ADR_FP64) bytes; the buffers
 * are carved out of it in a fixed order.  Call once, after assembly and before
 * adr_ilu0 / adr_batch_ilu0 / any solve (else ADR_ERR_STATE); a precision
 * needing more than the buffer holds later fails with ADR_ERR_NOMEM.  The
 * caller keeps the memory alive and untouched until adr_destroy, which does
 * not free it.  Histories, the stencil tables and the assembly arrays stay
 * library-allocated. */
size_t adr_workspace_bytes(const adr_problem *p, int32_t precision);
adr_status adr_bind_workspace(adr_problem *p, void *dev_ptr, size_t bytes);

const char *adr_status_str(int32_t status);
/* Message of the last call error on this thread ("" if none). */
const char *adr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ADR_H */
