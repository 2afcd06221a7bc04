/*
 * ta.h - C ABI of the MI355X (gfx950) Triangle Algorithm (TA) / Centering
 * Triangle Algorithm (CTA) library, libta.so.
 *
 * The methods are those of Lau & Kalantari, "On the Performance of a Novel
 * Class of Linear System Solvers and Comparison with State-of-The-Art
 * Algorithms" (arXiv 2304.12168): CTA is Algorithm 1 of section 3.2 with
 * H = A A^T (the choice the paper's implementation makes in section 5), TA is
 * Algorithm 3 (and Algorithm 2 with a fixed radius) of section 4.
 *
 * Conventions shared by every entry point
 *   - All array arguments are HIP DEVICE pointers owned by the caller.  The
 *     library never retains or frees them.  Scalars, option and info structs
 *     and the matrix descriptor itself live in HOST memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is ordered on it; solver calls return when the solve has finished
 *     (the host reads a device flag once per chunk of iterations).  Kernel-
 *     level calls (ta_spmv, ta_transpose, ...) return after enqueueing.
 *   - Workspace is taken with stream-ordered hipMallocAsync inside the call
 *     and released before return (cta_solve_plan_noalloc excepted).
 *   - Return value: 0 on success, a negative TA_E* code otherwise (see
 *     ta_strerror).  Not converging is not an error: it is reported in
 *     ta_info.stop.
 *   - One call per stream at a time; calls on different streams share no
 *     state.
 *   - Every reduction (inner products, norms, matrix rows) is evaluated with
 *     compensated (double-double) accumulation, so results do not depend on
 *     the summation order beyond the last bit.
 */
#ifndef TA_H
#define TA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define TA_OK 0
#define TA_EINVAL (-1)  /* bad shape, pointer, option value or malformed CSR */
#define TA_ENOMEM (-2)  /* device allocation failed */
#define TA_EHIP (-3)    /* a HIP runtime call failed; ta_strerror(TA_EHIP) has the text */
#define TA_ENOTSUP (-4) /* input outside what the kernels support (see ta_mat) */
#define TA_ESCRATCH (-5) /* cta_solve_plan_noalloc: the solve needs more device memory than
                            its fixed buffer holds (see there) */

/* ---- matrix kinds ---- */
#define TA_DENSE_ROWMAJOR 0
#define TA_CSR 1

/* ---- stop codes (ta_info.stop) ----
 * RESIDUAL : ||b - A x|| <= tol ||b|| on the true FP64 residual (Definition 1 (1),
 *            in relative form).
 * NORMAL   : ||A^T r|| <= tol_normal ||A^T b||, or A A^T r = 0 (Definition 1 (2);
 *            Example 1 and Theorem prop0TA (1): x solves the normal equation).
 * WITNESS  : ta_solve with fixed_rho only: b' = A x is a witness, so b is not in
 *            E_{A,rho} (Algorithm 2); info.rho_lo holds the lower bound of
 *            Corollary 1 on the norm of the minimum-norm solution.
 * MAXITER  : iteration budget spent.
 * BREAKDOWN: non-finite step quantities (e.g. NaN or Inf in A or b).          */
#define TA_STOP_RESIDUAL 1
#define TA_STOP_NORMAL 2
#define TA_STOP_WITNESS 3
#define TA_STOP_MAXITER 4
#define TA_STOP_BREAKDOWN 5

/* ---- precision of the matrix products ---- */
#define TA_FP64 0
#define TA_FP32 1
#define TA_BF16 2

/*
 * Matrix descriptor (host struct, device arrays).
 *   TA_CSR: row_ptr[m+1] (int32, row_ptr[0] = 0, nondecreasing, row_ptr[m] = nnz),
 *           col_idx[nnz] (int32 in [0, n)), val[nnz] (float64).  Column order
 *           inside a row is free; duplicates are allowed and act as a sum.
 *           A^T is built on the device inside each solver call.  Supported:
 *           nnz < 2^31 (a column may hold any number of them).
 *   TA_DENSE_ROWMAJOR: val[m*ld] row-major, ld >= n; row_ptr/col_idx unused.
 */
typedef struct ta_mat {
    int32_t kind;
    int64_t m, n, nnz, ld;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
} ta_mat;

/*
 * Options (host struct).  Inputs of the paper's algorithm headers:
 * epsilon -> tol (relative), epsilon' -> tol_normal (relative), t, rho.
 */
typedef struct ta_opts {
    double tol;            /* stop when ||b - A x|| <= tol ||b||; in [0, 1) */
    double tol_normal;     /* stop when ||A^T r|| <= tol_normal ||A^T b||; 0 = only A^T r = 0 */
    int32_t t;             /* CTA order, 1..8 and <= m (ignored by ta_solve) */
    int64_t max_iter;      /* iteration budget (>= 0) */
    int32_t precision;     /* TA_FP64 | TA_FP32 | TA_BF16: precision of the matrix products.
                              TA_FP32 / TA_BF16 are taken by cta_solve and cta_minnorm (one
                              shot; see there) and by cta_solve_batched; the plan solvers
                              and the TA solvers compute in FP64 only (TA_EINVAL) */
    int32_t replace_every; /* recompute r = b - A x every so many iterations; 0 = only at stop */
    int32_t warm_start;    /* cta_solve: 1 = start from the x passed in */
    double rho0;           /* ta_solve: initial radius (Algorithm 3 starts from 0) */
    int32_t fixed_rho;     /* ta_solve: 1 = Algorithm 2 (no radius growth, WITNESS exit) */
    int32_t chunk;         /* iterations per host poll of the stop flag; 0 = automatic */
    int32_t launch_mode;   /* 0 = each chunk of iterations is captured once as a HIP graph
                              and replayed (single-system solves: from the second chunk on,
                              not with t_cycle, not in cta_solve_plan_noalloc), 1 = kernels
                              launched one by one; results are identical */
    int32_t h_mode;        /* cta_solve and cta_solve_batched's x-form: 0 = H = A A^T
                              (section 5), 1 = H = A for a square symmetric positive
                              semidefinite A (not checked; in a batch every system square, a
                              dense batch in TA_FP64 only): t products per iteration instead
                              of 2t, phi_i = r^T A^i r.  Other solvers: 0 */
    int32_t t_cycle;       /* cta_solve / cta_minnorm / cta_solve_batched: 1 = the order of
                              iteration k (k = 0, 1, ...) cycles 1, 2, ..., t, t-1, ..., 2, 1,
                              2, ... (section 5.1's order cycling, read as a triangle wave of
                              period 2(t-1)); 0 = the fixed order t.  In a batch each column
                              takes the order of its own k, while the chain runs t steps for
                              all of them */
    int32_t nonneg;        /* ta_solve: 1 = LP feasibility {A x = b, x >= 0} (section 6): the
                              pivot uses c+ = max(A^T (b - b'), 0) in place of c (Proposition
                              eq. vrend2), so x stays >= 0; stop NORMAL when ||c+|| <=
                              tol_normal ||(A^T b)+|| (with b^T (b - b') > 0 this is a Farkas
                              certificate of infeasibility).  Other solvers: 0 */
    double rho_max;        /* ta_solve: > 0 = stop with WITNESS once the radius would grow
                              beyond rho_max (the termination bound section 6 asks for);
                              0 = no bound.  Other solvers: 0 */
    int32_t enhanced;      /* cta_solve / cta_minnorm / cta_solve_batched (per column): 1 =
                              the enhanced stop of section 3.2 (for
                              t >= 2): in every iteration of order t >= 2 the j-fold first-order
                              iterates f_j = F_1(f_{j-1}), f_0 = r, j = 1..t-1, are also tested,
                              and the first with ||A^T f_j|| <= tol_normal ||A^T b|| (||A f_j||
                              for h_mode 1) ends the solve with stop NORMAL at
                              x^ = x + sum_{i<j} (phi_1(f_i) / phi_2(f_i)) A^T f_i (f_i for
                              the y-form's y and for h_mode 1); that iteration counts.  The
                              tests and x^ come from the iteration's phi_1..phi_2t, with no
                              further products.  Needs tol_normal > 0 to act.  Other
                              solvers: 0 */
    int32_t normal_eq;     /* ta_solve / ta_minnorm: 1 = TA on the normal equation
                              A^T A x = A^T b (the inputs the rectangular hybrid of section
                              5.3 gives TA when A x = b is not solvable): the operator
                              M = A^T A is applied as A^T (A v) with A v rounded to FP64
                              (two passes, counted as two products; A^T b one more), the
                              true residual is A^T b - A^T (A x) as one compensated sum per
                              entry, hist[k] is relative to ||A^T b||, and rel_res /
                              rel_normal stay on (A, b).  Must be 0 (TA_EINVAL) for the
                              other solvers */
    double accel;          /* cta_solve / cta_minnorm: theta in (0, 1) = the convex-combination
                              step of the theorem on the dynamics of first-order CTA (section
                              3.4): after each step, if ||r_{k+1}|| >= theta ||r_k||, the iterate
                              becomes a r_k + (1 - a) r_{k+1} (and the same combination of x,
                              or y) with a = rho / (rho + 1), rho = ||r_{k+1}|| / ||r_k||, the
                              weight that makes the combination an eigenvector on a critical
                              line, so that the next step solves such a system; never twice in
                              a row.  The combination takes no product and is not counted as an
                              iteration; hist[k] holds the combined residual.  0 = off; a value
                              outside [0, 1) is TA_EINVAL.  cta_solve_batched: the same, each
                              column deciding on its own residuals.  Other solvers: 0 */
} ta_opts;

/* Result summary (host struct). */
typedef struct ta_info {
    int64_t iters;      /* while-loop bodies executed (TA radius updates included) */
    int64_t matvecs;    /* products with A or A^T, true-residual checks included */
    int32_t stop;       /* TA_STOP_* */
    double rel_res;     /* ||b - A x|| / ||b|| at exit, true FP64 residual */
    double rel_normal;  /* ||A^T (b - A x)|| / ||A^T b|| at exit */
    double rho, rho_lo; /* ta_solve: final radius and best witness lower bound */
} ta_info;

/*
 * The one-shot solvers below prepare A (see ta_plan_create) inside the call.
 *
 * cta_solve - Algorithm 1 (CTA of order t, H = A A^T), iterate form of
 * eq. CTAGEN7A: x'' = x' + sum_i alpha_i A^T H^{i-1} r'.
 *   A       : m x n matrix, any shape and rank.
 *   b       : device, m doubles (not modified).
 *   x       : device, n doubles; output (input too when opts->warm_start).
 *   hist    : device, hist_cap doubles or NULL; hist[k] = ||r_k|| / ||b|| for
 *             k = 0 .. min(iters, hist_cap - 1) (recurrence residual).
 *   info    : host, filled on return.
 * b = 0 returns x = 0, iters = 0, stop = RESIDUAL.
 * opts->precision TA_FP32 / TA_BF16: the Krylov chain's products use FP32 (or
 * BF16) copies of A and A^T and FP32 vectors, while the Gram entries, the
 * step, x and every true-residual check stay FP64; the call runs the batched
 * engine on this one system and one right-hand side (cta_solve_batched), so
 * the true residual replaces the recurrence after every chunk of iterations
 * and the solve stops only at a chunk's end.  hist is not written in that
 * form, and warm_start, replace_every, h_mode, t_cycle, enhanced and accel
 * must be 0 (TA_EINVAL otherwise).
 */
int cta_solve(const ta_mat *A, const double *b, double *x, const ta_opts *opts, double *hist,
              int64_t hist_cap, ta_info *info, void *stream);

/*
 * cta_minnorm - the same iteration in the y-form x = A^T y (Theorem 1 (4):
 * from x0 = 0 every iterate is A^T w_k, so on a consistent system the limit is
 * the minimum-norm solution).  The m-vector y is updated with
 * y'' = y' + sum_i alpha_i H^{i-1} r' and x = A^T y is formed at the end.
 * opts->warm_start is not supported (TA_EINVAL).  Arguments as cta_solve.
 */
int cta_minnorm(const ta_mat *A, const double *b, double *x, const ta_opts *opts, double *hist,
                int64_t hist_cap, ta_info *info, void *stream);

/*
 * ta_solve - Algorithm 3 (TA with rho <- max(2 rho, (b-b')^T b / ||c||)), or
 * Algorithm 2 when opts->fixed_rho (then opts->rho0 > 0 is required).
 * Pivot v_rho = rho A c / ||c|| with c = A^T (b - b') (eq. vr), strict-pivot
 * test rho ||c|| >= (b - b')^T b (eq. eqlem2), step to the point of segment
 * [b', v_rho] nearest to b (Proposition prop1TA).  Arguments as cta_solve;
 * opts->t is ignored.  opts->warm_start: start from the x passed in (b' = A x,
 * one product more); b = 0 still returns x = 0.
 */
int ta_solve(const ta_mat *A, const double *b, double *x, const ta_opts *opts, double *hist,
             int64_t hist_cap, ta_info *info, void *stream);

/*
 * ta_minnorm - Algorithm 4 (section 4.4, TA for an approximation to the
 * minimum-norm solution): from x_eps (device, n doubles, an approximate
 * solution: ||A x_eps - b|| <= tol ||b||) it bisects on the radius rho of
 * the ellipsoid E_{A,rho}.  Upper bound hi = ||x_eps||, lower bound lo = 0;
 * each test runs Algorithm 2 with rho = (hi + lo) / 2 from the last
 * witness's x (0 before the first witness): an approximate solution in the
 * ball lowers hi to rho (and becomes the answer), a witness raises lo to
 * (b - b')^T b / ||c|| (Corollary 1).  Ends when hi - lo <= tol ||x_eps||
 * (stop RESIDUAL), when a test ends on the normal equation (stop NORMAL, its
 * x returned), or when opts->max_iter TA iterations (summed over the tests)
 * are spent (stop MAXITER).  If a witness lifts lo above hi by more than the
 * gap tolerance, x_eps was no approximate solution of a consistent system
 * (Corollary 1 needs A x = b solvable): stop WITNESS.
 *   x     : device, n doubles, output (the last solution found, or x_eps);
 *   info  : iters / matvecs summed over the tests, rho = hi, rho_lo = lo,
 *           rel_res / rel_normal of the returned x;
 *   tests : host, may be NULL: number of Algorithm 2 tests run.
 * opts->tol, tol_normal, max_iter and chunk are used; fixed_rho, rho0, t and
 * warm_start are ignored.
 */
int ta_minnorm(const ta_mat *A, const double *b, const double *x_eps, double *x,
               const ta_opts *opts, ta_info *info, int64_t *tests, void *stream);

/* ---- prepared operators (plans) ----
 *
 * A plan holds what the solvers derive from A alone: A^T as a canonical CSR
 * built on the device (for a dense A, a row-major copy of A^T), and for A or
 * A^T with long rows (more than 16 nonzeros per row on average) one of two
 * regrouped copies: with at least 16384 columns and at least 3 entries per
 * (row, 8192-column tile) on average, the entries stored tile after tile
 * with 16-bit column offsets, so that each block stages one tile of x in LDS
 * and gathers from there (TA_FMT_CSR_TILED; one partial sum per row and
 * tile is merged afterwards); else, with at least 131072 columns, a copy with
 * sorted columns split into s = 8 g column slices (g doubling, up to 8, while a
 * slice of x exceeds 8 MB), run 8 at a time so that each XCD of the MI355X
 * gathers from its own slice of x (TA_FMT_CSR_SLICED).  A or A^T with short rows (16 or fewer
 * nonzeros on average) whose 64-row slices pad the entries by at most a
 * quarter is also copied into SELL-64 form (each slice stored position by
 * position, padded to its widest row), so its products need no row bounds
 * and make contiguous index loads; the sums keep the CSR order, so results
 * are unchanged.  A or A^T left to the row kernels whose longest row holds
 * at least 512 nonzeros and at least 32 times the average gets a merge-path
 * partition instead (TA_FMT_CSR_MERGE; Merrill and Garland's merge-based
 * SpMV, SC 2016): the row ends and the nonzeros form one sequence that is
 * cut into equal shares of 2048 items per block, 8 per thread, so that a
 * long row is split over many threads and blocks; the pieces of a row are
 * compensated sums merged in a fixed order, so results do not depend on
 * timing.  The partition is one int32 per 2048 items, and a call's
 * workspace holds 48 bytes per block for the pieces that cross blocks.
 * The one-shot solvers build the same; the one-shot products (ta_spmv,
 * ta_residual, ta_time_matvec) build the merge-path partition only.  Solving many
 * right-hand sides with one matrix builds them once.  The plan refers to A's device arrays (row_ptr,
 * col_idx, val, or the dense val): they must stay allocated and unchanged
 * while the plan lives.  A plan is read-only once created and may serve
 * calls on several streams at the same time.  Its device memory is taken
 * stream-ordered on `stream` and returned by ta_plan_destroy on that same
 * stream.  Errors as the one-shot calls (TA_EINVAL for a malformed CSR).
 */
typedef struct ta_plan ta_plan;

int ta_plan_create(const ta_mat *A, ta_plan **plan, void *stream);
int ta_plan_destroy(ta_plan *plan);

/* Storage the plan's products use for A (trans = 0) or A^T (trans = 1):
 * TA_FMT_CSR_ROWS, TA_FMT_DENSE_ROWS, TA_FMT_DENSE_COLS, TA_FMT_CSR_SLICED
 * (column slices), TA_FMT_SELL64, TA_FMT_CSR_TILED (LDS column tiles) or
 * TA_FMT_CSR_MERGE (merge-path partition), written to *format (host).
 * TA_EINVAL for a NULL argument. */
enum { TA_FMT_CSR_ROWS = 0, TA_FMT_DENSE_ROWS = 1, TA_FMT_DENSE_COLS = 2,
       TA_FMT_CSR_SLICED = 3, TA_FMT_SELL64 = 4, TA_FMT_CSR_TILED = 5,
       TA_FMT_CSR_MERGE = 6 };
int ta_plan_format(const ta_plan *plan, int32_t trans, int32_t *format);

/* The solvers above on a prepared operator; other arguments as there. */
int cta_solve_plan(const ta_plan *plan, const double *b, double *x, const ta_opts *opts,
                   double *hist, int64_t hist_cap, ta_info *info, void *stream);
int cta_minnorm_plan(const ta_plan *plan, const double *b, double *x, const ta_opts *opts,
                     double *hist, int64_t hist_cap, ta_info *info, void *stream);
int ta_solve_plan(const ta_plan *plan, const double *b, double *x, const ta_opts *opts,
                  double *hist, int64_t hist_cap, ta_info *info, void *stream);
int ta_minnorm_plan(const ta_plan *plan, const double *b, const double *x_eps, double *x,
                    const ta_opts *opts, ta_info *info, int64_t *tests, void *stream);

/*
 * ta_solve_halving - Algorithm 3 restarted as the remark after the theorem
 * on its properties (section 4.3) suggests: eps' (opts->tol_normal, or
 * opts->tol when that is 0) is halved each time a run ends with an
 * eps'-approximate solution of the normal equation (stop NORMAL), and TA
 * runs again from the x it returned (b' = A x, one product more), at most
 * max_halvings times; a consistent system whose normal-equation test fires
 * first thus still reaches ||b - A x|| <= tol ||b||.  The first run starts
 * from 0, or from the x passed in with opts->warm_start.
 *   x         : device, n doubles, output (input too with warm_start);
 *   info      : iters and matvecs summed over the runs; stop, rel_res,
 *               rel_normal, rho and rho_lo of the last run;
 *   halvings  : host, may be NULL: restarts made.
 * Each run has opts->max_iter iterations.  TA_EINVAL for max_halvings < 0 or
 * opts->normal_eq; other errors as ta_solve_plan.
 */
int ta_solve_halving(const ta_plan *plan, const double *b, double *x, const ta_opts *opts,
                     int32_t max_halvings, ta_info *info, int32_t *halvings, void *stream);

/*
 * cta_solve_plan_noalloc - cta_solve_plan for callers that cannot allocate
 * device memory (code that must not call hipMalloc, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, same kernels, same
 * results bit for bit.  The call allocates nothing: its workspace (the
 * Krylov vectors, the residual, the per-block partial sums, the solver
 * state) is carved from one fixed device buffer of TA_NOALLOC_SCRATCH_BYTES
 * that the library holds on each GPU it runs on until the process ends; the
 * State is set from a kernel argument and read back into host stack memory.
 * The plan itself is made beforehand with ta_plan_create (which allocates).
 *   Limit: the workspace is 8 (t + 1) (m + n) bytes (8 (m + n) more with
 *   accel, 16 s m or 16 s n more for a plan with s column slices, 16 m
 *   ceil(n / 8192) or 16 n ceil(m / 8192) more for one with column tiles, 48
 *   bytes per 2048 items of (rows + nonzeros) for a merge-path partition)
 *   plus the per-block partial sums; a solve that needs more than the buffer returns
 *   TA_ESCRATCH before any device work.  For t = 3 and m = n that is
 *   n up to about 1e6.
 *   Sharing: every call on one GPU uses that GPU's buffer, so calls that
 *   overlap in time on one GPU (from several host threads or streams) race
 *   and must be serialised by the caller.  Each call initialises what it
 *   reads; the buffer keeps the last call's contents.
 */
#define TA_NOALLOC_SCRATCH_BYTES (64u << 20)
int cta_solve_plan_noalloc(const ta_plan *plan, const double *b, double *x, const ta_opts *opts,
                           double *hist, int64_t hist_cap, ta_info *info, void *stream);

/* ---- batched solves: many systems, many right-hand sides, one set of kernels ----
 *
 * ta_batch_plan_create concatenates nsys systems (A[0..nsys-1], host array
 * of descriptors, sizes m_s x n_s, either all TA_CSR or all
 * TA_DENSE_ROWMAJOR; a mix is TA_EINVAL) into one block-diagonal operator on
 * the device, builds its transpose, and, for precision TA_FP32 or TA_BF16,
 * low-precision copies of the values.  The plan copies A's values, so A may
 * change or be freed afterwards.  Totals (sum of m_s, sum of n_s, and for
 * CSR sum of nnz_s) must stay below 2^31.  Dense systems are stored with rows
 * padded to a multiple of 16 and run their low-precision products on the
 * matrix cores (MFMA: FP32 16x16x4 in TA_FP32, BF16 16x16x16 with FP32
 * accumulation in TA_BF16, where the vector entries are rounded to BF16 too;
 * the FP64 true residuals of those solves use FP64 16x16x4, plain sums).  A
 * dense plan also holds the systems as CSR with every entry stored (when the
 * entries fit the CSR limits, sum below 2^31): FP64 solves (opts->precision
 * TA_FP64, on any dense plan) run there, with compensated sums like every
 * CSR plan.
 *
 * cta_solve_batched runs Algorithm 1 (CTA, H = A_s A_s^T, or H = A_s with
 * opts->h_mode 1) independently for every (system s, right-hand side c), all
 * advanced together:
 *   nrhs : host, nsys counts k_s in [0, 64];
 *   B    : host array of nsys device pointers, B[s] column-major m_s x k_s;
 *   X    : host array of nsys device pointers, X[s] column-major n_s x k_s (out);
 *   opts : as cta_solve; opts->precision is TA_FP64 or the plan's precision;
 *          opts->warm_start and opts->replace_every are not used; opts->chunk
 *          is the number of iterations between true-residual checks
 *          (0 = automatic); h_mode, t_cycle, enhanced and accel as cta_solve,
 *          per column;
 *   minnorm : 1 = the y-form of cta_minnorm (x = A^T y), 0 = the x-form;
 *   info : host, sum k_s entries, system-major (s, then c): iterations, products,
 *          stop code, FP64 true relative residual, normal-equation residual.
 * TA_FP64: each (s, c) follows exactly the single-right-hand-side iteration
 * (same iteration count and stop code as cta_solve / cta_minnorm on that
 * column), on CSR and on dense plans.  TA_FP32 / TA_BF16: products of the Krylov chain use the low
 * precision copies and FP32 vectors; Gram entries, steps, x (or y) and every
 * true-residual check are FP64, and the true residual replaces the recurrence
 * residual after every chunk (4, 8, 16, 32, then 64 iterations with TA_FP32,
 * 4 then 8 with TA_BF16, unless opts->chunk fixes it); a column can stop only
 * at a chunk's end; stop codes and residuals refer to FP64.
 * Systems are advanced in groups of equal vector width, a power of two: a
 * system's k_s columns form one piece (k_s rounded up to a power of two) or,
 * when that would pad more than a quarter, two (the widest power of two
 * K1 <= k_s and the rest, rounded up); low-precision groups are further split
 * by row length.  The groups run side by side, each on a host thread and a stream of its own that
 * start after the work already queued on `stream`; the call returns when all
 * are done.  Every column keeps its own iteration, so the results do not
 * depend on the grouping.
 */
typedef struct ta_batch_plan ta_batch_plan;

int ta_batch_plan_create(int32_t nsys, const ta_mat *A, int32_t precision, ta_batch_plan **plan,
                         void *stream);
int ta_batch_plan_destroy(ta_batch_plan *plan);
int cta_solve_batched(const ta_batch_plan *plan, const int32_t *nrhs, const double *const *B,
                      double *const *X, const ta_opts *opts, int32_t minnorm, ta_info *info,
                      void *stream);

/*
 * ta_batch_time_spmm - measurement hook: average milliseconds of one launch
 * of the SpMM kernel that a batched solve with K (1, 2, 4, ..., 64) columns
 * and the given precision runs on the plan's A (trans = 0) or A^T (trans = 1),
 * with its fused per-column ||y||^2 partial sums, over `reps` >= 1
 * back-to-back launches timed with HIP events on `stream` (input block
 * zero-filled).  Synchronises `stream`.
 */
int ta_batch_time_spmm(const ta_batch_plan *plan, int32_t K, int32_t trans, int32_t precision,
                       int32_t reps, double *avg_ms, void *stream);

/*
 * ta_validate - host-side argument checks only (shapes, pointers, options);
 * it reads no device memory and launches nothing, so it runs without a GPU.
 * `solver` is 0 for cta_solve, 1 for cta_minnorm, 2 for ta_solve.
 * Returns TA_OK or TA_EINVAL.
 */
int ta_validate(const ta_mat *A, const ta_opts *opts, int32_t solver);

/* Text for a return code (TA_EHIP: the last HIP error seen on this thread). */
const char *ta_strerror(int code);

/* ---- kernel-level entry points (the building blocks of every iteration) ---- */

/*
 * ta_spmv - y = A x (trans = 0) or y = A^T x (trans = 1), FP64, one
 * compensated sum per output entry.  For a CSR matrix with trans = 1 the
 * library builds A^T for the call.  If norm2 != NULL, *norm2 (device, one
 * double) receives ||y||^2.  Enqueues on `stream` and returns.
 */
int ta_spmv(const ta_mat *A, int32_t trans, const double *x, double *y, double *norm2,
            void *stream);

/* ta_spmv on a prepared operator: the product kernels the plan's solves use
 * (for long-row matrices, the XCD column-sliced kernels). */
int ta_spmv_plan(const ta_plan *plan, int32_t trans, const double *x, double *y, double *norm2,
                 void *stream);

/*
 * ta_residual - r = b - A x as one compensated sum per row (Definition 4);
 * *norm2 (device, may be NULL) receives ||r||^2.
 */
int ta_residual(const ta_mat *A, const double *b, const double *x, double *r, double *norm2,
                void *stream);

/*
 * ta_transpose - CSR of A^T from the CSR of A, built on the device:
 * at_row_ptr[n+1], at_col_idx[nnz], at_val[nnz] (device, caller-allocated).
 * Columns come out sorted inside each row, so the result is canonical and
 * deterministic (a row of A^T is put in the order of A's storage; rows of
 * more than 8192 entries are sorted by one block in global memory, more
 * slowly).  Synchronises `stream` before returning.
 */
int ta_transpose(const ta_mat *A, int32_t *at_row_ptr, int32_t *at_col_idx, double *at_val,
                 void *stream);

/*
 * ta_csr_outer - out[k] = (alpha * u[i]) * v[j] for the k-th stored entry
 * (i, j) of a CSR A (u: m entries, v: n entries, out: nnz entries, all
 * device).  Not in the paper: it is the gradient of a loss L of the solution
 * map x(A, b) = A^{-1} b (square nonsingular A, the limit of Algorithm 1,
 * Theorem 1 (4)) with respect to A's stored values, dL/da_ij = -lambda_i x_j
 * where A^T lambda = dL/dx, taken with alpha = -1, u = lambda, v = x.  The
 * CSR is checked on the device first (TA_EINVAL if malformed; this
 * synchronises `stream`); the product is then enqueued on `stream`.
 */
int ta_csr_outer(const ta_mat *A, const double *u, const double *v, double alpha, double *out,
                 void *stream);

/*
 * ta_time_matvec - measurement hook: average duration (milliseconds, host
 * double *avg_ms) of one launch of the FP64 matrix-product kernel that the
 * solvers use for y = A x (trans = 0) or A^T x (trans = 1), with its fused
 * ||y||^2 reduction, over `reps` >= 1 back-to-back launches timed with HIP
 * events on `stream`.  Preparation (checks, transpose) is outside the timed
 * launches.  Synchronises `stream`.
 */
int ta_time_matvec(const ta_mat *A, int32_t trans, const double *x, double *y, int32_t reps,
                   double *avg_ms, void *stream);
/* The same on a prepared operator (the kernels a plan's solves launch). */
int ta_time_matvec_plan(const ta_plan *plan, int32_t trans, const double *x, double *y,
                        int32_t reps, double *avg_ms, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TA_H */
