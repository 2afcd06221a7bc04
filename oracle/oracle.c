/*
 * Plain FP64 CPU oracle for the Centering Triangle Algorithm (CTA) and the
 * Triangle Algorithm (TA) of Lau & Kalantari, "On the Performance of a Novel
 * Class of Linear System Solvers and Comparison with State-of-The-Art
 * Algorithms" (arXiv 2304.12168).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file.  It shares no code,
 * header or constant generator with the GPU library, and the GPU library
 * never calls it.
 *
 * Everything is sequential, single-threaded and written for reading, not for
 * speed.  Build with -O2 -ffp-contract=off so that every a*b+c below is the
 * two-rounding expression it looks like, and every fma() is one rounding.
 *
 * Reductions.  Every inner product (matrix rows, matrix columns, norms) is
 * evaluated with the compensated algorithm Dot2 of Ogita, Rump and Oishi,
 * "Accurate sum and dot product", SIAM J. Sci. Comput. 26 (2005), Alg. 5.3:
 * the result is as accurate as if computed in twice the working precision
 * and then rounded once.  Terms are taken in index order.
 *
 * Stop codes: 1 residual, 2 normal equation, 3 witness, 4 iteration budget,
 * 5 breakdown (non-finite or degenerate step quantities).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_RESIDUAL = 1, OR_NORMAL = 2, OR_WITNESS = 3, OR_MAXITER = 4, OR_BREAKDOWN = 5 };
enum { OR_DENSE = 0, OR_CSR = 1 };

typedef struct {
    int32_t kind;           /* OR_DENSE (row-major, leading dimension ld) or OR_CSR */
    int64_t m, n, ld;
    const int32_t *row_ptr; /* CSR: m+1 */
    const int32_t *col_idx; /* CSR: nnz */
    const double *val;      /* CSR: nnz; dense: m*ld */
} or_mat;

typedef struct {
    double tol;        /* stop when ||b - A x|| <= tol ||b|| (true residual) */
    double tol_normal; /* stop when ||A^T r|| <= tol_normal ||A^T b||; 0: only A^T r = 0 */
    int32_t t;         /* CTA order */
    int64_t max_iter;
    int32_t replace_every; /* recompute r = b - A x every so many iterations; 0: never */
    int32_t warm_start;    /* CTA x-form: start from the given x */
    double rho0;           /* TA: initial radius */
    int32_t fixed_rho;     /* TA: 1 = fixed radius, stop at a witness */
    int32_t h_is_a;        /* CTA x-form: 1 = H = A (A square symmetric PSD), 0 = H = A A^T */
    int32_t t_cycle;       /* CTA: 1 = the order of iteration k is or_cycle_order(t, k) */
    int32_t nonneg;        /* TA: 1 = x >= 0 (LP feasibility): c replaced by c+ = max(c, 0) */
    double rho_max;        /* TA: > 0 = stop at a witness once the radius would exceed this */
    int32_t enhanced;      /* CTA, t >= 2: the enhanced stop (section 3.2) */
    int32_t normal_eq;     /* TA: 1 = run on the normal equation A^T A x = A^T b (the
                              rectangular hybrid's inputs for an inconsistent system) */
    double accel;          /* CTA: > 0 = convex-combination step when ||r_{k+1}|| >= accel ||r_k|| */
} or_opts;

/* Order cycling (section 5.1 cycles the order 1, ..., 5 and back), read as a
 * triangle wave of period 2 (t - 1): 1, 2, ..., t, t - 1, ..., 2, 1, 2, ... */
int or_cycle_order(int t, int64_t k) {
    if (t <= 1) return 1;
    const int64_t p = k % (2 * (int64_t)t - 2);
    return (int)(p < t ? p + 1 : 2 * (int64_t)t - 1 - p);
}

typedef struct {
    int64_t iters, matvecs;
    int32_t stop;
    double rel_res, rel_normal, rho, rho_lo;
} or_info;

/* ---------------------------------------------------------------------- */
/* Error-free transformations and the Dot2 accumulator                     */
/* ---------------------------------------------------------------------- */
typedef struct { double p, s; } acc2;

/* Knuth's TwoSum: a + b = x + y exactly. */
static void two_sum(double a, double b, double *x, double *y) {
    double z;
    *x = a + b;
    z = *x - a;
    *y = (a - (*x - z)) + (b - z);
}

/* TwoProduct with a fused multiply-add: a * b = x + y exactly. */
static void two_prod(double a, double b, double *x, double *y) {
    *x = a * b;
    *y = fma(a, b, -*x);
}

/* One Dot2 step: acc += a * b. */
static void acc_add(acc2 *c, double a, double b) {
    double h, r, q;
    two_prod(a, b, &h, &r);
    two_sum(c->p, h, &c->p, &q);
    c->s = c->s + (q + r);
}

static double acc_value(acc2 c) { return c.p + c.s; }

double or_dot2(int64_t n, const double *x, const double *y) {
    acc2 c = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) acc_add(&c, x[i], y[i]);
    return acc_value(c);
}

/* ---------------------------------------------------------------------- */
/* Matrix products: y = A x, w = A^T u, r = b - A x                         */
/* ---------------------------------------------------------------------- */
void or_apply(const or_mat *A, const double *x, double *y) {
    for (int64_t i = 0; i < A->m; ++i) {
        acc2 c = {0.0, 0.0};
        if (A->kind == OR_CSR) {
            for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k)
                acc_add(&c, A->val[k], x[A->col_idx[k]]);
        } else {
            const double *row = A->val + i * A->ld;
            for (int64_t j = 0; j < A->n; ++j) acc_add(&c, row[j], x[j]);
        }
        y[i] = acc_value(c);
    }
}

/* (A^T u)_j = sum over i of a_ij u_i, terms in increasing i. */
void or_apply_t(const or_mat *A, const double *u, double *w) {
    acc2 *c = (acc2 *)calloc((size_t)A->n, sizeof(acc2));
    for (int64_t i = 0; i < A->m; ++i) {
        if (A->kind == OR_CSR) {
            for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k)
                acc_add(&c[A->col_idx[k]], A->val[k], u[i]);
        } else {
            const double *row = A->val + i * A->ld;
            for (int64_t j = 0; j < A->n; ++j) acc_add(&c[j], row[j], u[i]);
        }
    }
    for (int64_t j = 0; j < A->n; ++j) w[j] = acc_value(c[j]);
    free(c);
}

/* r_i = b_i - (A x)_i as one compensated sum of the terms b_i, -a_i1 x_1, ... */
void or_residual(const or_mat *A, const double *b, const double *x, double *r) {
    for (int64_t i = 0; i < A->m; ++i) {
        acc2 c = {0.0, 0.0};
        acc_add(&c, b[i], 1.0);
        if (A->kind == OR_CSR) {
            for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k)
                acc_add(&c, -A->val[k], x[A->col_idx[k]]);
        } else {
            const double *row = A->val + i * A->ld;
            for (int64_t j = 0; j < A->n; ++j) acc_add(&c, -row[j], x[j]);
        }
        r[i] = acc_value(c);
    }
}

/* ---------------------------------------------------------------------- */
/* The auxiliary equation of CTA (section 3.1, eq. "eqcoeff")               */
/* ---------------------------------------------------------------------- */
/*
 * phi[1..2t] holds phi_i = r^T H^i r.  The auxiliary equation is the t x t
 * Hankel system M alpha = g with M_ij = phi_{i+j}, g_i = phi_i (i, j = 1..t).
 * The paper asks for its minimum-norm solution when it is not unique; the
 * reading used here is a ridge solution of a scaled system, which is
 * continuous in phi (no threshold):
 *
 *   1. te = t, lowered to i-1 at the first i with phi_{2i} <= 0 (then H^i r = 0
 *      and the higher Krylov directions carry nothing).
 *   2. te = 1: alpha_1 = phi_1 / phi_2 (Example 1's closed form).
 *   3. Otherwise scale by powers of two, s_i = 2^-k_i with k_i = floor((e_i-1)/2)
 *      where phi_{2i} = f 2^e_i, f in [0.5, 1), so that the scaled diagonal lies
 *      in [1, 4) and the scaling is exact:  Ms_ij = (phi_{i+j} s_i) s_j,
 *      gs_i = phi_i s_i.  Add a ridge to the diagonal,
 *      Ms_ii = fma(Ms_ii, 16 te^2 2^-53, Ms_ii).
 *   4. Unpivoted Cholesky Ms = L L^T, column by column; if a pivot is not
 *      positive at column j, te is lowered to j (the leading block is kept).
 *      If te drops to 1 the closed form of step 2 is used.
 *   5. Forward and back substitution, alpha_i = s_i * alpha~_i, zero past te.
 * Returns te (0: no usable direction).
 */
int or_gram_alpha(const double *phi, int t, double *alpha) {
    double s[16], Ms[16][16], gs[16], L[16][16], z[16], at[16];
    int te = t, i, j, k;
    for (i = 0; i < t; ++i) alpha[i] = 0.0;
    for (i = 1; i <= t; ++i) {
        if (!(phi[2 * i] > 0.0)) { te = i - 1; break; }
    }
    if (te <= 0) return 0;
    if (te >= 2) {
        double ridge;
        for (i = 0; i < te; ++i) {
            int e;
            (void)frexp(phi[2 * (i + 1)], &e);
            int kk = (int)floor((e - 1) / 2.0);
            s[i] = ldexp(1.0, -kk);
        }
        for (i = 0; i < te; ++i) {
            for (j = 0; j < te; ++j) Ms[i][j] = (phi[i + j + 2] * s[i]) * s[j];
            gs[i] = phi[i + 1] * s[i];
        }
        ridge = 16.0 * (double)te * (double)te * ldexp(1.0, -53);
        for (i = 0; i < te; ++i) Ms[i][i] = fma(Ms[i][i], ridge, Ms[i][i]);
        for (j = 0; j < te; ++j) {
            double d = Ms[j][j];
            for (k = 0; k < j; ++k) d = fma(-L[j][k], L[j][k], d);
            if (!(d > 0.0)) { te = j; break; }
            L[j][j] = sqrt(d);
            for (i = j + 1; i < te; ++i) {
                double v = Ms[i][j];
                for (k = 0; k < j; ++k) v = fma(-L[i][k], L[j][k], v);
                L[i][j] = v / L[j][j];
            }
        }
    }
    if (te == 1) {
        alpha[0] = phi[1] / phi[2];
        return 1;
    }
    for (i = 0; i < te; ++i) {
        double v = gs[i];
        for (k = 0; k < i; ++k) v = fma(-L[i][k], z[k], v);
        z[i] = v / L[i][i];
    }
    for (i = te - 1; i >= 0; --i) {
        double v = z[i];
        for (k = i + 1; k < te; ++k) v = fma(-L[k][i], at[k], v);
        at[i] = v / L[i][i];
    }
    for (i = 0; i < te; ++i) alpha[i] = s[i] * at[i];
    return te;
}

/* ---------------------------------------------------------------------- */
/* Algorithm 1 (CTA) with H = A A^T                                         */
/* ---------------------------------------------------------------------- */
static int finite_all(const double *v, int n) {
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static void exit_diagnostics(const or_mat *A, const double *b, const double *x, double nb,
                             double *rel_res, double *rel_normal) {
    double *rt = (double *)malloc(sizeof(double) * (size_t)A->m);
    double *w = (double *)malloc(sizeof(double) * (size_t)A->n);
    double nab, nw;
    or_residual(A, b, x, rt);
    *rel_res = sqrt(or_dot2(A->m, rt, rt)) / nb;
    or_apply_t(A, rt, w);
    nw = sqrt(or_dot2(A->n, w, w));
    or_apply_t(A, b, w);
    nab = sqrt(or_dot2(A->n, w, w));
    *rel_normal = nab > 0.0 ? nw / nab : 0.0;
    free(rt);
    free(w);
}

/*
 * CTA iterates F_t (section 3.1, eqs. CTAGEN7 / CTAGEN7A; Algorithm 1):
 *   w_j = A^T u_j, u_{j+1} = A w_j with u_0 = r (so u_j = H^j r, w_j = A^T H^j r),
 *   phi_{2j+1} = ||w_j||^2 = r^T H^{2j+1} r,  phi_{2j+2} = ||u_{j+1}||^2 = r^T H^{2j+2} r,
 *   r'' = r' - sum_i alpha_i u_i,
 *   x'' = x' + sum_i alpha_i w_{i-1}              (x-form, minnorm = 0)
 *   y'' = y' + sum_i alpha_i u_{i-1}, x = A^T y   (minnorm = 1; Theorem 1 (4):
 *                                                   the iterate stays in range(A^T)).
 * Start x = 0 (Algorithm 1's first choice), r = b.  The relative residual
 * ||r||/||b|| is tested with the recurrence residual; when it passes, the
 * true residual b - A x decides, and if it fails the recurrence residual is
 * replaced by it and the loop goes on without counting an iteration.
 * The second clause of Algorithm 1 (r^T H r small) is read as
 * ||A^T r|| <= tol_normal ||A^T b||, or phi_2 = 0 (Example 1: H r = 0 means x
 * solves the normal equation).
 */
/* The enhanced stop of section 3.2 (a variant of Algorithm 1 for t >= 2), taken
 * literally with explicit vectors: from the current residual f_0 = r, the
 * first-order steps f_j = F_1(f_{j-1}) = f_{j-1} - a_j H f_{j-1}, with
 * a_j = phi_1(f_{j-1}) / phi_2(f_{j-1}) (Example 1's order-1 step), for
 * j = 1, ..., t - 1; the first f_j that passes the normal-equation test (the
 * quadratic form f^T H f of section 3.2, read as ||A^T f_j|| against
 * tol_normal ||A^T b||; ||A f_j|| for H = A, as for the plain test) ends the
 * solve at x^ = x + sum_{i<j} a_{i+1} A^T f_i (H = A A^T), whose residual is
 * f_j.  For the y-form the increment is sum a_{i+1} f_i on y (x = A^T y); for
 * H = A it is sum a_{i+1} f_i on x.  The products made here are the oracle's
 * way of evaluating these quantities and are not counted as the method's:
 * the method gets them from the iteration's phi_1..phi_2t.
 * Returns 1 (and updates x or y and r) if some f_j passes, else 0. */
static int or_enhanced(const or_mat *A, const or_opts *o, int minnorm, int t, double *r,
                       double *xy, double nab) {
    const int64_t m = A->m, n = A->n;
    const int ha = o->h_is_a;
    const int64_t ng = ha ? m : n;           /* length of g = A^T f (or A f) */
    const int64_t nd = (minnorm || ha) ? m : n;
    double *f = (double *)malloc(sizeof(double) * (size_t)m);
    double *hf = (double *)malloc(sizeof(double) * (size_t)m);
    double *g = (double *)malloc(sizeof(double) * (size_t)ng);
    double *dx = (double *)calloc((size_t)nd, sizeof(double));
    int hit = 0;
    int64_t e;
    memcpy(f, r, sizeof(double) * (size_t)m);
    if (ha) or_apply(A, f, g); else or_apply_t(A, f, g);
    for (int j = 1; j < t && !hit; ++j) {
        double p1, p2, a;
        if (ha) {
            memcpy(hf, g, sizeof(double) * (size_t)m);   /* H f = A f */
            p1 = or_dot2(m, f, hf);
        } else {
            or_apply(A, g, hf);                          /* H f = A (A^T f) */
            p1 = or_dot2(n, g, g);
        }
        p2 = or_dot2(m, hf, hf);
        if (!(p2 > 0.0) || !isfinite(p1) || !isfinite(p2)) break;
        a = p1 / p2;
        if (minnorm || ha)
            for (e = 0; e < m; ++e) dx[e] = fma(a, f[e], dx[e]);
        else
            for (e = 0; e < n; ++e) dx[e] = fma(a, g[e], dx[e]);
        for (e = 0; e < m; ++e) f[e] = fma(-a, hf[e], f[e]);
        if (ha) or_apply(A, f, g); else or_apply_t(A, f, g);
        if (sqrt(or_dot2(ng, g, g)) <= o->tol_normal * nab) hit = 1;
    }
    if (hit) {
        for (e = 0; e < nd; ++e) xy[e] += dx[e];
        memcpy(r, f, sizeof(double) * (size_t)m);
    }
    free(f);
    free(hf);
    free(g);
    free(dx);
    return hit;
}

int or_cta(const or_mat *A, const double *b, double *x, const or_opts *o, int minnorm,
           double *hist, int64_t hist_cap, or_info *info) {
    const int64_t m = A->m, n = A->n;
    const int t = o->t;
    int stop = 0;
    int64_t k = 0, matvecs = 0, i, e;
    double nb, nab = 0.0, rr, phi[17], alpha[8];
    double *r, *y = NULL, *u[9], *w[8], *rt;
    /* convex-combination step (the theorem on the first-order dynamics,
       section 3.4): the previous residual and iterate, and whether the current
       iterate came from such a step */
    double *rp = NULL, *xp = NULL;
    int last_jump = 0;

    memset(info, 0, sizeof(*info));
    if (t < 1 || t > 8) return -1;
    nb = sqrt(or_dot2(m, b, b));
    if (nb == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        if (hist_cap > 0) hist[0] = 0.0;
        info->stop = OR_RESIDUAL;
        return 0;
    }
    r = (double *)malloc(sizeof(double) * (size_t)m);
    rt = (double *)malloc(sizeof(double) * (size_t)m);
    for (i = 0; i <= t; ++i) u[i] = (double *)malloc(sizeof(double) * (size_t)m);
    for (i = 0; i < t; ++i) w[i] = (double *)malloc(sizeof(double) * (size_t)n);
    if (minnorm) y = (double *)calloc((size_t)m, sizeof(double));
    if (o->accel > 0.0) {
        rp = (double *)malloc(sizeof(double) * (size_t)m);
        xp = (double *)malloc(sizeof(double) * (size_t)(minnorm ? m : n));
    }

    if (o->tol_normal > 0.0) {
        or_apply_t(A, b, w[0]);
        nab = sqrt(or_dot2(n, w[0], w[0]));
        ++matvecs;
    }
    if (o->warm_start && !minnorm) {
        or_residual(A, b, x, r);
        ++matvecs;
    } else {
        memset(x, 0, sizeof(double) * (size_t)n);
        memcpy(r, b, sizeof(double) * (size_t)m);
    }
    rr = or_dot2(m, r, r);
    if (hist_cap > 0) hist[0] = sqrt(rr) / nb;

    for (;;) {
        if (sqrt(rr) <= o->tol * nb) {
            if (minnorm) { or_apply_t(A, y, x); ++matvecs; }
            or_residual(A, b, x, rt);
            ++matvecs;
            double rrt = or_dot2(m, rt, rt);
            if (sqrt(rrt) <= o->tol * nb) { stop = OR_RESIDUAL; break; }
            memcpy(r, rt, sizeof(double) * (size_t)m);
            rr = rrt;
        }
        if (k >= o->max_iter) { stop = OR_MAXITER; break; }

        memcpy(u[0], r, sizeof(double) * (size_t)m);
        const int tk = o->t_cycle ? or_cycle_order(t, k) : t; /* order of this iteration */
        if (o->h_is_a) {
            /* H = A: u_{j+1} = A u_j, phi_{2j+1} = u_j^T A u_j, phi_{2j+2} = ||A u_j||^2 */
            for (int j = 0; j < tk; ++j) {
                or_apply(A, u[j], u[j + 1]);
                phi[2 * j + 1] = or_dot2(m, u[j], u[j + 1]);
                phi[2 * j + 2] = or_dot2(m, u[j + 1], u[j + 1]);
                matvecs += 1;
            }
        } else {
            for (int j = 0; j < tk; ++j) {
                or_apply_t(A, u[j], w[j]);
                phi[2 * j + 1] = or_dot2(n, w[j], w[j]);
                or_apply(A, w[j], u[j + 1]);
                phi[2 * j + 2] = or_dot2(m, u[j + 1], u[j + 1]);
                matvecs += 2;
            }
        }
        if (!finite_all(phi + 1, 2 * tk)) { stop = OR_BREAKDOWN; break; }
        /* normal-equation test on ||A^T r||: phi_1 for H = A A^T, phi_2 = ||A r||^2
           (A symmetric) for H = A; phi_2 = 0 means H r = 0 (Example 1) */
        if (sqrt(o->h_is_a ? phi[2] : phi[1]) <= o->tol_normal * nab || phi[2] == 0.0) {
            stop = OR_NORMAL;
            break;
        }
        if (o->enhanced && tk >= 2 && o->tol_normal > 0.0 &&
            or_enhanced(A, o, minnorm, tk, r, minnorm ? y : x, nab)) {
            ++k;
            rr = or_dot2(m, r, r);
            if (k < hist_cap) hist[k] = sqrt(rr) / nb;
            stop = OR_NORMAL;
            break;
        }
        or_gram_alpha(phi, tk, alpha);
        if (!finite_all(alpha, tk)) { stop = OR_BREAKDOWN; break; }

        const double rr_prev = rr;
        if (rp != NULL) {
            memcpy(rp, r, sizeof(double) * (size_t)m);
            if (minnorm)
                memcpy(xp, y, sizeof(double) * (size_t)m);
            else
                memcpy(xp, x, sizeof(double) * (size_t)n);
        }
        for (int j = 0; j < tk; ++j)
            for (e = 0; e < m; ++e) r[e] = fma(-alpha[j], u[j + 1][e], r[e]);
        if (minnorm) {
            for (int j = 0; j < tk; ++j)
                for (e = 0; e < m; ++e) y[e] = fma(alpha[j], u[j][e], y[e]);
        } else if (o->h_is_a) {
            /* r' = r - sum alpha_i A^i r = b - A (x + sum alpha_i A^{i-1} r) */
            for (int j = 0; j < tk; ++j)
                for (e = 0; e < n; ++e) x[e] = fma(alpha[j], u[j][e], x[e]);
        } else {
            for (int j = 0; j < tk; ++j)
                for (e = 0; e < n; ++e) x[e] = fma(alpha[j], w[j][e], x[e]);
        }
        ++k;
        rr = or_dot2(m, r, r);
        /* Convex-combination step: when ||r_{k+1}|| / ||r_k|| = rho >= accel
           (the residuals "do not differ by much"), the iterate becomes
           a r_k + (1 - a) r_{k+1} (and the same combination of x or y) with
           a = rho / (rho + 1), the weight that gives F_1(.) = 0 on a critical
           line.  Not twice in a row: the pair must be two steps of F_t. */
        if (rp != NULL) {
            const double rho = rr_prev > 0.0 ? sqrt(rr / rr_prev) : 0.0;
            if (!last_jump && rho >= o->accel) {
                const double a = rho / (rho + 1.0), a1 = 1.0 - a;
                double *xy = minnorm ? y : x;
                const int64_t nxy = minnorm ? m : n;
                for (e = 0; e < m; ++e) r[e] = fma(a, rp[e], a1 * r[e]);
                for (e = 0; e < nxy; ++e) xy[e] = fma(a, xp[e], a1 * xy[e]);
                rr = or_dot2(m, r, r);
                last_jump = 1;
            } else {
                last_jump = 0;
            }
        }
        if (k < hist_cap) hist[k] = sqrt(rr) / nb;
        if (o->replace_every > 0 && k % o->replace_every == 0) {
            if (minnorm) { or_apply_t(A, y, x); ++matvecs; }
            or_residual(A, b, x, r);
            ++matvecs;
            rr = or_dot2(m, r, r);
        }
    }
    if (minnorm) or_apply_t(A, y, x);

    info->iters = k;
    info->matvecs = matvecs;
    info->stop = stop;
    exit_diagnostics(A, b, x, nb, &info->rel_res, &info->rel_normal);

    free(r);
    free(rt);
    for (i = 0; i <= t; ++i) free(u[i]);
    for (i = 0; i < t; ++i) free(w[i]);
    free(y);
    free(rp);
    free(xp);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Algorithms 2 and 3 (TA)                                                  */
/* ---------------------------------------------------------------------- */
/*
 * Iterate b' = A x' inside the ellipsoid E_{A,rho} = {A x : ||x|| <= rho}
 * (section 4).  With r = b - b' and c = A^T r:
 *   - stop when ||r|| <= tol ||b|| (confirmed on the true residual b - A x);
 *   - stop when ||c|| <= tol_normal ||A^T b|| (Theorem prop0TA (1): c = 0 means
 *     x solves the normal equation);
 *   - v_rho = rho A c / ||c|| maximises c^T z over E_{A,rho} (eq. vr) and is a
 *     strict pivot iff rho ||c|| >= r^T b (eq. eqlem2).  Then b'' is the point
 *     of segment [b', v_rho] nearest to b (Proposition prop1TA, eq. alph):
 *     alpha = r^T (v - b') / ||v - b'||^2, clamped to [0, 1];
 *     b'' = b' + alpha (v - b'), x'' = (1 - alpha) x' + alpha rho c / ||c||.
 *   - otherwise b' is a witness: Algorithm 2 (fixed_rho) stops and reports the
 *     lower bound r^T b / ||c|| < ||x*|| of Corollary 1; Algorithm 3 sets
 *     rho = max(2 rho, r^T b / ||c||) and goes on.  When the new rho equals
 *     r^T b / ||c|| the next step is a strict pivot by eq. eqlem2 with equality,
 *     so it is taken as one whatever rounding says.
 * Each while-body is one iteration, radius updates included.  Rounding order:
 *   gamma = rho / ||c||, s = A c, d_i = fma(gamma, s_i, -b'_i) (= v_i - b'_i),
 *   b'_i = fma(alpha, d_i, b'_i), x_j = fma(alpha gamma, c_j, (1 - alpha) x_j).
 */
/* The operator TA works on: A itself, or M = A^T A (normal_eq), applied as
 * A^T (A v) with the inner product A v rounded to FP64.  M is symmetric, so
 * M^T = M; M's residual b~ - M x is b~ - A^T t, t = A x, one compensated sum
 * of b~_j and the terms -a_ij t_i per column. */
typedef struct {
    const or_mat *A;
    int ne;
    double *tmp; /* m entries */
} or_op;

static void op_apply(const or_op *P, const double *v, double *y) {
    if (P->ne) {
        or_apply(P->A, v, P->tmp);
        or_apply_t(P->A, P->tmp, y);
    } else {
        or_apply(P->A, v, y);
    }
}

static void op_apply_t(const or_op *P, const double *v, double *y) {
    if (P->ne)
        op_apply(P, v, y);
    else
        or_apply_t(P->A, v, y);
}

static void op_residual(const or_op *P, const double *b, const double *x, double *r) {
    const or_mat *A = P->A;
    if (!P->ne) {
        or_residual(A, b, x, r);
        return;
    }
    acc2 *c = (acc2 *)calloc((size_t)A->n, sizeof(acc2));
    or_apply(A, x, P->tmp);
    for (int64_t j = 0; j < A->n; ++j) acc_add(&c[j], b[j], 1.0);
    for (int64_t i = 0; i < A->m; ++i) {
        if (A->kind == OR_CSR) {
            for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k)
                acc_add(&c[A->col_idx[k]], -A->val[k], P->tmp[i]);
        } else {
            const double *row = A->val + i * A->ld;
            for (int64_t j = 0; j < A->n; ++j) acc_add(&c[j], -row[j], P->tmp[i]);
        }
    }
    for (int64_t j = 0; j < A->n; ++j) r[j] = acc_value(c[j]);
    free(c);
}

int or_ta(const or_mat *A, const double *b0, double *x, const or_opts *o, double *hist,
          int64_t hist_cap, or_info *info) {
    /* normal_eq: the system is A^T A x = A^T b; m below is its row count n and
       b its right-hand side A^T b; the exit diagnostics stay on (A, b) */
    const int ne = o->normal_eq != 0;
    const int64_t n = A->n, m = ne ? A->n : A->m;
    const int pm = ne ? 2 : 1; /* passes over A per operator product */
    double *btil = NULL;
    or_op P = {A, ne, NULL};
    const double *b = b0;
    int stop = 0, pass = 0, have_c = 0;
    int64_t k = 0, matvecs = 0, i;
    double nb, nab = 0.0, rr, rb, rho = o->rho0, rho_lo = 0.0, nc = 0.0;
    double *bp, *r, *c, *s, *d, *rt;

    memset(info, 0, sizeof(*info));
    if (ne) {
        P.tmp = (double *)malloc(sizeof(double) * (size_t)(A->m > 0 ? A->m : 1));
        btil = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        or_apply_t(A, b0, btil);
        b = btil;
        ++matvecs;
    }
    nb = sqrt(or_dot2(m, b, b));
    if (!o->warm_start || nb == 0.0) memset(x, 0, sizeof(double) * (size_t)n);
    if (nb == 0.0) {
        if (hist_cap > 0) hist[0] = 0.0;
        info->stop = OR_RESIDUAL;
        info->rho = rho;
        info->matvecs = matvecs;
        free(P.tmp);
        free(btil);
        return 0;
    }
    bp = (double *)calloc((size_t)m, sizeof(double));
    r = (double *)malloc(sizeof(double) * (size_t)m);
    rt = (double *)malloc(sizeof(double) * (size_t)m);
    s = (double *)malloc(sizeof(double) * (size_t)m);
    d = (double *)malloc(sizeof(double) * (size_t)m);
    c = (double *)malloc(sizeof(double) * (size_t)n);
    if (o->tol_normal > 0.0) {
        op_apply_t(&P, b, c);
        if (o->nonneg)
            for (i = 0; i < n; ++i) c[i] = c[i] > 0.0 ? c[i] : 0.0;
        nab = sqrt(or_dot2(n, c, c));
        matvecs += pm;
    }
    if (o->warm_start) {  /* start from the given x: b' = A x */
        op_apply(&P, x, bp);
        matvecs += pm;
    }
    for (i = 0; i < m; ++i) r[i] = b[i] - bp[i];
    rr = or_dot2(m, r, r);
    rb = or_dot2(m, r, b);
    if (hist_cap > 0) hist[0] = sqrt(rr) / nb;

    for (;;) {
        if (sqrt(rr) <= o->tol * nb) {
            op_residual(&P, b, x, rt);
            matvecs += pm;
            if (sqrt(or_dot2(m, rt, rt)) <= o->tol * nb) { stop = OR_RESIDUAL; break; }
            op_apply(&P, x, bp);
            matvecs += pm;
            for (i = 0; i < m; ++i) r[i] = b[i] - bp[i];
            rr = or_dot2(m, r, r);
            rb = or_dot2(m, r, b);
            have_c = 0;
        }
        if (k >= o->max_iter) { stop = OR_MAXITER; break; }
        if (!have_c) {
            op_apply_t(&P, r, c);
            /* LP feasibility (section 6): the best point of E_{A,rho} within the
               cone x >= 0 uses c+ (Proposition eq. vrend2) */
            if (o->nonneg)
                for (i = 0; i < n; ++i) c[i] = c[i] > 0.0 ? c[i] : 0.0;
            nc = sqrt(or_dot2(n, c, c));
            matvecs += pm;
            have_c = 1;
        }
        if (!isfinite(nc) || !isfinite(rb)) { stop = OR_BREAKDOWN; break; }
        if (nc <= o->tol_normal * nab) { stop = OR_NORMAL; break; }
        if (pass || rho * nc >= rb) {
            double gamma = rho / nc, rd, dd, alpha, beta, a1;
            op_apply(&P, c, s);
            matvecs += pm;
            for (i = 0; i < m; ++i) d[i] = fma(gamma, s[i], -bp[i]);
            rd = or_dot2(m, r, d);
            dd = or_dot2(m, d, d);
            if (!(dd > 0.0) || !isfinite(rd) || !isfinite(dd)) { stop = OR_BREAKDOWN; break; }
            alpha = rd / dd;
            if (alpha < 0.0) alpha = 0.0;
            if (alpha > 1.0) alpha = 1.0;
            for (i = 0; i < m; ++i) bp[i] = fma(alpha, d[i], bp[i]);
            beta = alpha * gamma;
            a1 = 1.0 - alpha;
            for (i = 0; i < n; ++i) x[i] = fma(beta, c[i], a1 * x[i]);
            pass = 0;
            have_c = 0;
            for (i = 0; i < m; ++i) r[i] = b[i] - bp[i];
            rr = or_dot2(m, r, r);
            rb = or_dot2(m, r, b);
        } else {
            double q = rb / nc;
            if (o->fixed_rho) { rho_lo = q; stop = OR_WITNESS; break; }
            if (q > rho_lo) rho_lo = q;
            if (o->rho_max > 0.0 && ((2.0 * rho >= q) ? 2.0 * rho : q) > o->rho_max) {
                stop = OR_WITNESS;  /* no solution within the radius bound */
                break;
            }
            pass = (q >= 2.0 * rho);
            rho = (2.0 * rho >= q) ? 2.0 * rho : q;
        }
        ++k;
        if (k < hist_cap) hist[k] = sqrt(rr) / nb;
    }
    info->iters = k;
    info->matvecs = matvecs;
    info->stop = stop;
    info->rho = rho;
    info->rho_lo = rho_lo;
    exit_diagnostics(A, b0, x, sqrt(or_dot2(A->m, b0, b0)), &info->rel_res,
                     &info->rel_normal);
    free(bp);
    free(r);
    free(rt);
    free(s);
    free(d);
    free(P.tmp);
    free(btil);
    free(c);
    return 0;
}

/* The restart of the remark that follows the theorem on Algorithm 3's
 * properties (section 4.3): take eps' = eps at first (tol_normal = 0 means
 * so); whenever a run ends with an eps'-approximate solution of the normal
 * equation, halve eps' and run Algorithm 3 again from the current
 * approximate solution (b' = A x first), at most max_halvings times.
 * Iterations and products are summed over the runs; stop, residuals and
 * radii are the last run's. */
int or_ta_halving(const or_mat *A, const double *b, double *x, const or_opts *o,
                  int32_t max_halvings, or_info *info, int32_t *halvings) {
    or_opts p = *o;
    if (!(p.tol_normal > 0.0)) p.tol_normal = p.tol;
    int64_t iters = 0, matvecs = 0;
    int32_t h = 0;
    for (;;) {
        or_info r;
        const int rc = or_ta(A, b, x, &p, NULL, 0, &r);
        if (rc != 0) return rc;
        iters += r.iters;
        matvecs += r.matvecs;
        *info = r;
        if (r.stop != OR_NORMAL || h >= max_halvings) break;
        p.tol_normal *= 0.5;
        p.warm_start = 1;
        ++h;
    }
    info->iters = iters;
    info->matvecs = matvecs;
    *halvings = h;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Gradient of the solution map (not in the paper)                         */
/* ---------------------------------------------------------------------- */
/*
 * For a square nonsingular A, x(A, b) = A^{-1} b is the limit of Algorithm 1
 * (Theorem 1 (4) with range(A^T) = R^n).  A loss L(x) has
 *   dL/db = lambda,   dL/da_ij = -lambda_i x_j,   where A^T lambda = dL/dx.
 * or_csr_outer writes the second formula on the stored pattern of a CSR A:
 * out[k] = (alpha * u[i]) * v[j] for the k-th stored entry (i, j).
 */
void or_csr_outer(const or_mat *A, const double *u, const double *v, double alpha, double *out) {
    for (int64_t i = 0; i < A->m; ++i)
        for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k)
            out[k] = (alpha * u[i]) * v[A->col_idx[k]];
}

/* ---------------------------------------------------------------------- */
/* TA for an approximate minimum-norm solution (Algorithm 4, section 4.4)  */
/* ---------------------------------------------------------------------- */
/*
 * Given x_eps with ||A x_eps - b|| <= tol ||b||, bisect on the radius rho of
 * the ellipsoid E_{A, rho}: the upper bound starts at ||x_eps||, the lower
 * bound at 0, and each test runs Algorithm 2 (TA with the fixed radius
 * rho = midpoint) until it finds an approximate solution in the ball
 * (the upper bound drops to rho, the solution is kept) or a witness (the
 * lower bound rises to (b - b')^T b / ||c|| >= rho, Corollary 1).  Each test
 * starts from the last witness's x (0 before the first witness).  The loop
 * ends when upper - lower <= tol * ||x_eps||, when a test ends on the normal
 * equation (its x is returned), or when the iteration budget o->max_iter,
 * counted over all tests, runs out.  Corollary 1's bound holds for consistent
 * systems; if a witness lifts the lower bound above the upper one by more
 * than the gap tolerance, the input was not an approximate solution of a
 * consistent system and the stop code is OR_WITNESS (x = the last solution
 * found, or x_eps).  info: iters and matvecs summed over the tests, rho =
 * upper bound, rho_lo = lower bound, rel_res / rel_normal of the returned x.
 * Returns the number of tests.
 */
int64_t or_ta_minnorm(const or_mat *A, const double *b, const double *x_eps, double *x,
                      const or_opts *o, or_info *info) {
    const int64_t m = A->m, n = A->n;
    double nb = sqrt(or_dot2(m, b, b));
    double hi = sqrt(or_dot2(n, x_eps, x_eps)), lo = 0.0;
    const double gap = o->tol * hi;
    double *xt = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *xw = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    int have_w = 0, stop = OR_RESIDUAL;
    int64_t tests = 0, iters = 0, matvecs = 0;

    memset(info, 0, sizeof(*info));
    memcpy(x, x_eps, sizeof(double) * (size_t)n);
    if (nb == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        hi = 0.0;
    }
    while (nb > 0.0 && hi - lo > gap) {
        or_opts t = *o;
        or_info ti;
        const double rho = 0.5 * (hi + lo);
        if (iters >= o->max_iter) { stop = OR_MAXITER; break; }
        t.fixed_rho = 1;
        t.rho0 = rho;
        t.warm_start = have_w;
        t.max_iter = o->max_iter - iters;
        if (have_w) memcpy(xt, xw, sizeof(double) * (size_t)n);
        or_ta(A, b, xt, &t, NULL, 0, &ti);
        ++tests;
        iters += ti.iters;
        matvecs += ti.matvecs;
        if (ti.stop == OR_RESIDUAL) {
            hi = rho;
            memcpy(x, xt, sizeof(double) * (size_t)n);
        } else if (ti.stop == OR_WITNESS) {
            lo = ti.rho_lo;
            memcpy(xw, xt, sizeof(double) * (size_t)n);
            have_w = 1;
        } else {
            if (ti.stop == OR_NORMAL) memcpy(x, xt, sizeof(double) * (size_t)n);
            stop = ti.stop;
            break;
        }
    }
    if (stop == OR_RESIDUAL && lo - hi > gap) stop = OR_WITNESS;
    info->iters = iters;
    info->matvecs = matvecs;
    info->stop = stop;
    info->rho = hi;
    info->rho_lo = lo;
    if (nb > 0.0) exit_diagnostics(A, b, x, nb, &info->rel_res, &info->rel_normal);
    free(xt);
    free(xw);
    return tests;
}
