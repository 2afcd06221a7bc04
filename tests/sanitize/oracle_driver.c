/*
 * Drives every entry point of the CPU oracle (oracle/oracle.c) on small dense
 * and CSR problems, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: out-of-bounds accesses, leaks, signed overflow
 * or misaligned loads anywhere in the oracle end the run with an error.
 * Prints one line per call; the test checks the exit status only.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

enum { OR_DENSE = 0, OR_CSR = 1 };
typedef struct {
    int32_t kind;
    int64_t m, n, ld;
    const int32_t *row_ptr, *col_idx;
    const double *val;
} or_mat;
typedef struct {
    double tol, tol_normal;
    int32_t t;
    int64_t max_iter;
    int32_t replace_every, warm_start;
    double rho0;
    int32_t fixed_rho, h_is_a, t_cycle, nonneg;
    double rho_max;
    int32_t enhanced, normal_eq;
    double accel;
} or_opts;
typedef struct {
    int64_t iters, matvecs;
    int32_t stop;
    double rel_res, rel_normal, rho, rho_lo;
} or_info;

double or_dot2(int64_t n, const double *x, const double *y);
void or_apply(const or_mat *A, const double *x, double *y);
void or_apply_t(const or_mat *A, const double *u, double *w);
void or_residual(const or_mat *A, const double *b, const double *x, double *r);
int or_gram_alpha(const double *phi, int t, double *alpha);
int or_cta(const or_mat *A, const double *b, double *x, const or_opts *o, int minnorm,
           double *hist, int64_t hist_cap, or_info *info);
int or_ta(const or_mat *A, const double *b, double *x, const or_opts *o, double *hist,
          int64_t hist_cap, or_info *info);
void or_csr_outer(const or_mat *A, const double *u, const double *v, double alpha, double *out);
int64_t or_ta_minnorm(const or_mat *A, const double *b, const double *x_eps, double *x,
                      const or_opts *o, or_info *info);

static uint64_t rs = 88172645463325252ull;
static double rnd(void) {  /* xorshift64, uniform in [-1, 1) */
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (double)(rs >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

int main(void) {
    enum { M = 13, N = 9 };
    double *a = malloc(sizeof(double) * M * N), *b = malloc(sizeof(double) * M);
    double *x = calloc(N, sizeof(double)), *xs = malloc(sizeof(double) * N);
    double *hist = malloc(sizeof(double) * 4001);
    int32_t *rp = malloc(sizeof(int32_t) * (M + 1)), *ci = malloc(sizeof(int32_t) * M * N);
    double *cv = malloc(sizeof(double) * M * N), *out = malloc(sizeof(double) * M * N);
    int64_t nnz = 0;
    for (int i = 0; i < M; ++i) {
        rp[i] = (int32_t)nnz;
        for (int j = 0; j < N; ++j) {
            a[i * N + j] = (i + j) % 3 == 0 ? 0.0 : rnd();
            if (a[i * N + j] != 0.0) {
                ci[nnz] = j;
                cv[nnz++] = a[i * N + j];
            }
        }
    }
    rp[M] = (int32_t)nnz;
    for (int j = 0; j < N; ++j) xs[j] = rnd();
    or_mat D = {OR_DENSE, M, N, N, NULL, NULL, a};
    or_mat C = {OR_CSR, M, N, 0, rp, ci, cv};
    or_apply(&D, xs, b);  /* consistent right-hand side */
    double w[N], r[M], phi[17] = {0, 3, 7, 2, 5, 1, 4, 2, 9}, alpha[8];
    or_apply_t(&C, b, w);
    or_residual(&C, b, xs, r);
    printf("dot2 %.3e gram %d\n", or_dot2(M, b, b), or_gram_alpha(phi, 4, alpha));
    or_csr_outer(&C, b, xs, -1.0, out);
    const or_mat *mats[2] = {&D, &C};
    for (int q = 0; q < 2; ++q) {
        for (int t = 1; t <= 4; ++t)
            for (int form = 0; form < 2; ++form) {
                or_opts o = {0};
                o.tol = 1e-9;
                o.t = t;
                o.max_iter = 4000;
                o.replace_every = t == 2 ? 3 : 0;
                o.tol_normal = t == 3 ? 1e-10 : 0.0;
                o.enhanced = t == 3;
                o.accel = t == 4 ? 0.5 : 0.0;
                o.t_cycle = t == 4 && form == 0;
                or_info info;
                memset(x, 0, sizeof(double) * N);
                or_cta(mats[q], b, x, &o, form, hist, 4001, &info);
                printf("cta q%d t%d form%d: stop %d iters %lld\n", q, t, form, info.stop,
                       (long long)info.iters);
            }
        for (int variant = 0; variant < 4; ++variant) {
            or_opts o = {0};
            o.tol = 1e-6;
            o.max_iter = 20000;
            o.normal_eq = variant == 1;
            o.nonneg = variant == 2;
            o.fixed_rho = variant == 3;
            o.rho0 = variant == 3 ? 0.5 : 0.0;
            o.tol_normal = 1e-12;
            or_info info;
            memset(x, 0, sizeof(double) * N);
            or_ta(mats[q], b, x, &o, hist, 4001, &info);
            printf("ta q%d v%d: stop %d iters %lld\n", q, variant, info.stop,
                   (long long)info.iters);
        }
        or_opts o = {0};
        o.tol = 1e-3;
        o.max_iter = 20000;
        or_info info;
        double xe[N];
        for (int j = 0; j < N; ++j) xe[j] = xs[j];
        int64_t tests = or_ta_minnorm(mats[q], b, xe, x, &o, &info);
        printf("minnorm q%d: %lld tests stop %d\n", q, (long long)tests, info.stop);
    }
    free(a); free(b); free(x); free(xs); free(hist); free(rp); free(ci); free(cv); free(out);
    return 0;
}
