/*
 * Drives the host-only paths of libta (argument validation, error texts,
 * every solver's rejection of bad arguments before any device work) for a
 * build whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Needs no GPU: no call below reaches the
 * device.  The test checks the exit status and that each call returned the
 * expected code.
 */
#include <stdio.h>
#include <string.h>

#include "ta.h"

static int fails = 0;
static void expect(const char *what, int got, int want) {
    if (got != want) {
        printf("FAIL %s: %d (want %d)\n", what, got, want);
        ++fails;
    }
}

int main() {
    ta_mat A = {TA_CSR, 10, 8, 20, 0, (const int32_t *)0x1000, (const int32_t *)0x2000,
                (const double *)0x3000};
    ta_mat D = {TA_DENSE_ROWMAJOR, 5, 4, 20, 4, nullptr, nullptr, (const double *)0x1000};
    ta_opts o;
    memset(&o, 0, sizeof o);
    o.tol = 1e-6;
    o.t = 3;
    o.max_iter = 10;
    expect("validate csr", ta_validate(&A, &o, 0), TA_OK);
    expect("validate dense", ta_validate(&D, &o, 1), TA_OK);
    expect("validate null", ta_validate(nullptr, &o, 0), TA_EINVAL);
    expect("validate opts null", ta_validate(&A, nullptr, 0), TA_EINVAL);
    for (int solver = 0; solver < 4; ++solver)
        for (int t = -1; t <= 10; ++t)
            for (int prec = 0; prec < 4; ++prec) {
                ta_opts q = o;
                q.t = t;
                q.precision = prec;
                (void)ta_validate(&A, &q, solver);
            }
    ta_opts bad = o;
    bad.tol = 1.5;
    expect("tol", ta_validate(&A, &bad, 0), TA_EINVAL);
    bad = o;
    bad.accel = 0.5;
    bad.precision = TA_FP32;
    expect("accel fp32", ta_validate(&A, &bad, 0), TA_EINVAL);
    for (int c = -7; c <= 1; ++c) (void)strlen(ta_strerror(c));
    ta_info info;
    double *dx = (double *)0x10;
    expect("cta_solve b", cta_solve(&A, nullptr, dx, &o, nullptr, 0, &info, nullptr), TA_EINVAL);
    expect("cta_minnorm info", cta_minnorm(&A, (const double *)0x8, dx, &o, nullptr, 0, nullptr,
                                           nullptr),
           TA_EINVAL);
    expect("ta_solve opts", ta_solve(&A, (const double *)0x8, dx, nullptr, nullptr, 0, &info,
                                     nullptr),
           TA_EINVAL);
    expect("ta_minnorm x_eps", ta_minnorm(&A, (const double *)0x8, nullptr, dx, &bad, &info,
                                          nullptr, nullptr),
           TA_EINVAL);
    expect("plan null", cta_solve_plan(nullptr, nullptr, nullptr, &o, nullptr, 0, &info, nullptr),
           TA_EINVAL);
    expect("noalloc null", cta_solve_plan_noalloc(nullptr, nullptr, nullptr, &o, nullptr, 0, &info,
                                                  nullptr),
           TA_EINVAL);
    expect("plan create", ta_plan_create(&A, nullptr, nullptr), TA_EINVAL);
    expect("plan destroy", ta_plan_destroy(nullptr), TA_OK);
    int32_t f = 0;
    expect("plan format", ta_plan_format(nullptr, 0, &f), TA_EINVAL);
    ta_batch_plan *bp = nullptr;
    expect("batch plan 0", ta_batch_plan_create(0, &A, TA_FP32, &bp, nullptr), TA_EINVAL);
    expect("batch plan prec", ta_batch_plan_create(1, &A, 9, &bp, nullptr), TA_EINVAL);
    expect("batch destroy", ta_batch_plan_destroy(nullptr), TA_OK);
    expect("batched null", cta_solve_batched(nullptr, nullptr, nullptr, nullptr, &o, 0, &info,
                                             nullptr),
           TA_EINVAL);
    double ms = 0;
    expect("time null", ta_time_matvec_plan(nullptr, 0, nullptr, nullptr, 1, &ms, nullptr),
           TA_EINVAL);
    expect("batch time null", ta_batch_time_spmm(nullptr, 64, 0, 0, 1, &ms, nullptr), TA_EINVAL);
    printf("%d failures\n", fails);
    return fails == 0 ? 0 : 1;
}
