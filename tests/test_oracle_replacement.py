"""Pins of the oracle's residual-replacement and candidate-rejection paths.

Algorithm 1 iterates F_t, a map of the current residual alone (section 3.1,
eqs. CTAGEN7 / CTAGEN7A): what the next iterate is depends only on (x, r),
never on how r was obtained.  Algorithm 3 iterates on (b', rho) with
b' = A x' (section 4, the update after Proposition prop1TA).  The reading of
both algorithms here carries r (or b') by recurrence, and
  * at a candidate stop lets the true residual b - A x decide; when it fails,
    the recurrence residual is replaced by the true one (CTA: r <- b - A x;
    TA: b' <- A x) and the loop goes on without counting an iteration;
  * with a period p > 0, replaces r by b - A x after every p-th iteration
    (x = A^T y first in the y-form).

None of these tests re-types the oracle's arithmetic.  They check what the
paper and the structure of the two algorithms force:
  * a replaced (or rejected) state equals a fresh start from the same iterate,
    bit for bit: the warm start computes exactly the quantities the
    replacement must produce, so any stale part (a kept recurrence vector,
    a stale norm, a skipped x = A^T y) shows up as a different trajectory;
  * with p = 1 the stop test sees the true residual, so a candidate can never
    be rejected: the product count is fixed by the iteration count;
  * replacement changes the trajectory by rounding only on a well-conditioned
    system, in both forms.
"""
import numpy as np
import pytest

import oracle
from workloads import convection_diffusion, dense_gaussian


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def three_singular_values(n=30, seed=0, svals=(1.0, 2.0, 4.0)):
    """A = Q1 diag(s) Q2^T with s taking three distinct values: H = A A^T has
    three distinct eigenvalues, so CTA-3 needs a couple of steps to reach the
    rounding floor, and tolerances below that floor force the candidate stop
    to reject the recurrence residual."""
    g = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(g.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(g.standard_normal((n, n)))
    s = np.array([svals[i % len(svals)] for i in range(n)])
    A = (Q1 * s) @ Q2.T
    return A, A @ g.standard_normal(n)


def _first_rejection(hist, tol, iters):
    """The recurrence norm tested at the top of iteration k is hist[k]; a test
    that passes at k < iters (the run went on) is a rejected candidate."""
    for k in range(min(len(hist), iters)):
        if hist[k] <= tol:
            return k
    return None


# --------------------------------------------------------------------------
# CTA, candidate rejection: r <- b - A x
# --------------------------------------------------------------------------
CTA_REJECT_CASES = [
    # (name, builder, t, tol, max_iter): tolerances just below what the
    # recurrence reaches first, so the candidate check rejects it
    ("three_sv_floor", lambda: three_singular_values(), 3, 1e-17, 8),
    ("convdiff8", lambda: (convection_diffusion(8).A, convection_diffusion(8).b), 3, 1e-14, 2000),
    ("gauss20", lambda: (dense_gaussian(20, seed=1).A, dense_gaussian(20, seed=1).b), 3, 1e-13,
     20000),
]


@pytest.mark.parametrize("case", CTA_REJECT_CASES, ids=lambda c: c[0])
def test_cta_rejected_candidate_restarts_from_the_true_residual(case):
    """After a rejected candidate at the top of iteration k, the run continues
    exactly as a fresh x-form run warm-started from x_k: same history entries
    bit for bit, same final x, same stop, and the product counts add up (the
    fresh run's own b - A x_k stands for the rejected check's)."""
    _, build, t, tol, K = case
    A, b = build()
    x, h, info = oracle.cta(A, b, tol=tol, t=t, max_iter=K)
    k = _first_rejection(h, tol, info.iters)
    assert k is not None and k >= 1, "the case must reject a candidate"
    # products: 2t per iteration plus the one rejected check
    xa, ha, ia = oracle.cta(A, b, tol=tol, t=t, max_iter=k)
    assert ia.stop == "maxiter" and ia.matvecs == 2 * t * k + 1
    np.testing.assert_array_equal(ha, h[:k + 1])
    xb, hb, ib = oracle.cta(A, b, tol=tol, t=t, max_iter=K - k, x0=xa)
    assert ib.stop == info.stop and ib.iters == info.iters - k
    np.testing.assert_array_equal(hb[1:], h[k + 1:])
    np.testing.assert_array_equal(xb, x)
    assert ia.matvecs + ib.matvecs - 1 == info.matvecs


# --------------------------------------------------------------------------
# CTA, periodic replacement
# --------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1, 3, 7])
def test_cta_periodic_replacement_is_a_warm_restart(p):
    """A replacement after iteration p leaves the state a warm start from x_p
    has: the run with period p equals (first p iterations) + (warm start from
    x_p with period p), bit for bit, in history, x and stop."""
    pr = convection_diffusion(8)
    tol, t, K = 1e-9, 3, 3000
    x, h, info = oracle.cta(pr.A, pr.b, tol=tol, t=t, max_iter=K, replace_every=p)
    assert info.stop == "residual" and info.iters > p
    xa, ha, _ = oracle.cta(pr.A, pr.b, tol=tol, t=t, max_iter=p)
    np.testing.assert_array_equal(ha, h[:p + 1])
    xb, hb, ib = oracle.cta(pr.A, pr.b, tol=tol, t=t, max_iter=K - p, x0=xa, replace_every=p)
    assert ib.stop == info.stop and ib.iters == info.iters - p
    np.testing.assert_array_equal(hb[1:], h[p + 1:])
    np.testing.assert_array_equal(xb, x)


@pytest.mark.parametrize("minnorm", [False, True], ids=["x-form", "y-form"])
def test_cta_replacement_every_iteration_never_rejects(minnorm):
    """With p = 1 the stop test always sees the freshly replaced true
    residual, so the candidate check at a stop recomputes the same value and
    passes, and below the rounding floor no check is ever made: the product
    count is exactly iters * (2t + 1) (x-form) or iters * (2t + 2) (y-form:
    x = A^T y before each residual), plus the final check at a RESIDUAL stop."""
    A, b = three_singular_values()
    t = 3
    per = 2 * t + (2 if minnorm else 1)
    fin = 2 if minnorm else 1
    for tol, K in ((1e-17, 10), (1e-15, 10), (1e-9, 10)):
        x, h, info = oracle.cta(A, b, tol=tol, t=t, max_iter=K, replace_every=1, minnorm=minnorm)
        if tol == 1e-17:
            assert info.stop == "maxiter"   # below what FP64 can reach
        assert info.matvecs == info.iters * per + (fin if info.stop == "residual" else 0), (
            tol, info)
    pr = convection_diffusion(8)
    x, h, info = oracle.cta(pr.A, pr.b, tol=1e-14, t=t, max_iter=3000, replace_every=1,
                            minnorm=minnorm)
    assert info.stop == "residual"
    assert info.matvecs == info.iters * per + fin


@pytest.mark.parametrize("minnorm", [False, True], ids=["x-form", "y-form"])
@pytest.mark.parametrize("p", [1, 4])
def test_cta_replacement_changes_the_trajectory_by_rounding_only(minnorm, p):
    """On a well-conditioned system the recurrence residual tracks b - A x to
    rounding, so replacing it every p iterations changes neither the
    iteration count nor, beyond rounding, the history and x (both forms)."""
    pr = dense_gaussian(40, seed=3, m=20)   # 20 x 40, full row rank
    t, tol = 2, 1e-10
    x0, h0, i0 = oracle.cta(pr.A, pr.b, tol=tol, t=t, max_iter=5000, minnorm=minnorm)
    x1, h1, i1 = oracle.cta(pr.A, pr.b, tol=tol, t=t, max_iter=5000, minnorm=minnorm,
                            replace_every=p)
    assert i0.stop == i1.stop == "residual"
    assert abs(i0.iters - i1.iters) <= 1
    n = min(len(h0), len(h1)) - 1
    np.testing.assert_allclose(h1[:n], h0[:n], rtol=1e-6, atol=1e-13)
    assert np.linalg.norm(x1 - x0) <= 1e-9 * np.linalg.norm(x0)
    # and the limit is the minimum-norm solution (full row rank: consistent)
    xs = np.linalg.pinv(pr.A.to_dense() if hasattr(pr.A, "to_dense") else pr.A) @ pr.b
    assert np.linalg.norm(x1 - xs) <= 1e-8 * np.linalg.norm(xs)


# --------------------------------------------------------------------------
# TA, candidate rejection: b' <- A x
# --------------------------------------------------------------------------
TA_REJECT_CASES = [
    ("gauss6x9", lambda: dense_gaussian(9, seed=2, m=6), 3e-16, 20000),
    ("convdiff8", lambda: convection_diffusion(8), 3e-15, 20000),
]


@pytest.mark.parametrize("case", TA_REJECT_CASES, ids=lambda c: c[0])
def test_ta_rejected_candidate_restarts_from_A_x(case):
    """After a rejected candidate at the top of iteration k (only possible
    right after a pivot step, which clears the tie flag), TA continues exactly
    as a fresh warm start from x_k with radius rho_k: b' = A x_k, the same
    history entries bit for bit, the same x and stop."""
    _, build, tol, K = case
    pr = build()
    x, h, info = oracle.ta(pr.A, pr.b, tol=tol, max_iter=K)
    k = _first_rejection(h, tol, info.iters)
    assert k is not None and k >= 1, "the case must reject a candidate"
    xa, ha, ia = oracle.ta(pr.A, pr.b, tol=tol, max_iter=k)
    np.testing.assert_array_equal(ha, h[:k + 1])
    xb, hb, ib = oracle.ta(pr.A, pr.b, tol=tol, max_iter=K - k, x0=xa, rho0=ia.rho)
    assert ib.stop == info.stop and ib.iters == info.iters - k
    np.testing.assert_array_equal(hb[1:], h[k + 1:])
    np.testing.assert_array_equal(xb, x)
    assert ib.rho == info.rho


@pytest.mark.parametrize("case", TA_REJECT_CASES, ids=lambda c: c[0])
def test_ta_exit_residual_is_the_true_one(case):
    """At a RESIDUAL stop the reported relative residual is the true
    ||b - A x|| / ||b|| (numpy, in extended precision via the oracle-free
    long double sum) and it meets the tolerance, even though the recurrence
    was rejected on the way."""
    _, build, tol, K = case
    pr = build()
    x, h, info = oracle.ta(pr.A, pr.b, tol=tol, max_iter=K)
    assert info.stop == "residual"
    a = pr.A if isinstance(pr.A, np.ndarray) else pr.A.to_dense()
    r = np.asarray(pr.b, np.longdouble) - a.astype(np.longdouble) @ x.astype(np.longdouble)
    rel = float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(np.asarray(pr.b, np.longdouble) ** 2)))
    assert rel <= tol * (1 + 1e-6)
    assert info.rel_res == pytest.approx(rel, rel=1e-2, abs=1e-19)
