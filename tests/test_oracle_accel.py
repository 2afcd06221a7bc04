"""Pins of the oracle's convex-combination step (the theorem on the dynamics
of first-order CTA, section 3.4): when ||r_{k+1}|| >= theta ||r_k||, the
iterate becomes a r_k + (1 - a) r_{k+1} with a = rho / (rho + 1),
rho = ||r_{k+1}|| / ||r_k||.

On an ij-critical line the first-order step zig-zags with the constant
factor rho_ij = (lambda_j - lambda_i) / (lambda_j + lambda_i), and that
combination is an eigenvector, which the next step solves exactly.  The
expected values are written in the eigenbasis, not by re-running the
oracle's arithmetic."""
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def _critical(lam_i, lam_j, n=6, seed=0):
    """A (n x n) with H = A A^T having eigenvalues lam_i (first half) and
    lam_j (second half) on orthonormal U; b on the ij-critical line:
    b = sqrt(lam_j) u + sqrt(lam_i) v with unit u, v in the two eigenspaces."""
    g = np.random.default_rng(seed)
    U, _ = np.linalg.qr(g.standard_normal((n, n)))
    h = n // 2
    s = np.concatenate([np.full(h, np.sqrt(lam_i)), np.full(n - h, np.sqrt(lam_j))])
    A = (U * s) @ U.T  # symmetric, A A^T = U diag(lam) U^T
    cu = g.standard_normal(h)
    cv = g.standard_normal(n - h)
    u = U[:, :h] @ (cu / np.linalg.norm(cu))
    v = U[:, h:] @ (cv / np.linalg.norm(cv))
    return A, np.sqrt(lam_j) * u + np.sqrt(lam_i) * v


@pytest.mark.parametrize("lams", [(1.0, 9.0), (0.5, 40.0)])
def test_critical_line_is_solved_after_one_combination(lams):
    A, b = _critical(*lams)
    rho = (lams[1] - lams[0]) / (lams[1] + lams[0])
    _, hist0, i0 = oracle.cta(A, b, tol=1e-12, t=1, max_iter=10_000)
    x, hist, info = oracle.cta(A, b, tol=1e-12, t=1, max_iter=10_000, accel=0.5)
    # plain first-order CTA zig-zags with the factor rho
    np.testing.assert_allclose(hist0[1:6] / hist0[0:5], rho, rtol=1e-10)
    assert i0.iters > 20
    # with the step: one first-order step, the combination (an eigenvector:
    # the larger-eigenvalue component cancels), then an exact step
    assert info.stop == "residual" and info.iters == 2
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-12, atol=1e-14)
    a = rho / (rho + 1.0)
    r1 = b - (np.dot(A.T @ b, A.T @ b) / np.dot(A @ (A.T @ b), A @ (A.T @ b))) * (A @ (A.T @ b))
    rbar = a * b + (1 - a) * r1
    np.testing.assert_allclose(hist[1], np.linalg.norm(rbar) / np.linalg.norm(b), rtol=1e-12)


def test_critical_line_y_form():
    A, b = _critical(1.0, 9.0, seed=3)
    xs = np.linalg.solve(A, b)
    xy, _, iy = oracle.cta_minnorm(A, b, tol=1e-12, t=1, max_iter=1000, accel=0.5)
    assert iy.stop == "residual" and iy.iters == 2
    np.testing.assert_allclose(xy, xs, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("t", [1, 2, 3])
def test_no_trigger_is_plain_cta(t):
    """A threshold the residual ratios never reach: plain CTA, bit for bit."""
    g = np.random.default_rng(4)
    A = np.eye(30) * 4.0 + 0.3 * g.standard_normal((30, 30))
    b = g.standard_normal(30)
    kw = dict(tol=1e-10, t=t, max_iter=200)
    x0, h0, i0 = oracle.cta(A, b, **kw)
    assert np.max(h0[1:] / h0[:-1]) < 0.9
    x1, h1, i1 = oracle.cta(A, b, accel=0.95, **kw)
    assert i0 == i1 and np.array_equal(x0, x1) and np.array_equal(h0, h1)


def test_combination_keeps_residual_consistent():
    """r is carried by recurrence through the combinations; the reported
    residual is the true one, within the tolerance, at a residual stop."""
    from workloads import kac_clement

    p = kac_clement(101)
    x, _, info = oracle.cta(p.A, p.b, tol=1e-8, t=1, max_iter=20_000, accel=0.5)
    assert info.stop == "residual" and info.rel_res <= 1e-8
    _, _, plain = oracle.cta(p.A, p.b, tol=1e-8, t=1, max_iter=20_000)
    assert info.iters < plain.iters
