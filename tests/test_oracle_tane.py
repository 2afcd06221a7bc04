"""Pins of the oracle's TA on the normal equation A^T A x = A^T b (the inputs
the rectangular hybrid of section 5.3 gives TA when the system is not
solvable): the limit is a least-squares solution, from x = 0 the
minimum-norm one (pinv), within the bound the normal-equation residual
allows; Algorithm 4 in this form certifies a bracket around ||pinv(A) b||,
where on (A, b) itself an inconsistent system ends with a witness."""
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def _rank_deficient(seed, m=14, n=10, r=6):
    g = np.random.default_rng(seed)
    A = g.standard_normal((m, r)) @ g.standard_normal((r, n))
    return A, g.standard_normal(m)


@pytest.mark.parametrize("seed", [0, 1])
def test_rank_deficient_limit_is_pinv(seed):
    """From x = 0 every TA iterate lies in range(A^T A) = range(A^T), so the
    limit is the minimum-norm least-squares solution pinv(A) b."""
    A, b = _rank_deficient(seed)
    x, _, info = oracle.ta(A, b, tol=1e-10, max_iter=500_000, normal_eq=True)
    assert info.stop == "residual"
    xp = np.linalg.pinv(A) @ b
    assert np.linalg.norm(x - xp) <= 1e-7 * np.linalg.norm(xp)
    # the exit diagnostics stay on (A, b): rel_normal is the tested quantity
    assert info.rel_normal <= 1e-10 * (1 + 1e-6)
    assert info.rel_res > 0.1  # inconsistent


def test_full_rank_error_bound():
    """Full column rank: ||x - x_ls|| <= ||A^T b - A^T A x|| / sigma_min(A)^2."""
    g = np.random.default_rng(3)
    A, b = g.standard_normal((14, 10)), g.standard_normal(14)
    x, _, info = oracle.ta(A, b, tol=1e-4, max_iter=500_000, normal_eq=True)
    assert info.stop == "residual"
    xl = np.linalg.lstsq(A, b, rcond=None)[0]
    smin = np.linalg.svd(A, compute_uv=False)[-1]
    bound = np.linalg.norm(A.T @ (b - A @ x)) / smin ** 2
    assert np.linalg.norm(x - xl) <= bound * (1 + 1e-9)
    assert np.linalg.norm(A.T @ (b - A @ x)) <= 1e-4 * np.linalg.norm(A.T @ b) * (1 + 1e-9)


def test_products_count_both_passes():
    """Each operator product is an A pass and an A^T pass; A^T b is one more."""
    A, b = _rank_deficient(2)
    _, _, info = oracle.ta(A, b, tol=1e-3, max_iter=100_000, normal_eq=True)
    assert info.matvecs % 2 == 1 and info.matvecs >= 2 * info.iters + 1


def test_algorithm4_certifies_on_the_normal_equation():
    A, b = _rank_deficient(0)
    xp = np.linalg.pinv(A) @ b
    null = np.linalg.svd(A)[2][6:].T
    xe = xp + null @ np.random.default_rng(9).standard_normal(4)  # LS, not minimum norm
    tol = 1e-3
    x, info, tests = oracle.ta_minnorm(A, b, xe, tol=tol, max_iter=500_000, normal_eq=True)
    assert info.stop == "residual" and tests > 1
    nx = np.linalg.norm(xp)
    assert info.rho_lo <= nx * (1 + 1e-12)            # Corollary 1: a certified lower bound
    assert nx <= info.rho + tol * np.linalg.norm(xe)  # within the gap of the upper bound
    assert info.rho - info.rho_lo <= tol * np.linalg.norm(xe)
    # the same input on (A, b): inconsistent, so the bounds cross (witness stop)
    _, info2, _ = oracle.ta_minnorm(A, b, xe, tol=tol, max_iter=500_000)
    assert info2.stop == "witness"


def test_consistent_system_same_limit():
    """For a consistent system both forms converge to solutions of A x = b."""
    A, _ = _rank_deficient(4)
    b = A @ np.random.default_rng(5).standard_normal(10)
    x, _, info = oracle.ta(A, b, tol=1e-8, max_iter=500_000, normal_eq=True)
    assert info.stop == "residual"
    assert np.linalg.norm(A @ x - b) <= 1e-6 * np.linalg.norm(b)
