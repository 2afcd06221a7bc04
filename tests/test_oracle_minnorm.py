"""Pins of the oracle's Algorithm 4 (TA for an approximate minimum-norm
solution, section 4.4) and of TA's warm start: a case worked by hand, and on
random systems the facts the paper and linear algebra fix -- Corollary 1's
lower bound, the residual and gap conditions of Definition 1, the bisection
count of the theorem after Algorithm 4, and a distance bound to pinv(A) b."""
import math

import numpy as np
import pytest

import oracle


def test_hand_case_1x2():
    """x1 + x2 = 2 from x_eps = (2, 0), tol 0.01 (gap <= 0.02).  Test 1
    (rho = 1): c = (2, 2), rho ||c|| = 2 sqrt 2 < r^T b = 4, a witness at
    once with lower bound 4 / (2 sqrt 2) = sqrt 2 = ||x_dagger||.  Every later
    test (rho between sqrt 2 and the upper bound) succeeds in one step with
    x' = (1, 1), so the gap 2 - sqrt 2 halves until <= 0.02: 5 more tests."""
    A = np.array([[1.0, 1.0]])
    x, info, tests = oracle.ta_minnorm(A, np.array([2.0]), np.array([2.0, 0.0]), tol=0.01,
                                      max_iter=1000)
    assert info.stop == "residual"
    assert tests == 6 and info.iters == 5
    assert info.rho_lo == pytest.approx(math.sqrt(2), rel=1e-15)
    assert info.rho == pytest.approx(math.sqrt(2) + (2 - math.sqrt(2)) / 32, rel=1e-14)
    assert np.allclose(x, [1.0, 1.0], rtol=0, atol=1e-14)


def test_ta_warm_start_counts_one_product():
    """TA from x0: b' = A x0 first (one product more than from 0); from the
    exact solution it stops at once."""
    g = np.random.default_rng(1)
    A = g.standard_normal((5, 9))
    xs = g.standard_normal(9)
    b = A @ xs
    x, _, info = oracle.ta(A, b, tol=1e-10, max_iter=10, x0=xs)
    assert info.stop == "residual" and info.iters == 0
    assert np.array_equal(x, xs)
    _, _, i0 = oracle.ta(A, b, tol=1e-3, max_iter=100000)
    _, _, i1 = oracle.ta(A, b, tol=1e-3, max_iter=100000, x0=np.zeros(9))
    assert i1.iters == i0.iters and i1.matvecs == i0.matvecs + 1


@pytest.mark.parametrize("shape,seed,tol", [((8, 20), 0, 1e-4), ((15, 40), 1, 1e-5),
                                           ((30, 31), 2, 1e-4)])
def test_random_consistent_systems(shape, seed, tol):
    g = np.random.default_rng(seed)
    m, n = shape
    A = g.standard_normal((m, n))
    b = A @ g.standard_normal(n)
    # an approximate solution that is not the minimum-norm one (x-form from a random x0)
    xe, _, ie = oracle.cta(A, b, tol=tol, t=3, max_iter=200000, x0=g.standard_normal(n))
    assert ie.stop == "residual"
    x, info, tests = oracle.ta_minnorm(A, b, xe, tol=tol, max_iter=5_000_000)
    assert info.stop == "residual"
    Ap = np.linalg.pinv(A)
    xd = Ap @ b
    nd, ne = np.linalg.norm(xd), np.linalg.norm(xe)
    hi, lo = info.rho, info.rho_lo
    # Corollary 1: a witness's bound never exceeds the minimum norm
    assert lo <= nd * (1 + 1e-12)
    # Definition 1: residual within tol, the norm within the final ball, gap closed
    res = np.linalg.norm(A @ x - b)
    assert res <= tol * np.linalg.norm(b) * (1 + 1e-9)
    assert np.linalg.norm(x) <= hi * (1 + 1e-12) and hi <= ne * (1 + 1e-15)
    assert hi - lo <= tol * ne
    # the theorem after Algorithm 4: at most k tests, ||x_eps|| / 2^k <= gap
    assert tests <= math.ceil(math.log2(ne / (tol * ne))) + 1
    # distance to pinv(A) b: x - x_dagger = z + e, e = A^+ (A x - b), z in null(A);
    # ||z||^2 = ||x||^2 - ||x_dagger + e||^2 <= hi^2 - (lo - ||e||)^2
    e = np.linalg.norm(Ap, 2) * res
    z = math.sqrt(max(hi * hi - max(lo - e, 0.0) ** 2, 0.0))
    assert np.linalg.norm(x - xd) <= (z + e) * (1 + 1e-9) + 1e-13


def test_inconsistent_system_crossed_bounds():
    """Corollary 1 is stated for the minimum-norm least-squares solution, but
    its proof needs A x* = b: on an inconsistent system a witness's bound
    (b - b')^T b / ||c|| can exceed ||x_ls||.  Here it does, the lower bound
    passes the upper one, and Algorithm 4 reports a witness (the input was
    not an approximate solution of a consistent system) and returns x_eps."""
    g = np.random.default_rng(3)
    A = g.standard_normal((12, 6))
    b = g.standard_normal(12)
    xl = np.linalg.lstsq(A, b, rcond=None)[0]
    xe = 1.5 * xl
    x, info, tests = oracle.ta_minnorm(A, b, xe, tol=1e-3, max_iter=2_000_000)
    assert info.rho_lo > np.linalg.norm(xl) * 1.5
    assert info.stop == "witness"
    assert np.array_equal(x, xe)
