"""Pins of the oracle's CTA with H = A (the specialisation to a symmetric
positive semidefinite A): one CTA-t iteration minimises ||r - sum_i alpha_i
A^i r|| over the Krylov space, i.e. it is one restart cycle of GMRES(t) on
A x = b itself (scipy), finite termination at the number of distinct
eigenvalues, and the closed-form step of Example 1 for t = 1."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from workloads import poisson5


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def _spd(n, seed, cond=50.0):
    g = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    lam = np.geomspace(1.0, cond, n)
    return (Q * lam) @ Q.T


@pytest.mark.parametrize("t", [1, 2, 3])
def test_h_a_equals_restarted_gmres(t):
    A = _spd(30, 20 + t)
    b = np.random.default_rng(t).standard_normal(30)
    K = 10
    x, hist, info = oracle.cta(A, b, tol=0.0, t=t, max_iter=K, h_is_a=True)
    assert info.matvecs == t * K  # t products per iteration
    xg = np.zeros(30)
    nb = np.linalg.norm(b)
    ref = [1.0]
    for _ in range(K):
        xg, _ = spla.gmres(A, b, x0=xg, restart=t, maxiter=1, rtol=0.0, atol=0.0)
        ref.append(np.linalg.norm(b - A @ xg) / nb)
    np.testing.assert_allclose(hist, ref, rtol=1e-8)
    np.testing.assert_allclose(x, xg, rtol=1e-7, atol=1e-10 * np.linalg.norm(x))


def test_h_a_t1_closed_form():
    """Example 1 with H = A: alpha = r^T A r / ||A r||^2, x1 = alpha b."""
    A = _spd(12, 3)
    b = np.random.default_rng(4).standard_normal(12)
    x, hist, info = oracle.cta(A, b, tol=0.0, t=1, max_iter=1, h_is_a=True)
    Ab = A @ b
    alpha = (b @ Ab) / (Ab @ Ab)
    np.testing.assert_allclose(x, alpha * b, rtol=1e-13)
    assert hist[1] == pytest.approx(np.linalg.norm(b - alpha * Ab) / np.linalg.norm(b), rel=1e-12)


def test_h_a_finite_termination():
    """A with 3 distinct eigenvalues: CTA-3 with H = A solves in one step."""
    g = np.random.default_rng(6)
    Q, _ = np.linalg.qr(g.standard_normal((20, 20)))
    lam = np.repeat([1.0, 4.0, 9.0], [7, 7, 6])
    A = (Q * lam) @ Q.T
    b = g.standard_normal(20)
    x, hist, info = oracle.cta(A, b, tol=0.0, t=3, max_iter=1, h_is_a=True)
    # exact in one step up to the rounding of the 3 x 3 Hankel solve; two
    # steps of CTA-2 on the same A leave a residual many orders larger
    assert hist[1] <= 1e-9
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-8)
    _, h2, _ = oracle.cta(A, b, tol=0.0, t=2, max_iter=1, h_is_a=True)
    assert h2[1] > 1e-4


def test_h_a_converges_faster_on_poisson():
    """On the Poisson matrix (SPD) H = A works with cond(A) instead of
    cond(A)^2: far fewer products to the same true residual."""
    A = poisson5(16)
    b = np.random.default_rng(7).uniform(-1, 1, A.m)
    _, _, ia = oracle.cta(A, b, tol=1e-8, t=3, max_iter=200000, h_is_a=True)
    _, _, ih = oracle.cta(A, b, tol=1e-8, t=3, max_iter=200000)
    assert ia.stop == ih.stop == "residual"
    assert ia.matvecs * 5 < ih.matvecs
