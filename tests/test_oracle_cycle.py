"""Pins of the oracle's CTA order cycling (section 5.1 cycles the order
1, ..., 5 and back; read as the triangle wave 1, 2, ..., t, ..., 2, 1, 2, ...):
the product count of a hand-counted schedule, and per iteration the
equivalence with one GMRES(t_k) restart cycle of the matching length."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def test_schedule_product_count():
    g = np.random.default_rng(0)
    A = g.standard_normal((20, 30))
    b = g.standard_normal(20)
    _, _, info = oracle.cta(A, b, tol=0.0, t=5, max_iter=8, t_cycle=True)
    # orders 1, 2, 3, 4, 5, 4, 3, 2: two products each
    assert info.matvecs == 2 * (1 + 2 + 3 + 4 + 5 + 4 + 3 + 2)
    _, _, info = oracle.cta(A, b, tol=0.0, t=5, max_iter=10, t_cycle=True)
    assert info.matvecs == 2 * (24 + 1 + 2)
    _, _, info = oracle.cta(A, b, tol=0.0, t=1, max_iter=7, t_cycle=True)
    assert info.matvecs == 14


@pytest.mark.parametrize("t", [2, 3, 5])
def test_cycle_equals_gmres_cycles(t):
    g = np.random.default_rng(30 + t)
    m, n = 25, 35
    A = g.standard_normal((m, n))
    b = g.standard_normal(m)
    H = A @ A.T
    K = 11
    x, hist, info = oracle.cta(A, b, tol=0.0, t=t, max_iter=K, t_cycle=True)
    orders = [min(p + 1, 2 * t - 1 - p) for p in (k % (2 * t - 2) for k in range(K))]
    y = np.zeros(m)
    ref = [1.0]
    for tk in orders:
        y, _ = spla.gmres(H, b, x0=y, restart=tk, maxiter=1, rtol=0.0, atol=0.0)
        ref.append(np.linalg.norm(b - H @ y) / np.linalg.norm(b))
    np.testing.assert_allclose(hist, ref, rtol=1e-8)
    np.testing.assert_allclose(x, A.T @ y, rtol=1e-6, atol=1e-9 * np.linalg.norm(x))
