"""Pins of the oracle's TA for LP feasibility {A x = b, x >= 0} (section 6:
c replaced by c+ = max(c, 0)): a Farkas case by hand, feasibility decided
like scipy's linprog on random instances, the infeasibility certificate at a
NORMAL stop (A^T r <= 0 up to the tolerance, r^T b > 0), and the radius
bound."""
import numpy as np
import pytest
from scipy.optimize import linprog

import oracle


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def test_farkas_by_hand():
    """x1 + x2 = -1 with x >= 0: at b' = 0, r = -1, c = A^T r = (-1, -1),
    c+ = 0: stop at once, r^T b = 1 > 0 certifies infeasibility."""
    A = np.array([[1.0, 1.0]])
    x, _, info = oracle.ta(A, np.array([-1.0]), tol=1e-8, max_iter=10, nonneg=True)
    assert info.stop == "normal" and info.iters == 0 and not x.any()


def _lp_feasible(A, b):
    res = linprog(np.zeros(A.shape[1]), A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    return res.status == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_feasible_instances(seed):
    g = np.random.default_rng(seed)
    A = g.standard_normal((20, 60))
    b = A @ np.abs(g.standard_normal(60))
    assert _lp_feasible(A, b)
    x, _, info = oracle.ta(A, b, tol=1e-6, max_iter=2_000_000, nonneg=True)
    assert info.stop == "residual"
    assert x.min() >= 0.0
    assert np.linalg.norm(A @ x - b) <= 1e-6 * np.linalg.norm(b) * (1 + 1e-9)


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_infeasible_instances_certified(seed):
    g = np.random.default_rng(seed)
    A = g.standard_normal((20, 15))
    b = g.standard_normal(20)
    assert not _lp_feasible(A, b)
    tn = 1e-8
    x, _, info = oracle.ta(A, b, tol=1e-6, max_iter=2_000_000, nonneg=True, tol_normal=tn)
    assert info.stop == "normal" and x.min() >= 0.0
    r = b - A @ x
    c = A.T @ r
    cb = np.maximum(A.T @ b, 0.0)
    # Farkas: y = r has A^T y <= 0 (to the stopping tolerance) and y^T b > 0
    assert np.linalg.norm(np.maximum(c, 0.0)) <= 1.01 * tn * np.linalg.norm(cb) + 1e-12
    assert r @ b > 0.0


def test_radius_bound():
    g = np.random.default_rng(6)
    A = g.standard_normal((10, 30))
    xs = np.abs(g.standard_normal(30))
    b = A @ xs
    _, _, ok = oracle.ta(A, b, tol=1e-6, max_iter=2_000_000, nonneg=True)
    assert ok.stop == "residual"
    # any x >= 0 with A x = b has norm >= the witness bound: a tiny bound stops early
    _, _, info = oracle.ta(A, b, tol=1e-6, max_iter=2_000_000, nonneg=True, rho_max=1e-3)
    assert info.stop == "witness" and info.rho <= 1e-3 and info.rho_lo > 1e-3
