"""TA for LP feasibility (c+ in place of c, optional radius bound) through
the C ABI, against the FP64 oracle: equal stop codes, iteration and product
counts, radius bounds within 1e-12 and x within 1e-9 relative."""
import numpy as np
import pytest

import oracle
import paper_2304_12168_amd as P
from workloads import csr_from_dense, lp_shaped

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load_library()
    oracle.build(force=False)


def _cmp(A, b, **kw):
    xg, hg, ig = P.ta_solve(A, b, nonneg=True, **kw)
    xo, ho, io = oracle.ta(A, b, nonneg=True, **kw)
    assert (ig.stop, ig.iters, ig.matvecs) == (io.stop, io.iters, io.matvecs), (ig, io)
    assert ig.rho == pytest.approx(io.rho, rel=1e-12, abs=1e-300)
    assert ig.rho_lo == pytest.approx(io.rho_lo, rel=1e-12, abs=1e-300)
    x = xg.cpu().numpy()
    assert np.linalg.norm(x - xo) <= 1e-9 * max(np.linalg.norm(xo), 1e-300)
    assert x.min() >= 0.0
    return ig


def test_farkas_by_hand():
    ig = _cmp(np.array([[1.0, 1.0]]), np.array([-1.0]), tol=1e-8, max_iter=10)
    assert ig.stop == "normal" and ig.iters == 0


@pytest.mark.parametrize("dense", [True, False], ids=["dense", "csr"])
@pytest.mark.parametrize("seed", [0, 1])
def test_feasible(seed, dense):
    g = np.random.default_rng(seed)
    a = g.standard_normal((20, 60))
    b = a @ np.abs(g.standard_normal(60))
    ig = _cmp(a if dense else csr_from_dense(a), b, tol=1e-6, max_iter=2_000_000)
    assert ig.stop == "residual"


@pytest.mark.parametrize("dense", [True, False], ids=["dense", "csr"])
@pytest.mark.parametrize("seed", [3, 4])
def test_infeasible(seed, dense):
    g = np.random.default_rng(seed)
    a = g.standard_normal((20, 15))
    b = g.standard_normal(20)
    ig = _cmp(a if dense else csr_from_dense(a), b, tol=1e-6, max_iter=2_000_000,
              tol_normal=1e-8)
    assert ig.stop == "normal"


def test_radius_bound():
    g = np.random.default_rng(6)
    A = g.standard_normal((10, 30))
    b = A @ np.abs(g.standard_normal(30))
    ig = _cmp(A, b, tol=1e-6, max_iter=2_000_000, rho_max=1e-3)
    assert ig.stop == "witness"


def test_lp_shaped_feasible():
    """LP-shaped sparse system (300 x 6000) with a nonnegative x*."""
    prob = lp_shaped(300, 6000, seed=4)
    b = prob.A.matvec(np.abs(np.random.default_rng(4).standard_normal(6000)))
    ig = _cmp(prob.A, b, tol=1e-5, max_iter=2_000_000)
    assert ig.stop == "residual"


def test_options_rejected_elsewhere():
    A = np.eye(3)
    with pytest.raises(P.TaError):
        P.cta_solve(A, np.ones(3), nonneg=True)
    with pytest.raises(P.TaError):
        P.ta_minnorm(A, np.ones(3), np.ones(3), nonneg=True)
