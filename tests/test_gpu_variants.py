"""CTA with H = A (symmetric positive semidefinite A) through the C ABI,
against the FP64 oracle: equal stop codes, iteration and product counts,
histories within 1e-10 and x within 1e-10 relative."""
import numpy as np
import pytest

import oracle
import paper_2304_12168_amd as P
from workloads import csr_from_dense, poisson5

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load_library()
    oracle.build(force=False)


def _spd(n, seed, cond=50.0):
    g = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    return (Q * np.geomspace(1.0, cond, n)) @ Q.T


CASES = {
    "poisson_16": lambda: (poisson5(16), 1e-8, 3),
    "poisson_40": lambda: (poisson5(40), 1e-6, 2),
    "spd_dense_30": lambda: (_spd(30, 1), 1e-10, 3),
    "spd_csr_30": lambda: (csr_from_dense(_spd(30, 2)), 1e-10, 1),
}


@pytest.mark.parametrize("case", list(CASES))
def test_h_a_matches_oracle(case):
    A, tol, t = CASES[case]()
    m = A.shape[0] if isinstance(A, np.ndarray) else A.m
    b = np.random.default_rng(3).uniform(-1, 1, m)
    xg, hg, ig = P.cta_solve(A, b, tol=tol, t=t, max_iter=200000, h_is_a=True)
    xo, ho, io = oracle.cta(A, b, tol=tol, t=t, max_iter=200000, h_is_a=True)
    assert (ig.stop, ig.iters, ig.matvecs) == (io.stop, io.iters, io.matvecs)
    np.testing.assert_allclose(hg.cpu().numpy(), ho, rtol=1e-10, atol=1e-300)
    assert np.linalg.norm(xg.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)


def test_h_a_rejects_rectangular_and_minnorm():
    A = np.random.default_rng(0).standard_normal((4, 5))
    with pytest.raises(P.TaError):
        P.cta_solve(A, np.ones(4), h_is_a=True)
    S = _spd(5, 0)
    with pytest.raises(P.TaError):
        P.cta_minnorm(S, np.ones(5), h_is_a=True)


@pytest.mark.slow
def test_h_a_poisson_512_first_iterations():
    """Full-size Poisson 512^2 (the stencil of the convection-diffusion case
    without convection): 100 iterations of CTA-3 with H = A match the
    oracle, and with half the products reach a smaller residual than 100
    iterations with H = A A^T."""
    A = poisson5(512)
    b = np.random.default_rng(5).uniform(0, 1, A.m)
    xg, hg, ig = P.cta_solve(A, b, tol=1e-12, t=3, max_iter=100, h_is_a=True)
    xo, ho, io = oracle.cta(A, b, tol=1e-12, t=3, max_iter=100, h_is_a=True)
    assert (ig.stop, ig.iters, ig.matvecs) == (io.stop, io.iters, io.matvecs)
    np.testing.assert_allclose(hg.cpu().numpy(), ho, rtol=1e-10)
    assert np.linalg.norm(xg.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    _, h2, i2 = P.cta_solve(A, b, tol=1e-12, t=3, max_iter=100)
    assert ig.matvecs * 2 == i2.matvecs
    assert float(hg[-1]) < float(h2[-1])


CYCLE_CASES = {
    "kac_101_t5": lambda: __import__("workloads").kac_clement(101),
    "convdiff_8_t3": lambda: __import__("workloads").convection_diffusion(8),
    "lp_200x5000_t4": lambda: __import__("workloads").lp_shaped(200, 5000, seed=3),
}


@pytest.mark.parametrize("case", list(CYCLE_CASES))
@pytest.mark.parametrize("minnorm", [False, True], ids=["x_form", "y_form"])
def test_order_cycling_matches_oracle(case, minnorm):
    p = CYCLE_CASES[case]()
    t = int(case.rsplit("_t", 1)[1])
    run_g = P.cta_minnorm if minnorm else P.cta_solve
    xg, hg, ig = run_g(p.A, p.b, tol=1e-8, t=t, max_iter=100000, t_cycle=True)
    xo, ho, io = oracle.cta(p.A, p.b, tol=1e-8, t=t, max_iter=100000, t_cycle=True,
                            minnorm=minnorm)
    assert (ig.stop, ig.iters, ig.matvecs) == (io.stop, io.iters, io.matvecs)
    np.testing.assert_allclose(hg.cpu().numpy(), ho, rtol=1e-10, atol=1e-300)
    assert np.linalg.norm(xg.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)


def test_cycling_and_h_a_together():
    A = poisson5(20)
    b = np.random.default_rng(4).uniform(-1, 1, A.m)
    xg, hg, ig = P.cta_solve(A, b, tol=1e-9, t=4, max_iter=100000, t_cycle=True, h_is_a=True)
    xo, ho, io = oracle.cta(A, b, tol=1e-9, t=4, max_iter=100000, t_cycle=True, h_is_a=True)
    assert (ig.stop, ig.iters, ig.matvecs) == (io.stop, io.iters, io.matvecs)
    assert np.linalg.norm(xg.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)


def test_batched_rejects_bad_variant_options():
    """Batches take every CTA variant (tested in test_gpu_batched.py and
    test_gpu_enhanced.py); theta must lie in [0, 1) and the flags be 0 or 1."""
    plan = P.BatchPlan([poisson5(4)], "fp64")
    for kw in (dict(accel=1.0), dict(accel=-0.5)):
        with pytest.raises(P.TaError, match="EINVAL"):
            P.cta_solve_batched(plan, [np.ones((16, 1))], **kw)
    plan.close()
