"""TA's warm start and Algorithm 4 (approximate minimum-norm solution by
bisection on the radius) through the C ABI, against the FP64 oracle: equal
stop codes, test counts, iteration and product counts; bounds within 1e-12
and x within 1e-9 relative."""
import math

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


def host(t):
    return t.detach().cpu().numpy()


def _same(ig, io, xg, xo, tg=None, to=None):
    assert (ig.stop, ig.iters, ig.matvecs) == (io.stop, io.iters, io.matvecs), (ig, io)
    assert tg == to
    assert ig.rho == pytest.approx(io.rho, rel=1e-12, abs=1e-300)
    assert ig.rho_lo == pytest.approx(io.rho_lo, rel=1e-12, abs=1e-300)
    assert np.linalg.norm(xg - xo) <= 1e-9 * max(np.linalg.norm(xo), 1e-300)


@pytest.mark.parametrize("dense", [True, False], ids=["dense", "csr"])
def test_ta_warm_start_matches_oracle(dense):
    g = np.random.default_rng(5)
    a = g.standard_normal((9, 14))
    A = a if dense else csr_from_dense(a)
    b = a @ g.standard_normal(14)
    x0 = 0.3 * g.standard_normal(14)
    xg, _, ig = P.ta_solve(A, b, tol=1e-6, max_iter=200000, x0=x0)
    xo, _, io = oracle.ta(A, b, tol=1e-6, max_iter=200000, x0=x0)
    _same(ig, io, host(xg), xo)


def test_hand_case_1x2():
    A = np.array([[1.0, 1.0]])
    x, info, tests = P.ta_minnorm(A, np.array([2.0]), np.array([2.0, 0.0]), tol=0.01,
                                  max_iter=1000)
    xo, io, to = oracle.ta_minnorm(A, np.array([2.0]), np.array([2.0, 0.0]), tol=0.01,
                                   max_iter=1000)
    assert tests == 6 and info.stop == "residual"
    _same(info, io, host(x), xo, tests, to)
    assert info.rho_lo == pytest.approx(math.sqrt(2), rel=1e-15)


@pytest.mark.parametrize("shape,seed,tol", [((8, 20), 0, 1e-4), ((15, 40), 1, 1e-5),
                                           ((30, 31), 2, 1e-4)])
@pytest.mark.parametrize("dense", [True, False], ids=["dense", "csr"])
def test_random_systems_match_oracle(shape, seed, tol, dense):
    g = np.random.default_rng(seed)
    m, n = shape
    a = g.standard_normal((m, n))
    b = a @ g.standard_normal(n)
    xe, _, _ = oracle.cta(a, b, tol=tol, t=3, max_iter=200000, x0=g.standard_normal(n))
    A = a if dense else csr_from_dense(a)
    x, info, tests = P.ta_minnorm(A, b, xe, tol=tol, max_iter=5_000_000)
    xo, io, to = oracle.ta_minnorm(A, b, xe, tol=tol, max_iter=5_000_000)
    assert io.stop == "residual"
    _same(info, io, host(x), xo, tests, to)


def test_inconsistent_reports_witness():
    g = np.random.default_rng(3)
    A = g.standard_normal((12, 6))
    b = g.standard_normal(12)
    xe = 1.5 * np.linalg.lstsq(A, b, rcond=None)[0]
    x, info, tests = P.ta_minnorm(A, b, xe, tol=1e-3, max_iter=2_000_000)
    xo, io, to = oracle.ta_minnorm(A, b, xe, tol=1e-3, max_iter=2_000_000)
    assert info.stop == "witness"
    _same(info, io, host(x), xo, tests, to)


def test_budget_and_zero_rhs():
    g = np.random.default_rng(9)
    A = g.standard_normal((6, 15))
    b = A @ g.standard_normal(15)
    xe, _, _ = oracle.cta(A, b, tol=1e-6, t=3, max_iter=100000, x0=g.standard_normal(15))
    x, info, tests = P.ta_minnorm(A, b, xe, tol=1e-6, max_iter=50)
    xo, io, to = oracle.ta_minnorm(A, b, xe, tol=1e-6, max_iter=50)
    assert info.stop == "maxiter"
    _same(info, io, host(x), xo, tests, to)
    x, info, tests = P.ta_minnorm(A, np.zeros(6), xe, tol=1e-6, max_iter=50)
    assert info.stop == "residual" and tests == 0 and not host(x).any()


def test_lp_shaped_plan_and_one_shot():
    """Sparse rectangular (LP-shaped, 200 x 5000): plan and one-shot agree
    with each other bit for bit and with the oracle."""
    prob = lp_shaped(200, 5000, seed=1)
    g = np.random.default_rng(2)
    xe, _, _ = oracle.cta(prob.A, prob.b, tol=1e-4, t=3, max_iter=100000,
                          x0=0.05 * g.standard_normal(5000))
    x1, i1, t1 = P.ta_minnorm(prob.A, prob.b, xe, tol=1e-4, max_iter=2_000_000)
    pl = P.plan(prob.A)
    x2, i2, t2 = P.ta_minnorm(pl, prob.b, xe, tol=1e-4, max_iter=2_000_000)
    assert np.array_equal(host(x1), host(x2)) and (i1, t1) == (i2, t2)
    xo, io, to = oracle.ta_minnorm(prob.A, prob.b, xe, tol=1e-4, max_iter=2_000_000)
    _same(i1, io, host(x1), xo, t1, to)


@pytest.mark.parametrize("N,tol", [(101, 1e-6), (301, 1e-6), (301, 1e-4)])
def test_halving_restarts_match_oracle(N, tol):
    """TA restarted with eps' halved after each stop on the normal equation
    (the remark after the theorem on Algorithm 3, section 4.3): equal stops,
    restart counts, summed iteration and product counts; x within 1e-9."""
    from workloads import kac_clement

    p = kac_clement(N)
    pl = P.plan(p.A)
    x, ig, hg = P.ta_solve_halving(pl, p.b, tol=tol, max_iter=200_000)
    xo, io, ho = oracle.ta_halving(p.A, p.b, tol=tol, max_iter=200_000)
    assert (ig.stop, ig.iters, ig.matvecs, hg) == (io.stop, io.iters, io.matvecs, ho), (ig, io)
    assert ig.stop == "residual" and hg >= 1
    assert np.linalg.norm(host(x) - xo) <= 1e-9 * np.linalg.norm(xo)
    with pytest.raises(P.TaError, match="EINVAL"):
        P.ta_solve_halving(pl, p.b, tol=tol, max_halvings=-1)
    with pytest.raises(P.TaError, match="EINVAL"):
        P.ta_solve_halving(pl, p.b, tol=tol, normal_eq=True)
    pl.close()
