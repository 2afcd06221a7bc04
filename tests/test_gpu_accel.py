"""The convex-combination step (the first-order dynamics theorem of section
3) through the C ABI, against the FP64 oracle: equal stop codes, iteration
and product counts, histories within 1e-10, x within 1e-9 relative; on a
critical line both solve the system after one step and one combination."""
import numpy as np
import pytest

import oracle
import paper_2304_12168_amd as P
from workloads import csr_from_dense, kac_clement, poisson5

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load_library()
    oracle.build(force=False)


def host(v):
    return v.detach().cpu().numpy()


def _compare(g, o, x_rtol=1e-9):
    x, hist, info = g
    xo, ho, io = o
    assert (info.stop, info.iters, info.matvecs) == (io.stop, io.iters, io.matvecs), (info, io)
    np.testing.assert_allclose(host(hist), ho, rtol=1e-10, atol=0)
    assert np.linalg.norm(host(x) - xo) <= x_rtol * np.linalg.norm(xo)


def _critical(lam_i=1.0, lam_j=9.0, n=6, seed=0):
    g = np.random.default_rng(seed)
    U, _ = np.linalg.qr(g.standard_normal((n, n)))
    h = n // 2
    s = np.concatenate([np.full(h, np.sqrt(lam_i)), np.full(n - h, np.sqrt(lam_j))])
    A = (U * s) @ U.T
    cu, cv = g.standard_normal(h), g.standard_normal(n - h)
    b = (np.sqrt(lam_j) * U[:, :h] @ (cu / np.linalg.norm(cu))
         + np.sqrt(lam_i) * U[:, h:] @ (cv / np.linalg.norm(cv)))
    return A, b


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_critical_line(kind):
    A, b = _critical()
    M = csr_from_dense(A) if kind == "csr" else A
    g = P.cta_solve(M, b, tol=1e-12, t=1, max_iter=1000, accel=0.5)
    o = oracle.cta(M, b, tol=1e-12, t=1, max_iter=1000, accel=0.5)
    assert o[2].iters == 2
    _compare(g, o, x_rtol=1e-12)


CASES = {
    "kac101_t1": (lambda: kac_clement(101), 1, 1e-8),
    "kac101_t3": (lambda: kac_clement(101), 3, 1e-8),
    "poisson16_t2": (lambda: poisson5(16), 2, 1e-6),
    "poisson16_t3": (lambda: poisson5(16), 3, 1e-6),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("form", ["x", "y"])
def test_matches_oracle(case, form):
    make, t, tol = CASES[case]
    p = make()
    A = p.A if hasattr(p, "A") else p
    b = p.b if hasattr(p, "b") else np.random.default_rng(1).uniform(-1, 1, A.m)
    kw = dict(tol=tol, t=t, max_iter=20_000, accel=0.5)
    if form == "x":
        _compare(P.cta_solve(A, b, **kw), oracle.cta(A, b, **kw))
    else:
        _compare(P.cta_minnorm(A, b, **kw), oracle.cta_minnorm(A, b, **kw))


def test_h_a_matches_oracle():
    A = poisson5(16)
    b = np.random.default_rng(2).uniform(-1, 1, A.m)
    kw = dict(tol=1e-8, t=3, max_iter=20_000, accel=0.5, h_is_a=True)
    _compare(P.cta_solve(A, b, **kw), oracle.cta(A, b, **kw))


def test_with_replacement_matches_oracle():
    p = kac_clement(101)
    kw = dict(tol=1e-8, t=2, max_iter=20_000, accel=0.5, replace_every=7)
    _compare(P.cta_solve(p.A, p.b, **kw), oracle.cta(p.A, p.b, **kw))


def test_no_trigger_is_plain():
    g = np.random.default_rng(4)
    A = np.eye(30) * 4.0 + 0.3 * g.standard_normal((30, 30))
    b = g.standard_normal(30)
    kw = dict(tol=1e-10, t=2, max_iter=200)
    x0, h0, i0 = P.cta_solve(A, b, **kw)
    x1, h1, i1 = P.cta_solve(A, b, accel=0.95, **kw)
    assert i0 == i1 and torch.equal(x0, x1) and torch.equal(h0, h1)


def test_accel_rejected_outside_cta():
    A, b = _critical()
    with pytest.raises(P.TaError, match="EINVAL"):
        P.ta_solve(A, b, accel=0.5)
    with pytest.raises(P.TaError, match="EINVAL"):
        P.cta_solve(A, b, accel=1.5)


def test_accel_in_the_batched_engine_with_order_cycling():
    """The batched engine takes the step per column (its own tests are in
    test_gpu_batched.py); here together with order cycling, against the
    oracle."""
    p = kac_clement(101)
    plan = P.BatchPlan([p.A], "fp64")
    kw = dict(tol=1e-8, t=3, max_iter=20_000, accel=0.5, t_cycle=True)
    X, infos = P.cta_solve_batched(plan, [np.asarray(p.b)], **kw)
    plan.close()
    xo, _, io = oracle.cta(p.A, p.b, **kw)
    ig = infos[0][0]
    assert (ig.stop, ig.iters, ig.matvecs) == (io.stop, io.iters, io.matvecs)
    assert np.linalg.norm(X[0][:, 0].cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("t", [3, 5])
def test_with_order_cycling_matches_oracle(t):
    p = kac_clement(101)
    kw = dict(tol=1e-8, t=t, max_iter=20_000, accel=0.5, t_cycle=True)
    _compare(P.cta_solve(p.A, p.b, **kw), oracle.cta(p.A, p.b, **kw))


@pytest.mark.parametrize("t,theta", [(2, 0.5), (3, 0.8)])
def test_with_enhanced_stop(t, theta):
    """Inconsistent Kac-Clement N = 1001: both sides stop NORMAL; the
    enhanced test's moment sums may decide one iteration apart (as without
    the step), so the counts agree within one and the true normal-equation
    residual meets the tolerance."""
    A = kac_clement(1001).A
    b = np.random.default_rng(11).standard_normal(1001)
    kw = dict(tol=1e-10, t=t, max_iter=200_000, tol_normal=1e-6, enhanced=True, accel=theta)
    _, _, ig = P.cta_solve(A, b, **kw)
    _, _, io = oracle.cta(A, b, **kw)
    assert ig.stop == io.stop == "normal"
    assert abs(ig.iters - io.iters) <= 1, (ig, io)
    assert ig.rel_normal <= 1e-6 * (1 + 1e-6)
