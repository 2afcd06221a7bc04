"""TA and Algorithm 4 on the normal equation A^T A x = A^T b (the rectangular
hybrid's inputs for an unsolvable system) through the C ABI, against the FP64
oracle: equal stop codes, iteration and product counts, histories within
1e-10, x within 1e-9 relative; Algorithm 4's tests and bracket equal.

The first device implementation never finished on the dense rank-deficient
case: the dense transposed product ignored the residual form of its epilogue
(it returned A^T t instead of A^T b - A^T t), so every candidate stop was
rejected and the chain advanced one iteration per host poll.  The dense
kernel now forms the residual like the other product kernels (the dense
cases below reach the oracle's RESIDUAL stop with its exact counts only if
the true residual is right), and after a first rejection the chains check
candidates after every iteration."""
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


def host(v):
    return v.detach().cpu().numpy() if hasattr(v, "detach") else np.asarray(v)


def _rank_deficient(seed, m=14, n=10, r=6):
    g = np.random.default_rng(seed)
    return g.standard_normal((m, r)) @ g.standard_normal((r, n)), g.standard_normal(m)


def _full_tall(seed):
    g = np.random.default_rng(seed)
    return g.standard_normal((14, 10)), g.standard_normal(14)


def _compare(g, o):
    x, hist, info = g
    xo, ho, io = o
    assert (info.stop, info.iters, info.matvecs) == (io.stop, io.iters, io.matvecs), (info, io)
    np.testing.assert_allclose(host(hist), ho, rtol=1e-10, atol=0)
    assert np.linalg.norm(host(x) - xo) <= 1e-9 * np.linalg.norm(xo)
    assert info.rel_res == pytest.approx(io.rel_res, rel=1e-8)
    assert info.rel_normal == pytest.approx(io.rel_normal, rel=1e-6, abs=1e-18)


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("case,tol", [("rank_deficient", 1e-6), ("full_tall", 1e-3)])
def test_ta_normal_eq_matches_oracle(kind, case, tol):
    A, b = (_rank_deficient if case == "rank_deficient" else _full_tall)(1)
    M = csr_from_dense(A) if kind == "csr" else A
    _compare(P.ta_solve(M, b, tol=tol, max_iter=200_000, normal_eq=True),
             oracle.ta(M, b, tol=tol, max_iter=200_000, normal_eq=True))


def test_ta_normal_eq_tall_sparse():
    """The transpose of an LP-shaped matrix (5000 x 200, sparse, full column
    rank) with a random, inconsistent right-hand side."""
    At = lp_shaped(200, 5000, seed=2).A.to_scipy().T.tocsr()
    from workloads.gen import Csr
    A = Csr(At.shape[0], At.shape[1], At.indptr.astype(np.int32),
            At.indices.astype(np.int32), At.data.astype(np.float64))
    b = np.random.default_rng(4).standard_normal(A.m)
    _compare(P.ta_solve(A, b, tol=1e-3, max_iter=100_000, normal_eq=True),
             oracle.ta(A, b, tol=1e-3, max_iter=100_000, normal_eq=True))


def test_algorithm4_on_normal_eq():
    A, b = _rank_deficient(0)
    xp = np.linalg.pinv(A) @ b
    xe = xp + np.linalg.svd(A)[2][6:].T @ np.random.default_rng(9).standard_normal(4)
    xg, ig, tg = P.ta_minnorm(A, b, xe, tol=1e-3, max_iter=500_000, normal_eq=True)
    xo, io, to = oracle.ta_minnorm(A, b, xe, tol=1e-3, max_iter=500_000, normal_eq=True)
    assert (ig.stop, tg, ig.iters, ig.matvecs) == (io.stop, to, io.iters, io.matvecs)
    assert ig.rho == pytest.approx(io.rho, rel=1e-12) and ig.rho_lo == pytest.approx(io.rho_lo,
                                                                                  rel=1e-9)
    assert np.linalg.norm(host(xg) - xo) <= 1e-9 * np.linalg.norm(xo)
    assert ig.rho_lo <= np.linalg.norm(xp) <= ig.rho + 1e-3 * np.linalg.norm(xe)


def test_normal_eq_is_a_ta_option_only():
    """Host-side validation: CTA takes no normal_eq (TA_EINVAL)."""
    A, b = _full_tall(0)
    with pytest.raises(P.TaError, match="EINVAL"):
        P.cta_solve(A, b, normal_eq=True)
    with pytest.raises(P.TaError, match="EINVAL"):
        P.cta_minnorm(A, b, normal_eq=True)


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_normal_eq_from_a_warm_start(kind):
    """The remark after the theorem on Algorithm 3 lets TA move to the normal
    equation from the current iterate when A x = b does not look solvable:
    TA on (A, b) until its normal-equation test at 1e-3, then TA with normal_eq warm-started
    from its x (b' = A^T A x first), against the oracle doing the same."""
    A, b = _rank_deficient(7)
    M = csr_from_dense(A) if kind == "csr" else A
    x1, _, i1 = P.ta_solve(M, b, tol=1e-6, tol_normal=1e-3, max_iter=200_000)
    xo1, _, io1 = oracle.ta(M, b, tol=1e-6, tol_normal=1e-3, max_iter=200_000)
    assert (i1.stop, i1.iters) == (io1.stop, io1.iters) and io1.stop == "normal"
    _compare(P.ta_solve(M, b, tol=1e-6, max_iter=200_000, normal_eq=True, x0=x1),
             oracle.ta(M, b, tol=1e-6, max_iter=200_000, normal_eq=True, x0=xo1))
