"""A batch whose systems fall into every width group (K = 1 .. 64) and both
row-length parts (stencils at most 6 nonzeros per row, random sparse rows
longer): the groups and parts run side by side on their own streams, and
each system must get what it gets when solved alone.

FP64: equal stop codes, iteration and product counts, x within 1e-12
relative (the row lanes, and so the order of the compensated sums, may
differ with the group's composition).  FP32 products with FP64 refinement:
every column stops as when solved alone.  The iteration cap sits far from
every column's count: the stencils stop at it, the random systems converge
in under 60 iterations."""
import numpy as np
import pytest

import oracle
import paper_2304_12168_amd as P
from workloads import poisson5, random_diag_dominant

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


def _batch():
    g = np.random.default_rng(31)
    ks = [1, 2, 3, 6, 12, 20, 40, 64, 5, 33]
    A = []
    for i, k in enumerate(ks):
        if i % 2 == 0:
            A.append(poisson5(12 + 2 * i))
        else:
            A.append(random_diag_dominant(300 + 40 * i, 7, seed=i))
    B = [g.uniform(-1, 1, (a.m, k)) for a, k in zip(A, ks)]
    return A, B


def _solve(A, B, prec, **kw):
    plan = P.BatchPlan([P.to_device(a) for a in A], prec)
    X, infos = P.cta_solve_batched(plan, B, precision=prec, **kw)
    torch.cuda.synchronize()
    out = [host(x) for x in X]
    plan.close()
    return out, infos


@pytest.mark.parametrize("minnorm", [False, True], ids=["x_form", "y_form"])
def test_fp64_side_by_side_equals_alone(minnorm):
    A, B = _batch()
    kw = dict(tol=1e-8, t=3, max_iter=1500, minnorm=minnorm)
    X, infos = _solve(A, B, "fp64", **kw)
    for s in range(len(A)):
        Xs, inf_s = _solve([A[s]], [B[s]], "fp64", **kw)
        for c in range(B[s].shape[1]):
            a, b = infos[s][c], inf_s[0][c]
            assert (a.stop, a.iters, a.matvecs) == (b.stop, b.iters, b.matvecs), (s, c, a, b)
        assert np.linalg.norm(X[s] - Xs[0]) <= 1e-12 * np.linalg.norm(Xs[0])


def test_fp32_side_by_side_reaches_tolerance():
    A, B = _batch()
    kw = dict(tol=1e-6, t=3, max_iter=1500)
    X, infos = _solve(A, B, "fp32", **kw)
    for s in range(len(A)):
        _, inf_s = _solve([A[s]], [B[s]], "fp32", **kw)
        for c in range(B[s].shape[1]):
            assert infos[s][c].stop == inf_s[0][c].stop, (s, c)
            if infos[s][c].stop == "residual":
                r = B[s][:, c] - A[s].to_scipy() @ X[s][:, c]
                assert np.linalg.norm(r) <= 1e-6 * np.linalg.norm(B[s][:, c]) * (1 + 1e-9)
