"""The precision option (FP32 / BF16 matrix products, FP64 refinement) at the
single-system boundary, through the C ABI, on every solver that takes it,
and its rejection by those that compute in FP64 only.

cta_solve / cta_minnorm with TA_FP32 or TA_BF16 run the batched engine on one
system and one right-hand side: the column must stop on the FP64 true
residual at the tolerance, agree with the one-column cta_solve_batched call,
and x must agree with the FP64 oracle's x within 1e-6 relative
(mixed-mode bar; both x lie in range(A^T) and the systems are well
conditioned there)."""
import numpy as np
import pytest

import oracle
import paper_2304_12168_amd as P
from workloads import dense_gaussian, lp_shaped, random_diag_dominant

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


def _cases():
    g = np.random.default_rng(8)
    lp = lp_shaped(400, 9000, seed=3)
    rd = random_diag_dominant(3000, 7, seed=2)
    dg = dense_gaussian(120, seed=4, m=60)
    out = []
    for name, A in (("lp_shaped", lp.A), ("diag_dominant", rd), ("dense_wide", dg.A)):
        a = A if isinstance(A, np.ndarray) else A.to_scipy()
        b = a @ g.standard_normal(a.shape[1])
        out.append((name, A, b))
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("minnorm", [False, True], ids=["cta_solve", "cta_minnorm"])
def test_low_precision_single_system(prec, minnorm):
    tol, t = 1e-8, 3
    solve = P.cta_minnorm if minnorm else P.cta_solve
    run = oracle.cta_minnorm if minnorm else oracle.cta
    for name, A, b in _cases():
        x, _, info = solve(A, b, tol=tol, t=t, max_iter=4000, precision=prec)
        assert info.stop == "residual" and info.rel_res <= tol, (name, info)
        a = A if isinstance(A, np.ndarray) else A.to_scipy()
        xg = host(x)
        assert np.linalg.norm(b - a @ xg) <= tol * (1 + 1e-6) * np.linalg.norm(b), name
        xo, _, io = run(A, b, tol=tol, t=t, max_iter=20000)
        assert io.stop == "residual", (name, io)
        assert np.linalg.norm(xg - xo) <= 1e-6 * np.linalg.norm(xo), name
        # the same engine as one column of cta_solve_batched (whose row-lane
        # tuner times the kernels per plan, so the sums, and the last bits,
        # may be taken in another order): the same x to the mixed-mode bar
        plan = P.BatchPlan([A], prec)
        X, infos = P.cta_solve_batched(plan, [b.reshape(-1, 1)], tol=tol, t=t, max_iter=4000,
                                       minnorm=minnorm, precision=prec)
        plan.close()
        assert infos[0][0].stop == "residual"
        assert np.linalg.norm(host(X[0][:, 0]) - xg) <= 1e-6 * np.linalg.norm(xg), name


def test_low_precision_rejected_where_fp64_only():
    name, A, b = _cases()[1]
    pl = P.Plan(A)
    try:
        for call in (lambda: P.cta_solve(pl, b, precision="fp32"),
                     lambda: P.cta_minnorm(pl, b, precision="bf16"),
                     lambda: P.cta_solve_noalloc(pl, b, precision="fp32"),
                     lambda: P.ta_solve(A, b, precision="fp32"),
                     lambda: P.ta_solve(pl, b, precision="bf16"),
                     lambda: P.ta_minnorm(A, b, np.zeros(A.n), precision="fp32"),
                     lambda: P.cta_solve(A, b, precision="fp32", x0=np.zeros(A.n)),
                     lambda: P.cta_solve(A, b, precision="fp32", accel=0.5)):
            with pytest.raises(P.TaError, match="EINVAL"):
                call()
    finally:
        pl.close()


def test_low_precision_empty_and_zero_rhs():
    """b = 0: x = 0 at once, as in FP64."""
    A = random_diag_dominant(500, 7, seed=1)
    x, _, info = P.cta_solve(A, np.zeros(500), tol=1e-6, t=3, precision="fp32")
    assert info.stop == "residual" and info.iters == 0 and not host(x).any()
