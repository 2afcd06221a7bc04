"""cta_solve_plan_noalloc (the variant of cta_solve_plan for callers that
cannot allocate device memory) through the C ABI, against cta_solve_plan on
the same plan: the same kernels on a workspace carved from the library's
fixed per-GPU buffer, so x, the history and the counts must agree bit for
bit.  Two calls in a row, the second on a smaller system (the buffer keeps
the first call's contents), then a solve too large for the buffer, which
must be refused before any device work."""
import numpy as np
import pytest

import paper_2304_12168_amd as P
from workloads import convection_diffusion, csr_from_coo, dense_gaussian, lp_shaped, skewed_rows

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load_library()


def _same(a, b):
    xa, ha, ia = a
    xb, hb, ib = b
    assert (ia.stop, ia.iters, ia.matvecs) == (ib.stop, ib.iters, ib.matvecs), (ia, ib)
    assert torch.equal(xa, xb)
    assert torch.equal(ha, hb)
    assert ia.rel_res == ib.rel_res and ia.rel_normal == ib.rel_normal


def test_noalloc_equals_plan_solve_on_two_calls_the_second_smaller():
    big = convection_diffusion(48)       # n = 2304, SELL-64 products
    small = dense_gaussian(40, seed=5)   # 40 x 40 dense rows
    for p, kw in ((big, dict(tol=1e-6, t=3, max_iter=400)),
                  (small, dict(tol=1e-9, t=2, max_iter=20000))):
        pl = P.Plan(p.A)
        try:
            ref = P.cta_solve(pl, p.b, **kw)
            got = P.cta_solve_noalloc(pl, p.b, **kw)
            _same(got, ref)
            assert np.isfinite(got[2].rel_res)
        finally:
            pl.close()


def test_noalloc_options_follow_the_plan_solve():
    """Replacement, warm start and the convex-combination step take the same
    paths (the last one reserves two more vectors)."""
    p = convection_diffusion(24)
    pl = P.Plan(p.A)
    try:
        x0 = np.random.default_rng(3).standard_normal(p.A.n) * 1e-3
        for kw in (dict(replace_every=5), dict(x0=x0), dict(accel=0.5)):
            _same(P.cta_solve_noalloc(pl, p.b, tol=1e-6, t=2, max_iter=300, **kw),
                  P.cta_solve(pl, p.b, tol=1e-6, t=2, max_iter=300, **kw))
    finally:
        pl.close()


def test_noalloc_refuses_a_solve_larger_than_its_buffer():
    """A diagonal 3e6 x 3e6 system at t = 3 needs about 8 (t + 1)(m + n) =
    192 MB of workspace, past the 64 MiB buffer: TA_ESCRATCH, and x is
    untouched (no device work was enqueued)."""
    n = 3_000_000
    idx = np.arange(n)
    A = csr_from_coo(n, n, idx, idx, np.full(n, 2.0))
    pl = P.Plan(A)
    try:
        b = torch.ones(n, dtype=torch.float64, device="cuda")
        with pytest.raises(P.TaError, match="TA_ESCRATCH"):
            P.cta_solve_noalloc(pl, b, tol=1e-6, t=3, max_iter=10)
        # the plan solve itself still works on it
        x, _, info = P.cta_solve(pl, b, tol=1e-6, t=3, max_iter=10)
        assert info.stop == "residual" and torch.allclose(x, torch.full_like(x, 0.5))
    finally:
        pl.close()


def test_noalloc_on_regrouped_plans():
    """Plans whose A is stored in LDS column tiles (per-(tile, row) partials),
    XCD column slices (per-(slice, row) partials) or a merge-path partition
    (per-block head and carry slots): those are carved from the buffer too."""
    cases = [(lambda: lp_shaped(2000, 200_000, seed=5), "csr_tiled"),
             (lambda: lp_shaped(20_000, 200_000, seed=5), "csr_sliced"),
             (lambda: skewed_rows(20_000, 20_000, seed=1, empty_frac=0.1, dense_rows=1), "csr_merge")]
    for make, fmt in cases:
        p = make()
        pl = P.Plan(p.A)
        try:
            assert pl.format(False) == fmt
            kw = dict(tol=1e-8, t=3, max_iter=200)
            _same(P.cta_solve_noalloc(pl, p.b, **kw), P.cta_solve(pl, p.b, **kw))
        finally:
            pl.close()
