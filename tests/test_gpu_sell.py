"""SELL-64 storage of a prepared operator (64-row slices stored position by
position): chosen for short rows of even length, and its products equal the
oracle's compensated row sums bit for bit -- the same terms in the same
order -- including a ragged last slice, empty rows, explicit zeros and
unsorted columns; solves through it match the oracle as the CSR kernels do
(every epilogue: norms, residual replacement, the TA step)."""
import numpy as np
import pytest

import oracle
import paper_2304_12168_amd as P
from workloads import (convection_diffusion, csr_from_coo, dense_gaussian, kac_clement,
                       poisson5, random_diag_dominant)

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


def _ragged_tail(m=1001, n=997, seed=0):
    """Row lengths 0, 3, 4 or 5 (m not a multiple of 64), unsorted columns,
    some stored values exactly zero."""
    g = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(m):
        k = int(g.choice([0, 3, 4, 5], p=[0.05, 0.15, 0.3, 0.5]))
        rows += [i] * k
        cols += list(g.choice(n, size=k, replace=False))
    vals = g.standard_normal(len(rows))
    vals[::17] = 0.0
    A = csr_from_coo(m, n, np.array(rows), np.array(cols), vals)
    for i in range(m):
        s, e = A.row_ptr[i], A.row_ptr[i + 1]
        p = g.permutation(e - s)
        A.col_idx[s:e] = A.col_idx[s:e][p]
        A.val[s:e] = A.val[s:e][p]
    return A


def _uneven(m=640, n=700, seed=1):
    """Every 64th row holds 40 entries, the others 2: SELL would pad each
    slice to 40 positions, so the plan keeps CSR."""
    g = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(m):
        k = 40 if i % 64 == 0 else 2
        rows += [i] * k
        cols += list(g.choice(n, size=k, replace=False))
    return csr_from_coo(m, n, np.array(rows), np.array(cols), g.standard_normal(len(rows)))


SELL = {
    "poisson_64": lambda: poisson5(64),
    "kac_1001": lambda: kac_clement(1001).A,
    "convdiff_33": lambda: convection_diffusion(33).A,
    "randsparse_3000": lambda: random_diag_dominant(3000, 7, seed=2),
    "ragged_tail": _ragged_tail,
}


def _expected(rp):
    """The plan's rule, recomputed: one thread per row (16 or fewer entries
    per row on average) and 64-row slices padded by at most a quarter."""
    rp = np.asarray(rp, dtype=np.int64)
    rows, nnz = rp.size - 1, int(rp[-1])
    if rows == 0 or nnz == 0 or nnz / rows > 16.0:
        return "csr_rows"
    lens = np.diff(rp)
    pad = np.zeros(-(-rows // 64) * 64, dtype=np.int64)
    pad[:rows] = lens
    slots = 64 * int(pad.reshape(-1, 64).max(axis=1).sum())
    return "sell64" if slots <= nnz + nnz // 4 else "csr_rows"


def test_format_choice():
    for name, make in sorted(SELL.items()) + [("uneven", _uneven)]:
        A = make()
        S = A.to_scipy().T.tocsr()
        pl = P.plan(A)
        assert pl.format(False) == _expected(A.row_ptr), name
        assert pl.format(True) == _expected(S.indptr), name
    # the cases the rule is meant for, and one it must refuse
    assert P.plan(poisson5(64)).format(True) == "sell64"
    assert P.plan(kac_clement(1001).A).format(True) == "sell64"
    assert P.plan(_uneven()).format(False) == "csr_rows"
    d = P.plan(dense_gaussian(50, seed=1).A)
    assert (d.format(False), d.format(True)) == ("dense_rows", "dense_rows")


@pytest.mark.parametrize("name", sorted(SELL))
def test_products_bit_exact(name):
    A = SELL[name]()
    pl = P.plan(A)
    assert pl.format(False) == "sell64"
    g = np.random.default_rng(5)
    x, u = g.standard_normal(A.n), g.standard_normal(A.m)
    y, ny = P.spmv(pl, x, want_norm=True)
    w = P.spmv(pl, u, trans=True)
    torch.cuda.synchronize()
    y_o = oracle.apply(A, x)
    assert np.array_equal(host(y), y_o)
    assert np.array_equal(host(w), oracle.apply_t(A, u))
    assert host(ny)[0] == pytest.approx(oracle.dot2(y_o, y_o), rel=4e-16)
    # the one-shot product (CSR kernel) gives the same bits
    assert np.array_equal(host(P.spmv(A, x)), host(y))


def _cmp(g, o, x_rtol=1e-10):
    x, hist, info = g
    xo, ho, io = o
    assert (info.stop, info.iters, info.matvecs) == (io.stop, io.iters, io.matvecs), (info, io)
    np.testing.assert_allclose(host(hist), ho, rtol=1e-10, atol=0)
    assert np.linalg.norm(host(x) - xo) <= x_rtol * max(np.linalg.norm(xo), 1e-300)


def test_solves_through_sell_match_oracle():
    p = kac_clement(1001)
    pl = P.plan(p.A)
    assert pl.format(False) == "sell64"
    kw = dict(tol=1e-8, t=3, max_iter=20_000, replace_every=5)
    _cmp(P.cta_solve(pl, p.b, **kw), oracle.cta(p.A, p.b, **kw))
    _cmp(P.cta_minnorm(pl, p.b, **kw), oracle.cta_minnorm(p.A, p.b, **kw))
    A = convection_diffusion(33).A
    b = np.random.default_rng(3).uniform(-1, 1, A.m)
    kw = dict(tol=1e-4, max_iter=50_000)
    _cmp(P.ta_solve(P.plan(A), b, **kw), oracle.ta(A, b, **kw), x_rtol=1e-9)


def test_ragged_tail_solve_matches_oracle():
    A = _ragged_tail(m=700, n=700, seed=4)
    # a diagonal keeps the square system solvable
    d = csr_from_coo(700, 700, np.arange(700), np.arange(700), np.full(700, 6.0))
    S = (A.to_scipy() + d.to_scipy()).tocsr()
    from workloads import Csr

    B = Csr(700, 700, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.copy())
    pl = P.plan(B)
    assert pl.format(False) == "sell64"
    b = np.random.default_rng(8).standard_normal(700)
    kw = dict(tol=1e-9, t=2, max_iter=20_000)
    _cmp(P.cta_solve(pl, b, **kw), oracle.cta(B, b, **kw))
