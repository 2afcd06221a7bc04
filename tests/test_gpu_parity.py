"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars:
  * index work (the device transpose) is bit-exact;
  * matrix products and residuals agree to 1 ulp per entry (both sides use
    compensated row sums; one-thread-per-row kernels are bit-exact);
  * FP64 solves: equal iteration counts and stop codes, residual histories
    within 1e-10 relative, x within 1e-10 relative (the tolerance the FP64
    path is held to).
"""

import numpy as np
import pytest

import oracle
import paper_2304_12168_amd as P
from workloads import (Csr, convection_diffusion, csr_from_coo, csr_from_dense, dense_gaussian,
                       kac_clement, lp_shaped, poisson5, random_diag_dominant, skewed_rows)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HIST_RTOL = 1e-10
X_RTOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load_library()
    oracle.build(force=False)


def host(t):
    return t.detach().cpu().numpy()


def ulps(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.spacing(np.maximum(np.abs(a), np.abs(b)))
    scale[scale == 0] = np.finfo(np.float64).tiny
    return np.abs(a - b) / scale


def _ragged_csr(m, n, seed, long_rows=()):
    """Random CSR with empty rows, a few very long rows and unsorted columns."""
    g = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(m):
        k = 0 if g.random() < 0.1 else int(g.integers(1, 9))
        if i in long_rows:
            k = min(n, 3000)
        c = g.choice(n, size=k, replace=False)
        rows.append(np.full(k, i))
        cols.append(c)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    A = csr_from_coo(m, n, rows, cols, g.standard_normal(rows.size))
    # shuffle columns inside each row (the ABI allows any order)
    for i in range(m):
        s, e = A.row_ptr[i], A.row_ptr[i + 1]
        p = g.permutation(e - s)
        A.col_idx[s:e] = A.col_idx[s:e][p]
        A.val[s:e] = A.val[s:e][p]
    return A


def _long_columns():
    """50000 x 40 with columns of 50000 (dense), 8192, 8193, 16384, 16385 and
    40000 entries and the rest about 10: A^T rows past the 8192 entries the
    transpose sorts in LDS at once."""
    g = np.random.default_rng(26)
    m, n = 50_000, 40
    lens = [m, 8192, 8193, 16384, 16385, 40_000] + [int(w) for w in g.integers(1, 20, size=n - 6)]
    cols = np.concatenate([np.full(w, j) for j, w in enumerate(lens)])
    rows = np.concatenate([g.choice(m, size=w, replace=False) for w in lens])
    return csr_from_coo(m, n, rows, cols, g.standard_normal(rows.size))


def _dense_columns():
    """2e6 x 3: a dense column, one of 1e6 random rows and one of 10: A^T rows
    that the transpose sorts through merges of up to 2^21 entries."""
    g = np.random.default_rng(30)
    m = 2_000_000
    parts = [np.arange(m), g.choice(m, size=1_000_000, replace=False), g.choice(m, size=10, replace=False)]
    rows = np.concatenate(parts)
    cols = np.concatenate([np.full(p.size, j) for j, p in enumerate(parts)])
    return csr_from_coo(m, 3, rows, cols, g.standard_normal(rows.size))


MATS = {
    "kac_1001": lambda: kac_clement(1001).A,
    "long_columns_50000x40": _long_columns,
    "dense_columns_2e6x3": _dense_columns,
    # one dense row (the merge path on A) and one dense column (a 1e5-entry A^T row)
    "one_row_1x100000": lambda: csr_from_dense(
        np.random.default_rng(31).standard_normal((1, 100_000))),
    "one_column_100000x1": lambda: csr_from_dense(
        np.random.default_rng(32).standard_normal((100_000, 1))),
    "convdiff_33": lambda: convection_diffusion(33).A,
    "ragged_700x517": lambda: _ragged_csr(700, 517, 1, long_rows=(5, 300)),
    "lp_500x20000": lambda: lp_shaped(500, 20000, seed=3).A,
    "randsparse_3000": lambda: random_diag_dominant(3000, 7, seed=2),
    "dense_257x131": lambda: dense_gaussian(131, seed=2, m=257).A,
    "dense_64x300": lambda: dense_gaussian(300, seed=3, m=64).A,
    # merge-path partitions (skewed rows; a few long rows; block-edge lengths)
    "skewed_20000": lambda: skewed_rows(20_000, 20_000, seed=1, empty_frac=0.1, dense_rows=1).A,
    "few_long_rows_4x20000": lambda: _few_long_rows().A,
    "merge_edges_400x6000": lambda: _merge_edges().A,
}


@pytest.mark.parametrize("name", sorted(MATS))
def test_products_match_oracle(name):
    A = MATS[name]()
    m, n = (A.shape if isinstance(A, np.ndarray) else (A.m, A.n))
    g = np.random.default_rng(7)
    x = g.standard_normal(n)
    u = g.standard_normal(m)
    b = g.standard_normal(m)
    dA = P.to_device(A)
    y, ny = P.spmv(dA, x, want_norm=True)
    w, nw = P.spmv(dA, u, trans=True, want_norm=True)
    r, nr = P.residual(dA, b, x, want_norm=True)
    torch.cuda.synchronize()
    y_o, w_o, r_o = oracle.apply(A, x), oracle.apply_t(A, u), oracle.residual(A, b, x)
    assert ulps(host(y), y_o).max() <= 1
    assert ulps(host(w), w_o).max() <= 1
    assert ulps(host(r), r_o).max() <= 1
    # squared norms: compensated on both sides
    assert host(ny)[0] == pytest.approx(oracle.dot2(y_o, y_o), rel=4e-16)
    assert host(nw)[0] == pytest.approx(oracle.dot2(w_o, w_o), rel=4e-16)
    assert host(nr)[0] == pytest.approx(oracle.dot2(r_o, r_o), rel=4e-16)


@pytest.mark.parametrize("name", ["kac_1001", "convdiff_33", "randsparse_3000"])
def test_one_thread_per_row_products_are_bit_exact(name):
    A = MATS[name]()
    x = np.random.default_rng(3).standard_normal(A.n)
    y = host(P.spmv(P.to_device(A), x))
    w = host(P.spmv(P.to_device(A), x[: A.m], trans=True))
    assert np.array_equal(y, oracle.apply(A, x))
    assert np.array_equal(w, oracle.apply_t(A, x[: A.m]))


@pytest.mark.parametrize("name", ["kac_1001", "ragged_700x517", "lp_500x20000", "convdiff_33",
                                  "long_columns_50000x40", "dense_columns_2e6x3",
                                  "one_column_100000x1"])
def test_transpose_is_exact(name):
    A = MATS[name]()
    rp, ci, v = P.transpose(P.to_device(A))
    ref = A.to_scipy().T.tocsr()
    ref.sort_indices()
    assert np.array_equal(host(rp), ref.indptr.astype(np.int32))
    assert np.array_equal(host(ci), ref.indices.astype(np.int32))
    assert np.array_equal(host(v), ref.data)


def test_transpose_with_duplicates_keeps_storage_order():
    # duplicates (i, j) act as a sum; A^T keeps them in A's storage order
    A = Csr(3, 3, np.array([0, 3, 4, 6], np.int32), np.array([1, 1, 0, 2, 1, 1], np.int32),
            np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0]))
    rp, ci, v = P.transpose(P.to_device(A))
    assert host(rp).tolist() == [0, 1, 5, 6]
    assert host(ci).tolist() == [0, 0, 0, 2, 2, 1]
    assert host(v).tolist() == [3.0, 1.0, 2.0, 5.0, 6.0, 4.0]


def test_products_deterministic():
    A = lp_shaped(300, 40000, seed=1).A
    x = np.random.default_rng(0).standard_normal(A.n)
    dA = P.to_device(A)
    a = host(P.spmv(dA, x))
    b = host(P.spmv(dA, x))
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------
def _compare(res_gpu, res_or, x_rtol=X_RTOL):
    x, hist, info = res_gpu
    xo, ho, io = res_or
    assert info.stop == io.stop, (info, io)
    assert info.iters == io.iters, (info, io)
    assert info.matvecs == io.matvecs, (info, io)
    h = host(hist)
    assert h.shape == ho.shape
    np.testing.assert_allclose(h, ho, rtol=HIST_RTOL, atol=0)
    xg = host(x)
    nx = np.linalg.norm(xo)
    assert np.linalg.norm(xg - xo) <= x_rtol * max(nx, 1e-300)
    assert info.rel_res == pytest.approx(io.rel_res, rel=1e-8, abs=1e-300)
    assert info.rel_normal == pytest.approx(io.rel_normal, rel=1e-6, abs=1e-18)


CTA_CASES = [
    ("kac_101_t3", lambda: kac_clement(101), 3, 1e-10, 10000),
    ("kac_1001_t3", lambda: kac_clement(1001), 3, 1e-6, 10000),
    ("kac_1001_t1", lambda: kac_clement(1001), 1, 1e-6, 100000),
    ("convdiff_8_t3", lambda: convection_diffusion(8), 3, 1e-6, 10000),
    ("convdiff_16_t2", lambda: convection_diffusion(16), 2, 1e-6, 20000),
    ("convdiff_16_t5", lambda: convection_diffusion(16), 5, 1e-6, 20000),
    ("dense_gauss_12_t2", lambda: dense_gaussian(12, seed=4), 2, 1e-8, 200000),
    ("dense_gauss_40x25_t3", lambda: dense_gaussian(25, seed=1, m=40), 3, 1e-6, 5000),
    ("lp_200x5000_t3", lambda: lp_shaped(200, 5000), 3, 1e-10, 1000),
    ("rand_5000_t3", lambda: type("Pb", (), {"A": random_diag_dominant(5000, 7, seed=3),
                                               "b": np.random.default_rng(1).uniform(-1, 1, 5000)})(),
     3, 1e-12, 1000),
]


@pytest.mark.parametrize("case", CTA_CASES, ids=[c[0] for c in CTA_CASES])
def test_cta_solve_matches_oracle(case):
    _, make, t, tol, budget = case
    p = make()
    g = P.cta_solve(p.A, p.b, tol=tol, t=t, max_iter=budget)
    o = oracle.cta(p.A, p.b, tol=tol, t=t, max_iter=budget)
    _compare(g, o)


@pytest.mark.parametrize("case", [c for c in CTA_CASES if c[0].startswith(("kac", "lp", "conv"))],
                         ids=lambda c: c[0])
def test_cta_minnorm_matches_oracle(case):
    _, make, t, tol, budget = case
    p = make()
    g = P.cta_minnorm(p.A, p.b, tol=tol, t=t, max_iter=budget)
    o = oracle.cta_minnorm(p.A, p.b, tol=tol, t=t, max_iter=budget)
    _compare(g, o)


def test_cta_budget_and_history_cap():
    p = convection_diffusion(16)
    g = P.cta_solve(p.A, p.b, tol=1e-12, t=3, max_iter=37, hist_cap=10)
    o = oracle.cta(p.A, p.b, tol=1e-12, t=3, max_iter=37, hist_cap=10)
    assert g[2].stop == o[2].stop == "maxiter" and g[2].iters == 37
    assert g[1].shape[0] == 10
    np.testing.assert_allclose(host(g[1]), o[1], rtol=HIST_RTOL)


def test_cta_warm_start_and_replacement():
    p = convection_diffusion(12)
    x0 = np.random.default_rng(2).uniform(0, 1, p.A.n)
    g = P.cta_solve(p.A, p.b, tol=1e-8, t=2, max_iter=50000, x0=x0, replace_every=25)
    o = oracle.cta(p.A, p.b, tol=1e-8, t=2, max_iter=50000, x0=x0, replace_every=25)
    _compare(g, o)
    g = P.cta_minnorm(p.A, p.b, tol=1e-8, t=3, max_iter=50000, replace_every=10)
    o = oracle.cta_minnorm(p.A, p.b, tol=1e-8, t=3, max_iter=50000, replace_every=10)
    _compare(g, o)


def test_cta_normal_equation_stop_on_inconsistent():
    g0 = np.random.default_rng(4)
    A = g0.standard_normal((40, 15))
    b = g0.standard_normal(40)
    for dense in (True, False):
        M = A if dense else csr_from_dense(A)
        g = P.cta_solve(M, b, tol=1e-6, tol_normal=1e-9, t=2, max_iter=100000)
        o = oracle.cta(M, b, tol=1e-6, tol_normal=1e-9, t=2, max_iter=100000)
        _compare(g, o)
        assert g[2].stop == "normal"


def test_cta_edge_cases():
    p = kac_clement(11)
    # b = 0
    x, h, info = P.cta_solve(p.A, np.zeros(11), t=3)
    assert info.stop == "residual" and info.iters == 0 and not host(x).any()
    # zero budget
    x, h, info = P.cta_solve(p.A, p.b, tol=1e-6, t=3, max_iter=0)
    assert info.stop == "maxiter" and info.iters == 0 and host(h)[0] == 1.0
    # NaN in b
    bn = p.b.copy()
    bn[3] = np.nan
    x, h, info = P.cta_solve(p.A, bn, tol=1e-6, t=2, max_iter=10)
    assert info.stop == "breakdown"
    # A = 0 (every direction vanishes): normal equation stop at once
    Z = csr_from_coo(5, 4, [], [], [])
    x, h, info = P.cta_solve(Z, np.ones(5), t=2, max_iter=10)
    o = oracle.cta(Z, np.ones(5), t=2, max_iter=10)
    assert info.stop == o[2].stop == "normal" and info.iters == 0
    # t = m (order equal to the row count)
    q = kac_clement(5)
    _compare(P.cta_solve(q.A, q.b, tol=1e-12, t=5, max_iter=10),
             oracle.cta(q.A, q.b, tol=1e-12, t=5, max_iter=10))


def test_malformed_csr_is_rejected():
    bad = Csr(3, 3, np.array([0, 2, 1, 3], np.int32), np.array([0, 1, 2], np.int32),
              np.ones(3))
    with pytest.raises(P.TaError, match="EINVAL"):
        P.cta_solve(bad, np.ones(3), t=1)
    bad2 = Csr(3, 3, np.array([0, 1, 2, 3], np.int32), np.array([0, 5, 2], np.int32),
               np.ones(3))
    with pytest.raises(P.TaError, match="EINVAL"):
        P.spmv(bad2, np.ones(3))


def test_solve_deterministic():
    p = convection_diffusion(16)
    a = P.cta_solve(p.A, p.b, tol=1e-6, t=3, max_iter=500)
    b = P.cta_solve(p.A, p.b, tol=1e-6, t=3, max_iter=500)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


# ---------------------------------------------------------------------------
# TA
# ---------------------------------------------------------------------------
TA_CASES = [
    ("ta_scalar", lambda: (np.array([[11.0]]), np.array([15.0])), {}, 1e-15, 10),
    ("ta_6x9", lambda: _consistent(6, 9, 11), {}, 1e-6, 2000000),
    ("ta_20x20_fixed", lambda: _consistent(20, 20, 3), {"fixed_rho": True, "rho0": 50.0}, 1e-8,
     20000),
    ("ta_kac_101", lambda: (kac_clement(101).A, kac_clement(101).b), {}, 1e-3, 200000),
    ("ta_csr_incons", lambda: (csr_from_dense(np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])),
                               np.array([1.0, 2.0, 3.0])), {"tol_normal": 1e-9}, 1e-9, 100000),
]


def _consistent(m, n, seed):
    g = np.random.default_rng(seed)
    A = g.standard_normal((m, n))
    return A, A @ g.standard_normal(n)


@pytest.mark.parametrize("case", TA_CASES, ids=[c[0] for c in TA_CASES])
def test_ta_solve_matches_oracle(case):
    _, make, kw, tol, budget = case
    A, b = make()
    for M in ((A, csr_from_dense(A)) if isinstance(A, np.ndarray) else (A,)):
        g = P.ta_solve(M, b, tol=tol, max_iter=budget, **kw)
        o = oracle.ta(M, b, tol=tol, max_iter=budget, **kw)
        _compare(g, o, x_rtol=1e-9)
        assert g[2].rho == o[2].rho and g[2].rho_lo == o[2].rho_lo


def test_ta_witness():
    A, b = _consistent(8, 8, 9)
    nx = np.linalg.norm(np.linalg.solve(A, b))
    g = P.ta_solve(A, b, tol=1e-12, max_iter=100000, rho0=0.5 * nx, fixed_rho=True)
    o = oracle.ta(A, b, tol=1e-12, max_iter=100000, rho0=0.5 * nx, fixed_rho=True)
    _compare(g, o, x_rtol=1e-9)
    assert g[2].stop == "witness" and g[2].rho_lo == o[2].rho_lo < nx


# ---------------------------------------------------------------------------
# full-size workloads: sampled parity
# ---------------------------------------------------------------------------
@pytest.mark.slow
def test_kac_10001_full_solve():
    p = kac_clement(10001)
    _compare(P.cta_solve(p.A, p.b, tol=1e-6, t=3, max_iter=100000),
             oracle.cta(p.A, p.b, tol=1e-6, t=3, max_iter=100000))


@pytest.mark.slow
def test_convdiff_512_first_iterations():
    p = convection_diffusion(512)
    _compare(P.cta_solve(p.A, p.b, tol=1e-6, t=3, max_iter=4),
             oracle.cta(p.A, p.b, tol=1e-6, t=3, max_iter=4))


@pytest.mark.slow
def test_lp_shaped_full_minnorm():
    p = lp_shaped()
    _compare(P.cta_minnorm(p.A, p.b, tol=1e-6, t=3, max_iter=100),
             oracle.cta_minnorm(p.A, p.b, tol=1e-6, t=3, max_iter=100))


@pytest.mark.slow
def test_dense_500_first_iterations():
    p = dense_gaussian(500, seed=0)
    _compare(P.cta_solve(p.A, p.b, tol=1e-8, t=2, max_iter=30),
             oracle.cta(p.A, p.b, tol=1e-8, t=2, max_iter=30))
    _compare(P.ta_solve(p.A, p.b, tol=1e-8, max_iter=30),
             oracle.ta(p.A, p.b, tol=1e-8, max_iter=30), x_rtol=1e-9)


# ---------------------------------------------------------------------------
# prepared operators, the LDS column-tiled and the XCD column-sliced kernels
# ---------------------------------------------------------------------------
def _transpose(p):  # A^T has the long rows and is the regrouped operand
    At = p.A.to_scipy().T.tocsr()
    At.sort_indices()
    A = Csr(At.shape[0], At.shape[1], At.indptr.astype(np.int32), At.indices.astype(np.int32),
            At.data.copy())
    xs = np.random.default_rng(11).standard_normal(A.n)
    return type("Pb", (), {"A": A, "b": A.to_scipy() @ xs})()


def _wide():  # 600 nonzeros per row, 200k columns: 25 tiles, ~24 entries per (row, tile)
    return lp_shaped(2000, 200_000, seed=5)


def _wide_sliced():  # 61 per row over 25 tiles is too thin for tiles: column slices
    return lp_shaped(20_000, 200_000, seed=6)


def _ragged_tiles():
    """3 tiles (20000 columns, the last one ragged), ~200 entries per row at
    random columns, every 7th row and the last row empty, a few rows whose
    entries all fall in one tile."""
    g = np.random.default_rng(21)
    m, n = 301, 20_000
    rows, cols = [], []
    for i in range(m):
        if i % 7 == 3 or i == m - 1:
            continue
        if i % 11 == 5:
            c = g.choice(np.arange(8192, 16384), size=150, replace=False)
        else:
            c = g.choice(n, size=int(g.integers(150, 250)), replace=False)
        rows += [i] * len(c)
        cols += list(c)
    A = csr_from_coo(m, n, np.array(rows), np.array(cols), g.standard_normal(len(rows)))
    x = g.standard_normal(n)
    return type("Pb", (), {"A": A, "b": A.to_scipy() @ x})()


def _two_tiles():
    """Exactly 2 tiles (16384 columns, the smallest tiled width), 300 random
    entries per row."""
    g = np.random.default_rng(22)
    m, n = 257, 16_384
    rows = np.repeat(np.arange(m), 300)
    cols = np.concatenate([g.choice(n, size=300, replace=False) for _ in range(m)])
    A = csr_from_coo(m, n, rows, cols, g.standard_normal(rows.size))
    x = g.standard_normal(n)
    return type("Pb", (), {"A": A, "b": A.to_scipy() @ x})()


def _few_long_rows():
    """4 rows of about 10000 random entries over 20000 columns: the row
    kernels would run one block, the merge path 20."""
    g = np.random.default_rng(23)
    m, n = 4, 20_000
    cols = [g.choice(n, size=int(g.integers(9000, 11000)), replace=False) for _ in range(m)]
    rows = np.concatenate([np.full(c.size, i) for i, c in enumerate(cols)])
    A = csr_from_coo(m, n, rows, np.concatenate(cols), g.standard_normal(rows.size))
    x = g.standard_normal(n)
    return type("Pb", (), {"A": A, "b": A.to_scipy() @ x})()


def _merge_edges():
    """Row lengths placed against the merge path's 2048-item blocks and
    8-item threads: a 3000-entry row first, empty rows (also last), rows of
    7, 8, 9, 2047, 2048, 2049 and 4096 entries among short ones."""
    g = np.random.default_rng(24)
    m, n = 400, 6000
    lens = g.integers(0, 10, size=m)
    lens[0] = 3000
    lens[m - 1] = 0
    for i, w in zip((3, 50, 51, 52, 120, 121, 122, 300, 301), (0, 7, 8, 9, 2047, 2048, 2049, 4096, 0)):
        lens[i] = w
    rows = np.repeat(np.arange(m), lens)
    cols = np.concatenate([g.choice(n, size=int(w), replace=False) for w in lens])
    A = csr_from_coo(m, n, rows, cols, g.standard_normal(rows.size))
    x = g.standard_normal(n)
    return type("Pb", (), {"A": A, "b": A.to_scipy() @ x})()


def _lp_dense_row():
    """The LP shape (2000 x 200000, about 600 entries per row) with a dense
    linking row appended: too skewed for column tiles, so the merge path."""
    B = lp_shaped(2000, 200_000, seed=5).A.to_scipy().tocoo()
    g = np.random.default_rng(25)
    n = B.shape[1]
    rows = np.concatenate([B.row, np.full(n, B.shape[0])])
    cols = np.concatenate([B.col, np.arange(n)])
    A = csr_from_coo(B.shape[0] + 1, n, rows, cols, np.concatenate([B.data, g.standard_normal(n)]))
    x = g.standard_normal(n)
    return type("Pb", (), {"A": A, "b": A.to_scipy() @ x})()


def _wide_random(m, n, per_row, seed):
    """m rows of per_row random columns (repeats summed) over n columns: too
    few entries per (row, 8192-column tile) for tiles, so column slices:
    8 g of them, g the least power of two with n <= g 2^23 (x's slice within
    8 MB): 16 at n = 1.1e7, 32 at n = 2e7."""
    g = np.random.default_rng(seed)
    rows = np.repeat(np.arange(m), per_row)
    cols = g.integers(0, n, size=rows.size)
    A = csr_from_coo(m, n, rows, cols, g.standard_normal(rows.size))
    x = g.standard_normal(n)
    return type("Pb", (), {"A": A, "b": A.to_scipy() @ x})()


REGROUPED = {
    "sliced16_A": (lambda: _wide_random(1000, 11_000_000, 600, 28), ("csr_sliced", None)),
    "sliced32_A": (lambda: _wide_random(500, 20_000_000, 600, 29), ("csr_sliced", None)),
    "lp_dense_row_merge_A": (_lp_dense_row, ("csr_merge", None)),
    "skewed_merge_A": (lambda: skewed_rows(20_000, 20_000, seed=1, empty_frac=0.1, dense_rows=1),
                       ("csr_merge", None)),
    "skewed_merge_AT": (lambda: _transpose(skewed_rows(6000, 8000, seed=2)), (None, "csr_merge")),
    "few_long_rows_merge_A": (_few_long_rows, ("csr_merge", None)),
    "edges_merge_A": (_merge_edges, ("csr_merge", None)),
    "wide_tiled_A": (_wide, ("csr_tiled", None)),
    "two_tiles_A": (_two_tiles, ("csr_tiled", None)),
    "tall_tiled_AT": (lambda: _transpose(_wide()), (None, "csr_tiled")),
    "ragged_tiled_A": (_ragged_tiles, ("csr_tiled", None)),
    "wide_sliced_A": (_wide_sliced, ("csr_sliced", None)),
    "tall_sliced_AT": (lambda: _transpose(_wide_sliced()), (None, "csr_sliced")),
}


def _plan_checked(make, fmt):
    p = make()
    pl = P.plan(p.A)
    for trans, f in ((False, fmt[0]), (True, fmt[1])):
        if f is not None:
            assert pl.format(trans) == f
    return p, pl


@pytest.mark.parametrize("case", sorted(REGROUPED))
def test_regrouped_products_match_oracle(case):
    make, fmt = REGROUPED[case]
    p, pl = _plan_checked(make, fmt)
    A = p.A
    g = np.random.default_rng(4)
    x = g.standard_normal(A.n)
    u = g.standard_normal(A.m)
    # the plan's product kernels are the ones the solvers launch
    for trans, vec, ref in ((False, x, oracle.apply(A, x)), (True, u, oracle.apply_t(A, u))):
        y = host(P.spmv(pl, vec, trans=trans))
        assert ulps(y, ref).max() <= 1
    pl.close()


@pytest.mark.parametrize("case", sorted(REGROUPED))
def test_regrouped_solves_match_oracle(case):
    make, fmt = REGROUPED[case]
    p, pl = _plan_checked(make, fmt)
    g = P.cta_minnorm(pl, p.b, tol=1e-10, t=3, max_iter=200)
    o = oracle.cta_minnorm(p.A, p.b, tol=1e-10, t=3, max_iter=200)
    _compare(g, o)
    g = P.cta_solve(pl, p.b, tol=1e-10, t=2, max_iter=200)
    o = oracle.cta(p.A, p.b, tol=1e-10, t=2, max_iter=200)
    _compare(g, o)
    g = P.ta_solve(pl, p.b, tol=1e-3, max_iter=300)
    o = oracle.ta(p.A, p.b, tol=1e-3, max_iter=300)
    _compare(g, o, x_rtol=1e-9)
    pl.close()


def test_long_rows_keep_their_column_tiles():
    """256 rows of 20000 random entries over 10^6 columns: column tiles (984
    blocks), built from (A^T)^T, whose rows are longer than one LDS sort;
    products and a short CTA solve against the oracle."""
    g = np.random.default_rng(27)
    m, n, w = 256, 1_000_000, 20_000
    rows = np.repeat(np.arange(m), w)
    cols = np.concatenate([g.choice(n, size=w, replace=False) for _ in range(m)])
    A = csr_from_coo(m, n, rows, cols, g.standard_normal(rows.size))
    pl = P.plan(A)
    assert pl.format(False) == "csr_tiled"
    x = g.standard_normal(n)
    u = g.standard_normal(m)
    assert ulps(host(P.spmv(pl, x)), oracle.apply(A, x)).max() <= 1
    assert ulps(host(P.spmv(pl, u, trans=True)), oracle.apply_t(A, u)).max() <= 1
    b = A.to_scipy() @ g.standard_normal(n)
    _compare(P.cta_minnorm(pl, b, tol=1e-10, t=3, max_iter=20),
             oracle.cta_minnorm(A, b, tol=1e-10, t=3, max_iter=20))
    pl.close()


def _skewed_spd(n=3000, seed=5):
    """B + B^T plus a dominant diagonal, B with skewed rows and one dense row:
    symmetric positive definite, with a dense row and column."""
    from scipy import sparse

    B = skewed_rows(n, n, seed=seed, dense_rows=1).A.to_scipy()
    S = (B + B.T).tocsr()
    S = (S + sparse.diags(abs(S).sum(axis=1).A1 + 1.0)).tocsr()
    S.sort_indices()
    return Csr(n, n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.copy())


def test_merge_path_epilogues_in_solves():
    """The merge-path product under the epilogues of H = A (CTA, the dot with
    the input) and of TA's LP-feasibility form (the positive part), against
    the oracle."""
    S = _skewed_spd()
    pl = P.plan(S)
    assert pl.format(False) == pl.format(True) == "csr_merge"
    b = S.to_scipy() @ np.random.default_rng(3).standard_normal(S.n)
    kw = dict(tol=1e-8, t=3, max_iter=5000, h_is_a=True)
    _compare(P.cta_solve(pl, b, **kw), oracle.cta(S, b, **kw))
    pl.close()
    A = skewed_rows(2000, 20_000, seed=6, dense_rows=1).A
    xs = np.abs(np.random.default_rng(4).standard_normal(A.n))
    b = A.to_scipy() @ xs
    pl = P.plan(A)
    assert pl.format(False) == "csr_merge"
    kw = dict(tol=1e-4, max_iter=20_000, nonneg=True)
    _compare(P.ta_solve(pl, b, **kw), oracle.ta(A, b, **kw), x_rtol=1e-9)
    pl.close()


def test_plan_and_one_shot_are_identical():
    p = kac_clement(3001)
    pl = P.plan(p.A)
    a = P.cta_solve(pl, p.b, tol=1e-6, t=3, max_iter=5000)
    b = P.cta_solve(p.A, p.b, tol=1e-6, t=3, max_iter=5000)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert a[2] == b[2]
    c = P.ta_solve(pl, p.b, tol=1e-2, max_iter=5000)
    d = oracle.ta(p.A, p.b, tol=1e-2, max_iter=5000)
    _compare(c, d, x_rtol=1e-9)
    pl.close()


def test_plan_rejects_malformed_csr():
    bad = Csr(3, 3, np.array([0, 2, 1, 3], np.int32), np.array([0, 1, 2], np.int32), np.ones(3))
    with pytest.raises(P.TaError, match="EINVAL"):
        P.plan(bad)


@pytest.mark.parametrize("case", ["cta_x", "cta_y", "ta", "ta_ne", "cta_accel_replace", "cta_cycle",
                                  "cta_merge", "cta_tiled", "cta_sliced"])
def test_graph_replay_equals_plain_launches(case):
    """Single-system chains replay their chunks from captured HIP graphs
    (launch_mode 0, the default) or launch every kernel (launch_mode 1): the
    same kernels with the same arguments, so x, the history and every count
    must agree bit for bit.  The solves run many chunks, so each graph is
    replayed several times, with the other mode's eager work in between."""
    p = convection_diffusion(12)
    g = np.random.default_rng(4)
    A = p.A
    kw = dict(tol=1e-10, max_iter=3000)
    if case == "cta_x":
        run = lambda **o: P.cta_solve(A, p.b, t=3, **kw, **o)
    elif case == "cta_y":
        run = lambda **o: P.cta_minnorm(A, p.b, t=2, **kw, **o)
    elif case == "ta":
        q = dense_gaussian(20, seed=3, m=12)
        run = lambda **o: P.ta_solve(q.A, q.b, tol=1e-9, max_iter=20000, **o)
    elif case == "ta_ne":
        a = g.standard_normal((30, 12))
        bb = g.standard_normal(30)
        run = lambda **o: P.ta_solve(a, bb, tol=1e-7, max_iter=20000, normal_eq=True, **o)
    elif case == "cta_accel_replace":
        run = lambda **o: P.cta_solve(A, p.b, t=2, accel=0.5, replace_every=7, **kw, **o)
    elif case in ("cta_merge", "cta_tiled", "cta_sliced"):
        # plans whose products take the merge path (with its fix-up kernel),
        # column tiles or column slices (each with its combine kernel)
        q = {"cta_merge": lambda: skewed_rows(5000, 5000, seed=8, dense_rows=1),
             "cta_tiled": _wide, "cta_sliced": _wide_sliced}[case]()
        pl = P.plan(q.A)
        assert pl.format(False) == {"cta_merge": "csr_merge", "cta_tiled": "csr_tiled",
                                    "cta_sliced": "csr_sliced"}[case]
        run = lambda **o: P.cta_minnorm(pl, q.b, t=3, tol=1e-20, max_iter=200, **o)
    else:
        run = lambda **o: P.cta_solve(A, p.b, t=4, t_cycle=True, **kw, **o)
    for _ in range(2):
        xg, hg, ig = run(graph=True)
        xl, hl, il = run(graph=False)
        assert (ig.stop, ig.iters, ig.matvecs) == (il.stop, il.iters, il.matvecs)
        assert ig.iters > 64, ig  # several chunks, graphs replayed
        assert torch.equal(xg, xl) and torch.equal(hg, hl)
        assert ig.rel_res == il.rel_res and ig.rho == il.rho


FULL = {
    # the bandwidth sweep's sizes, in the layouts the benchmark times
    "skewed_1e6_merge": (lambda: skewed_rows(1_000_000, 1_000_000, seed=0).A, "csr_merge"),
    "poisson_2896_sell_nt": (lambda: poisson5(2896), "sell64"),
    "lp_1e7_sliced16": (lambda: lp_shaped(100_000, 10_000_000, seed=0).A, "csr_sliced"),
}


@pytest.mark.parametrize("case", sorted(FULL))
def test_full_size_products_match_oracle(case):
    """Every output entry of the A and A^T products at the benchmark's sizes
    (the merge path on 8e6 skewed nonzeros, SELL-64 with non-temporal loads on
    4.2e7, 16 column slices on 6e7) within 1 ulp of the oracle."""
    make, fmt = FULL[case]
    A = make()
    pl = P.plan(A)
    assert pl.format(False) == fmt
    g = np.random.default_rng(5)
    x = g.standard_normal(A.n)
    u = g.standard_normal(A.m)
    assert ulps(host(P.spmv(pl, x)), oracle.apply(A, x)).max() <= 1
    assert ulps(host(P.spmv(pl, u, trans=True)), oracle.apply_t(A, u)).max() <= 1
    pl.close()
