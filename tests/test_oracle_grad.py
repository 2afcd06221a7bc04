"""Pins of the oracle's gradient of the solution map x(A, b) = A^{-1} b
(square nonsingular A; not in the paper), each against something other than
the oracle: a hand-worked case, central finite differences of the oracle's
own forward solves, and PyTorch's autograd through dense LU and SVD solves."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from workloads import csr_from_coo, perturbed_stencil


def test_csr_outer_by_hand():
    # pattern {(0,1), (1,0), (1,2)}; out_k = (alpha u_i) v_j
    A = csr_from_coo(2, 3, [0, 1, 1], [1, 0, 2], [9.0, 9.0, 9.0])
    out = oracle.csr_outer(A, [2.0, 3.0], [5.0, 7.0, 11.0], -1.0)
    assert out.tolist() == [-14.0, -15.0, -33.0]


def test_csr_outer_rounding():
    g = np.random.default_rng(4)
    A = perturbed_stencil(6, seed=1).A
    u, v = g.standard_normal(A.m), g.standard_normal(A.n)
    out = oracle.csr_outer(A, u, v, -0.7)
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
    for k in range(len(out)):
        exact = Fraction(-0.7) * Fraction(u[rows[k]]) * Fraction(v[A.col_idx[k]])
        assert abs(Fraction(out[k]) - exact) <= abs(exact) * Fraction(2.3e-16)


def _loss_parts(p):
    xt = p.meta["x_target"]
    return xt, (lambda x: float(np.sum((x - xt) ** 2))), (lambda x: 2.0 * (x - xt))


def test_gradient_matches_central_differences():
    """h = 1e-6 central differences of L(x(A, b)) with the oracle's forward
    solve (CTA-3 to 1e-14) against the adjoint gradient, for entries of b and
    stored values of A."""
    p = perturbed_stencil(4, sigma=0.1, seed=0)
    xt, L, dL = _loss_parts(p)
    kw = dict(tol=1e-14, t=3, max_iter=100000)
    x, lam, gv, fi, ai = oracle.cta_grad(p.A, p.b, dL, **kw)
    assert fi.stop == ai.stop == "residual"
    h = 1e-6

    def loss_b(bb):
        return L(oracle.cta(p.A, bb, hist_cap=1, **kw)[0])

    def loss_v(vals):
        A = perturbed_stencil(4, sigma=0.1, seed=0).A
        A.val = vals
        return L(oracle.cta(A, p.b, hist_cap=1, **kw)[0])

    for i in (0, 5, 15):
        e = np.zeros(p.A.m)
        e[i] = h
        fd = (loss_b(p.b + e) - loss_b(p.b - e)) / (2 * h)
        assert fd == pytest.approx(lam[i], rel=1e-6, abs=1e-9)
    for k in (0, 7, len(p.A.val) - 1):
        d = np.zeros(len(p.A.val))
        d[k] = h
        fd = (loss_v(p.A.val + d) - loss_v(p.A.val - d)) / (2 * h)
        assert fd == pytest.approx(gv[k], rel=1e-6, abs=1e-9)


@pytest.mark.slow
def test_gradient_matches_dense_autograd_n400():
    """Perturbed 20 x 20 stencil (n = 400): the oracle's adjoint gradient
    (CTA-8 to 1e-10 for both solves) against PyTorch autograd through the
    dense solve (LU) and through pinv (SVD), restricted to the stored
    pattern."""
    torch = pytest.importorskip("torch")
    p = perturbed_stencil(20, sigma=0.1, seed=0)
    xt, L, dL = _loss_parts(p)
    x, lam, gv, fi, ai = oracle.cta_grad(p.A, p.b, dL, tol=1e-10, t=8, max_iter=200000)
    assert fi.stop == ai.stop == "residual"
    rows = np.repeat(np.arange(p.A.m), np.diff(p.A.row_ptr))
    cols = p.A.col_idx
    # a posteriori bounds: relative error <= cond(A) x relative residual
    # (the adjoint right-hand side 2(x - x_target) carries the forward error)
    kappa = np.linalg.cond(p.A.to_dense())
    ex = 1.01 * kappa * fi.rel_res
    g = dL(x)
    el = 1.01 * kappa * (ai.rel_res + 2 * ex * np.linalg.norm(x) / np.linalg.norm(g))
    assert ex < 1e-4 and el < 1e-4
    for how in ("solve", "pinv"):
        Ad = torch.tensor(p.A.to_dense(), dtype=torch.float64, requires_grad=True)
        bd = torch.tensor(p.b, dtype=torch.float64, requires_grad=True)
        xd = torch.linalg.solve(Ad, bd) if how == "solve" else torch.linalg.pinv(Ad) @ bd
        loss = ((xd - torch.tensor(xt)) ** 2).sum()
        loss.backward()
        gA = Ad.grad.numpy()[rows, cols]
        gb = bd.grad.numpy()
        xr = xd.detach().numpy()
        assert np.linalg.norm(x - xr) <= ex * np.linalg.norm(xr)
        assert np.linalg.norm(lam - gb) <= el * np.linalg.norm(gb), how
        # -lambda_i x_j: the two relative errors add (to first order)
        assert np.linalg.norm(gv - gA) <= 2 * (ex + el) * np.linalg.norm(gA), how
