"""Pins of the CPU oracle against the paper and against mathematics.

Each test checks the oracle against something other than itself: exact
rational arithmetic, closed forms stated in the paper, textbook equivalences
(restarted GMRES, Frank-Wolfe), brute force (pseudo-inverse, least squares)
or invariants the paper proves.  None of them re-types the oracle's formulas.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from workloads import (convection_diffusion, csr_from_dense, dense_gaussian, kac_clement,
                       lp_shaped, poisson5)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


# --------------------------------------------------------------------------
# compensated reductions and products: exact rational arithmetic
# --------------------------------------------------------------------------
def _exact_dot(x, y):
    return sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))


@pytest.mark.parametrize("seed", range(6))
def test_dot2_is_nearly_correctly_rounded(seed):
    g = np.random.default_rng(seed)
    n = 200
    x = g.standard_normal(n) * np.exp(g.uniform(-20, 20, n))
    y = g.standard_normal(n)
    # heavy cancellation: append the negated products
    x = np.concatenate([x, -x[: n // 2] * (1 + 1e-9)])
    y = np.concatenate([y, y[: n // 2]])
    ex = _exact_dot(x, y)
    got = oracle.dot2(x, y)
    nn = x.size
    gamma = nn * U / (1 - nn * U)
    bound = U * abs(float(ex)) + gamma ** 2 * float(np.sum(np.abs(x * y)))
    assert abs(Fraction(got) - ex) <= Fraction(bound) * 1.0000001


def test_dot2_exact_on_integers():
    x = np.arange(1, 1001, dtype=np.float64)
    assert oracle.dot2(x, x) == sum(i * i for i in range(1, 1001))


def _tiny_csr(seed, m=7, n=5, dens=0.5):
    g = np.random.default_rng(seed)
    a = g.standard_normal((m, n)) * (g.random((m, n)) < dens)
    return a, csr_from_dense(a)


@pytest.mark.parametrize("seed", range(4))
def test_products_match_exact_rationals(seed):
    a, A = _tiny_csr(seed)
    g = np.random.default_rng(100 + seed)
    x = g.standard_normal(a.shape[1])
    u = g.standard_normal(a.shape[0])
    b = g.standard_normal(a.shape[0])
    for M in (a, A):
        y = oracle.apply(M, x)
        w = oracle.apply_t(M, u)
        r = oracle.residual(M, b, x)
        for i in range(a.shape[0]):
            ex = _exact_dot(a[i], x)
            assert abs(Fraction(y[i]) - ex) <= Fraction(2 * U * abs(float(ex)) + 1e-300)
            exr = Fraction(float(b[i])) - ex
            assert abs(Fraction(r[i]) - exr) <= Fraction(2 * U * abs(float(exr)) + 1e-300)
        for j in range(a.shape[1]):
            ex = _exact_dot(a[:, j], u)
            assert abs(Fraction(w[j]) - ex) <= Fraction(2 * U * abs(float(ex)) + 1e-300)


def test_transposed_product_is_product_with_the_transpose():
    """A^T u must equal the product with the explicitly transposed matrix,
    bit for bit (same terms, same order)."""
    a, A = _tiny_csr(7, m=30, n=17, dens=0.3)
    u = np.random.default_rng(1).standard_normal(30)
    w1 = oracle.apply_t(A, u)
    w2 = oracle.apply(csr_from_dense(a.T.copy()), u)
    w3 = oracle.apply_t(a, u)
    assert np.array_equal(w1, w2) and np.array_equal(w1, w3)


def test_dense_and_csr_agree_bitwise():
    a, A = _tiny_csr(3, m=40, n=25, dens=1.0)
    A_full = csr_from_dense(a, keep_zeros=True)
    x = np.random.default_rng(2).standard_normal(25)
    assert np.array_equal(oracle.apply(a, x), oracle.apply(A_full, x))


# --------------------------------------------------------------------------
# the auxiliary equation: closed forms of Example 1, least squares
# --------------------------------------------------------------------------
def _phis(H, r, t):
    # phi_i = r^T H^i r by repeated products (numpy, plain)
    out = []
    v = r.copy()
    for _ in range(2 * t):
        v = H @ v
        out.append(float(r @ v))
    return np.array(out)


def test_gram_t1_closed_form():
    """Example 1: alpha_{1,1} = phi_1 / phi_2 exactly."""
    for phi1, phi2 in [(3.0, 7.0), (1e-30, 3e-29), (2.5e10, 1.25e21)]:
        a, te = oracle.gram_alpha([phi1, phi2], 1)
        assert te == 1 and a[0] == phi1 / phi2


@pytest.mark.parametrize("seed", range(5))
def test_gram_t2_matches_example1_cramer(seed):
    """Example 1: alpha_{2,1} = (phi1 phi4 - phi2 phi3) / (phi2 phi4 - phi3^2),
    alpha_{2,2} = (phi2^2 - phi1 phi3) / (phi2 phi4 - phi3^2)."""
    g = np.random.default_rng(seed)
    lam = g.uniform(0.5, 3.0, 6)
    r = g.standard_normal(6)
    H = np.diag(lam)
    p1, p2, p3, p4 = _phis(H, r, 2)
    det = p2 * p4 - p3 * p3
    a21 = (p1 * p4 - p2 * p3) / det
    a22 = (p2 * p2 - p1 * p3) / det
    a, te = oracle.gram_alpha([p1, p2, p3, p4], 2)
    assert te == 2
    assert a[0] == pytest.approx(a21, rel=1e-11)
    assert a[1] == pytest.approx(a22, rel=1e-11)


@pytest.mark.parametrize("t", [2, 3, 4])
def test_gram_solves_the_least_squares_problem(t):
    """alpha = argmin ||r - sum alpha_i H^i r|| (the definition of alpha_t(r))."""
    g = np.random.default_rng(t)
    m = 12
    B = g.standard_normal((m, m))
    H = B @ B.T / m + 0.3 * np.eye(m)
    r = g.standard_normal(m)
    K = np.stack([np.linalg.matrix_power(H, i) @ r for i in range(1, t + 1)], axis=1)
    a_ls = np.linalg.lstsq(K, r, rcond=None)[0]
    a, te = oracle.gram_alpha(_phis(H, r, t), t)
    assert te == t
    res_ls = np.linalg.norm(r - K @ a_ls)
    res = np.linalg.norm(r - K @ a)
    assert res <= res_ls * (1 + 1e-8) + 1e-12 * np.linalg.norm(r)


def test_gram_singular_gives_the_optimal_residual():
    """r has only two eigen-components, so the 3x3 Hankel matrix is singular;
    any least-squares alpha (the paper picks the minimum-norm one) gives the
    same new residual, which is zero (minimal polynomial of degree 2)."""
    lam = np.array([1.0, 2.0, 5.0, 7.0])
    H = np.diag(lam)
    r = np.array([1.0, 0.0, 2.0, 0.0])
    a, te = oracle.gram_alpha(_phis(H, r, 3), 3)
    K = np.stack([np.linalg.matrix_power(H, i) @ r for i in range(1, 4)], axis=1)
    assert np.linalg.norm(r - K @ a) <= 1e-7 * np.linalg.norm(r)
    a_pinv = np.linalg.pinv(K) @ r
    assert np.linalg.norm(K @ (a - a_pinv)) <= 1e-7


def test_gram_truncates_when_krylov_vector_vanishes():
    a, te = oracle.gram_alpha([1.0, 2.0, 0.0, 0.0, 0.0, 0.0], 3)
    assert te == 1 and a[0] == 0.5 and a[1] == 0 and a[2] == 0
    a, te = oracle.gram_alpha([0.0] * 6, 3)
    assert te == 0 and not a.any()


# --------------------------------------------------------------------------
# CTA trajectories: paper theorems and textbook equivalences
# --------------------------------------------------------------------------
def _critical_line_cases():
    with open(os.path.join(GOLDEN, "critical_line.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _critical_line_cases(), ids=lambda c: f"{c['lam_i']}-{c['lam_j']}")
def test_cta1_critical_line_zigzag(case):
    """Theorem (dynamics of F_1) (iv): on an ij-critical line the residual norm
    shrinks by exactly rho_ij per step and alternates between r+ and r-."""
    li, lj = case["lam_i"], case["lam_j"]
    A = np.diag([math.sqrt(li), math.sqrt(lj)])  # H = A A^T = diag(li, lj)
    ai, aj = math.sqrt(lj / (li + lj)), math.sqrt(li / (li + lj))
    b = np.array([ai, aj])  # r+ (unit norm)
    K = len(case["expected_rel_res"]) - 1
    x, hist, info = oracle.cta(A, b, tol=0.0, t=1, max_iter=K)
    assert info.iters == K
    np.testing.assert_allclose(hist, case["expected_rel_res"], rtol=1e-12, atol=0)
    r = oracle.residual(A, b, x)
    sign = -1.0 if K % 2 else 1.0
    np.testing.assert_allclose(r, case["expected_rel_res"][-1] * np.array([ai, sign * aj]),
                               rtol=1e-9, atol=1e-15)


def test_cta1_eigenvector_converges_in_one_step():
    """Theorem (dynamics) (iii): an eigenvector of H is solved in one step."""
    g = np.random.default_rng(5)
    A = g.standard_normal((8, 8))
    Uu, s, Vt = np.linalg.svd(A)
    b = 3.0 * Uu[:, 2]  # eigenvector of H = A A^T
    x, hist, info = oracle.cta(A, b, tol=1e-12, t=1, max_iter=5)
    assert info.stop == "residual" and info.iters == 1


@pytest.mark.parametrize("m,spread,floor", [(2, "lin", 1e-10), (3, "lin", 1e-10), (4, "lin", 1e-8),
                                             (6, "sqrt", 1e-5)])
def test_finite_termination_at_minimal_polynomial_degree(m, spread, floor):
    """Theorem 2 (ii): F_s(r0) = 0 for a solvable system when s is the degree of
    the minimal polynomial of r0 with respect to H (here s = m).  Exact in exact
    arithmetic; in FP64 the monomial Krylov basis makes the Hankel system
    ill-conditioned as t grows, which leaves a floor (a wrong term leaves O(1))."""
    g = np.random.default_rng(m)
    Q = np.linalg.qr(g.standard_normal((m, m)))[0]
    sv = np.linspace(1.0, 2.0, m) if spread == "lin" else np.sqrt(np.arange(1.0, m + 1))
    A = Q @ np.diag(sv)
    b = g.standard_normal(m)
    x, hist, info = oracle.cta(A, b, tol=1e-9, t=m, max_iter=1)
    assert hist[1] <= floor
    # one order less leaves a clearly nonzero residual
    x, hist, info = oracle.cta(A, b, tol=1e-9, t=m - 1, max_iter=1)
    assert hist[1] > 100 * floor


def test_finite_termination_inconsistent_gives_normal_solution():
    """Theorem 2 (iii): for an unsolvable system F_s(r0) != 0 but A^T F_s(r0) = 0."""
    A = np.array([[1.0, 0.0], [0.0, 2.0], [0.0, 0.0]])
    b = np.array([1.0, 1.0, 1.0])
    x, hist, info = oracle.cta(A, b, tol=1e-12, t=2, max_iter=1)
    np.testing.assert_allclose(x, [1.0, 0.5], rtol=1e-12)
    assert hist[1] == pytest.approx(1 / math.sqrt(3), rel=1e-12)
    assert info.rel_normal <= 1e-11


@pytest.mark.parametrize("t", [1, 2, 3])
def test_cta_equals_restarted_gmres_on_AAt(t):
    """One CTA-t iteration with H = A A^T is one restart cycle of GMRES(t) on
    A A^T y = b with x = A^T y (both minimise ||b - H y|| over the same
    Krylov space), so the residual histories coincide."""
    g = np.random.default_rng(10 + t)
    m, n = 30, 40
    A = g.standard_normal((m, n))
    b = g.standard_normal(m)
    H = A @ A.T
    K = 12
    x, hist, info = oracle.cta(A, b, tol=0.0, t=t, max_iter=K)
    y = np.zeros(m)
    nb = np.linalg.norm(b)
    ref = [1.0]
    for _ in range(K):
        y, _ = spla.gmres(H, b, x0=y, restart=t, maxiter=1, rtol=0.0, atol=0.0)
        ref.append(np.linalg.norm(b - H @ y) / nb)
    np.testing.assert_allclose(hist, ref, rtol=1e-8)
    np.testing.assert_allclose(x, A.T @ y, rtol=1e-6, atol=1e-9 * np.linalg.norm(x))


@pytest.mark.parametrize("t", [1, 2, 3])
def test_cta_residual_history_nonincreasing(t):
    p = convection_diffusion(8)
    x, hist, info = oracle.cta(p.A, p.b, tol=1e-8, t=t, max_iter=3000)
    assert np.all(hist[1:] <= hist[:-1] * (1 + 1e-13))


def test_cta_min_norm_on_rank_deficient_consistent():
    """Theorem 1 (4): from x0 = 0 the iterates stay in range(A^T) and tend to
    the minimum-norm solution pinv(A) b."""
    g = np.random.default_rng(3)
    A = g.standard_normal((8, 5)) @ g.standard_normal((5, 12))  # rank 5
    b = A @ g.standard_normal(12)
    xp = np.linalg.pinv(A) @ b
    sv = np.linalg.svd(A, compute_uv=False)
    smin = sv[sv > 1e-10 * sv[0]].min()
    Vt = np.linalg.svd(A)[2]
    Pnull = Vt[5:].T @ Vt[5:]
    for minnorm in (False, True):
        x, hist, info = oracle.cta(A, b, tol=1e-10, t=2, max_iter=200000, minnorm=minnorm)
        assert info.stop == "residual"
        assert np.linalg.norm(Pnull @ x) <= 1e-12 * np.linalg.norm(x)
        bound = info.rel_res * np.linalg.norm(b) / smin
        assert np.linalg.norm(x - xp) <= 2 * bound + 1e-13 * np.linalg.norm(xp)


def test_cta_inconsistent_reaches_normal_equation():
    """Theorem 1: A^T b - A^T A x_k -> 0 even when A x = b is unsolvable."""
    g = np.random.default_rng(4)
    A = g.standard_normal((12, 6))
    b = g.standard_normal(12)
    x, hist, info = oracle.cta(A, b, tol=1e-6, tol_normal=1e-9, t=2, max_iter=100000)
    assert info.stop == "normal"
    xl = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.linalg.norm(x - xl) <= 1e-6 * np.linalg.norm(xl)


def test_cta_pinv_limit_dense_gaussian():
    p = dense_gaussian(12, seed=4)
    x, hist, info = oracle.cta(p.A, p.b, tol=1e-10, t=2, max_iter=500000)
    assert info.stop == "residual" and info.rel_res <= 1e-10
    sv = np.linalg.svd(p.A, compute_uv=False)
    bound = info.rel_res * np.linalg.norm(p.b) / sv[-1]
    assert np.linalg.norm(x - np.linalg.pinv(p.A) @ p.b) <= 2 * bound


def test_cta_kac_min_norm():
    """Kac N=101 is singular and consistent; the limit is pinv(A) b."""
    p = kac_clement(101)
    a = p.A.to_dense()
    x, hist, info = oracle.cta(p.A, p.b, tol=1e-10, t=3, max_iter=100000)
    assert info.stop == "residual"
    xp = np.linalg.pinv(a) @ p.b
    sv = np.linalg.svd(a, compute_uv=False)
    smin = sv[sv > 1e-9 * sv[0]].min()
    assert np.linalg.norm(x - xp) <= 2 * info.rel_res * np.linalg.norm(p.b) / smin


def test_cta_minnorm_lp_shaped_small():
    p = lp_shaped(60, 900, seed=2)
    a = p.A.to_dense()
    x, hist, info = oracle.cta_minnorm(p.A, p.b, tol=1e-12, t=3, max_iter=2000)
    assert info.stop == "residual"
    xp = np.linalg.pinv(a) @ p.b
    assert np.linalg.norm(x - xp) <= 1e-9 * np.linalg.norm(xp)


def test_cta_zero_rhs_and_budget():
    p = kac_clement(11)
    x, hist, info = oracle.cta(p.A, np.zeros(11), tol=1e-6, t=3)
    assert info.stop == "residual" and info.iters == 0 and not x.any()
    x, hist, info = oracle.cta(p.A, p.b, tol=1e-14, t=1, max_iter=3)
    assert info.stop == "maxiter" and info.iters == 3 and hist.size == 4


def test_cta_warm_start_resumes_the_same_trajectory():
    """CTA is memoryless: stopping after k iterations and restarting from x_k
    continues the same residual sequence (x-form)."""
    p = convection_diffusion(8)
    x1, h1, _ = oracle.cta(p.A, p.b, tol=0.0, t=2, max_iter=40)
    xa, ha, _ = oracle.cta(p.A, p.b, tol=0.0, t=2, max_iter=25)
    xb, hb, _ = oracle.cta(p.A, p.b, tol=0.0, t=2, max_iter=15, x0=xa)
    # the restart recomputes r = b - A x, so agreement is to rounding only
    np.testing.assert_allclose(hb, h1[25:41], rtol=1e-6)
    np.testing.assert_allclose(xb, x1, rtol=1e-6, atol=1e-9)


# --------------------------------------------------------------------------
# generators: closed-form spectra
# --------------------------------------------------------------------------
def test_kac_spectrum():
    for N in (5, 8, 11):
        a = kac_clement(N).A.to_dense()
        ev = np.sort(np.linalg.eigvals(a).real)
        np.testing.assert_allclose(ev, np.arange(-(N - 1), N, 2), atol=1e-8)


def test_convdiff_spectrum():
    """Kronecker sum of two tridiagonal Toeplitz matrices:
    lambda_jk = 4 - 2 sqrt(1 - (g h / 2)^2) (cos(j pi h) + cos(k pi h))."""
    N, gam = 6, 10.0
    h = 1 / (N + 1)
    a = convection_diffusion(N, gam).A.to_dense()
    ev = np.sort(np.linalg.eigvals(a).real)
    c = math.sqrt(1 - (gam * h / 2) ** 2)
    ref = np.sort([4 - 2 * c * (math.cos(j * math.pi * h) + math.cos(k * math.pi * h))
                   for j in range(1, N + 1) for k in range(1, N + 1)])
    np.testing.assert_allclose(ev, ref, atol=1e-10)
    p = poisson5(5).to_dense()
    assert np.allclose(p, p.T) and np.all(np.linalg.eigvalsh(p) > 0)


# --------------------------------------------------------------------------
# TA: hand-solved cases, Frank-Wolfe equivalence, witness bound
# --------------------------------------------------------------------------
def test_ta_scalar_case_by_hand():
    """1x1 system a x = b from rho = 0: the first iteration is a radius update
    to |b|/|a| (a witness at b' = 0), the second a full step to b' = b."""
    x, hist, info = oracle.ta(np.array([[4.0]]), np.array([3.0]), tol=1e-15, max_iter=10)
    assert info.stop == "residual" and info.iters == 2
    assert x[0] == 0.75 and info.rho == 0.75 and info.rho_lo == 0.75
    np.testing.assert_array_equal(hist, [1.0, 1.0, 0.0])


def test_ta_radius_tie_is_a_strict_pivot():
    """11 x = 15 from rho = 0: the radius update sets rho = (b-b')^T b / ||c|| =
    fl(225/165), and then rho ||c|| = fl(fl(15/11) * 165) < 225 in floating
    point although equality holds exactly.  Theorem prop0TA (3) makes equality
    a strict pivot, so the second iteration is a full step (alpha = 1): two
    iterations, rho = fl(15/11).  Treating the tie as a failed pivot test
    would double rho and take a third iteration."""
    rho = 225.0 / 165.0
    assert rho * 165.0 < 225.0  # the tie is decided by rounding here
    x, hist, info = oracle.ta(np.array([[11.0]]), np.array([15.0]), tol=1e-15, max_iter=10)
    assert info.stop == "residual" and info.iters == 2
    assert info.rho == rho
    assert x[0] == pytest.approx(15.0 / 11.0, rel=1e-15)


def _frank_wolfe(A, b, rho, K):
    """Conditional gradient with exact line search for min 1/2||Ax-b||^2 over
    the ball ||x|| <= rho (linear minimisation oracle rho g/||g|| with
    g = A^T (b - A x))."""
    x = np.zeros(A.shape[1])
    hist = [1.0]
    nb = np.linalg.norm(b)
    for _ in range(K):
        res = b - A @ x
        g = A.T @ res
        s = rho * g / np.linalg.norm(g)
        dvec = A @ (s - x)
        lam = min(max((res @ dvec) / (dvec @ dvec), 0.0), 1.0)
        x = x + lam * (s - x)
        hist.append(np.linalg.norm(b - A @ x) / nb)
    return x, np.array(hist)


def test_ta_fixed_radius_is_frank_wolfe():
    g = np.random.default_rng(8)
    A = g.standard_normal((10, 14))
    b = A @ g.standard_normal(14)
    rho = 2.0 * np.linalg.norm(np.linalg.pinv(A) @ b)  # b is inside E_{A,rho}
    K = 60
    x, hist, info = oracle.ta(A, b, tol=0.0, max_iter=K, rho0=rho, fixed_rho=True)
    assert info.stop == "maxiter"
    xf, hf = _frank_wolfe(A, b, rho, K)
    np.testing.assert_allclose(hist, hf, rtol=1e-7)
    np.testing.assert_allclose(x, xf, rtol=1e-6, atol=1e-9)
    assert np.linalg.norm(x) <= rho * (1 + 1e-12)


def test_ta_witness_lower_bound():
    """Algorithm 2 with rho < ||x*|| must end at a witness, and Corollary 1
    gives (b-b')^T b / ||A^T (b-b')|| < ||x*||."""
    g = np.random.default_rng(9)
    A = g.standard_normal((8, 8))
    b = A @ g.standard_normal(8)
    nx = np.linalg.norm(np.linalg.solve(A, b))
    x, hist, info = oracle.ta(A, b, tol=1e-12, max_iter=100000, rho0=0.5 * nx, fixed_rho=True)
    assert info.stop == "witness"
    assert 0 < info.rho_lo < nx
    assert np.linalg.norm(x) <= 0.5 * nx * (1 + 1e-12)


def test_ta_alg3_solves_and_bounds():
    g = np.random.default_rng(11)
    A = g.standard_normal((6, 9))
    b = A @ g.standard_normal(9)
    x, hist, info = oracle.ta(A, b, tol=1e-6, max_iter=2000000)
    assert info.stop == "residual" and info.rel_res <= 1e-6
    xs = np.linalg.pinv(A) @ b
    assert info.rho_lo < np.linalg.norm(xs)  # every radius update used a witness
    assert np.linalg.norm(x) <= info.rho * (1 + 1e-12)
    assert np.all(hist[1:] <= hist[:-1] * (1 + 1e-13))


def test_ta_normal_equation_stop_on_inconsistent():
    A = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    b = np.array([1.0, 2.0, 3.0])
    x, hist, info = oracle.ta(A, b, tol=1e-9, tol_normal=1e-9, max_iter=100000)
    assert info.stop == "normal"
    np.testing.assert_allclose(x, [1.0, 2.0], rtol=1e-8)
