"""Pins of the oracle's enhanced stop (section 3.2: for t >= 2, the j-fold
first-order iterates F_1^j(r), j < t, are tested as well, and the first that
passes the normal-equation test ends the solve at x^).

The expected values come from an eigen-decomposition of H, where a
first-order step acts coordinate-wise: f <- f (1 - a lambda) with
a = sum lambda f^2 / sum lambda^2 f^2 (Example 1's order-1 step).  The test
quantity is ||A^T f||^2 = sum lambda f^2 for H = A A^T and ||A f||^2 =
sum lambda^2 f^2 for H = A.  The tolerance is placed just above or just below
these values, so a wrong index, step or test quantity in the oracle moves its
stop."""
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def _first_order_chain(lam, V, r, steps, h_is_a=False):
    """f_0 = r, f_j = F_1(f_{j-1}) in the eigenbasis of H = V diag(lam) V^T.
    Returns the iterates (original basis), the steps a_j and the test values
    sqrt(f_j^T H f_j) (H = A A^T) or ||A f_j|| (H = A)."""
    c = V.T @ r
    fs, steps_a, tests = [V @ c], [], []
    for _ in range(steps):
        a = np.sum(lam * c * c) / np.sum(lam * lam * c * c)
        c = c * (1.0 - a * lam)
        steps_a.append(a)
        fs.append(V @ c)
        q = np.sum(lam * lam * c * c) if h_is_a else np.sum(lam * c * c)
        tests.append(np.sqrt(max(q, 0.0)))
    return fs, steps_a, tests


def _tall(seed, m=14, n=10):
    g = np.random.default_rng(seed)
    return g.standard_normal((m, n)), g.standard_normal(m)


def test_t2_window_at_j1():
    """t = 2: the only extra iterate is f_1 = F_1(b).  With the tolerance just
    above its test value the solve stops after one iteration at x^ = a_1 A^T b;
    just below, it does not."""
    A, b = _tall(0)
    lam, V = np.linalg.eigh(A @ A.T)
    fs, a, q = _first_order_chain(lam, V, b, 1)
    nab = np.linalg.norm(A.T @ b)
    x, hist, info = oracle.cta(A, b, tol=1e-12, t=2, max_iter=50,
                               tol_normal=1.001 * q[0] / nab, enhanced=True)
    assert info.stop == "normal" and info.iters == 1
    np.testing.assert_allclose(x, a[0] * (A.T @ b), rtol=1e-12)
    np.testing.assert_allclose(hist[1], np.linalg.norm(fs[1]) / np.linalg.norm(b), rtol=1e-10)
    # just below: no extra iterate passes, so the run is plain CTA-2's
    kw = dict(tol=1e-12, t=2, max_iter=50, tol_normal=0.999 * q[0] / nab)
    x2, h2, info2 = oracle.cta(A, b, enhanced=True, **kw)
    x3, h3, info3 = oracle.cta(A, b, **kw)
    assert info2 == info3 and np.array_equal(x2, x3) and np.array_equal(h2, h3)
    assert not np.allclose(x2, a[0] * (A.T @ b), rtol=1e-6)


def _seed_with_window(make, lam_of, steps):
    """First seed whose test values fall strictly (q_2 < q_1 / 2), so that a
    tolerance between them selects j = 2."""
    for seed in range(200):
        A, b = make(seed)
        lam, V = lam_of(A)
        fs, a, q = _first_order_chain(lam, V, b, steps, h_is_a=make is _spd_case)
        if q[1] < 0.5 * q[0]:
            return seed, A, b, fs, a, q
    raise AssertionError("no seed with a window")


def test_t3_stops_at_j2_x_and_y_form():
    seed, A, b, fs, a, q = _seed_with_window(_tall, lambda A: np.linalg.eigh(A @ A.T), 2)
    nab = np.linalg.norm(A.T @ b)
    tol_ne = np.sqrt(q[0] * q[1]) / nab  # between the j = 2 and j = 1 values
    xh = A.T @ (a[0] * fs[0] + a[1] * fs[1])
    x, hist, info = oracle.cta(A, b, tol=1e-12, t=3, max_iter=50, tol_normal=tol_ne,
                               enhanced=True)
    assert info.stop == "normal" and info.iters == 1, (seed, info)
    np.testing.assert_allclose(x, xh, rtol=1e-11)
    assert info.rel_normal <= tol_ne * (1 + 1e-8)
    xy, _, infoy = oracle.cta_minnorm(A, b, tol=1e-12, t=3, max_iter=50, tol_normal=tol_ne,
                                      enhanced=True)
    assert infoy.stop == "normal" and infoy.iters == 1
    np.testing.assert_allclose(xy, xh, rtol=1e-11)


def _spd_case(seed, n=12):
    g = np.random.default_rng(100 + seed)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    lam = np.concatenate([np.geomspace(1.0, 30.0, n - 3), np.zeros(3)])  # singular PSD
    return (Q * lam) @ Q.T, g.standard_normal(n)


def test_h_a_stops_at_j2():
    """H = A (symmetric PSD, singular, b not in its range): the test quantity
    is ||A f_j|| and x^ = x + sum a_i f_{i-1}."""
    seed, A, b, fs, a, q = _seed_with_window(_spd_case, np.linalg.eigh, 2)
    nab = np.linalg.norm(A @ b)
    tol_ne = np.sqrt(q[0] * q[1]) / nab
    x, _, info = oracle.cta(A, b, tol=1e-12, t=3, max_iter=50, tol_normal=tol_ne,
                            enhanced=True, h_is_a=True)
    assert info.stop == "normal" and info.iters == 1, (seed, info)
    np.testing.assert_allclose(x, a[0] * fs[0] + a[1] * fs[1], rtol=1e-11)


@pytest.mark.parametrize("t", [2, 3, 4])
def test_without_a_hit_the_run_is_plain_cta(t):
    """A tolerance no iterate reaches: every number equals plain CTA's."""
    A, b = _tall(7)
    kw = dict(tol=1e-10, t=t, max_iter=40, tol_normal=1e-13)
    x0, h0, i0 = oracle.cta(A, b, **kw)
    x1, h1, i1 = oracle.cta(A, b, enhanced=True, **kw)
    assert i0 == i1
    assert np.array_equal(x0, x1) and np.array_equal(h0, h1)


def test_t1_has_no_extra_iterates():
    A, b = _tall(3)
    kw = dict(tol=1e-10, t=1, max_iter=30, tol_normal=0.5)
    assert oracle.cta(A, b, **kw)[2] == oracle.cta(A, b, enhanced=True, **kw)[2]
