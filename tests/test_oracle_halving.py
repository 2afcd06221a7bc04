"""Pins of the oracle's restarted TA (the remark after the theorem on
Algorithm 3's properties, section 4.3: halve eps' and restart from the
current approximate solution when a run ends on the normal equation).  On
consistent Kac-Clement systems, where plain TA with eps' = eps ends on the
normal equation first, the restarted runs reach the residual test, checked
on the true residual computed here with numpy; without halvings it is plain
TA; and one halving is plain TA followed by a warm-started run with eps'/2."""
import numpy as np
import pytest

import oracle
from workloads import kac_clement


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


@pytest.mark.parametrize("N", [101, 301])
@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_restarts_reach_the_residual_test(N, tol):
    p = kac_clement(N)
    _, _, plain = oracle.ta(p.A, p.b, tol=tol, tol_normal=tol, max_iter=200_000)
    assert plain.stop == "normal"  # the case the remark is about
    x, info, h = oracle.ta_halving(p.A, p.b, tol=tol, max_iter=200_000)
    assert info.stop == "residual" and h >= 1
    r = np.linalg.norm(p.b - p.A.to_scipy() @ x)
    assert r <= tol * np.linalg.norm(p.b) * (1 + 1e-12)


def test_no_halving_is_plain_ta():
    p = kac_clement(101)
    x0, _, i0 = oracle.ta(p.A, p.b, tol=1e-6, tol_normal=1e-6, max_iter=200_000)
    x1, i1, h = oracle.ta_halving(p.A, p.b, tol=1e-6, max_halvings=0, max_iter=200_000)
    assert h == 0 and np.array_equal(x0, x1)
    assert (i0.stop, i0.iters, i0.matvecs) == (i1.stop, i1.iters, i1.matvecs)


def test_one_halving_is_a_warm_restart_with_half_eps():
    p = kac_clement(101)
    xa, _, ia = oracle.ta(p.A, p.b, tol=1e-6, tol_normal=1e-6, max_iter=200_000)
    xb, _, ib = oracle.ta(p.A, p.b, tol=1e-6, tol_normal=0.5e-6, max_iter=200_000, x0=xa)
    x, info, h = oracle.ta_halving(p.A, p.b, tol=1e-6, max_halvings=1, max_iter=200_000)
    assert h == 1 and np.array_equal(x, xb)
    assert (info.iters, info.matvecs, info.stop) == (ia.iters + ib.iters, ia.matvecs + ib.matvecs,
                                                     ib.stop)
