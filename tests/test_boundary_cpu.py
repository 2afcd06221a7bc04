"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol the header declares, and its host-only validation rejects bad input."""
import ctypes as C
import os
import re

import pytest

import paper_2304_12168_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "ta.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB_PATH):
        import paper_2304_12168_amd.build as B

        B.build()
    return P.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert set(names) == set(P.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -5, -99):
        assert isinstance(lib.ta_strerror(code), bytes)


def _csr_desc(m=10, n=8, nnz=20):
    return P.TaMat(P.TA_CSR, m, n, nnz, 0, 0x1000, 0x2000, 0x3000)


def test_validate_accepts_good_arguments(lib):
    assert P.validate(_csr_desc(), 0, t=3) == 0
    assert P.validate(_csr_desc(), 1, t=8) == 0
    assert P.validate(_csr_desc(), 2) == 0
    assert P.validate(_csr_desc(), 2, rho0=1.5, fixed_rho=True) == 0
    dense = P.TaMat(P.TA_DENSE_ROWMAJOR, 5, 4, 20, 4, None, None, 0x1000)
    assert P.validate(dense, 0, t=2) == 0


@pytest.mark.parametrize("kw", [dict(t=0), dict(t=9), dict(t=11), dict(tol=1.0), dict(tol=-1e-3),
                                dict(tol=float("nan")), dict(max_iter=-1),
                                dict(tol_normal=2.0), dict(replace_every=-2),
                                dict(precision=7)])
def test_validate_rejects_bad_options(lib, kw):
    assert P.validate(_csr_desc(), 0, **kw) == -1


def test_validate_rejects_bad_matrices(lib):
    assert P.validate(P.TaMat(5, 3, 3, 0, 0, 0x1, 0x1, 0x1), 0, t=1) == -1  # kind
    assert P.validate(P.TaMat(P.TA_CSR, -1, 3, 0, 0, 0x1, 0x1, 0x1), 0, t=1) == -1
    assert P.validate(P.TaMat(P.TA_CSR, 3, 3, 4, 0, None, 0x1, 0x1), 0, t=1) == -1  # row_ptr
    assert P.validate(P.TaMat(P.TA_CSR, 3, 3, 4, 0, 0x1, None, 0x1), 0, t=1) == -1  # col_idx
    assert P.validate(P.TaMat(P.TA_DENSE_ROWMAJOR, 3, 4, 12, 3, None, None, 0x1), 0, t=1) == -1
    assert P.validate(P.TaMat(P.TA_CSR, 2, 3, 4, 0, 0x1, 0x1, 0x1), 0, t=3) == -1  # t > m


def test_minnorm_rejects_warm_start_and_ta_fixed_rho_needs_radius(lib):
    assert P.validate(_csr_desc(), 1, t=2, warm_start=True) == -1
    assert P.validate(_csr_desc(), 2, fixed_rho=True, rho0=0.0) == -1
    assert P.validate(_csr_desc(), 2, rho0=float("inf")) == -1


def test_null_descriptor(lib):
    o = P.make_opts()
    assert lib.ta_validate(None, C.byref(o), 0) == -1


def test_validate_variant_options(lib):
    import ctypes

    sq = _csr_desc(m=8, n=8)
    rect = _csr_desc(m=3, n=5)
    assert P.validate(sq, 0, t=3, h_is_a=True) == 0
    assert P.validate(rect, 0, t=2, h_is_a=True) == -1   # H = A needs a square A
    assert P.validate(sq, 1, t=2, h_is_a=True) == -1     # x-form only
    assert P.validate(sq, 2, h_is_a=True) == -1          # not for TA
    assert P.validate(rect, 0, t=3, t_cycle=True) == 0
    assert P.validate(rect, 1, t=3, t_cycle=True) == 0
    assert P.validate(rect, 2, t_cycle=True) == -1       # TA has no order
    assert P.validate(rect, 0, t=3, enhanced=True) == 0
    assert P.validate(rect, 1, t=3, enhanced=True) == 0
    assert P.validate(sq, 0, t=3, enhanced=True, h_is_a=True) == 0
    assert P.validate(rect, 2, enhanced=True) == -1      # a CTA stop
    assert P.validate(rect, 2, normal_eq=True) == 0      # TA on the normal equation
    assert P.validate(rect, 0, t=2, normal_eq=True) == -1  # a TA input form
    assert P.validate(rect, 1, t=2, normal_eq=True) == -1
    assert P.validate(rect, 0, t=3, accel=0.5) == 0
    assert P.validate(rect, 1, t=1, accel=0.9) == 0
    assert P.validate(sq, 0, t=2, accel=0.5, h_is_a=True) == 0
    assert P.validate(rect, 2, accel=0.5) == -1          # a CTA step
    assert P.validate(rect, 0, t=2, accel=1.0) == -1     # theta in [0, 1)
    assert P.validate(rect, 0, t=2, accel=-0.1) == -1
    assert P.validate(rect, 0, t=2, accel=float("nan")) == -1
    oe = P.make_opts(t=3)
    oe.enhanced = 2
    assert lib.ta_validate(ctypes.byref(rect), ctypes.byref(oe), 0) == -1
    o = P.make_opts(t=3)
    o.launch_mode = 2
    assert lib.ta_validate(ctypes.byref(sq), ctypes.byref(o), 0) == -1


def test_validate_precision_per_solver(lib):
    """FP32 / BF16 products are a CTA option (one-shot solves and batched);
    TA computes in FP64 only; the per-iteration CTA options need FP64."""
    d = _csr_desc()
    for prec in (P.TA_FP32, P.TA_BF16, "fp32", "bf16"):
        assert P.validate(d, 0, t=3, precision=prec) == 0
        assert P.validate(d, 1, t=3, precision=prec) == 0
        assert P.validate(d, 2, precision=prec) == -1
        for kw in (dict(warm_start=True), dict(replace_every=4), dict(t_cycle=True),
                   dict(enhanced=True), dict(accel=0.5)):
            assert P.validate(d, 0, t=3, precision=prec, **kw) == -1, kw
    assert P.validate(_csr_desc(m=8, n=8), 0, t=3, precision="fp32", h_is_a=True) == -1


def test_strerror_of_every_code(lib):
    for code, name in P.ERRORS.items():
        assert lib.ta_strerror(code).decode() != "unknown error", name
