"""CPU oracle for the TA / CTA solvers (ctypes wrapper over ``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU library never does, and
this package never imports the GPU library.

The arithmetic lives in ``oracle.c`` (plain sequential FP64 C).  This module
only marshals numpy arrays and builds the shared object with gcc.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STOP_NAMES = {0: "none", 1: "residual", 2: "normal", 3: "witness", 4: "maxiter", 5: "breakdown"}


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Mat(C.Structure):
    _fields_ = [("kind", C.c_int32), ("m", C.c_int64), ("n", C.c_int64), ("ld", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("tol_normal", C.c_double), ("t", C.c_int32),
                ("max_iter", C.c_int64), ("replace_every", C.c_int32), ("warm_start", C.c_int32),
                ("rho0", C.c_double), ("fixed_rho", C.c_int32), ("h_is_a", C.c_int32),
                ("t_cycle", C.c_int32), ("nonneg", C.c_int32), ("rho_max", C.c_double),
                ("enhanced", C.c_int32), ("normal_eq", C.c_int32), ("accel", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int64), ("matvecs", C.c_int64), ("stop", C.c_int32),
                ("rel_res", C.c_double), ("rel_normal", C.c_double), ("rho", C.c_double),
                ("rho_lo", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.or_dot2.restype = C.c_double
        lib.or_dot2.argtypes = [C.c_int64, P, P]
        lib.or_apply.argtypes = [C.POINTER(_Mat), P, P]
        lib.or_apply_t.argtypes = [C.POINTER(_Mat), P, P]
        lib.or_residual.argtypes = [C.POINTER(_Mat), P, P, P]
        lib.or_gram_alpha.restype = C.c_int
        lib.or_gram_alpha.argtypes = [P, C.c_int, P]
        lib.or_cta.restype = C.c_int
        lib.or_cta.argtypes = [C.POINTER(_Mat), P, P, C.POINTER(_Opts), C.c_int, P, C.c_int64,
                               C.POINTER(_Info)]
        lib.or_csr_outer.argtypes = [C.POINTER(_Mat), P, P, C.c_double, P]
        lib.or_ta.restype = C.c_int
        lib.or_ta.argtypes = [C.POINTER(_Mat), P, P, C.POINTER(_Opts), P, C.c_int64,
                              C.POINTER(_Info)]
        lib.or_ta_minnorm.restype = C.c_int64
        lib.or_ta_minnorm.argtypes = [C.POINTER(_Mat), P, P, P, C.POINTER(_Opts),
                                      C.POINTER(_Info)]
        lib.or_ta_halving.restype = C.c_int
        lib.or_ta_halving.argtypes = [C.POINTER(_Mat), P, P, C.POINTER(_Opts), C.c_int32,
                                      C.POINTER(_Info), C.POINTER(C.c_int32)]
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class _MatRef:
    """Keeps the numpy buffers alive while the C struct points at them."""

    def __init__(self, A):
        if isinstance(A, np.ndarray):
            a = _f64(A)
            self.keep = (a,)
            self.s = _Mat(0, a.shape[0], a.shape[1], a.shape[1], None, None, _ptr(a).value)
            self.m, self.n = a.shape
        else:
            rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
            ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
            v = _f64(A.val)
            self.keep = (rp, ci, v)
            self.s = _Mat(1, A.m, A.n, 0, _ptr(rp).value, _ptr(ci).value, _ptr(v).value)
            self.m, self.n = A.m, A.n


@dataclasses.dataclass
class Info:
    iters: int
    matvecs: int
    stop: str
    rel_res: float
    rel_normal: float
    rho: float
    rho_lo: float


def _info(i: _Info) -> Info:
    return Info(int(i.iters), int(i.matvecs), STOP_NAMES.get(int(i.stop), str(i.stop)),
                float(i.rel_res), float(i.rel_normal), float(i.rho), float(i.rho_lo))


def dot2(x, y) -> float:
    """Compensated dot product (Ogita-Rump-Oishi Dot2), terms in index order."""
    x, y = _f64(x), _f64(y)
    return float(_load().or_dot2(x.size, _ptr(x), _ptr(y)))


def apply(A, x) -> np.ndarray:
    """y = A x with a compensated sum per row."""
    M = _MatRef(A)
    x = _f64(x)
    y = np.empty(M.m)
    _load().or_apply(C.byref(M.s), _ptr(x), _ptr(y))
    return y


def apply_t(A, u) -> np.ndarray:
    """w = A^T u with a compensated sum per column (rows taken in order)."""
    M = _MatRef(A)
    u = _f64(u)
    w = np.empty(M.n)
    _load().or_apply_t(C.byref(M.s), _ptr(u), _ptr(w))
    return w


def residual(A, b, x) -> np.ndarray:
    """r = b - A x as one compensated sum per row."""
    M = _MatRef(A)
    b, x = _f64(b), _f64(x)
    r = np.empty(M.m)
    _load().or_residual(C.byref(M.s), _ptr(b), _ptr(x), _ptr(r))
    return r


def gram_alpha(phi, t: int):
    """Step coefficients from phi_1..phi_2t (``phi[0]`` is phi_1)."""
    p = np.zeros(2 * t + 1)
    p[1:2 * t + 1] = np.asarray(phi, dtype=np.float64)[:2 * t]
    a = np.zeros(t)
    te = _load().or_gram_alpha(_ptr(p), int(t), _ptr(a))
    return a, int(te)


def _opts(tol, tol_normal, t, max_iter, replace_every, warm_start, rho0, fixed_rho,
          h_is_a=False, t_cycle=False, nonneg=False, rho_max=0.0, enhanced=False,
          normal_eq=False, accel=0.0):
    return _Opts(float(tol), float(tol_normal), int(t), int(max_iter), int(replace_every),
                 int(warm_start), float(rho0), int(fixed_rho), int(bool(h_is_a)),
                 int(bool(t_cycle)), int(bool(nonneg)), float(rho_max), int(bool(enhanced)),
                 int(bool(normal_eq)), float(accel))


def cta(A, b, tol=1e-6, t=3, max_iter=100000, tol_normal=0.0, replace_every=0,
        x0: Optional[np.ndarray] = None, minnorm=False, hist_cap: Optional[int] = None,
        h_is_a=False, t_cycle=False, enhanced=False, accel=0.0):
    """Algorithm 1 (CTA, H = A A^T; with h_is_a, H = A for a square symmetric
    positive semidefinite A, x-form only; with t_cycle, the order of
    iteration k cycles 1, 2, ..., t, ..., 2, 1, ...; with enhanced, the
    enhanced stop of section 3.2 on the j-fold first-order iterates; with accel
    = theta in (0, 1), the convex-combination step of the first-order dynamics
    theorem whenever ||r_{k+1}|| >= theta ||r_k||).  Returns (x, hist, info)."""
    if h_is_a:
        mm, nn = A.shape if isinstance(A, np.ndarray) else (A.m, A.n)
        if minnorm or mm != nn:
            raise ValueError("H = A takes a square A and the x-form")
    M = _MatRef(A)
    b = _f64(b)
    cap = int(max_iter) + 1 if hist_cap is None else int(hist_cap)
    hist = np.full(max(cap, 1), np.nan)
    x = np.zeros(M.n) if x0 is None else _f64(x0).copy()
    o = _opts(tol, tol_normal, t, max_iter, replace_every, x0 is not None, 0.0, 0, h_is_a,
              t_cycle, enhanced=enhanced, accel=accel)
    inf = _Info()
    rc = _load().or_cta(C.byref(M.s), _ptr(b), _ptr(x), C.byref(o), int(bool(minnorm)),
                        _ptr(hist), cap, C.byref(inf))
    if rc != 0:
        raise ValueError("oracle cta: invalid arguments")
    info = _info(inf)
    return x, hist[:min(info.iters + 1, cap)], info


def cta_minnorm(A, b, **kw):
    return cta(A, b, minnorm=True, **kw)


def ta(A, b, tol=1e-6, max_iter=100000, tol_normal=0.0, rho0=0.0, fixed_rho=False,
       hist_cap: Optional[int] = None, x0: Optional[np.ndarray] = None, nonneg=False,
       rho_max=0.0, normal_eq=False):
    """Algorithm 3 (or Algorithm 2 with ``fixed_rho``), from x0 (b' = A x0) if
    given, else from 0; with ``nonneg``, the LP-feasibility form (x >= 0, c
    replaced by c+) and an optional radius bound ``rho_max``; with
    ``normal_eq``, on A^T A x = A^T b (the products are A^T (A v); the exit
    diagnostics stay on (A, b)).  Returns (x, hist, info)."""
    M = _MatRef(A)
    b = _f64(b)
    cap = int(max_iter) + 1 if hist_cap is None else int(hist_cap)
    hist = np.full(max(cap, 1), np.nan)
    x = np.zeros(M.n) if x0 is None else _f64(x0).copy()
    o = _opts(tol, tol_normal, 1, max_iter, 0, x0 is not None, rho0, fixed_rho,
              nonneg=nonneg, rho_max=rho_max, normal_eq=normal_eq)
    inf = _Info()
    _load().or_ta(C.byref(M.s), _ptr(b), _ptr(x), C.byref(o), _ptr(hist), cap, C.byref(inf))
    info = _info(inf)
    return x, hist[:min(info.iters + 1, cap)], info


def ta_halving(A, b, tol=1e-6, tol_normal=0.0, max_halvings=20, max_iter=100000, rho0=0.0,
               fixed_rho=False, x0: Optional[np.ndarray] = None):
    """Algorithm 3 restarted with eps' halved each time it ends on the normal
    equation (the remark after the theorem on its properties, section 4.3),
    at most ``max_halvings`` times; eps' starts at ``tol_normal``, or at tol
    when 0.  Returns (x, info, halvings): iterations and products summed over
    the runs, the rest of info from the last run."""
    M = _MatRef(A)
    b = _f64(b)
    x = np.zeros(M.n) if x0 is None else _f64(x0).copy()
    o = _opts(tol, tol_normal, 1, max_iter, 0, x0 is not None, rho0, fixed_rho)
    inf = _Info()
    h = C.c_int32(0)
    rc = _load().or_ta_halving(C.byref(M.s), _ptr(b), _ptr(x), C.byref(o), int(max_halvings),
                               C.byref(inf), C.byref(h))
    if rc != 0:
        raise RuntimeError(f"or_ta_halving: {rc}")
    return x, _info(inf), int(h.value)


def csr_outer(A, u, v, alpha=1.0) -> np.ndarray:
    """out[k] = (alpha u_i) v_j for the k-th stored entry (i, j) of a CSR A."""
    M = _MatRef(A)
    if M.s.kind != 1:
        raise ValueError("csr_outer takes a CSR matrix")
    u, v = _f64(u), _f64(v)
    out = np.empty(len(A.val))
    _load().or_csr_outer(C.byref(M.s), _ptr(u), _ptr(v), float(alpha), _ptr(out))
    return out


def cta_grad(A, b, dldx_of_x, tol=1e-12, t=3, max_iter=100000):
    """Forward solve and adjoint gradient of a loss of x(A, b) = A^{-1} b for a
    square nonsingular CSR A (not in the paper; the derivative of the solution
    map).  Algorithm 1 solves A x = b, then A^T lambda = dL/dx on the
    transposed CSR (built with scipy), and the gradient is dL/db = lambda,
    dL/da_ij = -lambda_i x_j on the stored pattern.  dldx_of_x maps x to dL/dx.
    Returns (x, lambda, grad_vals, info_forward, info_adjoint)."""
    import scipy.sparse as sps

    sp = sps.csr_matrix((np.asarray(A.val, np.float64), np.asarray(A.col_idx),
                         np.asarray(A.row_ptr)), shape=(A.m, A.n))
    At = sp.T.tocsr()
    At.sort_indices()

    class _T:
        pass

    T = _T()
    T.m, T.n = A.n, A.m
    T.row_ptr = At.indptr.astype(np.int32)
    T.col_idx = At.indices.astype(np.int32)
    T.val = At.data.astype(np.float64)
    x, _, fi = cta(A, b, tol=tol, t=t, max_iter=max_iter, hist_cap=1)
    g = np.asarray(dldx_of_x(x), dtype=np.float64)
    lam, _, ai = cta(T, g, tol=tol, t=t, max_iter=max_iter, hist_cap=1)
    return x, lam, csr_outer(A, lam, x, -1.0), fi, ai


def ta_minnorm(A, b, x_eps, tol=1e-6, max_iter=100000, tol_normal=0.0, normal_eq=False):
    """Algorithm 4: from an approximate solution x_eps, bisect on the radius
    with Algorithm 2 tests (on A^T A x = A^T b with ``normal_eq``).  Returns
    (x, info, tests); info.rho and info.rho_lo are the final upper and lower
    bounds on the norm."""
    M = _MatRef(A)
    b, xe = _f64(b), _f64(x_eps)
    x = np.zeros(M.n)
    o = _opts(tol, tol_normal, 1, max_iter, 0, 0, 0.0, False, normal_eq=normal_eq)
    inf = _Info()
    tests = _load().or_ta_minnorm(C.byref(M.s), _ptr(b), _ptr(xe), _ptr(x), C.byref(o),
                                   C.byref(inf))
    return x, _info(inf), int(tests)
