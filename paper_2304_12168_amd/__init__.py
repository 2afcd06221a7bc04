"""MI355X (gfx950) Triangle Algorithm / Centering Triangle Algorithm solvers.

Thin ctypes binding over ``libta.so`` (C ABI declared in ``include/ta.h``).
This module only marshals arguments: every step of a solve runs in the HIP
kernels of the library.  PyTorch provides device memory and the stream.
There is no CPU fallback: if the library is missing, importing the solver
entry points raises.

Methods: Lau & Kalantari, arXiv 2304.12168 -- CTA (Algorithm 1, H = A A^T)
and TA (Algorithms 2 and 3).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libta.so")

TA_DENSE_ROWMAJOR = 0
TA_CSR = 1
TA_FP64, TA_FP32, TA_BF16 = 0, 1, 2
STOP_NAMES = {0: "none", 1: "residual", 2: "normal", 3: "witness", 4: "maxiter", 5: "breakdown"}
ERRORS = {-1: "TA_EINVAL", -2: "TA_ENOMEM", -3: "TA_EHIP", -4: "TA_ENOTSUP", -5: "TA_ESCRATCH"}

# every symbol the header declares
EXPORTS = ("cta_solve", "cta_minnorm", "ta_solve", "ta_validate", "ta_strerror", "ta_spmv",
           "ta_residual", "ta_transpose", "ta_time_matvec", "ta_plan_create", "ta_plan_destroy",
           "cta_solve_plan", "cta_minnorm_plan", "ta_solve_plan", "ta_time_matvec_plan",
           "ta_spmv_plan", "ta_batch_plan_create", "ta_batch_plan_destroy", "cta_solve_batched",
           "ta_batch_time_spmm", "ta_csr_outer", "ta_minnorm", "ta_minnorm_plan", "ta_plan_format",
           "cta_solve_plan_noalloc", "ta_solve_halving")
# storage of a plan's products (ta_plan_format)
FORMATS = {0: "csr_rows", 1: "dense_rows", 2: "dense_cols", 3: "csr_sliced", 4: "sell64",
           5: "csr_tiled", 6: "csr_merge"}


class TaMat(C.Structure):
    _fields_ = [("kind", C.c_int32), ("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("ld", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("val", C.c_void_p)]


class TaOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("tol_normal", C.c_double), ("t", C.c_int32),
                ("max_iter", C.c_int64), ("precision", C.c_int32), ("replace_every", C.c_int32),
                ("warm_start", C.c_int32), ("rho0", C.c_double), ("fixed_rho", C.c_int32),
                ("chunk", C.c_int32), ("launch_mode", C.c_int32), ("h_mode", C.c_int32),
                ("t_cycle", C.c_int32), ("nonneg", C.c_int32), ("rho_max", C.c_double),
                ("enhanced", C.c_int32), ("normal_eq", C.c_int32), ("accel", C.c_double)]


class TaInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("matvecs", C.c_int64), ("stop", C.c_int32),
                ("rel_res", C.c_double), ("rel_normal", C.c_double), ("rho", C.c_double),
                ("rho_lo", C.c_double)]


class TaError(RuntimeError):
    pass


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libta.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise TaError(f"{path} not found: build it with `python -m paper_2304_12168_amd.build`")
        lib = C.CDLL(path)
        P, I64, I32 = C.c_void_p, C.c_int64, C.c_int32
        MP, OP, IP = C.POINTER(TaMat), C.POINTER(TaOpts), C.POINTER(TaInfo)
        for name in ("cta_solve", "cta_minnorm", "ta_solve"):
            f = getattr(lib, name)
            f.restype = C.c_int
            f.argtypes = [MP, P, P, OP, P, I64, IP, P]
        for name in ("cta_solve_plan", "cta_minnorm_plan", "ta_solve_plan",
                     "cta_solve_plan_noalloc"):
            f = getattr(lib, name)
            f.restype = C.c_int
            f.argtypes = [P, P, P, OP, P, I64, IP, P]
        lib.ta_plan_create.restype = C.c_int
        lib.ta_plan_create.argtypes = [MP, C.POINTER(C.c_void_p), P]
        lib.ta_plan_destroy.restype = C.c_int
        lib.ta_plan_destroy.argtypes = [P]
        lib.ta_plan_format.restype = C.c_int
        lib.ta_plan_format.argtypes = [P, I32, C.POINTER(C.c_int32)]
        lib.ta_batch_plan_create.restype = C.c_int
        lib.ta_batch_plan_create.argtypes = [I32, P, I32, C.POINTER(C.c_void_p), P]
        lib.ta_batch_plan_destroy.restype = C.c_int
        lib.ta_batch_plan_destroy.argtypes = [P]
        lib.ta_batch_time_spmm.restype = C.c_int
        lib.ta_batch_time_spmm.argtypes = [P, I32, I32, I32, I32, C.POINTER(C.c_double), P]
        lib.cta_solve_batched.restype = C.c_int
        lib.cta_solve_batched.argtypes = [P, P, P, P, OP, I32, P, P]
        lib.ta_spmv_plan.restype = C.c_int
        lib.ta_spmv_plan.argtypes = [P, I32, P, P, P, P]
        lib.ta_time_matvec_plan.restype = C.c_int
        lib.ta_time_matvec_plan.argtypes = [P, I32, P, P, I32, C.POINTER(C.c_double), P]
        lib.ta_validate.restype = C.c_int
        lib.ta_validate.argtypes = [MP, OP, I32]
        lib.ta_strerror.restype = C.c_char_p
        lib.ta_strerror.argtypes = [C.c_int]
        lib.ta_spmv.restype = C.c_int
        lib.ta_spmv.argtypes = [MP, I32, P, P, P, P]
        lib.ta_residual.restype = C.c_int
        lib.ta_residual.argtypes = [MP, P, P, P, P, P]
        lib.ta_transpose.restype = C.c_int
        lib.ta_transpose.argtypes = [MP, P, P, P, P]
        for name in ("ta_minnorm", "ta_minnorm_plan"):
            f = getattr(lib, name)
            f.restype = C.c_int
            f.argtypes = [P if name.endswith("plan") else MP, P, P, P, OP, IP,
                          C.POINTER(C.c_int64), P]
        lib.ta_solve_halving.restype = C.c_int
        lib.ta_solve_halving.argtypes = [P, P, P, OP, I32, IP, C.POINTER(C.c_int32), P]
        lib.ta_csr_outer.restype = C.c_int
        lib.ta_csr_outer.argtypes = [MP, P, P, C.c_double, P, P]
        lib.ta_time_matvec.restype = C.c_int
        lib.ta_time_matvec.argtypes = [MP, I32, P, P, I32, C.POINTER(C.c_double), P]
        _lib = lib
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = load_library().ta_strerror(rc).decode()
        raise TaError(f"{what}: {ERRORS.get(rc, rc)}: {msg}")


# ---------------------------------------------------------------------------
# device matrices
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class DeviceMatrix:
    """A matrix resident in device memory (torch tensors) plus its descriptor."""

    kind: int
    m: int
    n: int
    nnz: int
    ld: int
    row_ptr: Optional[object] = None  # torch.int32, m+1
    col_idx: Optional[object] = None  # torch.int32, nnz
    val: Optional[object] = None      # torch.float64, nnz or (m, ld)

    def desc(self) -> TaMat:
        def ptr(t):
            return None if t is None else t.data_ptr()

        return TaMat(self.kind, self.m, self.n, self.nnz, self.ld, ptr(self.row_ptr),
                     ptr(self.col_idx), ptr(self.val))

    @property
    def shape(self):
        return (self.m, self.n)


def to_device(A, device="cuda") -> DeviceMatrix:
    """Copy a host matrix (dense numpy array, or any object with m, n, row_ptr,
    col_idx, val as numpy arrays) to the GPU."""
    import torch

    if isinstance(A, DeviceMatrix):
        return A
    if isinstance(A, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float64)).to(device)
        m, n = a.shape
        return DeviceMatrix(TA_DENSE_ROWMAJOR, m, n, m * n, n, val=a)
    rp = torch.from_numpy(np.ascontiguousarray(A.row_ptr, dtype=np.int32)).to(device)
    ci = torch.from_numpy(np.ascontiguousarray(A.col_idx, dtype=np.int32)).to(device)
    v = torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float64)).to(device)
    return DeviceMatrix(TA_CSR, int(A.m), int(A.n), int(v.numel()), 0, rp, ci, v)


def _vec(v, device="cuda"):
    import torch

    if isinstance(v, np.ndarray):
        return torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(device)
    if v.dtype != torch.float64 or not v.is_contiguous():
        raise TaError("vectors must be contiguous float64 tensors")
    return v


def _stream():
    import torch

    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclasses.dataclass
class Info:
    iters: int
    matvecs: int
    stop: str
    rel_res: float
    rel_normal: float
    rho: float
    rho_lo: float


def _info(i: TaInfo) -> Info:
    return Info(int(i.iters), int(i.matvecs), STOP_NAMES.get(int(i.stop), str(i.stop)),
                float(i.rel_res), float(i.rel_normal), float(i.rho), float(i.rho_lo))


def make_opts(tol=1e-6, t=3, max_iter=100000, tol_normal=0.0, replace_every=0, warm_start=False,
              rho0=0.0, fixed_rho=False, chunk=0, precision=TA_FP64, graph=True,
              h_is_a=False, t_cycle=False, nonneg=False, rho_max=0.0,
              enhanced=False, normal_eq=False, accel=0.0) -> TaOpts:
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    return TaOpts(float(tol), float(tol_normal), int(t), int(max_iter), int(precision),
                  int(replace_every), int(bool(warm_start)), float(rho0), int(bool(fixed_rho)),
                  int(chunk), 0 if graph else 1, 1 if h_is_a else 0, 1 if t_cycle else 0,
                  1 if nonneg else 0, float(rho_max), 1 if enhanced else 0,
                  1 if normal_eq else 0, float(accel))


class Plan:
    """A prepared operator (ta_plan): A^T and, for long rows, the LDS column
    tiles or the XCD column slices of A (or A^T); for short even rows, SELL-64
    copies of A and A^T.  Built once on the device.  Keeps the matrix alive."""

    def __init__(self, A):
        lib = load_library()
        self.A = to_device(A)
        self._desc = self.A.desc()
        h = C.c_void_p()
        _check(lib.ta_plan_create(C.byref(self._desc), C.byref(h), _stream()), "ta_plan_create")
        self.handle = h

    @property
    def m(self):
        return self.A.m

    def format(self, trans: bool = False) -> str:
        """Storage the products of A (or A^T) use: a FORMATS value."""
        f = C.c_int32(-1)
        _check(load_library().ta_plan_format(self.handle, int(bool(trans)), C.byref(f)),
               "ta_plan_format")
        return FORMATS[f.value]

    @property
    def n(self):
        return self.A.n

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load_library().ta_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan(A) -> Plan:
    return Plan(A)


def _solve(name, A, b, x0=None, hist_cap=None, **kw):
    import torch

    lib = load_library()
    if isinstance(A, Plan):
        return _solve_plan(name, A, b, x0=x0, hist_cap=hist_cap, **kw)
    dA = to_device(A)
    bd = _vec(b)
    opts = make_opts(**kw)
    x = torch.zeros(dA.n, dtype=torch.float64, device=bd.device)
    if x0 is not None:
        x.copy_(_vec(x0))
    cap = int(opts.max_iter) + 1 if hist_cap is None else int(hist_cap)
    hist = torch.full((max(cap, 1),), float("nan"), dtype=torch.float64, device=bd.device)
    info = TaInfo()
    d = dA.desc()
    rc = getattr(lib, name)(C.byref(d), C.c_void_p(bd.data_ptr()), C.c_void_p(x.data_ptr()),
                            C.byref(opts), C.c_void_p(hist.data_ptr()), cap, C.byref(info),
                            _stream())
    _check(rc, name)
    inf = _info(info)
    return x, hist[: min(inf.iters + 1, cap)], inf


def _solve_plan(name, pl, b, x0=None, hist_cap=None, _suffix="_plan", **kw):
    import torch

    lib = load_library()
    bd = _vec(b)
    opts = make_opts(**kw)
    x = torch.zeros(pl.n, dtype=torch.float64, device=bd.device)
    if x0 is not None:
        x.copy_(_vec(x0))
    cap = int(opts.max_iter) + 1 if hist_cap is None else int(hist_cap)
    hist = torch.full((max(cap, 1),), float("nan"), dtype=torch.float64, device=bd.device)
    info = TaInfo()
    rc = getattr(lib, name + _suffix)(pl.handle, C.c_void_p(bd.data_ptr()),
                                      C.c_void_p(x.data_ptr()), C.byref(opts),
                                      C.c_void_p(hist.data_ptr()), cap, C.byref(info), _stream())
    _check(rc, name + _suffix)
    inf = _info(info)
    return x, hist[: min(inf.iters + 1, cap)], inf


def cta_solve(A, b, tol=1e-6, t=3, max_iter=100000, x0=None, **kw):
    """Algorithm 1 (CTA of order t, H = A A^T), from x0 if given (warm start),
    else from 0.  Returns (x, hist, info)."""
    return _solve("cta_solve", A, b, x0=x0, tol=tol, t=t, max_iter=max_iter,
                  warm_start=x0 is not None, **kw)


def cta_solve_noalloc(pl: "Plan", b, tol=1e-6, t=3, max_iter=100000, x0=None, **kw):
    """cta_solve on a prepared operator through ``cta_solve_plan_noalloc``:
    the library takes its workspace from a fixed per-GPU device buffer and
    allocates nothing (the output tensors here are allocated by torch, as for
    every binding call).  Returns (x, hist, info)."""
    if not isinstance(pl, Plan):
        raise TaError("cta_solve_noalloc takes a Plan")
    return _solve_plan("cta_solve", pl, b, x0=x0, tol=tol, t=t, max_iter=max_iter,
                       warm_start=x0 is not None, _suffix="_plan_noalloc", **kw)


def cta_minnorm(A, b, tol=1e-6, t=3, max_iter=100000, **kw):
    """Algorithm 1 in the form x = A^T y (minimum-norm limit).  Returns (x, hist, info)."""
    return _solve("cta_minnorm", A, b, tol=tol, t=t, max_iter=max_iter, **kw)


def ta_solve(A, b, tol=1e-6, max_iter=100000, rho0=0.0, fixed_rho=False, x0=None, **kw):
    """Algorithm 3 (or Algorithm 2 with ``fixed_rho``), from x0 (b' = A x0) if
    given, else from 0.  Returns (x, hist, info)."""
    return _solve("ta_solve", A, b, x0=x0, tol=tol, t=1, max_iter=max_iter, rho0=rho0,
                  fixed_rho=fixed_rho, warm_start=x0 is not None, **kw)


def validate(A, solver: int = 0, **kw) -> int:
    """Host-side argument checks only (no device access).  Returns the code."""
    lib = load_library()
    if isinstance(A, TaMat):
        d = A
    elif isinstance(A, DeviceMatrix):
        d = A.desc()
    else:
        raise TaError("validate takes a TaMat or a DeviceMatrix")
    o = make_opts(**kw)
    return int(lib.ta_validate(C.byref(d), C.byref(o), int(solver)))


def spmv(A, x, trans: bool = False, want_norm: bool = False):
    """y = A x or A^T x (FP64, compensated rows).  Returns y (and ||y||^2)."""
    import torch

    lib = load_library()
    xd = _vec(x)
    if isinstance(A, Plan):
        y = torch.empty(A.n if trans else A.m, dtype=torch.float64, device=xd.device)
        nrm = torch.zeros(1, dtype=torch.float64, device=xd.device) if want_norm else None
        rc = lib.ta_spmv_plan(A.handle, int(bool(trans)), C.c_void_p(xd.data_ptr()),
                              C.c_void_p(y.data_ptr()),
                              C.c_void_p(nrm.data_ptr() if nrm is not None else 0), _stream())
        _check(rc, "ta_spmv_plan")
        return (y, nrm) if want_norm else y
    dA = to_device(A)
    y = torch.empty(dA.n if trans else dA.m, dtype=torch.float64, device=xd.device)
    nrm = torch.zeros(1, dtype=torch.float64, device=xd.device) if want_norm else None
    d = dA.desc()
    rc = lib.ta_spmv(C.byref(d), int(bool(trans)), C.c_void_p(xd.data_ptr()),
                     C.c_void_p(y.data_ptr()), C.c_void_p(nrm.data_ptr() if nrm is not None else 0),
                     _stream())
    _check(rc, "ta_spmv")
    return (y, nrm) if want_norm else y


def residual(A, b, x, want_norm: bool = False):
    """r = b - A x (FP64, one compensated sum per row)."""
    import torch

    lib = load_library()
    dA = to_device(A)
    bd, xd = _vec(b), _vec(x)
    r = torch.empty(dA.m, dtype=torch.float64, device=bd.device)
    nrm = torch.zeros(1, dtype=torch.float64, device=bd.device) if want_norm else None
    d = dA.desc()
    rc = lib.ta_residual(C.byref(d), C.c_void_p(bd.data_ptr()), C.c_void_p(xd.data_ptr()),
                         C.c_void_p(r.data_ptr()),
                         C.c_void_p(nrm.data_ptr() if nrm is not None else 0), _stream())
    _check(rc, "ta_residual")
    return (r, nrm) if want_norm else r


def transpose(A):
    """CSR of A^T built on the device: (row_ptr, col_idx, val) tensors."""
    import torch

    lib = load_library()
    dA = to_device(A)
    dev = dA.val.device
    rp = torch.empty(dA.n + 1, dtype=torch.int32, device=dev)
    ci = torch.empty(max(dA.nnz, 1), dtype=torch.int32, device=dev)
    v = torch.empty(max(dA.nnz, 1), dtype=torch.float64, device=dev)
    d = dA.desc()
    rc = lib.ta_transpose(C.byref(d), C.c_void_p(rp.data_ptr()), C.c_void_p(ci.data_ptr()),
                          C.c_void_p(v.data_ptr()), _stream())
    _check(rc, "ta_transpose")
    return rp, ci[: dA.nnz], v[: dA.nnz]


def ta_minnorm(A, b, x_eps, tol=1e-6, max_iter=100000, **kw):
    """Algorithm 4 from an approximate solution x_eps.  Returns (x, info,
    tests); info.rho and info.rho_lo are the final upper and lower bounds on
    the norm of the minimum-norm solution."""
    import torch

    lib = load_library()
    bd, xe = _vec(b), _vec(x_eps)
    opts = make_opts(tol=tol, max_iter=max_iter, **kw)
    info = TaInfo()
    tests = C.c_int64(0)
    if isinstance(A, Plan):
        x = torch.zeros(A.n, dtype=torch.float64, device=bd.device)
        rc = lib.ta_minnorm_plan(A.handle, C.c_void_p(bd.data_ptr()), C.c_void_p(xe.data_ptr()),
                                 C.c_void_p(x.data_ptr()), C.byref(opts), C.byref(info),
                                 C.byref(tests), _stream())
        _check(rc, "ta_minnorm_plan")
    else:
        dA = to_device(A)
        d = dA.desc()
        x = torch.zeros(dA.n, dtype=torch.float64, device=bd.device)
        rc = lib.ta_minnorm(C.byref(d), C.c_void_p(bd.data_ptr()), C.c_void_p(xe.data_ptr()),
                            C.c_void_p(x.data_ptr()), C.byref(opts), C.byref(info),
                            C.byref(tests), _stream())
        _check(rc, "ta_minnorm")
    return x, _info(info), int(tests.value)


def ta_solve_halving(plan, b, tol=1e-6, tol_normal=0.0, max_halvings=20, max_iter=100000,
                     **kw):
    """TA restarted with eps' halved after each stop on the normal equation
    (ta_solve_halving), on a Plan.  Returns (x, info, halvings)."""
    import torch

    lib = load_library()
    if not isinstance(plan, Plan):
        raise TypeError("ta_solve_halving takes a Plan")
    bd = _vec(b)
    x = torch.zeros(plan.n, dtype=torch.float64, device=bd.device)
    opts = make_opts(tol=tol, tol_normal=tol_normal, max_iter=max_iter, **kw)
    info = TaInfo()
    h = C.c_int32(0)
    rc = lib.ta_solve_halving(plan.handle, C.c_void_p(bd.data_ptr()), C.c_void_p(x.data_ptr()),
                              C.byref(opts), int(max_halvings), C.byref(info), C.byref(h),
                              _stream())
    _check(rc, "ta_solve_halving")
    return x, _info(info), int(h.value)


def csr_outer(A, u, v, alpha: float = 1.0):
    """out[k] = (alpha u_i) v_j for the k-th stored entry (i, j) of a CSR A."""
    import torch

    lib = load_library()
    dA = to_device(A)
    ud, vd = _vec(u), _vec(v)
    out = torch.empty(max(dA.nnz, 1), dtype=torch.float64, device=ud.device)
    d = dA.desc()
    rc = lib.ta_csr_outer(C.byref(d), C.c_void_p(ud.data_ptr()), C.c_void_p(vd.data_ptr()),
                          float(alpha), C.c_void_p(out.data_ptr()), _stream())
    _check(rc, "ta_csr_outer")
    return out[: dA.nnz]


def time_matvec(A, x, trans: bool = False, reps: int = 50) -> float:
    """Average milliseconds of one launch of the solvers' FP64 product kernel(s)."""
    import torch

    lib = load_library()
    xd = _vec(x)
    ms = C.c_double(0.0)
    if isinstance(A, Plan):
        y = torch.empty(A.n if trans else A.m, dtype=torch.float64, device=xd.device)
        rc = lib.ta_time_matvec_plan(A.handle, int(bool(trans)), C.c_void_p(xd.data_ptr()),
                                     C.c_void_p(y.data_ptr()), int(reps), C.byref(ms), _stream())
    else:
        dA = to_device(A)
        y = torch.empty(dA.n if trans else dA.m, dtype=torch.float64, device=xd.device)
        d = dA.desc()
        rc = lib.ta_time_matvec(C.byref(d), int(bool(trans)), C.c_void_p(xd.data_ptr()),
                                C.c_void_p(y.data_ptr()), int(reps), C.byref(ms), _stream())
    _check(rc, "ta_time_matvec")
    return float(ms.value)


PRECISIONS = {"fp64": TA_FP64, "fp32": TA_FP32, "bf16": TA_BF16}


class BatchPlan:
    """Block-diagonal operator over several systems (ta_batch_plan), all CSR or
    all dense, with low-precision copies of the values for ``precision``
    'fp32' or 'bf16'.  Dense systems run their products on the matrix cores."""

    def __init__(self, systems, precision: str = "fp64"):
        lib = load_library()
        self.systems = [to_device(A) for A in systems]
        kinds = {d.kind for d in self.systems}
        if len(kinds) != 1:
            raise TaError("a batch holds CSR systems or dense systems, not both")
        self.dense = kinds == {TA_DENSE_ROWMAJOR}
        self.precision = PRECISIONS[precision]
        descs = (TaMat * len(self.systems))(*[d.desc() for d in self.systems])
        h = C.c_void_p()
        _check(lib.ta_batch_plan_create(len(self.systems), descs, self.precision, C.byref(h),
                                        _stream()), "ta_batch_plan_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load_library().ta_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cta_solve_batched(plan: BatchPlan, B, tol=1e-6, t=3, max_iter=100000, minnorm=False,
                      precision: str = "fp64", **kw):
    """Solve every column of every B[s] (an (m_s, k_s) float64 tensor or
    array) with CTA.  Returns (X, infos): X[s] is (n_s, k_s), infos[s] a list
    of Info per column."""
    import torch

    lib = load_library()
    S = len(plan.systems)
    if len(B) != S:
        raise TaError("one right-hand-side block per system")
    cols, xs, ks = [], [], []
    for d, b in zip(plan.systems, B):
        bt = b if isinstance(b, torch.Tensor) else torch.from_numpy(np.asarray(b, dtype=np.float64))
        if bt.dim() == 1:
            bt = bt[:, None]
        bt = bt.to(device="cuda", dtype=torch.float64)
        k = int(bt.shape[1])
        cm = bt.t().contiguous()  # (k, m) storage = column-major m x k
        cols.append(cm)
        xs.append(torch.zeros((k, d.n), dtype=torch.float64, device=cm.device))
        ks.append(k)
    nrhs = (C.c_int32 * S)(*ks)
    bp = (C.c_void_p * S)(*[c.data_ptr() for c in cols])
    xp = (C.c_void_p * S)(*[x.data_ptr() for x in xs])
    opts = make_opts(tol=tol, t=t, max_iter=max_iter, precision=PRECISIONS[precision], **kw)
    total = max(sum(ks), 1)
    infos = (TaInfo * total)()
    rc = lib.cta_solve_batched(plan.handle, nrhs, bp, xp, C.byref(opts), int(bool(minnorm)),
                               infos, _stream())
    _check(rc, "cta_solve_batched")
    out_info, i = [], 0
    for k in ks:
        out_info.append([_info(infos[i + c]) for c in range(k)])
        i += k
    return [x.t() for x in xs], out_info


def batch_time_spmm(plan: BatchPlan, K: int, trans: bool = False, precision: str = "fp64",
                    reps: int = 20) -> float:
    """Average milliseconds of one launch of the batched SpMM kernel."""
    lib = load_library()
    ms = C.c_double(0.0)
    rc = lib.ta_batch_time_spmm(plan.handle, int(K), int(bool(trans)), PRECISIONS[precision],
                                int(reps), C.byref(ms), _stream())
    _check(rc, "ta_batch_time_spmm")
    return float(ms.value)
