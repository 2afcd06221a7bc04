"""Differentiable CTA solve: x(A, b) with a hand-written adjoint.

Not in the paper.  For a square nonsingular A the limit of Algorithm 1 is
x = A^{-1} b (Theorem 1 (4), range(A^T) = R^n), and a loss L(x) has

    dL/db = lambda,    dL/da_ij = -lambda_i x_j,    A^T lambda = dL/dx.

The forward solve and the adjoint solve are CTA solves through the C ABI:
``cta_solve`` in FP64, or the batched engine with FP32 / BF16 products and
FP64 refinement.  A^T is built on the device (``ta_transpose``) and the
gradient of A's stored values is the sparse-pattern outer product
``ta_csr_outer``.  Every step runs in the library's kernels; this module only
wires them into ``torch.autograd``.

The formulas above hold at the solution only: a forward or adjoint solve that
stops short of the tolerance (iteration budget, normal-equation stop,
breakdown) yields an x and a gradient that are not those of x(A, b), so such
a stop raises ``TaError`` unless the caller passes ``allow_unconverged=True``
(for timing runs to a fixed budget, whose gradients carry no guarantee).
"""
from __future__ import annotations

from typing import List, Optional

from . import (TA_CSR, BatchPlan, DeviceMatrix, Info, TaError, csr_outer, cta_solve,
               cta_solve_batched, to_device, transpose)


def _check(stage, info, allow):
    if info.stop != "residual" and not allow:
        raise TaError(f"cta_solve_diff: the {stage} solve stopped with '{info.stop}' at relative "
                      f"residual {info.rel_res:.3e}; its x and gradient are not those of the "
                      f"solution map (pass allow_unconverged=True to accept them)")


def _solve(A: DeviceMatrix, b, tol, t, max_iter, precision):
    if precision == "fp64":
        x, _, info = cta_solve(A, b, tol=tol, t=t, max_iter=max_iter, hist_cap=1)
        return x, info
    plan = BatchPlan([A], precision)
    try:
        X, infos = cta_solve_batched(plan, [b.reshape(-1, 1)], tol=tol, t=t, max_iter=max_iter,
                                     precision=precision)
    finally:
        plan.close()
    return X[0][:, 0].contiguous(), infos[0][0]


def _make_fn():
    import torch

    class CTASolve(torch.autograd.Function):
        """x = CTA solve of A x = b, differentiable in A's stored values and b."""

        @staticmethod
        def forward(ctx, vals, b, row_ptr, col_idx, m, n, opts):
            tol, t, max_iter, precision, log, allow = opts
            A = DeviceMatrix(TA_CSR, m, n, int(vals.numel()), 0, row_ptr, col_idx,
                             vals.detach().contiguous())
            x, info = _solve(A, b.detach().contiguous(), tol, t, max_iter, precision)
            if log is not None:
                log.append(("forward", info))
            _check("forward", info, allow)
            ctx.save_for_backward(vals.detach(), x)
            ctx.struct = (row_ptr, col_idx, m, n)
            ctx.opts = opts
            return x

        @staticmethod
        def backward(ctx, gx):
            vals, x = ctx.saved_tensors
            row_ptr, col_idx, m, n = ctx.struct
            tol, t, max_iter, precision, log, allow = ctx.opts
            A = DeviceMatrix(TA_CSR, m, n, int(vals.numel()), 0, row_ptr, col_idx,
                             vals.contiguous())
            trp, tci, tval = transpose(A)
            AT = DeviceMatrix(TA_CSR, n, m, int(vals.numel()), 0, trp, tci, tval)
            lam, info = _solve(AT, gx.contiguous(), tol, t, max_iter, precision)
            if log is not None:
                log.append(("adjoint", info))
            _check("adjoint", info, allow)
            gvals = csr_outer(A, lam, x, -1.0) if ctx.needs_input_grad[0] else None
            gb = lam if ctx.needs_input_grad[1] else None
            return gvals, gb, None, None, None, None, None

    return CTASolve


_FN = None


def cta_solve_diff(A, vals, b, tol: float = 1e-8, t: int = 3, max_iter: int = 100000,
                   precision: str = "fp64", log: Optional[List] = None,
                   allow_unconverged: bool = False):
    """x(A, b) for a square CSR A whose stored values are the tensor ``vals``
    (float64, device, nnz entries, in A's storage order); differentiable in
    ``vals`` and ``b``.  ``A`` supplies the sparsity pattern (a host CSR or a
    DeviceMatrix).  ``precision`` 'fp64' uses cta_solve; 'fp32' / 'bf16' the
    batched engine's low-precision products with FP64 refinement.  If ``log``
    is a list, (stage, Info) pairs of the forward and adjoint solves are
    appended to it.  A solve that does not reach ``tol`` raises TaError unless
    ``allow_unconverged``."""
    global _FN
    if _FN is None:
        _FN = _make_fn()
    dA = to_device(A)
    if dA.kind != TA_CSR or dA.m != dA.n:
        raise TaError("cta_solve_diff takes a square CSR matrix")
    if int(vals.numel()) != dA.nnz:
        raise TaError("vals must hold one entry per stored entry of A")
    return _FN.apply(vals, b, dA.row_ptr, dA.col_idx, dA.m, dA.n,
                     (float(tol), int(t), int(max_iter), precision, log,
                      bool(allow_unconverged)))


__all__ = ["cta_solve_diff", "Info"]
