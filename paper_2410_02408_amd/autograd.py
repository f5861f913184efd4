"""Differentiable block-Jacobi PCG solve (adjoint backward).

``pcg_solve_diff(values, b, pattern, block_size)`` returns x = A^-1 b for
the CSR matrix with the given pattern and ``values``.  Its backward is the
adjoint: one more PCG solve with the same preconditioner and right-hand side
dL/dx gives lambda = A^-1 dL/dx (A symmetric), so

    dL/db      = lambda
    dL/dvalues = -lambda_i x_j on every stored entry (i, j)   (bjp_value_grad)

Both solves and the gradient gather run in the library's kernels; torch only
routes the tensors.  Values must describe a symmetric matrix; the gradient is
that of the stored entries taken as independent (for a symmetric
parametrisation, chain through the assembly, e.g. with index_add).
"""
from __future__ import annotations

import dataclasses

import torch

from . import bjp


@dataclasses.dataclass
class Pattern:
    """CSR structure on the device (int32)."""

    n: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor

    @classmethod
    def from_host(cls, A, device="cuda"):
        dev = torch.device(device)
        return cls(A.n, torch.as_tensor(A.row_ptr, device=dev), torch.as_tensor(A.col_idx, device=dev))


class PCGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, b, pattern: Pattern, block_size: int, tol: float, info_out):
        A = bjp.DeviceCsr(pattern.n, pattern.row_ptr, pattern.col_idx, values.detach().contiguous())
        M = bjp.precondition(A, block_size=block_size)
        ws = bjp.PcgWorkspace(A)
        x, info = bjp.pcg_solve(A, M, b.detach(), tol=tol, workspace=ws)
        if info.status != "OK":
            raise bjp.BjpError(-3, f"forward PCG: {info.status}")
        if info_out is not None:
            info_out.append(info)
        ctx.A, ctx.M, ctx.ws, ctx.tol, ctx.info_out = A, M, ws, tol, info_out
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        lam, info = bjp.pcg_solve(ctx.A, ctx.M, gx.contiguous().to(torch.float64), tol=ctx.tol,
                                  workspace=ctx.ws)
        if info.status != "OK":
            raise bjp.BjpError(-3, f"adjoint PCG: {info.status}")
        if ctx.info_out is not None:
            ctx.info_out.append(info)
        gv = bjp.value_grad(ctx.A, lam, x) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return gv, gb, None, None, None, None


def pcg_solve_diff(values: torch.Tensor, b: torch.Tensor, pattern: Pattern, block_size: int,
                   tol: float = 1e-10, info_out: list | None = None) -> torch.Tensor:
    return PCGSolve.apply(values, b, pattern, block_size, tol, info_out)


class EdgeAssembly:
    """Maps per-edge conductivities to the CSR values of the 2D edge Poisson
    matrix on a fixed pattern (differentiable with torch)."""

    def __init__(self, graph, A, device="cuda"):
        import numpy as np

        dev = torch.device(device)
        rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
        key = rows.astype(np.int64) * A.n + A.col_idx
        order = np.argsort(key)

        def slot(i, j):
            pos = np.searchsorted(key[order], np.asarray(i, np.int64) * A.n + np.asarray(j, np.int64))
            return order[pos]

        m = len(graph.ei)
        self.nnz = A.nnz
        self.s_ii = torch.as_tensor(slot(graph.ei, graph.ei), device=dev)
        self.s_jj = torch.as_tensor(slot(graph.ej, graph.ej), device=dev)
        self.s_ij = torch.as_tensor(slot(graph.ei, graph.ej), device=dev)
        self.s_ji = torch.as_tensor(slot(graph.ej, graph.ei), device=dev)
        self.s_bb = torch.as_tensor(slot(graph.bi, graph.bi), device=dev)
        self.m = m

    def assemble(self, c: torch.Tensor) -> torch.Tensor:
        ce, cb = c[: self.m], c[self.m:]
        v = torch.zeros(self.nnz, dtype=c.dtype, device=c.device)
        v = v.index_add(0, self.s_ii, ce).index_add(0, self.s_jj, ce)
        v = v.index_add(0, self.s_ij, -ce).index_add(0, self.s_ji, -ce)
        return v.index_add(0, self.s_bb, cb)
