"""torch.autograd wrappers around the assembly adjoint and the shared CG solve.

    values = assemble(logE, x, asm, E)     # A(logE, x) on asm's current mask
    u      = solve(values, f, asm)         # A u = f, Jacobi-PCG
    L      = (f * u).sum(); L.backward()   # -> logE.grad, x.grad

Argument marshalling only: the forward passes are sta_set_params +
sta_full_rebuild and sta_cg_solve, the backward passes are sta_cg_solve
(adjoint solve, A symmetric), sta_slot_outer (-lambda u^T on the pattern)
and sta_adjoint.  The adjoint uses the assembler's parameters and mask at
backward time: run backward before editing or re-parameterising it.

The moduli E = exp(logE) enter the matrix as data.  Pass them as E (computed
once, e.g. on the host, as the CPU oracle takes them) to fix their bits;
without E they are computed here with torch.exp on the device, whose last
bit can differ from another exp routine's, and then so can the matrix.
"""
from __future__ import annotations

import torch


class AssembleFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, logE, x, asm, E):
        if E is None:
            E = torch.exp(logE.detach().to(torch.float64))
        asm.set_params(x.detach().to(torch.float64).contiguous(), E.detach().to(torch.float64).contiguous())
        asm.full_rebuild()
        ctx.asm = asm
        return asm.values()

    @staticmethod
    def backward(ctx, g_values):
        g_logE, g_x = ctx.asm.adjoint(g_values.contiguous())
        return g_logE, g_x, None, None


class SolveFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, f, asm, rtol):
        u, _, _ = asm.cg_solve(f.reshape(-1).contiguous(), values.contiguous(), rtol=rtol)
        ctx.save_for_backward(values, u)
        ctx.asm, ctx.rtol, ctx.fshape = asm, rtol, f.shape
        return u

    @staticmethod
    def backward(ctx, g_u):
        values, u = ctx.saved_tensors
        lam, _, _ = ctx.asm.cg_solve(g_u.reshape(-1).contiguous(), values, rtol=ctx.rtol)
        g_values = ctx.asm.slot_outer(lam, u, -1.0)
        return g_values, lam.reshape(ctx.fshape), None, None


def assemble(logE: torch.Tensor, x: torch.Tensor, asm, E: torch.Tensor | None = None) -> torch.Tensor:
    """CSR values of A at moduli exp(logE) (given as E when not None) and nodes x."""
    return AssembleFunction.apply(logE, x, asm, E)


def solve(values: torch.Tensor, f: torch.Tensor, asm, rtol: float = 1e-12) -> torch.Tensor:
    return SolveFunction.apply(values, f, asm, rtol)
