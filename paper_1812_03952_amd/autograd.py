"""torch.autograd.Functions over the library: the CPR-GMRES solve with a
hand-written adjoint, and the Jacobian assembly from log-permeability.

For J(x) with A(theta) x = b:  dJ/db = lambda,  dJ/dA_ij = -lambda_i x_j^T
(A^T lambda = dJ/dx), and dJ/dtheta follows from dJ/dA through the
transmissibility chain rule of the assembly.  Every step runs in the
library's kernels (rs_gmres_solve, rs_adjoint_solve, rs_grad_vals,
rs_assemble, rs_grad_logk).
"""
from __future__ import annotations

import torch

from . import rsolve as rs


class SolveSpec:
    """Pattern, grid and solver options shared by forward and backward."""

    def __init__(self, nx, ny, nz, row_ptr, col_idx, method=rs.ABF, prec=64, cpr=None, gmres=None):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.row_ptr, self.col_idx = row_ptr, col_idx
        self.method, self.prec = method, prec
        self.cpr = cpr if cpr is not None else rs.cpr_opts()
        self.gmres = gmres if gmres is not None else rs.gmres_opts()
        self.last_info = None
        self.last_adjoint_info = None


class SolveFn(torch.autograd.Function):
    """x = A(vals)^{-1} b by CPR-preconditioned GMRES."""

    @staticmethod
    def forward(ctx, vals, b, spec: SolveSpec):
        A = rs.bsr_create(spec.nx, spec.ny, spec.nz, spec.row_ptr, spec.col_idx, vals.detach().contiguous())
        D = rs.decouple(A, spec.method, spec.prec)
        M = rs.cpr_setup(A, D, spec.cpr)
        x = torch.zeros_like(b)
        spec.last_info = rs.gmres_solve(A, M, b.detach().contiguous(), x, spec.gmres)
        ctx.A, ctx.spec = A, spec
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        A, spec = ctx.A, ctx.spec
        lam = torch.zeros_like(x)
        spec.last_adjoint_info = rs.adjoint_solve(A, gx.contiguous(), lam, spec.method, spec.prec,
                                                  spec.cpr, spec.gmres)
        G = None
        if ctx.needs_input_grad[0]:
            G = torch.empty(16 * A.nnzb, dtype=torch.float64, device=x.device)
            rs.grad_vals(A, lam, x, G)
        return G, lam if ctx.needs_input_grad[1] else None, None


class AssembleFn(torch.autograd.Function):
    """BSR values of the synthetic Jacobian as a function of log k."""

    @staticmethod
    def forward(ctx, logk, prob: "rs.DeviceProblem"):
        vals = torch.empty(16 * prob.col_idx.numel(), dtype=torch.float64, device=logk.device)
        prob.assemble(logk.detach().contiguous(), vals)
        ctx.prob = prob
        ctx.save_for_backward(logk)
        return vals

    @staticmethod
    def backward(ctx, G):
        (logk,) = ctx.saved_tensors
        p = ctx.prob
        g = torch.empty_like(logk)
        rs.grad_logk(p.nx, p.ny, p.nz, logk.detach().contiguous(), p.kvkh, p.tscale, p.Mf, p.Mb, p.wcell,
                     p.wu, p.row_ptr, G.contiguous(), g)
        return g, None
