"""Differentiable GaBP solves (torch.autograd) on top of the C ABI.

Forward: solve A(v) x = b with the context's mode and precision (FP32 messages inside FP64
refinement for the training use case). Backward: solve A^T lambda = dL/dx with the same
GaBP on the transposed graph (A_ij and A_ji exchanged in every message rule), then
dL/dA_e = -lambda_row(e) x_col(e) for every stored entry (HIP scatter kernel) and
dL/db = lambda. Only x and the matrix values are saved between the passes: the forward
messages are not stored, the backward recomputes its own (including its own precomputed Lt
for A^T).

``ThetaField`` is an example coefficient model: per-node log-diffusion theta on an upwind
convection-diffusion grid (face coefficient exp((theta_a + theta_b)/2), boundary faces
exp(theta_a), rotating velocity), assembled with torch ops so that autograd carries
dL/dvalues back onto theta. It reproduces ``workloads.theta_operator`` value for value.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gabp as B
from . import workloads as W


class GaBPSolve(torch.autograd.Function):
    """x = A(values)^{-1} b with the sparsity pattern and options of ``solver``.

    The solver holds one matrix at a time. The forward saves its (detached) values and the
    solver's value version; when another forward on the same solver has replaced the
    values before this backward runs (several solves summed into one loss), the backward
    uploads its own values again before the transposed solve."""

    @staticmethod
    def forward(ctx, values, b, solver, tol, max_sweeps):
        v = values.detach().contiguous()
        solver.update_values(v)
        x, info = solver.solve(b.detach().contiguous(), tol, max_sweeps)
        solver.last_forward_info = info
        if info.status != B.OK:
            raise B.GaBPError(info.status, f"forward solve did not converge: {info}")
        ctx.solver, ctx.tol, ctx.max_sweeps = solver, tol, max_sweeps
        ctx.version = solver.values_version
        ctx.save_for_backward(x, v)
        return x

    @staticmethod
    def backward(ctx, gx):
        x, v = ctx.saved_tensors
        s = ctx.solver
        if s.values_version != ctx.version:
            s.update_values(v)
            ctx.version = s.values_version
        lam, info = s.solve_transposed(gx.contiguous(), ctx.tol, ctx.max_sweeps)
        s.last_backward_info = info
        if info.status != B.OK:
            raise B.GaBPError(info.status, f"adjoint solve did not converge: {info}")
        G, _ = s.adjoint_scatter(lam, x)
        return G, lam, None, None, None


def gabp_solve(values, b, solver, tol=1e-10, max_sweeps=2_000_000):
    return GaBPSolve.apply(values, b, solver, tol, max_sweeps)


class ThetaField:
    """Upwind convection-diffusion operator A(theta) on an n x n grid, assembled in torch."""

    def __init__(self, n: int, vscale: float = 20.0, device="cuda"):
        self.n = n
        theta0 = np.zeros(n * n)
        a, pos = W.theta_operator(n, theta0, vscale, with_index=True)
        self.pattern = a                      # rowptr/col of every A(theta)
        h = 1.0 / (n + 1)
        t = (np.arange(n) + 1) * h
        y, x = np.meshgrid(t, t, indexing="ij")
        vx, vy = -vscale * (y - 0.5), vscale * (x - 0.5)
        conv = np.stack([h * np.maximum(vy, 0), h * np.maximum(vx, 0),
                         h * (np.abs(vx) + np.abs(vy)), h * np.maximum(-vx, 0),
                         h * np.maximum(-vy, 0)], -1).reshape(n * n, 5)
        self.conv = torch.as_tensor(conv, device=device)
        keep = pos.reshape(-1) >= 0
        self.keep = torch.as_tensor(np.nonzero(keep)[0], device=device)
        self.device = device

    def values(self, theta: torch.Tensor) -> torch.Tensor:
        n = self.n
        th = theta.reshape(n, n)
        kx = torch.cat([torch.exp(th[:, :1]), torch.exp(0.5 * (th[:, :-1] + th[:, 1:])),
                        torch.exp(th[:, -1:])], dim=1)
        ky = torch.cat([torch.exp(th[:1, :]), torch.exp(0.5 * (th[:-1, :] + th[1:, :])),
                        torch.exp(th[-1:, :])], dim=0)
        kw, ke = kx[:, :-1], kx[:, 1:]
        ks, kn = ky[:-1, :], ky[1:, :]
        c = self.conv.reshape(n, n, 5)
        coef = torch.stack([-(ks + c[..., 0]), -(kw + c[..., 1]),
                            kw + ke + ks + kn + c[..., 2], -(ke + c[..., 3]),
                            -(kn + c[..., 4])], dim=-1)
        return coef.reshape(-1)[self.keep]
