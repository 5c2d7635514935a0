"""Port inductance as a differentiable function of the per-voxel kinetic
parameter p_k = lambda_k^-2 (London depth, eq. 3).

Forward: set the two-fluid material, solve every port (svh_solve), form
Z_port = Y^-1 and L = Im(Z_port) / w.  Backward: adjoint solve (svh_solve with
transpose = 1), the admittance derivative per voxel (svh_port_gradient) and
its contraction with W = Z G Z (svh_gradient_contract), since
dL/dp_k = -Im(Z dY_k Z) / w.  All arithmetic runs in the HIP library; this
module only moves arguments.
"""
from __future__ import annotations

import numpy as np
import torch


class PortInductance(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pvec, problem, sigma0, freq, rre):
        lam = np.sqrt(1.0 / pvec.detach().cpu().numpy().astype(np.float64))
        s0 = np.broadcast_to(np.asarray(sigma0, dtype=np.float64), lam.shape).copy()
        problem.set_material([freq], s0, lam, per_voxel=True)
        X, Y, info = problem.solve(0, rre=rre)
        Z = np.linalg.inv(Y)
        w = 2 * np.pi * freq
        ctx.problem, ctx.freq, ctx.rre, ctx.Z, ctx.X = problem, freq, rre, Z, X
        ctx.info = info
        return torch.from_numpy(Z.imag / w).to(pvec.device)

    @staticmethod
    def backward(ctx, gL):
        p = ctx.problem
        w = 2 * np.pi * ctx.freq
        Xa, _, _ = p.solve(0, rre=ctx.rre, transpose=True)
        dY = p.port_gradient(0, ctx.X, Xa)
        G = gL.detach().cpu().numpy().astype(np.float64)
        W = ctx.Z @ G @ ctx.Z
        grad = p.gradient_contract(dY, W, -1.0 / w)
        return grad.to(gL.device), None, None, None, None


def port_inductance(problem, pvec, sigma0, freq, rre=1e-12):
    """L (nports x nports) for p = lambda^-2 per voxel; differentiable in pvec."""
    return PortInductance.apply(pvec, problem, sigma0, freq, rre)
