"""Port inductance as a differentiable function of the per-voxel kinetic
parameter p_k = lambda_k^-2 (London depth, eq. 3).

Forward: set the two-fluid material, solve every port (svh_solve), and take
Z_port = Y^-1 and L = Im(Z_port) / w (svh_port_inductance).  Backward: the
material of the forward call is applied again (so a solve or a material change
between forward and backward cannot leak in), then the adjoint solve
(svh_solve with transpose = 1), the admittance derivative per voxel
(svh_port_gradient) and its contraction with the loss weights G = dLoss/dL
(svh_gradient_contract, which forms W = Z^T G Z^T itself, since
dL/dp_k = -Im(Z dY_k Z) / w).  The arithmetic runs in the HIP library; this
module moves arguments.
"""
from __future__ import annotations

import numpy as np
import torch


def _apply_material(problem, pvec, sigma0, freq):
    lam = np.sqrt(1.0 / pvec.detach().cpu().numpy().astype(np.float64))
    s0 = np.broadcast_to(np.asarray(sigma0, dtype=np.float64), lam.shape).copy()
    problem.set_material([freq], s0, lam, per_voxel=True)


class PortInductance(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pvec, problem, sigma0, freq, rre):
        _apply_material(problem, pvec, sigma0, freq)
        X, Y, info = problem.solve(0, rre=rre)
        _, L = problem.port_inductance(0, Y)
        ctx.save_for_backward(pvec)
        ctx.problem, ctx.sigma0, ctx.freq, ctx.rre, ctx.Y, ctx.X = problem, sigma0, freq, rre, Y, X
        ctx.info = info
        return torch.from_numpy(L).to(pvec.device)

    @staticmethod
    def backward(ctx, gL):
        (pvec,) = ctx.saved_tensors
        p = ctx.problem
        _apply_material(p, pvec, ctx.sigma0, ctx.freq)  # the material X was solved with
        Xa, _, _ = p.solve(0, rre=ctx.rre, transpose=True)
        dY = p.port_gradient(0, ctx.X, Xa)
        G = gL.detach().cpu().numpy().astype(np.float64)
        grad = p.gradient_contract(0, ctx.Y, G, dY)
        return grad.to(gL.device), None, None, None, None


def port_inductance(problem, pvec, sigma0, freq, rre=1e-12):
    """L (nports x nports) for p = lambda^-2 per voxel; differentiable in pvec."""
    return PortInductance.apply(pvec, problem, sigma0, freq, rre)
