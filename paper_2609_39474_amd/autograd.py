"""Differentiable march: a ``torch.autograd.Function`` over the library's BDF
dual-time march and its discrete adjoint (C ABI ``msc_set_recording``,
``msc_bdf2_adjoint``, ``msc_init_adjoint``).

The forward creates a context from device FP64 tensors (p_hat0, u0), records
one checkpoint per physical step, advances ``nsteps`` steps and returns the
final hydrodynamic field (p_hat, u) as device tensors.  The backward feeds the
output gradients into the m^n slot of the state adjoint, reverses the recorded
steps and applies the adjoint of the initial map.  The gradient is that of the
discrete map at the forward's accepted inner counts (the counts themselves are
piecewise constant in the inputs), which is what a replayed schedule
differentiates by finite differences.

``biot_savart`` is the control map of the vorticity experiment (u0 from a
periodic 2D vorticity field by the spectral stream function); it is plain
torch (differentiable by torch) and not a step of the method.
"""
from __future__ import annotations

import math

import torch

from . import msc as M


def biot_savart(omega: torch.Tensor) -> torch.Tensor:
    """u = (d_y psi, -d_x psi) with psi_hat = omega_hat / |k|^2 on the
    periodic unit-spaced N x N grid; the k = 0 and Nyquist modes are zeroed."""
    N0, N1 = omega.shape
    kx = torch.fft.fftfreq(N0, d=1.0 / N0, dtype=torch.float64, device=omega.device) * (2 * math.pi / N0)
    ky = torch.fft.fftfreq(N1, d=1.0 / N1, dtype=torch.float64, device=omega.device) * (2 * math.pi / N1)
    KX, KY = torch.meshgrid(kx, ky, indexing="ij")
    k2 = KX * KX + KY * KY
    keep = (k2 > 0)
    keep &= (torch.arange(N0, device=omega.device) != N0 // 2).reshape(-1, 1)
    keep &= (torch.arange(N1, device=omega.device) != N1 // 2).reshape(1, -1)
    W = torch.fft.fft2(omega.to(torch.float64))
    psi = torch.where(keep, W / torch.where(keep, k2, torch.ones_like(k2)), torch.zeros_like(W))
    ux = torch.fft.ifft2(1j * KY * psi).real
    uy = torch.fft.ifft2(-1j * KX * psi).real
    return torch.stack([ux, uy])


class _March(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phat0, u0, params, nsteps, schedule, info):
        phat0 = phat0.detach().to(torch.float64).contiguous()
        u0 = u0.detach().to(torch.float64).contiguous()
        stream = torch.cuda.current_stream(phat0.device).cuda_stream
        s = M.Solver(params, phat0, u0, stream=stream)
        s.set_recording(True)
        if schedule is not None:
            s.set_schedule(schedule)
        _, stats = s.bdf2_step(int(nsteps))
        out_p = torch.empty_like(phat0)
        out_u = torch.empty_like(u0)
        s.moments_device(out_p.data_ptr(), out_u.data_ptr())
        if info is not None:
            info["stats"] = stats
            info["schedule"] = [st["iters"] for st in stats]
        ctx.solver = s
        ctx.nsteps = int(nsteps)
        ctx.save_for_backward(phat0, u0)
        return out_p, out_u

    @staticmethod
    def backward(ctx, g_p, g_u):
        phat0, u0 = ctx.saved_tensors
        s = ctx.solver
        d, Q, NS = s.d, s.Q, s.NS
        FQ = Q * NS
        lam = torch.zeros(s.state_size(), dtype=torch.float64, device=phat0.device)
        if g_p is not None:
            lam[3 * FQ:3 * FQ + NS] = g_p.reshape(-1).to(torch.float64)
        if g_u is not None:
            lam[3 * FQ + NS:3 * FQ + (d + 1) * NS] = g_u.reshape(-1).to(torch.float64)
        s.bdf2_adjoint_device(ctx.nsteps, lam.data_ptr())
        lp = torch.empty_like(phat0)
        lu = torch.empty_like(u0)
        s.init_adjoint_device(phat0.data_ptr(), u0.data_ptr(), lam.data_ptr(), lp.data_ptr(), lu.data_ptr())
        s.close()
        ctx.solver = None
        return lp, lu, None, None, None, None


def march(phat0: torch.Tensor, u0: torch.Tensor, params: M.msc_params, nsteps: int, schedule=None,
          info: dict | None = None):
    """Differentiable BDF march of nsteps physical steps from (p_hat0, u0)
    (device tensors, FP64).  ``schedule``: inner counts to replay (fixed
    acceptance), e.g. for finite differences; ``info`` receives the per-step
    statistics and the accepted counts."""
    return _March.apply(phat0, u0, params, nsteps, schedule, info)
