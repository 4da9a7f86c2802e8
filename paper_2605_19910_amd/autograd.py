"""torch.autograd.Function around the forward solve and the adjoint kernel.

``transmission(eps, H, sigma_L, sigma_R, energies)`` returns T(E) for the system
whose on-site energies are shifted by ``eps`` (H_ii,ss += eps[i, s], real); its
gradient with respect to ``eps`` comes from rgf_backward (dG = G dH G), not from
autograd through torch ops.  The shift itself is applied to a copy of H before the
solve (input preparation); every step of the solve and of the adjoint runs in the
HIP library.
"""
from __future__ import annotations

import torch

from . import binding


class RGFTransmission(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, H, sigma_L, sigma_R, energies, checkpoint_domains: int = 8):
        l, b = H.shape[1], H.shape[2]
        ne = energies.shape[0]
        if H.shape[0] != 3:
            raise ValueError("the adjoint supports block-tridiagonal systems (w = 1)")
        Hs = H.clone()
        idx = torch.arange(b, device=H.device)
        Hs[1][:, idx, idx] += eps.to(torch.complex128)
        plan = binding.Plan(l, b, 1, ne, want_backward=True, checkpoint_domains=checkpoint_domains)
        ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=H.device)
        G, T, info = binding.solve(Hs, sigma_L, sigma_R, energies, plan=plan, workspace=ws)
        ctx.plan, ctx.ws = plan, ws
        ctx.save_for_backward(sigma_L, sigma_R, G)
        ctx.info = info
        return T

    @staticmethod
    def backward(ctx, dT):
        sigma_L, sigma_R, G = ctx.saved_tensors
        plan = ctx.plan
        d = torch.empty((plan.l, plan.b), dtype=torch.float64, device=G.device)
        stream = torch.cuda.current_stream(G.device).cuda_stream
        binding.rgf_backward(plan, sigma_L, sigma_R, G, dT.contiguous().to(torch.float64), d, ctx.ws, stream)
        return d, None, None, None, None, None


def transmission(eps, H, sigma_L, sigma_R, energies, checkpoint_domains: int = 8):
    return RGFTransmission.apply(eps, H, sigma_L, sigma_R, energies, checkpoint_domains)
