"""torch.autograd.Function wrappers around the forward solve and the adjoint kernel.

``transmission(eps, H, sigma_L, sigma_R, energies)``: T(E) for the system whose
on-site energies are shifted by the real ``eps`` (H_ii,ss += eps[i, s]); its
gradient with respect to ``eps`` comes from rgf_backward.

``transmission_h(H, sigma_L, sigma_R, energies)``: T(E) as a function of the
complex band H itself (every entry an independent parameter, H not assumed
Hermitian); its gradient with respect to H (PyTorch's convention dL/dRe + i dL/dIm)
is the band gradient of rgf_backward.

Between forward and backward only the adjoint's checkpoints (the prefix of the
workspace the plan names) and the diagonal blocks of G are kept; the backward gets a
fresh workspace whose prefix receives the checkpoints.  The on-site shift is applied
to a copy of H before the solve (input preparation); every step of the solve and of
the adjoint runs in the HIP library.
"""
from __future__ import annotations

import torch

from . import binding


def _forward(H, sigma_L, sigma_R, energies, eta_d, checkpoint_domains, flags):
    l, b = H.shape[1], H.shape[2]
    ne = energies.shape[0]
    if H.shape[0] != 3:
        raise ValueError("the adjoint supports block-tridiagonal systems (w = 1)")
    plan = binding.Plan(l, b, 1, ne, want_backward=flags, checkpoint_domains=checkpoint_domains)
    ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=H.device)
    G, T, info = binding.solve(H, sigma_L, sigma_R, energies, eta_d=eta_d, plan=plan, workspace=ws)
    ck = ws[:plan.checkpoint_bytes].clone()
    G_diag = G[:, 1].contiguous()
    return plan, ck, G_diag, T, info


def _backward(plan, ck, H, sigma_L, sigma_R, energies, eta_d, G_diag, dT, dH, d_onsite):
    ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=H.device)
    ws[:plan.checkpoint_bytes].copy_(ck)
    stream = torch.cuda.current_stream(H.device).cuda_stream
    binding.rgf_backward(plan, H, sigma_L, sigma_R, energies, eta_d, G_diag, 0,
                         dT.contiguous().to(torch.float64), dH, d_onsite, ws, stream)


class RGFTransmission(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, H, sigma_L, sigma_R, energies, checkpoint_domains: int = 8, eta_d: float = 0.0):
        b = H.shape[2]
        Hs = H.clone()
        idx = torch.arange(b, device=H.device)
        Hs[1][:, idx, idx] += eps.to(torch.complex128)
        plan, ck, G_diag, T, info = _forward(Hs, sigma_L, sigma_R, energies, eta_d, checkpoint_domains,
                                             binding.BACKWARD_ONSITE)
        ctx.plan, ctx.ck, ctx.eta_d = plan, ck, eta_d
        ctx.save_for_backward(Hs, sigma_L, sigma_R, energies, G_diag)
        ctx.info = info
        return T

    @staticmethod
    def backward(ctx, dT):
        Hs, sigma_L, sigma_R, energies, G_diag = ctx.saved_tensors
        plan = ctx.plan
        d = torch.empty((plan.l, plan.b), dtype=torch.float64, device=Hs.device)
        _backward(plan, ctx.ck, Hs, sigma_L, sigma_R, energies, ctx.eta_d, G_diag, dT, None, d)
        return d, None, None, None, None, None, None


class RGFTransmissionH(torch.autograd.Function):
    @staticmethod
    def forward(ctx, H, sigma_L, sigma_R, energies, checkpoint_domains: int = 8, eta_d: float = 0.0):
        H = H.contiguous()
        plan, ck, G_diag, T, info = _forward(H, sigma_L, sigma_R, energies, eta_d, checkpoint_domains,
                                             binding.BACKWARD_BAND)
        ctx.plan, ctx.ck, ctx.eta_d = plan, ck, eta_d
        ctx.save_for_backward(H, sigma_L, sigma_R, energies, G_diag)
        ctx.info = info
        return T

    @staticmethod
    def backward(ctx, dT):
        H, sigma_L, sigma_R, energies, G_diag = ctx.saved_tensors
        dH = torch.zeros_like(H)
        _backward(ctx.plan, ctx.ck, H, sigma_L, sigma_R, energies, ctx.eta_d, G_diag, dT, dH, None)
        return dH, None, None, None, None, None


def transmission(eps, H, sigma_L, sigma_R, energies, checkpoint_domains: int = 8, eta_d: float = 0.0):
    return RGFTransmission.apply(eps, H, sigma_L, sigma_R, energies, checkpoint_domains, eta_d)


def transmission_h(H, sigma_L, sigma_R, energies, checkpoint_domains: int = 8, eta_d: float = 0.0):
    return RGFTransmissionH.apply(H, sigma_L, sigma_R, energies, checkpoint_domains, eta_d)
