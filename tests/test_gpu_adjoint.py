"""Adjoint on the GPU: dT/d eps (on-site energies) and dT/dH (every entry of the
band of H) against the oracle's gradients (first-order perturbation dG = G dH G,
pinned by finite differences on the CPU), through torch.autograd and through the
C ABI directly; independent of the number of checkpoint domains (bitwise); the
memory kept between forward and backward; and against central finite differences
of the GPU forward at the full 256 x 64, 256-energy size."""
import numpy as np
import pytest

import oracle
from workloads import make_config, make_random

from test_gpu_rgf import rel

pytestmark = pytest.mark.gpu


def dev_inputs(wl):
    import torch
    d = torch.device("cuda:0")
    return (torch.from_numpy(wl.H).to(d), torch.from_numpy(wl.sigma_L).to(d),
            torch.from_numpy(wl.sigma_R).to(d), torch.from_numpy(wl.energies).to(d))


def gpu_grad(wl, nd=8, weights=None):
    import torch
    from paper_2605_19910_amd import autograd as ag
    H, sL, sR, E = dev_inputs(wl)
    eps = torch.zeros((wl.l, wl.b), dtype=torch.float64, device=H.device, requires_grad=True)
    T = ag.transmission(eps, H, sL, sR, E, checkpoint_domains=nd)
    w = torch.ones_like(T) if weights is None else torch.as_tensor(weights, device=T.device)
    (T * w).sum().backward()
    torch.cuda.synchronize()
    return T.detach().cpu().numpy(), eps.grad.cpu().numpy()


@pytest.mark.parametrize("l,b,ne,nd", [(12, 16, 3, 3), (9, 37, 2, 8), (16, 64, 2, 1), (20, 128, 2, 4),
                                       (1, 8, 2, 1), (7, 20, 2, 7)])
def test_adjoint_matches_oracle(lib, l, b, ne, nd):
    wl = make_random(l, b, 1, ne, seed=4100 + l + b, eta=1e-3)
    w = np.linspace(0.5, 1.5, ne)
    T, g = gpu_grad(wl, nd, w)
    ref = np.zeros((l, b))
    for e in range(ne):
        Te, ge = oracle.grad_onsite(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        ref += w[e] * ge
        assert abs(T[e] - Te) <= 1e-10 * max(1, abs(Te))
    assert rel(g, ref) <= 1e-10, rel(g, ref)


def gpu_grad_h(wl, nd=8, weights=None):
    import torch
    from paper_2605_19910_amd import autograd as ag
    H, sL, sR, E = dev_inputs(wl)
    H.requires_grad_(True)
    T = ag.transmission_h(H, sL, sR, E, checkpoint_domains=nd)
    w = torch.ones_like(T) if weights is None else torch.as_tensor(weights, device=T.device)
    (T * w).sum().backward()
    torch.cuda.synchronize()
    return T.detach().cpu().numpy(), H.grad.cpu().numpy()


@pytest.mark.parametrize("l,b,ne,nd", [(12, 16, 3, 3), (9, 37, 2, 8), (16, 64, 2, 1), (20, 128, 2, 4),
                                       (1, 8, 2, 1), (2, 8, 2, 2), (7, 20, 2, 7)])
def test_band_gradient_matches_oracle(lib, l, b, ne, nd):
    wl = make_random(l, b, 1, ne, seed=4300 + l + b, eta=1e-3)
    w = np.linspace(0.5, 1.5, ne)
    T, g = gpu_grad_h(wl, nd, w)
    ref = np.zeros((3, l, b, b), dtype=np.complex128)
    for e in range(ne):
        Te, ge = oracle.grad_band(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        ref += w[e] * ge
        assert abs(T[e] - Te) <= 1e-10 * max(1, abs(Te))
    assert rel(g, ref) <= 1e-10, rel(g, ref)
    # blocks outside the matrix get no gradient
    assert np.all(g[0, 0] == 0) and np.all(g[2, l - 1] == 0)


def test_band_gradient_through_the_c_abi_from_the_output_band(lib):
    """rgf_backward reading the diagonal blocks straight from the forward's output
    band (pointer G + l b^2, stride 3 l b^2), both gradients at once, against the
    oracle."""
    import torch
    from paper_2605_19910_amd import binding
    wl = make_random(10, 24, 1, 3, seed=71, eta=1e-3)
    H, sL, sR, E = dev_inputs(wl)
    l, b, ne = wl.l, wl.b, wl.ne
    plan = binding.Plan(l, b, 1, ne, want_backward=binding.BACKWARD_ONSITE | binding.BACKWARD_BAND,
                        checkpoint_domains=3)
    ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=H.device)
    G, T, info = binding.solve(H, sL, sR, E, plan=plan, workspace=ws)
    dLdT = torch.tensor([1.0, -0.5, 2.0], dtype=torch.float64, device=H.device)
    dH = torch.zeros_like(H)
    d_on = torch.empty((l, b), dtype=torch.float64, device=H.device)
    Gd = G[:, 1]   # view into the band: first diagonal block of energy e at G + e 3 l b^2 + l b^2
    stream = torch.cuda.current_stream().cuda_stream
    binding.rgf_backward(plan, H, sL, sR, E, 0.0, Gd, 3 * l * b * b, dLdT, dH, d_on, ws, stream)
    torch.cuda.synchronize()
    ref = np.zeros((3, l, b, b), dtype=np.complex128)
    ref_on = np.zeros((l, b))
    for e in range(ne):
        ref += dLdT[e].item() * oracle.grad_band(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])[1]
        ref_on += dLdT[e].item() * oracle.grad_onsite(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])[1]
    assert rel(dH.cpu().numpy(), ref) <= 1e-10
    assert rel(d_on.cpu().numpy(), ref_on) <= 1e-10
    # the on-site gradient is the real part of the band gradient's diagonal entries
    np.testing.assert_allclose(d_on.cpu().numpy(), np.real(np.diagonal(dH[1].cpu().numpy(), axis1=1, axis2=2)),
                               rtol=0, atol=1e-12 * np.abs(ref_on).max())


def test_checkpoint_count_does_not_change_the_result(lib):
    """P and R are recomputed from checkpoints with the same products in the same
    order as the forward's sequential recursion: bitwise identical gradients."""
    wl = make_random(24, 32, 1, 3, seed=77, eta=1e-3)
    _, g1 = gpu_grad(wl, 1)
    _, g3 = gpu_grad(wl, 3)
    _, g8 = gpu_grad(wl, 8)
    assert np.array_equal(g1, g3) and np.array_equal(g1, g8)
    _, h1 = gpu_grad_h(wl, 1)
    _, h5 = gpu_grad_h(wl, 5)
    assert np.array_equal(h1, h5)


def test_config5_adjoint_vs_finite_differences(lib):
    """L = sum over 256 energies of T(E), 256 layers x 64 orbitals (16384 on-site
    parameters), 8 checkpoint domains.  32 parameters drawn by default_rng(105):
    central differences of the GPU forward at h = 1e-6.  At this step the quotient
    is limited by the forward's rounding noise divided by h (the FD error grows as h
    shrinks: measured with the oracle, 9e-8 at h = 1e-4, 4e-5 at 1e-6, 1e-2 at 1e-8),
    so the bound is 10 x (noise / 2h + |FD(h) - FD(2h)|) with the noise of L measured
    at each parameter; a second quotient at h = 1e-4 must agree to 1e-6.  Plus the
    oracle adjoint on two energies."""
    import torch
    from paper_2605_19910_amd import binding
    wl = make_config(5)
    T, g = gpu_grad(wl, 8)
    assert np.all(np.isfinite(g))
    H, sL, sR, E = dev_inputs(wl)
    # memory kept between forward and backward: checkpoints + diagonal blocks of G,
    # against the forward's workspace + the whole band of G that a non-checkpointed
    # adjoint would need
    pb = binding.Plan(wl.l, wl.b, 1, wl.ne, want_backward=True, checkpoint_domains=8)
    plain = binding.Plan(wl.l, wl.b, 1, wl.ne)
    blk = wl.b * wl.b * 16
    held = pb.checkpoint_bytes + wl.ne * wl.l * blk
    full = plain.workspace_bytes + wl.ne * 3 * wl.l * blk
    print(f"kept between forward and backward: {held / 2**30:.2f} GiB vs {full / 2**30:.2f} GiB", flush=True)
    assert held <= full / 4
    plan = binding.Plan(wl.l, wl.b, 1, wl.ne)
    ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=H.device)
    G = torch.empty((wl.ne, 3, wl.l, wl.b, wl.b), dtype=torch.complex128, device=H.device)
    Tt = torch.empty((wl.ne,), dtype=torch.float64, device=H.device)
    info = torch.empty((wl.ne,), dtype=torch.int32, device=H.device)

    def Lsum(i, s, delta):
        Hp = H.clone()
        Hp[1, i, s, s] += delta
        binding.solve(Hp, sL, sR, E, plan=plan, workspace=ws, out=(G, Tt, info))
        torch.cuda.synchronize()
        return float(Tt.sum().item())

    params = np.random.default_rng(105).choice(wl.l * wl.b, 32, replace=False)
    h = 1e-6
    worst = 0.0
    gmax = abs(g).max()
    for p in params:
        i, s = divmod(int(p), wl.b)
        fd1 = (Lsum(i, s, h) - Lsum(i, s, -h)) / (2 * h)
        fd2 = (Lsum(i, s, 2 * h) - Lsum(i, s, -2 * h)) / (4 * h)
        # rounding noise of the forward's L around this parameter: the exact change
        # for a shift of 1e-13 is ~1e-13 |g|, far below what rounding causes
        noise = abs(Lsum(i, s, 1e-13) - Lsum(i, s, -1e-13))
        bound = 10 * (noise / (2 * h) + abs(fd1 - fd2)) + 1e-9 * max(1.0, gmax)
        diff = abs(fd1 - g[i, s])
        worst = max(worst, diff)
        assert diff <= bound, (i, s, g[i, s], fd1, fd2, noise)
        # a wider step, where truncation (h^2) dominates instead of rounding noise
        H4 = 1e-4
        fd4 = (Lsum(i, s, H4) - Lsum(i, s, -H4)) / (2 * H4)
        assert abs(fd4 - g[i, s]) <= 1e-6 * max(1.0, abs(g[i, s])), (i, s, g[i, s], fd4)
    print(f"max |adjoint - FD(h=1e-6)| over 32 parameters: {worst:.3e}; max |grad| {gmax:.3e}")
    # oracle adjoint on two energies (weights 1 on those, 0 elsewhere)
    for e in (17, 200):
        w = np.zeros(wl.ne)
        w[e] = 1.0
        _, ge = gpu_grad(wl, 8, w)
        Te, ref = oracle.grad_onsite(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        rn = oracle.rgf(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], pivot_noise=9, extras=False)
        r0 = oracle.rgf(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], extras=False)
        tol = max(1e-10, 8 * rel(rn["G"], r0["G"]))
        assert rel(ge, ref) <= tol, (e, rel(ge, ref), tol)
