"""Observables read off a solved band on the GPU (rgf_dos, rgf_density, rgf_bond_current): the density
of states against the oracle's definition on the same band (bitwise: one division per
entry) and against the uniform chain's closed form, and the electron density against
the oracle's and against the equilibrium identity density = sum_e w_e f_e DOS_e.

Bounds.  The uniform chain's band is exact on the GPU to ~1e-13 relative (its pivots
are well conditioned), so the closed form is checked at 1e-9 relative.  The equilibrium
identity holds exactly; both sides come from the same GPU sweep (G^< from its
multipliers), so they agree to the sweep's rounding times the pivots' conditioning,
well inside 1e-9 relative for these systems (pivot kappa below 1e4); the same holds for the
bond currents against T(E) (f_L - f_R) / 2pi.  Against the
oracle's density the same 1e-9 holds (FP64 rule of the sweep at b = 16, kappa <= 1e4:
2 b u kappa ~ 1e-11, summed over a handful of energies)."""
import numpy as np
import pytest

import oracle
from test_gpu_rgf import free_gpu
from workloads import make_random, make_uniform_chain

pytestmark = pytest.mark.gpu


def to_dev(*xs):
    import torch
    d = torch.device("cuda:0")
    return [torch.from_numpy(np.ascontiguousarray(x)).to(d) for x in xs]


def test_dos_matches_definition_on_the_same_band(lib):
    import torch
    wl = make_random(20, 24, 2, 3, seed=41, eta=1e-3)
    H, sL, sR, E = to_dev(wl.H, wl.sigma_L, wl.sigma_R, wl.energies)
    G, T, info = lib.solve(H, sL, sR, E, eta_d=0.0)
    d = lib.dos(G)
    torch.cuda.synchronize()
    Gh, dh = G.cpu().numpy(), d.cpu().numpy()
    for e in range(wl.ne):
        want = oracle.dos(Gh[e], 2)
        assert np.max(np.abs(dh[e] - want)) <= 1e-15 * np.max(np.abs(want)), e


def test_dos_uniform_chain_closed_form(lib):
    """Uniform chain with eta_d = eta: DOS of every orbital -(1/pi) Im (V diag(1/r_c) V^H)_ss."""
    import torch
    l, b = 64, 32
    wl = make_uniform_chain(l, b, 8, seed=106, eta=1e-2, eta_d=1e-2)
    V, eps = wl.meta["V"], wl.meta["eps"]
    H, sL, sR, E = to_dev(wl.H, wl.sigma_L, wl.sigma_R, wl.energies)
    G, T, info = lib.solve(H, sL, sR, E, eta_d=wl.eta_d)
    d = lib.dos(G)
    torch.cuda.synchronize()
    assert bool((info == 0).all())
    dh = d.cpu().numpy().reshape(wl.ne, l, b)
    worst = 0.0
    for e in range(wl.ne):
        z = wl.energies[e] + 1j * wl.eta - eps
        r = np.sqrt(z - 2.0) * np.sqrt(z + 2.0)
        want = -np.imag(np.diagonal((V / r[None, :]) @ V.conj().T)) / np.pi
        worst = max(worst, np.max(np.abs(dh[e] - want[None, :])) / np.max(np.abs(want)))
    print(f"uniform chain DOS: worst relative deviation from the closed form {worst:.2e}", flush=True)
    assert worst <= 1e-9


def test_density_equilibrium_and_oracle(lib):
    import torch
    wl = make_random(12, 16, 1, 6, seed=43, eta=1e-3)
    f = 1.0 / (1.0 + np.exp((wl.energies + 0.2) / 0.25))
    wts = np.full(wl.ne, 4.0 / wl.ne)
    H, sL, sR, E, fd, wd = to_dev(wl.H, wl.sigma_L, wl.sigma_R, wl.energies, f, wts)
    G, Gl, T, info = lib.solve_lesser(H, sL, sR, E, fd, fd, eta_d=0.0)
    n = lib.density(Gl, wd)
    d = lib.dos(G)
    torch.cuda.synchronize()
    assert bool((info == 0).all())
    nh, dh = n.cpu().numpy(), d.cpu().numpy()
    ident = np.sum((wts * f)[:, None] * dh, axis=0)
    e1 = np.max(np.abs(nh - ident)) / np.max(np.abs(ident))
    bands = [oracle.lesser(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], f[e], f[e], 0.0)[1]
             for e in range(wl.ne)]
    want = oracle.density(bands, wts, 1)
    e2 = np.max(np.abs(nh - want)) / np.max(np.abs(want))
    print(f"density: vs equilibrium identity {e1:.2e}, vs oracle {e2:.2e}", flush=True)
    assert e1 <= 1e-9 and e2 <= 1e-9
    free_gpu()


@pytest.mark.parametrize("fL,fR", [(1.0, 0.0), (0.25, 0.75)])
def test_bond_current_conserved_and_landauer(lib, fL, fR):
    """Every bond carries T(E) (f_L - f_R) / 2pi (GPU T), and the kernel agrees with the
    oracle's trace on the same G^< band."""
    import torch
    wl = make_random(16, 24, 1, 4, seed=47, eta=1e-3)
    H, sL, sR, E = to_dev(wl.H, wl.sigma_L, wl.sigma_R, wl.energies)
    fl, fr = to_dev(np.full(wl.ne, fL), np.full(wl.ne, fR))
    G, Gl, T, info = lib.solve_lesser(H, sL, sR, E, fl, fr, eta_d=0.0)
    j = lib.bond_current(H, Gl)
    torch.cuda.synchronize()
    assert bool((info == 0).all())
    jh, Th, Glh = j.cpu().numpy(), T.cpu().numpy(), Gl.cpu().numpy()
    worst_id = worst_or = 0.0
    for e in range(wl.ne):
        want = Th[e] * (fL - fR) / (2 * np.pi)
        worst_id = max(worst_id, np.max(np.abs(jh[e] - want)) / max(abs(want), 1e-3))
        ref = oracle.bond_current(wl.H, Glh[e])
        worst_or = max(worst_or, np.max(np.abs(jh[e] - ref)) / max(np.max(np.abs(ref)), 1e-3))
    print(f"bond current: vs Landauer {worst_id:.2e}, vs oracle trace {worst_or:.2e}", flush=True)
    assert worst_id <= 1e-9 and worst_or <= 1e-12
