"""Lead self-energies by decimation on the GPU (rgf_lead_self_energy), against
closed forms, the oracle's decimation and the Dyson fixed point, and end to end:
GPU self-energies of the uniform chain's own leads fed to rgf_solve give the
integer transmission of the infinite chain.

Bounds.  At the energies used here (at least 1/32 from the on-site levels of the
closed-form leads; broadening 1e-3 for the random leads) the oracle's FP64
decimation matches the closed forms to 1e-11 or better (oracle pins), so 1e-9
relative (Frobenius, per energy) is the bound against closed forms and against the
oracle.  Step counts are compared exactly: both sides decide convergence in FP64,
and the coupling norms fall by orders of magnitude per step near convergence.
"""
import numpy as np
import pytest

import oracle
from parity import rel
from test_gpu_rgf import free_gpu
from workloads import make_uniform_chain, surface_sigma

pytestmark = pytest.mark.gpu


def gpu_leads(lib, H00, H01, Hc, E, eta, tol=1e-14, max_steps=100):
    import torch
    d = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to(d)
    S, steps = lib.lead_self_energy(t(H00), t(H01), t(Hc), torch.from_numpy(np.asarray(E, dtype=np.float64)).to(d),
                                    eta, tol, max_steps)
    torch.cuda.synchronize()
    return S.cpu().numpy(), steps.cpu().numpy()


def random_lead(b, seed):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((b, b)) + 1j * rng.standard_normal((b, b))) / 4
    H00 = (A + A.conj().T) / 2
    H01 = (rng.standard_normal((b, b)) + 1j * rng.standard_normal((b, b))) / (3 * np.sqrt(b))
    Hc = (rng.standard_normal((b, b)) + 1j * rng.standard_normal((b, b))) / (2 * np.sqrt(b))
    return H00, H01, Hc


@pytest.mark.parametrize("b", [8, 64, 128])
def test_rotated_stack_closed_form(lib, b):
    """H00 = V diag(eps) V^H, H01 = Hc = I: g_s = V diag(sigma(z - eps_c)) V^H; the
    64 midpoint energies of [-2, 2] at eta = 1e-6."""
    wl = make_uniform_chain(2, b, 64, eta=1e-6)
    V, eps = wl.meta["V"], wl.meta["eps"]
    I = np.eye(b)
    S, steps = gpu_leads(lib, wl.H[1, 0], I, I, wl.energies, 1e-6)
    assert np.all(steps > 0), steps
    worst = 0.0
    for e, E in enumerate(wl.energies):
        want = (V * surface_sigma(E + 1e-6j - eps)[None, :]) @ V.conj().T
        worst = max(worst, rel(S[e], want))
    print(f"rotated stack b={b}: worst relative error {worst:.2e}, steps {steps.min()}..{steps.max()}", flush=True)
    assert worst <= 1e-9
    # step counts as the oracle's, at a few energies
    for e in (0, 17, 40, 63):
        _, k = oracle.surface_gf(wl.H[1, 0], I, wl.energies[e] + 1e-6j)
        assert steps[e] == k, (e, steps[e], k)


@pytest.mark.parametrize("b,seed", [(1, 1), (7, 2), (32, 3), (100, 4), (128, 5)])
def test_random_lead_against_oracle(lib, b, seed):
    """Random Hermitian H00, random H01 and Hc, 24 energies in [-3, 3] at eta = 1e-3:
    sigma and the step count against the oracle, and the GPU's surface function
    (Hc = I) through the Dyson fixed point."""
    H00, H01, Hc = random_lead(b, seed)
    E = np.linspace(-3.0, 3.0, 24) + 0.0137
    S, steps = gpu_leads(lib, H00, H01, Hc, E, 1e-3)
    G, _ = gpu_leads(lib, H00, H01, np.eye(b), E, 1e-3)
    worst = worst_fp = 0.0
    for e in range(len(E)):
        want, k = oracle.lead_self_energy(H00, H01, Hc, E[e], 1e-3)
        assert steps[e] == k, (e, steps[e], k)
        worst = max(worst, rel(S[e], want))
        z = E[e] + 1e-3j
        g = G[e]
        fp = g - np.linalg.inv(z * np.eye(b) - H00 - H01 @ g @ H01.conj().T)
        worst_fp = max(worst_fp, np.linalg.norm(fp) / np.linalg.norm(g))
    print(f"random lead b={b}: worst vs oracle {worst:.2e}, fixed-point residual {worst_fp:.2e}", flush=True)
    assert worst <= 1e-9 and worst_fp <= 1e-9


def test_not_converged_reported(lib):
    """Two steps are not enough at eta = 1e-6 inside the band: steps = -1, NaN."""
    I = np.eye(4)
    S, steps = gpu_leads(lib, np.zeros((4, 4)), I, I, [0.3, 1.1], 1e-6, max_steps=2)
    assert np.all(steps == -1) and np.all(np.isnan(S))


def test_argument_errors(lib):
    import torch
    d = torch.device("cuda:0")
    x = torch.zeros((4, 4), dtype=torch.complex128, device=d)
    E = torch.zeros(2, dtype=torch.float64, device=d)
    for kw, code in ((dict(tolerance=0.0), 1), (dict(max_steps=0), 1), (dict(eta=-1.0), 1)):
        args = dict(eta=1e-3)
        args.update(kw)
        with pytest.raises(lib.RgfError) as ei:
            lib.lead_self_energy(x, x, x, E, **args)
        assert ei.value.code == code


def test_end_to_end_uniform_chain_transmission(lib):
    """The uniform chain (256 layers of 128) with self-energies from the GPU
    decimation of its own leads: in-band T(E) is the integer number of open
    channels, and the band of G matches the run with closed-form self-energies."""
    import torch
    l, b, ne = 256, 128, 64
    wl = make_uniform_chain(l, b, ne, eta=1e-6)
    eps = wl.meta["eps"]
    I = np.eye(b)
    S, steps = gpu_leads(lib, wl.H[1, 0], I, I, wl.energies, wl.eta)
    assert np.all(steps > 0)
    d = torch.device("cuda:0")
    H = torch.from_numpy(np.ascontiguousarray(wl.H)).to(d)
    Sd = torch.from_numpy(S).to(d)
    E = torch.from_numpy(wl.energies).to(d)
    G, T, info = lib.solve(H, Sd, Sd, E, eta_d=0.0)
    torch.cuda.synchronize()
    assert bool((info == 0).all())
    n_open = np.array([np.sum(np.abs(x - eps) < 2) for x in wl.energies])
    dT = np.max(np.abs(T.cpu().numpy() - n_open))
    print(f"end to end: max |T - open channels| {dT:.2e}", flush=True)
    assert dT < 1e-7
    del G
    free_gpu()
