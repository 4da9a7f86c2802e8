"""GPU parity of the lesser Green's function on the band, G^< = G^R Sigma^< G^A with
the leads' lesser self-energies i f_X Gamma_X, through the C ABI (rgf_solve_lesser).

Bound: G^< is a sum of products C A C^H of the first and last block columns of G^R,
each known to the FP64 rule's 2 b u kappa_max (tests/parity.py); the product
doubles the relative error, so per energy the band of G^< is compared with the
oracle within 2 * fp64_bound(kappa_max, b), relative Frobenius over the band.
Cases: small ragged systems with random occupations (with and without device
broadening), the 256 x 128 system at 9 energies with the Fermi functions of two
leads at different chemical potentials, the uniform chain against its closed form
at the full size, a singular pivot, and block n-diagonal systems (w = 2, 3, 4, with
one and several workgroups per energy in the sweep) against the dense definition.
"""
import numpy as np
import pytest

import oracle
from parity import fp64_bound, mask_band, oracle_results, rel
from test_gpu_rgf import free_gpu, to_dev
from workloads import make_config, make_random, make_uniform_chain, surface_sigma

pytestmark = pytest.mark.gpu


def fermi(E, mu, kT):
    return 1.0 / (1.0 + np.exp((np.asarray(E) - mu) / kT))


def run(lib, wl, fL, fR, eta_d=0.0, split=0):
    import torch
    H, sL, sR, E = to_dev(wl)
    d = H.device
    plan = lib.Plan(wl.l, wl.b, wl.w, wl.ne)
    plan.set_split(split, 0)
    G, Gl, T, info = lib.solve_lesser(H, sL, sR, E, torch.from_numpy(np.asarray(fL, dtype=np.float64)).to(d),
                                      torch.from_numpy(np.asarray(fR, dtype=np.float64)).to(d), eta_d, plan=plan)
    torch.cuda.synchronize()
    plan.close()
    return G, Gl, T, info


def check(label, Gl, energies, refs, b):
    bad = []
    for e, r in zip(energies, refs):
        err = rel(mask_band(Gl[e].cpu().numpy(), 1), r["G"])
        tol = 2.0 * fp64_bound(r["kappa"], b)
        print(f"{label} energy {e}: kappa {r['kappa']:.2e} |dG<|/|G<| {err:.2e} bound {tol:.2e}", flush=True)
        if not err <= tol:
            bad.append((e, err, tol))
    assert not bad, bad


@pytest.mark.parametrize("l,b,eta_d", [(1, 8, 0.0), (2, 16, 0.0), (9, 24, 0.05), (17, 37, 0.0), (12, 64, 0.0),
                                       (6, 128, 0.05), (20, 100, 0.0), (33, 48, 0.0)])
def test_lesser_small(lib, l, b, eta_d):
    wl = make_random(l, b, 1, 3, seed=4100 + l + b, eta=1e-3)
    rng = np.random.default_rng(l * b)
    fL, fR = rng.uniform(0, 1, 3), rng.uniform(0, 1, 3)
    G, Gl, T, info = run(lib, wl, fL, fR, eta_d)
    assert bool((info == 0).all())
    refs = oracle_results("lesser", wl, range(3), eta_d=eta_d, occ=list(zip(fL, fR)))
    check(f"lesser l={l} b={b} eta_d={eta_d}", Gl, range(3), refs, b)


def test_lesser_config2(lib):
    """256 x 128, 64 energies; leads at chemical potentials +-0.2 and kT = 0.025 (the
    bias window is where f_L != f_R); 9 energies against the oracle, and the one- and
    four-workgroup sweeps give the same G^< bitwise."""
    import torch
    wl = make_config(2)
    fL, fR = fermi(wl.energies, 0.2, 0.025), fermi(wl.energies, -0.2, 0.025)
    G, Gl, T, info = run(lib, wl, fL, fR)
    assert bool((info == 0).all())
    es = [0, 8, 16, 28, 30, 32, 35, 48, 63]
    refs = oracle_results("lesser", ("config", 2), es, occ=[(fL[e], fR[e]) for e in es])
    check("config2 lesser", Gl, es, refs, wl.b)
    del G
    G1, Gl1, T1, info1 = run(lib, wl, fL, fR, split=1)
    for X in (Gl, Gl1):
        X[:, 0, 0] = 0
        X[:, 2, wl.l - 1] = 0
    assert torch.equal(Gl, Gl1) and torch.equal(T, T1)
    del G1, Gl1, Gl
    free_gpu()


def test_lesser_uniform_chain_closed_form(lib):
    """Uniform chain, 256 layers of 128, eta_d = eta: G_{i,0} = V diag(s_c^i / r_c) V^H
    and G_{i,l-1} = V diag(s_c^(l-1-i) / r_c) V^H, Gamma = V diag(-2 Im s_c) V^H, so
    with one lead occupied every band block of G^< has a closed form."""
    l, b, ne = 256, 128, 16
    wl = make_uniform_chain(l, b, ne, eta=1e-6, eta_d=1e-6)
    V, eps = wl.meta["V"], wl.meta["eps"]
    for fL, fR in ((1.0, 0.0), (0.0, 1.0)):
        G, Gl, T, info = run(lib, wl, np.full(ne, fL), np.full(ne, fR), eta_d=wl.eta_d)
        assert bool((info == 0).all())
        for e in (0, 5, 11, 15):
            z = wl.energies[e] + 1j * wl.eta - eps
            s = surface_sigma(z)
            r = np.sqrt(z - 2.0) * np.sqrt(z + 2.0)
            gam = -2.0 * s.imag
            Ge = Gl[e].cpu().numpy()
            num = den = 0.0
            for i in (0, 1, 77, 254, 255):
                for k in (-1, 0, 1):
                    j = i + k
                    if not 0 <= j < l:
                        continue
                    if fL:
                        d = 1j * s ** i * np.conj(s) ** j * gam / np.abs(r) ** 2
                    else:
                        d = 1j * s ** (l - 1 - i) * np.conj(s) ** (l - 1 - j) * gam / np.abs(r) ** 2
                    ex = (V * d[None, :]) @ V.conj().T
                    num += np.linalg.norm(Ge[1 + k, i] - ex) ** 2
                    den += np.linalg.norm(ex) ** 2
            err = np.sqrt(num / den)
            print(f"uniform chain lesser f=({fL},{fR}) energy {e}: rel err {err:.2e}", flush=True)
            assert err <= 1e-9, (fL, e, err)
        del G, Gl
    free_gpu()


def test_lesser_singular_pivot(lib):
    """The energy whose first Schur pivot is exactly zero gets info = l and NaN in G^<;
    the others match the oracle."""
    wl = make_random(6, 8, 1, 2, seed=3, eta=1e-3)
    wl.sigma_R[0] = 0.0
    wl.H[1, 5] = wl.energies[0] * np.eye(8)
    G, Gl, T, info = run(lib, wl, [0.5, 0.5], [0.1, 0.1])
    inf = info.cpu().numpy()
    assert inf[0] == 6 and inf[1] == 0
    assert np.all(np.isnan(Gl[0].cpu().numpy()))
    refs = oracle_results("lesser", wl, [1], occ=[(0.5, 0.1)])
    check("lesser next to a singular energy", Gl, [1], refs, 8)


def test_lesser_rejects_other_plans(lib):
    import torch
    wl = make_random(8, 16, 1, 2, seed=9, eta=1e-3)
    H, sL, sR, E = to_dev(wl)
    f = torch.zeros(2, dtype=torch.float64, device=H.device)
    for kw in (dict(precision="fp32"), dict(want_backward=True)):
        plan = lib.Plan(8, 16, 1, 2, **kw)
        with pytest.raises(lib.RgfError) as ei:
            lib.solve_lesser(H, sL, sR, E, f, f, plan=plan)
        assert ei.value.code == 2
        plan.close()


@pytest.mark.parametrize("l,b,w,eta_d", [(7, 8, 2, 0.0), (12, 20, 3, 0.0), (9, 16, 2, 0.05), (20, 37, 2, 0.0),
                                         (10, 64, 4, 0.0), (6, 128, 2, 0.0), (3, 5, 2, 0.0)])
def test_lesser_ndiagonal(lib, l, b, w, eta_d):
    """Block n-diagonal G^< (first column by the sweep's downward recursion, last column
    through the transfer products of its multipliers) against the dense definition
    M^{-1} Sigma^< M^{-H}, within twice the FP64 rule of the n-diagonal sweep."""
    wl = make_random(l, b, w, 3, seed=4300 + l + b + w, eta=1e-3)
    rng = np.random.default_rng(l * b + w)
    fL, fR = rng.uniform(0, 1, 3), rng.uniform(0, 1, 3)
    G, Gl, T, info = run(lib, wl, fL, fR, eta_d)
    assert bool((info == 0).all())
    kap = oracle_results("nrgf", wl, range(3), eta_d=eta_d)
    bad = []
    for e in range(3):
        want = oracle.lesser_dense(wl.H, w, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], fL[e], fR[e], eta_d)
        err = rel(mask_band(Gl[e].cpu().numpy(), w), want)
        tol = 2.0 * fp64_bound(kap[e]["kappa"], b)
        print(f"lesser l={l} b={b} w={w} energy {e}: kappa {kap[e]['kappa']:.2e} |dG<|/|G<| {err:.2e} "
              f"bound {tol:.2e}", flush=True)
        if not err <= tol:
            bad.append((e, err, tol))
    assert not bad, bad
