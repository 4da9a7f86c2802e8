"""Pins of the oracle's lead self-energies (decimation) and lesser Green's function
against what the mathematics fixes independently of them:

* decimation against the closed-form surface Green's function of a chain and of a
  unitarily rotated stack of chains, against the surface block of a long finite
  chain inverted densely, and through the Dyson fixed point it must satisfy;
* the lesser function against its definition (dense M^{-1} Sigma^< M^{-H}),
  against the equilibrium identity G^< = -f (G^R - G^A), against the closed form of
  a uniform chain, and by anti-Hermiticity.
"""
import numpy as np
import pytest

import oracle
from workloads import make_random, make_uniform_chain, surface_sigma



def rel_err(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _chain_gs(z, eps, t):
    """Closed form for a b = 1 chain with on-site eps and hopping t: the root of
    t^2 g^2 - (z - eps) g + 1 = 0 that is the surface sigma of the unit chain
    rescaled, g = sigma((z - eps) / t) / t."""
    return surface_sigma((z - eps) / t) / t


@pytest.mark.parametrize("eps,t", [(0.0, 1.0), (0.3, 0.7), (-0.5, 1.4)])
def test_decimation_scalar_chain_closed_form(eps, t):
    """Energies inside and outside the band |E - eps| < 2|t|, none within 0.1 |t| of
    the on-site level: there the first decimation step inverts z - eps ~ i eta and the
    iteration cancels terms of size 1/eta (3e-5 lost at E = eps, eta = 1e-6, also in
    this closed-form case), which says nothing about the implementation."""
    offs = np.array([0.13, 0.4, 0.77, 1.2, 1.6, 1.95, 2.4, 3.1])
    for E in eps + t * np.concatenate([-offs, offs]):
        for eta in (1e-6, 1e-3, 0.1):
            z = E + 1j * eta
            g, steps = oracle.surface_gf(np.array([[eps]], complex), np.array([[t]], complex), z)
            assert steps > 0
            want = _chain_gs(z, eps, t)
            assert abs(g[0, 0] - want) <= 1e-9 * max(1.0, abs(want)), (E, eta, g[0, 0], want)


def test_decimation_rotated_stack_closed_form():
    """H00 = V diag(eps) V^H, H01 = I: independent chains in the rotated basis, so
    g_s = V diag(sigma(z - eps_c)) V^H, and Sigma with Hc = I equals it."""
    wl = make_uniform_chain(2, 8, 4, seed=9)
    V, eps = wl.meta["V"], wl.meta["eps"]
    H00 = wl.H[1, 0]
    H01 = np.eye(8, dtype=complex)
    # every energy at least 0.1 from the chain levels eps_c in {-1.5, -0.5, 0.5, 1.5}
    for E in (-2.5, -1.2, 0.1, 0.9, 3.1):
        z = E + 1e-6j
        g, steps = oracle.surface_gf(H00, H01, z)
        want = (V * surface_sigma(z - eps)[None, :]) @ V.conj().T
        assert rel_err(g, want) < 1e-9, E
        S, _ = oracle.lead_self_energy(H00, H01, np.eye(8), E, 1e-6)
        assert rel_err(S, want) < 1e-9


def test_decimation_against_long_finite_chain():
    """With broadening eta = 0.05 the surface block of (z - H_N)^{-1} for a finite
    chain of N layers approaches g_s exponentially in N (dense inverse, N = 300)."""
    rng = np.random.default_rng(12)
    b = 3
    A = (rng.standard_normal((b, b)) + 1j * rng.standard_normal((b, b))) / 4
    H00 = (A + A.conj().T) / 2
    H01 = (rng.standard_normal((b, b)) + 1j * rng.standard_normal((b, b))) / 3
    N = 300
    Hn = np.zeros((N * b, N * b), dtype=complex)
    for i in range(N):
        Hn[i * b:(i + 1) * b, i * b:(i + 1) * b] = H00
        if i + 1 < N:
            Hn[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = H01
            Hn[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = H01.conj().T
    for E in (-1.0, 0.2, 1.3):
        z = E + 0.05j
        gN = np.linalg.inv(z * np.eye(N * b) - Hn)[:b, :b]
        g, _ = oracle.surface_gf(H00, H01, z)
        assert rel_err(g, gN) < 1e-6, E


def test_decimation_fixed_point_and_causality():
    rng = np.random.default_rng(3)
    for b in (1, 4, 7):
        A = (rng.standard_normal((b, b)) + 1j * rng.standard_normal((b, b))) / 4
        H00 = (A + A.conj().T) / 2
        H01 = (rng.standard_normal((b, b)) + 1j * rng.standard_normal((b, b))) / 3
        for E in (-2.0, -0.4, 0.0, 0.7, 2.6):
            z = E + 1e-4j
            g, steps = oracle.surface_gf(H00, H01, z)
            assert steps > 0
            resid = g - np.linalg.inv(z * np.eye(b) - H00 - H01 @ g @ H01.conj().T)
            assert np.linalg.norm(resid) <= 1e-8 * np.linalg.norm(g)
            # retarded: the spectral function i (g - g^H) is positive semidefinite
            ev = np.linalg.eigvalsh(1j * (g - g.conj().T))
            assert ev.min() >= -1e-9 * max(1.0, ev.max())


def test_decimation_reports_no_convergence():
    g, steps = oracle.surface_gf(np.zeros((2, 2), complex), np.eye(2, dtype=complex), 0.5 + 1e-9j, max_iter=2)
    assert steps == -1 and np.all(np.isnan(g))


@pytest.mark.parametrize("l,b,w", [(1, 3, 1), (2, 2, 1), (5, 4, 1), (8, 3, 1), (6, 5, 2), (7, 2, 3)])
def test_lesser_matches_definition(l, b, w):
    wl = make_random(l, b, 1, 3, seed=40 + l * 7 + b, eta=1e-3)
    rng = np.random.default_rng(l + b)
    for e in range(wl.ne):
        fL, fR = rng.uniform(0, 1, 2)
        for eta_d in (0.0, 0.05):
            args = (wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
            dense = oracle.lesser_dense(wl.H, 1, *args[1:], fL, fR, eta_d)
            G, Gl = oracle.lesser(*args, fL, fR, eta_d)
            assert rel_err(Gl, dense) < 1e-11, (e, eta_d)


def test_lesser_equilibrium_identity():
    """Equal occupations and no device broadening: G^< = G^R Sigma^< G^A with
    Sigma^< = i f (Gamma_L + Gamma_R) = -f (Sigma^R - Sigma^A) gives
    G^< = -f (G^R - G^A) block by block (the optical theorem G^R - G^A =
    G^R (Sigma^R - Sigma^A) G^A)."""
    wl = make_random(9, 6, 1, 4, seed=5, eta=1e-3)
    for e in range(wl.ne):
        f = 0.37
        G, Gl = oracle.lesser(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], f, f, 0.0)
        l = wl.l
        for i in range(l):
            assert rel_err(Gl[1, i], -f * (G[1, i] - G[1, i].conj().T)) < 1e-10
            if i + 1 < l:
                # block (i, i+1) against G_{i,i+1} and G_{i+1,i}
                assert rel_err(Gl[2, i], -f * (G[2, i] - G[0, i + 1].conj().T)) < 1e-10


def test_lesser_anti_hermitian():
    wl = make_random(7, 5, 1, 2, seed=6, eta=1e-3)
    G, Gl = oracle.lesser(wl.H, wl.energies[1], wl.sigma_L[1], wl.sigma_R[1], 0.9, 0.1, 0.0)
    for i in range(wl.l):
        assert np.allclose(Gl[1, i], -Gl[1, i].conj().T, atol=1e-13)
        if i + 1 < wl.l:
            assert np.allclose(Gl[2, i], -Gl[0, i + 1].conj().T, atol=1e-13)


def test_lesser_uniform_chain_closed_form():
    """Uniform chain with eta_d = eta (a segment of the infinite chain): the first
    and last block columns are G_{i,0} = V diag(s_c^i / r_c) V^H and
    G_{i,l-1} = V diag(s_c^(l-1-i) / r_c) V^H (s_c = sigma(z - eps_c),
    r_c = sqrt(z - eps_c - 2) sqrt(z - eps_c + 2)), Gamma = V diag(-2 Im s_c) V^H,
    so with occupations (1, 0) and (0, 1) every band block of G^< has a closed form."""
    l, b = 40, 8
    wl = make_uniform_chain(l, b, 6, seed=106, eta=1e-2, eta_d=1e-2)
    V, eps = wl.meta["V"], wl.meta["eps"]
    for e in range(wl.ne):
        z = wl.energies[e] + 1j * wl.eta - eps
        s = surface_sigma(z)
        r = np.sqrt(z - 2.0) * np.sqrt(z + 2.0)
        gam = -2.0 * s.imag
        for fL, fR in ((1.0, 0.0), (0.0, 1.0)):
            G, Gl = oracle.lesser(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], fL, fR, wl.eta_d)
            for i in range(l):
                for k in (-1, 0, 1):
                    j = i + k
                    if not 0 <= j < l:
                        continue
                    if fL:
                        d = 1j * s ** i * np.conj(s) ** j * gam / np.abs(r) ** 2
                    else:
                        d = 1j * s ** (l - 1 - i) * np.conj(s) ** (l - 1 - j) * gam / np.abs(r) ** 2
                    want = (V * d[None, :]) @ V.conj().T
                    assert np.linalg.norm(Gl[1 + k, i] - want) <= 1e-10 * max(1e-300, np.linalg.norm(want)) + 1e-13


def test_dos_uniform_chain_closed_form():
    """A segment of the uniform chain with eta_d = eta is the infinite chain seen on l
    layers, whose on-site Green's function is V diag(1 / r_c) V^H with
    r_c = sqrt(z - eps_c - 2) sqrt(z - eps_c + 2): the DOS of every orbital is
    -(1/pi) Im (V diag(1 / r_c) V^H)_ss, and a layer's total is sum_c -(1/pi) Im(1/r_c),
    which for eta -> 0 inside a channel's band is 1 / (pi sqrt(4 - (E - eps_c)^2))."""
    l, b = 24, 8
    wl = make_uniform_chain(l, b, 5, seed=106, eta=1e-2, eta_d=1e-2)
    V, eps = wl.meta["V"], wl.meta["eps"]
    for e in range(wl.ne):
        z = wl.energies[e] + 1j * wl.eta - eps
        r = np.sqrt(z - 2.0) * np.sqrt(z + 2.0)
        want = -np.imag(np.diagonal((V / r[None, :]) @ V.conj().T)) / np.pi
        G = oracle.rgf(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], wl.eta_d)["G"]
        d = oracle.dos(G, 1).reshape(l, b)
        assert np.max(np.abs(d - want[None, :])) <= 1e-10 * np.max(np.abs(want))
        assert np.allclose(d.sum(axis=1), np.sum(-np.imag(1.0 / r)) / np.pi, rtol=1e-10)
    # the eta -> 0 limit of one channel inside its band
    x = 0.7
    zz = x + 1e-9j
    assert abs(-np.imag(1.0 / (np.sqrt(zz - 2.0) * np.sqrt(zz + 2.0))) / np.pi
               - 1.0 / (np.pi * np.sqrt(4.0 - x * x))) < 1e-7


def test_density_equilibrium_is_occupation_times_dos():
    """With both leads at the same occupation f(E) and no device broadening,
    G^< = i f A with A = i (G^R - G^A) = -2 Im-part on the diagonal, so the density is
    sum_e w_e f_e dos_e orbital by orbital (the definition of G^< via the dense inverse
    on one side, the DOS of the RGF band on the other)."""
    wl = make_random(8, 5, 1, 6, seed=12, eta=1e-3)
    f = 1.0 / (1.0 + np.exp((wl.energies - 0.1) / 0.3))
    wts = np.full(wl.ne, 4.0 / wl.ne)
    bands, want = [], 0.0
    for e in range(wl.ne):
        bands.append(oracle.lesser_dense(wl.H, 1, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], f[e], f[e], 0.0))
        G = oracle.rgf(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], 0.0)["G"]
        want = want + wts[e] * f[e] * oracle.dos(G, 1)
    got = oracle.density(bands, wts, 1)
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))
    assert np.all(got > 0)


def test_density_dos_pick_the_diagonal():
    """A planted band: the DOS and density read the s-th diagonal entry of the diagonal
    blocks only (an off-diagonal entry or block changes nothing)."""
    l, b, w = 3, 2, 2
    G = np.zeros((2 * w + 1, l, b, b), dtype=np.complex128)
    for i in range(l):
        for s in range(b):
            G[w, i, s, s] = 1.0 - 1j * (1 + i * b + s)
    G[w, 1, 0, 1] = 5j
    G[w + 1, 0] = 7j
    assert np.allclose(oracle.dos(G, w), np.arange(1, l * b + 1) / np.pi)
    assert np.allclose(oracle.density([G, 2 * G], [0.5, 0.25], w), -np.arange(1, l * b + 1) / (2 * np.pi))


@pytest.mark.parametrize("fL,fR", [(1.0, 0.0), (0.3, 0.8)])
def test_bond_current_is_conserved_and_landauer(fL, fR):
    """In steady state without device broadening the particle current is the same
    through every bond and equals the Landauer current T(E) (f_L - f_R) / 2pi, T the
    Caroli transmission (a relation between the lesser band and G_{0,l-1} alone)."""
    wl = make_random(10, 6, 1, 5, seed=21, eta=1e-3)
    for e in range(wl.ne):
        G, Gl = oracle.lesser(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], fL, fR, 0.0)
        r = oracle.rgf(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], 0.0)
        T = oracle.transmission(r["row0"][wl.l - 1], wl.sigma_L[e], wl.sigma_R[e])
        j = oracle.bond_current(wl.H, Gl)
        want = T * (fL - fR) / (2 * np.pi)
        assert np.max(np.abs(j - want)) <= 1e-10 * max(abs(want), 1e-3), (e, j, want)


def test_bond_current_uniform_chain_counts_channels():
    """Uniform chain, leads (1, 0): every bond carries (open channels) / 2pi."""
    wl = make_uniform_chain(12, 8, 6, seed=106, eta=1e-6)
    eps = wl.meta["eps"]
    for e in range(wl.ne):
        _, Gl = oracle.lesser(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], 1.0, 0.0, 0.0)
        j = oracle.bond_current(wl.H, Gl)
        n_open = np.sum(np.abs(wl.energies[e] - eps) < 2)
        assert np.max(np.abs(j - n_open / (2 * np.pi))) < 1e-6
