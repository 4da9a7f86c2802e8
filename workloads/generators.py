"""Seeded generators for block n-diagonal NEGF test systems.

Inputs only: a Hermitian block band H, the retarded lead self-energies of two
semi-infinite one-dimensional leads, and a midpoint energy grid.  The matrix whose
selected inverse is wanted is M(E) = (E + i*eta_d) I - H - Sigma_L(E) (+) Sigma_R(E),
with Sigma_L on the first layer and Sigma_R on the last one (paper, Sec. 2
introduction: M := E I - H - Sigma^r).  The paper's own test matrices are synthetic
and random (Sec. 4, footnote of Sec. 2); the exact recipe below is this project's.

Band layout used everywhere in this repository: ``H[w + k, i]`` is the b x b block
(i, i + k) for k in [-w, w]; blocks whose column i + k falls outside [0, l) are
zero and never read.  Blocks are row-major complex128 (interleaved re/im pairs).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np


# ----------------------------------------------------------------------------
# Lead self-energy and energy grid
# ----------------------------------------------------------------------------

def surface_sigma(z):
    """Closed-form surface Green's function of a semi-infinite chain with on-site
    energy 0 and hopping 1, i.e. the self-energy a unit hopping adds to the site the
    chain is attached to:  sigma(z) = (z - sqrt(z - 2) * sqrt(z + 2)) / 2, with
    principal square roots.  For Im z > 0 this is the retarded branch: Im sigma < 0
    inside the band |Re z| < 2 and |sigma| < 1 outside it."""
    z = np.asarray(z, dtype=np.complex128)
    return 0.5 * (z - np.sqrt(z - 2.0) * np.sqrt(z + 2.0))


def midpoint_grid(lo: float, hi: float, n: int) -> np.ndarray:
    """n energies at the midpoints of n equal cells of [lo, hi]; never hits the
    band edges lo, hi themselves."""
    k = np.arange(n, dtype=np.float64)
    return lo + (hi - lo) * (k + 0.5) / n


def lead_sigma(energies: np.ndarray, eta: float, b: int,
               onsite: Optional[np.ndarray] = None,
               basis: Optional[np.ndarray] = None) -> np.ndarray:
    """Retarded self-energy [nE, b, b] of a lead made of b independent unit-hopping
    chains, one per orbital of the contact layer.  With ``onsite``/``basis`` the b
    chains have on-site energies eps_c and are rotated by the unitary ``basis``:
    Sigma = V diag(sigma(E + i*eta - eps_c)) V^H."""
    energies = np.asarray(energies, dtype=np.float64)
    ne = energies.shape[0]
    z = energies + 1j * eta
    out = np.zeros((ne, b, b), dtype=np.complex128)
    if onsite is None:
        s = surface_sigma(z)
        idx = np.arange(b)
        out[:, idx, idx] = s[:, None]
        return out
    eps = np.asarray(onsite, dtype=np.float64)
    s = surface_sigma(z[:, None] - eps[None, :])          # [nE, b]
    V = np.asarray(basis, dtype=np.complex128)
    for e in range(ne):
        out[e] = (V * s[e][None, :]) @ V.conj().T
    return out


# ----------------------------------------------------------------------------
# Random Hermitian block band
# ----------------------------------------------------------------------------

def _cn(rng: np.random.Generator, shape) -> np.ndarray:
    """Complex Gaussian with real and imaginary parts iid N(0, 1) / 4 (real part
    drawn first)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / 4.0


def random_hermitian_band(l: int, b: int, w: int, seed, far_scale: float = 0.3) -> np.ndarray:
    """Hermitian block band H[2w+1, l, b, b].

    Draw order: the l diagonal blocks A_i (H_ii = (A_i + A_i^H)/2), then the l-1
    nearest-neighbour blocks B_i = H_{i,i+1} (H_{i+1,i} = B_i^H), then for each
    further distance d = 2..w the l-d blocks far_scale**(d-1) * C_i = H_{i,i+d}."""
    if w < 1 or l < 1 or b < 1:
        raise ValueError("need l >= 1, b >= 1, w >= 1")
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    H = np.zeros((2 * w + 1, l, b, b), dtype=np.complex128)
    A = _cn(rng, (l, b, b))
    H[w] = 0.5 * (A + np.conj(np.swapaxes(A, 1, 2)))
    for d in range(1, w + 1):
        n = l - d
        if n <= 0:
            # draw nothing for bands wider than the chain
            continue
        C = _cn(rng, (n, b, b))
        if d > 1:
            C = C * (far_scale ** (d - 1))
        H[w + d, :n] = C
        H[w - d, d:] = np.conj(np.swapaxes(C, 1, 2))
    return H


def band_block(H: np.ndarray, w: int, i: int, j: int) -> Optional[np.ndarray]:
    """Block (i, j) of a band array, or None when |i - j| > w or out of range."""
    l = H.shape[1]
    k = j - i
    if abs(k) > w or not (0 <= i < l) or not (0 <= j < l):
        return None
    return H[w + k, i]


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    """One system: band H, energies and the two lead self-energies per energy."""
    name: str
    l: int
    b: int
    w: int
    H: np.ndarray                 # [2w+1, l, b, b] complex128
    energies: np.ndarray          # [nE] float64
    sigma_L: np.ndarray           # [nE, b, b] complex128 (retarded, includes +i*eta)
    sigma_R: np.ndarray           # [nE, b, b] complex128
    eta: float                    # broadening used inside the lead self-energy
    eta_d: float = 0.0            # optional broadening added on the device diagonal
    domains: int = 0              # DDRGF interior/separator pairs used by the config
    meta: Dict = field(default_factory=dict)

    @property
    def ne(self) -> int:
        return int(self.energies.shape[0])

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx)
        return Workload(self.name + "[sub]", self.l, self.b, self.w, self.H,
                        self.energies[idx], self.sigma_L[idx], self.sigma_R[idx],
                        self.eta, self.eta_d, self.domains, dict(self.meta))


def make_random(l: int, b: int, w: int, ne: int, seed, e_lo=-2.0, e_hi=2.0,
                eta=1e-6, eta_d=0.0, domains=0, name="random") -> Workload:
    H = random_hermitian_band(l, b, w, seed)
    E = midpoint_grid(e_lo, e_hi, ne)
    sig = lead_sigma(E, eta, b)
    return Workload(name, l, b, w, H, E, sig, sig.copy(), eta, eta_d, domains)


def make_uniform_chain(l: int, b: int, ne: int, seed: int = 106, eta: float = 1e-6,
                       eta_d: float = 0.0, e_lo=-2.0, e_hi=2.0,
                       levels=(-1.5, -0.5, 0.5, 1.5)) -> Workload:
    """Segment of an infinite uniform chain: H_ii = V diag(eps) V^H, H_{i,i+-1} = I,
    leads are the same chain continued to +-infinity.  V is a Haar-like unitary
    (QR of a complex Gaussian, phases of R's diagonal moved into Q)."""
    rng = np.random.default_rng(seed)
    X = _cn(rng, (b, b))
    Q, R = np.linalg.qr(X)
    d = np.diag(R)
    Q = Q * (d / np.abs(d))[None, :]
    if b % len(levels) == 0:
        eps = np.repeat(np.asarray(levels, dtype=np.float64), b // len(levels))
    else:
        eps = np.resize(np.asarray(levels, dtype=np.float64), b)
    w = 1
    H = np.zeros((3, l, b, b), dtype=np.complex128)
    H0 = (Q * eps[None, :]) @ Q.conj().T
    H0 = 0.5 * (H0 + H0.conj().T)
    H[1] = H0[None]
    I = np.eye(b, dtype=np.complex128)
    H[2, : l - 1] = I
    H[0, 1:] = I
    E = midpoint_grid(e_lo, e_hi, ne)
    sig = lead_sigma(E, eta, b, onsite=eps, basis=Q)
    wl = Workload("uniform_chain", l, b, w, H, E, sig, sig.copy(), eta, eta_d)
    wl.meta.update(V=Q, eps=eps)
    return wl


def make_dominant(l: int, b: int, w: int, ne: int, seed, e_lo=-2.0, e_hi=2.0, eta=1e-6,
                  name="dominant") -> Workload:
    """Block diagonally dominant random system, the class of test matrices of the
    paper's numerical experiments (Sec. "Numerical experiments", RGF n = 3): the
    random Hermitian band of :func:`random_hermitian_band` with every diagonal block
    shifted by s I, s = ||H_ii||_2 max + 2 (sum over j != i of ||H_ij||_2) max +
    max(|e_lo|, |e_hi|) + 1 (the lead self-energy has |sigma| <= 1).  Then
    ||(E - H_ii - s - Sigma)^{-1}|| * sum_j ||H_ij|| <= 1/2 at every energy of the
    grid, so every Schur pivot and every closed DDRGF interior is well
    conditioned.  The device levels sit far above the lead band, so T is
    tiny; the point is the selected inverse."""
    H = random_hermitian_band(l, b, w, seed)
    off = np.zeros(l)
    for k in range(-w, w + 1):
        if k == 0:
            continue
        for i in range(l):
            if 0 <= i + k < l:
                off[i] += np.linalg.norm(H[w + k, i], 2)
    diag = max(np.linalg.norm(H[w, i], 2) for i in range(l))
    s = diag + 2.0 * off.max() + max(abs(e_lo), abs(e_hi)) + 1.0
    H[w] += s * np.eye(b)[None]
    E = midpoint_grid(e_lo, e_hi, ne)
    sig = lead_sigma(E, eta, b)
    wl = Workload(name, l, b, w, H, E, sig, sig.copy(), eta)
    wl.meta.update(shift=s)
    return wl


# The five benchmark workloads (sizes, grids and broadenings) plus the uniform chain.
CONFIGS = {
    1: dict(l=16, b=16, w=1, ne=4, e_lo=-1.0, e_hi=1.0, eta=1e-3, seed=101, domains=2),
    2: dict(l=256, b=128, w=1, ne=64, e_lo=-2.0, e_hi=2.0, eta=1e-6, seed=102, domains=8),
    3: dict(l=512, b=64, w=2, ne=128, e_lo=-2.0, e_hi=2.0, eta=1e-4, seed=103, domains=16),
    4: dict(devices=64, ne=16, e_lo=-2.0, e_hi=2.0, eta=1e-6, seed=104,
            b_choices=(32, 64, 96, 128), l_lo=64, l_hi=512),
    5: dict(l=256, b=64, w=1, ne=256, e_lo=-2.0, e_hi=2.0, eta=1e-6, seed=105, domains=8),
}


def make_config(n: int, **over):
    """Workload for benchmark configuration n (1..5).  Keyword overrides replace
    entries of the recipe (e.g. ``ne=8`` for a cheaper subset).  Configuration 4
    returns a list of per-device workloads."""
    cfg = dict(CONFIGS[n])
    cfg.update(over)
    if n == 4:
        meta_rng = np.random.default_rng(cfg["seed"])
        nd = cfg["devices"]
        bs = meta_rng.choice(np.asarray(cfg["b_choices"]), size=nd)
        ls = meta_rng.integers(cfg["l_lo"], cfg["l_hi"] + 1, size=nd)
        seeds = np.random.SeedSequence(cfg["seed"]).spawn(nd)
        out: List[Workload] = []
        for d in range(nd):
            wl = make_random(int(ls[d]), int(bs[d]), 1, cfg["ne"], np.random.default_rng(seeds[d]),
                             cfg["e_lo"], cfg["e_hi"], cfg["eta"], name=f"config4/device{d}")
            out.append(wl)
        return out
    wl = make_random(cfg["l"], cfg["b"], cfg["w"], cfg["ne"], cfg["seed"], cfg["e_lo"], cfg["e_hi"],
                     cfg["eta"], cfg.get("eta_d", 0.0), cfg.get("domains", 0), name=f"config{n}")
    return wl
