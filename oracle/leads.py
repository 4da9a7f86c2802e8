"""Retarded self-energies of semi-infinite periodic leads.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper takes the retarded lead self-energies as given inputs of the selected
inversion (Sec. 2, where M = E I - H - Sigma^r is introduced).  The step before the
path computes them.  A lead is a half-infinite repetition of identical principal
layers with on-layer block H00 and coupling H01 from each layer to the next one
away from the device.  Its surface Green's function g_s is the solution of the
Dyson fixed point g_s = (z - H00 - H01 g_s H10)^{-1}, z = E + i eta, H10 = H01^H,
with negative semidefinite Im part; the self-energy the lead adds to the device
layer it touches is Sigma = Hc g_s Hc^H, Hc the coupling from that device layer to
the lead's surface layer.

g_s is computed here by the decimation iteration of Lopez Sancho, Lopez Sancho and
Rubio (J. Phys. F 15, 851 (1985)).  Every step eliminates every other layer of the
remaining chain, so the couplings alpha (away from the device) and beta (towards
it) then reach twice as far:
    g      = (z - eps)^{-1}
    eps_s <- eps_s + alpha g beta
    eps   <- eps + alpha g beta + beta g alpha
    alpha <- alpha g alpha,   beta <- beta g beta
starting from eps_s = eps = H00, alpha = H01, beta = H10, until
max|alpha| + max|beta| < tol; then g_s = (z - eps_s)^{-1}.  The number of steps
grows like log2 of the decay length 1/eta.
"""
from __future__ import annotations

import numpy as np


def surface_gf(H00: np.ndarray, H01: np.ndarray, z: complex, tol: float = 1e-14, max_iter: int = 100):
    """Surface Green's function of the semi-infinite lead by decimation.

    Returns (g_s, steps): steps is the number of decimation steps taken when the
    couplings fell below ``tol``; (NaN block, -1) when ``max_iter`` steps did not get
    there."""
    b = H00.shape[0]
    eye = np.eye(b, dtype=np.complex128)
    eps_s = np.array(H00, dtype=np.complex128)
    eps = eps_s.copy()
    alpha = np.array(H01, dtype=np.complex128)
    beta = alpha.conj().T.copy()
    for step in range(1, max_iter + 1):
        g = np.linalg.inv(z * eye - eps)
        ag = alpha @ g
        bg = beta @ g
        agb = ag @ beta
        bga = bg @ alpha
        eps_s = eps_s + agb
        eps = eps + agb + bga
        alpha = ag @ alpha
        beta = bg @ beta
        if np.abs(alpha).max() + np.abs(beta).max() < tol:
            return np.linalg.inv(z * eye - eps_s), step
    return np.full((b, b), np.nan + 1j * np.nan), -1


def lead_self_energy(H00, H01, Hc, E: float, eta: float, tol: float = 1e-14, max_iter: int = 100):
    """Sigma = Hc g_s Hc^H at one energy.  Returns (Sigma, steps)."""
    gs, steps = surface_gf(H00, H01, E + 1j * eta, tol, max_iter)
    Hc = np.asarray(Hc, dtype=np.complex128)
    return Hc @ gs @ Hc.conj().T, steps


def lead_self_energies(H00, H01, Hc, energies, eta: float, tol: float = 1e-14, max_iter: int = 100):
    """Sigma at every energy of a grid: (Sigma [nE, b, b], steps [nE])."""
    out = [lead_self_energy(H00, H01, Hc, float(E), eta, tol, max_iter) for E in energies]
    return np.stack([s for s, _ in out]), np.array([k for _, k in out], dtype=np.int32)
