"""Selected blocks of the lesser Green's function — test infrastructure only (see the
package docstring).

The Keldysh equation G^< = G^R Sigma^< G^A is the step after the Dyson equation the
paper solves (Sec. 1, and the outlook's recursive Keldysh stage).  Here the only
lesser self-energies are the two leads': Sigma^<_X = i f_X Gamma_X on the layer lead
X attaches to, Gamma_X = i (Sigma_X - Sigma_X^H), f_X the lead's occupation at this
energy.  Device broadening eta_d, when present, enters G^R only; it carries no
lesser self-energy of its own.

* :func:`lesser_dense` is the definition, on the assembled matrix;
* :func:`lesser` uses the first and last block columns of G^R from Algorithm 1's
  extras (:func:`rgf`): G^<_ij = G_{i,0} Sigma^<_L G_{j,0}^H + G_{i,l-1} Sigma^<_R
  G_{j,l-1}^H for |i - j| <= 1.
"""
from __future__ import annotations

import numpy as np

from .rgf_oracle import dense_matrix, gamma_of, rgf


def lesser_dense(H, w, E, sigma_L, sigma_R, f_L: float, f_R: float, eta_d=0.0):
    """Band of G^< = M^{-1} Sigma^< M^{-H} (layout [2w+1, l, b, b])."""
    l, b = H.shape[1], H.shape[2]
    G = np.linalg.inv(dense_matrix(H, w, E, sigma_L, sigma_R, eta_d))
    S = np.zeros((l * b, l * b), dtype=np.complex128)
    S[:b, :b] += 1j * f_L * gamma_of(sigma_L)
    S[(l - 1) * b:, (l - 1) * b:] += 1j * f_R * gamma_of(sigma_R)
    Gl = G @ S @ G.conj().T
    out = np.zeros((2 * w + 1, l, b, b), dtype=np.complex128)
    for i in range(l):
        for k in range(-w, w + 1):
            j = i + k
            if 0 <= j < l:
                out[w + k, i] = Gl[i * b:(i + 1) * b, j * b:(j + 1) * b]
    return out


def lesser(H, E, sigma_L, sigma_R, f_L: float, f_R: float, eta_d=0.0):
    """Block tridiagonal systems: (band of G^R, band of G^<), each [3, l, b, b]."""
    res = rgf(H, E, sigma_L, sigma_R, eta_d, extras=True)
    l, b = H.shape[1], H.shape[2]
    sl_L = 1j * f_L * gamma_of(sigma_L)
    sl_R = 1j * f_R * gamma_of(sigma_R)
    c0, cL = res["col0"], res["colL"]
    out = np.zeros((3, l, b, b), dtype=np.complex128)
    for i in range(l):
        for k in (-1, 0, 1):
            j = i + k
            if 0 <= j < l:
                out[1 + k, i] = c0[i] @ sl_L @ c0[j].conj().T + cL[i] @ sl_R @ cL[j].conj().T
    return res["G"], out


# ----------------------------------------------------------------------------
# Observables on a solved band (the densities the Dyson and Keldysh stages give)
# ----------------------------------------------------------------------------

def dos(G_band: np.ndarray, w: int) -> np.ndarray:
    """Orbital-resolved density of states of one energy, -(1/pi) Im G^R_{ii,ss},
    from the diagonal blocks of a band [2w+1, l, b, b]; returns [l * b]."""
    diag = G_band[w]
    return -np.imag(np.diagonal(diag, axis1=1, axis2=2)).reshape(-1) / np.pi


def density(Gless_bands, weights, w: int) -> np.ndarray:
    """Orbital-resolved electron density, the energy quadrature
    sum_e weights[e] (1/2pi) Im G^<_{ii,ss}(E_e) (G^<_ss = i a with a >= 0, so
    -i G^<_ss / 2pi is the spectral density of occupied states); [l * b]."""
    out = None
    for g, wt in zip(Gless_bands, weights):
        x = wt * np.imag(np.diagonal(g[w], axis1=1, axis2=2)).reshape(-1) / (2.0 * np.pi)
        out = x if out is None else out + x
    return out


def bond_current(H: np.ndarray, Gless_band: np.ndarray) -> np.ndarray:
    """Spectral particle current from layer i to layer i+1 at one energy (w = 1,
    hbar = 1, spin not counted): with rho = <c^dag c> = -i int dE/2pi G^<, the rate
    of change of the charge on layer i through the bond (i, i+1) gives
    j_i(E) = (1/pi) Re Tr[H_{i,i+1} G^<_{i+1,i}(E)]; returns [l - 1]."""
    l = H.shape[1]
    out = np.empty(l - 1)
    for i in range(l - 1):
        out[i] = np.real(np.trace(H[2, i] @ Gless_band[0, i + 1])) / np.pi
    return out
