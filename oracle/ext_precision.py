"""Extended-precision reference for the selected inverse — test infrastructure only.

The FP64 oracle and the GPU path both run the block elimination of the paper
without pivoting across blocks, so both carry rounding errors amplified by the
condition numbers of the Schur pivots.  To tell how far each of them is from the
exact selected inverse, this module runs the same elimination (Sec. 2.3: the
n-diagonal upward pass of Proposition 3 and the downward recursions for the band;
Sec. 2.2, Algorithm 1 is its w = 1 case) in the x87 80-bit extended format
(NumPy ``longdouble``: 64-bit significand, unit roundoff 2^-64 ~ 5.4e-20, i.e.
2048 times smaller than FP64's).  LAPACK has no such precision, so the LU
factorisation with partial row pivoting and the triangular solves are written out
here; products use NumPy's own (non-BLAS) long-double loops.

At a pivot condition number kappa the result is accurate to roughly kappa * 1e-19,
so for kappa up to ~1e8 it serves as the exact answer against which FP64 errors of
1e-13 .. 1e-8 are measured.  Slow by design: about 30 s per energy for a chain of
256 layers of 128 orbitals.
"""
from __future__ import annotations

from typing import Callable, Dict, Optional

import numpy as np

CT = np.clongdouble


def lu_factor_ext(A: np.ndarray):
    """P A = L U with partial row pivoting (largest |a| in each column), in extended
    precision.  Returns (LU, perm) with L unit lower (below the diagonal of LU), U
    upper, and perm such that A[perm] = L U."""
    LU = np.array(A, dtype=CT, copy=True)
    n = LU.shape[0]
    perm = np.arange(n)
    for k in range(n):
        p = k + int(np.argmax(np.abs(LU[k:, k])))
        if LU[p, k] == 0:
            raise np.linalg.LinAlgError("singular pivot")
        if p != k:
            LU[[k, p]] = LU[[p, k]]
            perm[[k, p]] = perm[[p, k]]
        LU[k + 1:, k] /= LU[k, k]
        LU[k + 1:, k + 1:] -= np.outer(LU[k + 1:, k], LU[k, k + 1:])
    return LU, perm


def lu_solve_ext(lu, B: np.ndarray) -> np.ndarray:
    """A^{-1} B from the factors of A (forward then back substitution)."""
    LU, perm = lu
    n = LU.shape[0]
    X = np.array(B, dtype=CT, copy=True)[perm]
    for i in range(1, n):
        X[i] -= LU[i, :i] @ X[:i]
    for i in range(n - 1, -1, -1):
        if i + 1 < n:
            X[i] -= LU[i, i + 1:] @ X[i + 1:]
        X[i] /= LU[i, i]
    return X


def lu_solve_right_ext(B: np.ndarray, lu) -> np.ndarray:
    """B A^{-1} from the factors of A:  with A = P^T L U,  B A^{-1} = B U^{-1} L^{-1} P,
    solved column block by column block (right substitutions)."""
    LU, perm = lu
    n = LU.shape[0]
    Y = np.array(B, dtype=CT, copy=True)
    # Y U = B  (columns left to right)
    for j in range(n):
        if j:
            Y[:, j] -= Y[:, :j] @ LU[:j, j]
        Y[:, j] /= LU[j, j]
    # Z L = Y  (columns right to left, L unit lower)
    for j in range(n - 2, -1, -1):
        Y[:, j] -= Y[:, j + 1:] @ LU[j + 1:, j]
    # undo the row permutation of A: B A^{-1} = Z P, i.e. column j of Z goes to column perm[j]
    out = np.empty_like(Y)
    out[:, perm] = Y
    return out


def nrgf_ext(Mb: Callable[[int, int], Optional[np.ndarray]], l: int, b: int, w: int,
             first_row: bool = True) -> Dict[str, np.ndarray]:
    """Band of M^{-1} for the block n-diagonal matrix whose blocks ``Mb`` returns, by
    the n-diagonal RGF of Sec. 2.3 in extended precision.

    Upward pass, layers l-1 .. 0: factor the Schur pivot S_ii; form
    U_{c,i} = S_{c,i} S_ii^{-1} and L_{i,c} = S_ii^{-1} S_{i,c} for c in
    C_i = [max(0, i-w), i-1]; update S_{a,c} -= S_{a,i} L_{i,c} for a, c in C_i.
    Downward pass: G_00 = S_00^{-1}; then for i = 1 .. l-1 and a in C_i,
    G_{a,i} = -sum_c G_{a,c} U_{c,i}, G_{i,a} = -sum_c L_{i,c} G_{c,a}, and
    G_ii = S_ii^{-1} - sum_c L_{i,c} G_{c,i}.  With ``first_row`` also the first block
    row G_{0,i} = -sum_c G_{0,c} U_{c,i} (for the transmission).

    Returns {"G": band [2w+1, l, b, b] (clongdouble), "row0": [l, b, b]}."""
    S: Dict[tuple, np.ndarray] = {}
    for i in range(l):
        for j in range(max(0, i - w), min(l, i + w + 1)):
            S[(i, j)] = np.array(Mb(i, j), dtype=CT, copy=True)
    lu = [None] * l
    U: Dict[tuple, np.ndarray] = {}
    L: Dict[tuple, np.ndarray] = {}
    for i in range(l - 1, -1, -1):
        lu[i] = lu_factor_ext(S[(i, i)])
        C = range(max(0, i - w), i)
        for c in C:
            U[(c, i)] = lu_solve_right_ext(S[(c, i)], lu[i])
            L[(i, c)] = lu_solve_ext(lu[i], S[(i, c)])
        for a in C:
            for c in C:
                S[(a, c)] = S[(a, c)] - S[(a, i)] @ L[(i, c)]
    eye = np.eye(b, dtype=CT)
    G: Dict[tuple, np.ndarray] = {(0, 0): lu_solve_ext(lu[0], eye)}
    row0 = np.zeros((l, b, b), dtype=CT)
    row0[0] = G[(0, 0)]
    for i in range(1, l):
        C = list(range(max(0, i - w), i))
        for a in C:
            acc = np.zeros((b, b), dtype=CT)
            for c in C:
                acc -= G[(a, c)] @ U[(c, i)]
            G[(a, i)] = acc
            acc = np.zeros((b, b), dtype=CT)
            for c in C:
                acc -= L[(i, c)] @ G[(c, a)]
            G[(i, a)] = acc
        acc = lu_solve_ext(lu[i], eye)
        for c in C:
            acc = acc - L[(i, c)] @ G[(c, i)]
        G[(i, i)] = acc
        if first_row:
            if 0 in C:
                row0[i] = G[(0, i)]
            else:
                acc = np.zeros((b, b), dtype=CT)
                for c in C:
                    acc -= row0[c] @ U[(c, i)]
                row0[i] = acc
    band = np.zeros((2 * w + 1, l, b, b), dtype=CT)
    for (i, j), blk in G.items():
        band[w + j - i, i] = blk
    return {"G": band, "row0": row0}


def block_accessor_ext(H, w, E, sigma_L, sigma_R, eta_d=0.0):
    """Blocks of M(E) = (E + i eta_d) I - H - Sigma_L (+) Sigma_R (Sec. 2 introduction),
    formed in extended precision from the FP64 inputs (the inputs are exact in both
    formats; only the arithmetic differs)."""
    l, b = H.shape[1], H.shape[2]
    z = CT(E) + CT(1j) * CT(eta_d)
    eye = np.eye(b, dtype=CT)

    def M(i, j):
        k = j - i
        if abs(k) > w or not (0 <= i < l) or not (0 <= j < l):
            return None
        if k != 0:
            return -np.asarray(H[w + k, i], dtype=CT)
        blk = z * eye - np.asarray(H[w, i], dtype=CT)
        if i == 0:
            blk = blk - np.asarray(sigma_L, dtype=CT)
        if i == l - 1:
            blk = blk - np.asarray(sigma_R, dtype=CT)
        return blk

    return M


def transmission_ext(G_first_last, sigma_L, sigma_R) -> float:
    """T = Re Tr[Gamma_L G_{0,l-1} Gamma_R G_{0,l-1}^H], Gamma = i (Sigma - Sigma^H),
    evaluated in extended precision."""
    sl = np.asarray(sigma_L, dtype=CT)
    sr = np.asarray(sigma_R, dtype=CT)
    gl = CT(1j) * (sl - sl.conj().T)
    gr = CT(1j) * (sr - sr.conj().T)
    R = np.asarray(G_first_last, dtype=CT)
    return float(np.real(np.trace(gl @ R @ gr @ R.conj().T)))


def solve_energy_ext(H, w, E, sigma_L, sigma_R, eta_d=0.0):
    """(band of G in extended precision, T) for one energy of a workload."""
    l, b = H.shape[1], H.shape[2]
    r = nrgf_ext(block_accessor_ext(H, w, E, sigma_L, sigma_R, eta_d), l, b, w)
    return r["G"], transmission_ext(r["row0"][l - 1], sigma_L, sigma_R)
