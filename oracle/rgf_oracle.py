"""Plain FP64 CPU oracle — test infrastructure only (never called by the GPU path).

Everything here works on ONE energy at a time, in complex128, with LAPACK (through
SciPy) for LU factorisations and triangular solves and NumPy for products.  No
blocking, fusion or reordering beyond what the paper's algorithms state.

Paper: "Revisiting recursive methods for Dyson and Keldysh in NEGF: Part I".
  * Sec. 2.1, eqs. (2x2 UDL factorisation / explicit inverse): one Schur step.
  * Sec. 2.2, Algorithm 1 (RGF for block tridiagonal systems), eqs. (2x2 / 4x4
    exact RGF) and the cost model eq. (cost_model_RGF).
  * Sec. 2.3, Proposition 3 and the prose description of the n-diagonal downward
    pass; op counts eq. (cost_model_general_RGF).
  * Sec. 3, eqs. (T_hat structure, 2x2 explicit inverse for DDRGF, Schur
    complement in DDRGF), Proposition 4, the data-dependency discussion and
    Algorithm 2 (DDRGF).
Transmission and the on-site gradient are not in the paper (it stops at G^R); the
readings used here are the Caroli trace with leads on the first and last layer and
the first-order perturbation dG = G dH G.

Band layout: H[w + k, i] is block (i, i + k); the same layout is used for outputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np
import scipy.linalg as sla


# ----------------------------------------------------------------------------
# Operation counter (for the paper's op-count formulas)
# ----------------------------------------------------------------------------

@dataclass
class OpCounter:
    lu: int = 0
    getrs: int = 0
    gemm: int = 0
    extra_gemm: int = 0      # products spent on halos/extras, not in the paper's RGF count

    def as_tuple(self):
        return (self.lu, self.getrs, self.gemm)


class _Ops:
    """LU / GETRS / GEMM with optional counting."""

    def __init__(self, counter: Optional[OpCounter], extra: bool = False):
        self.c = counter
        self.extra = extra

    def lu(self, A):
        if self.c is not None:
            self.c.lu += 1
        return sla.lu_factor(A, check_finite=False)

    def solve_left(self, lu, B):
        """S^{-1} B (GETRS)."""
        if self.c is not None:
            self.c.getrs += 1
        return sla.lu_solve(lu, B, trans=0, check_finite=False)

    def solve_right(self, B, lu):
        """B S^{-1}, computed as (S^T)^{-1} B^T transposed (GETRS on the transpose)."""
        if self.c is not None:
            self.c.getrs += 1
        return sla.lu_solve(lu, B.T, trans=1, check_finite=False).T

    def gemm(self, A, B):
        if self.c is not None:
            if self.extra:
                self.c.extra_gemm += 1
            else:
                self.c.gemm += 1
        return A @ B


# ----------------------------------------------------------------------------
# Assembly of M(E) = (E + i eta_d) I - H - Sigma_L (+) Sigma_R   (Sec. 2 intro)
# ----------------------------------------------------------------------------

def block_accessor(H: np.ndarray, w: int, E: float, sigma_L: np.ndarray, sigma_R: np.ndarray,
                   eta_d: float = 0.0) -> Callable[[int, int], Optional[np.ndarray]]:
    """Return M(i, j): block (i, j) of M(E), or None outside the band."""
    l, b = H.shape[1], H.shape[2]
    z = E + 1j * eta_d
    eye = np.eye(b, dtype=np.complex128)

    def M(i: int, j: int):
        k = j - i
        if abs(k) > w or i < 0 or j < 0 or i >= l or j >= l:
            return None
        if k != 0:
            return -H[w + k, i]
        blk = z * eye - H[w, i]
        if i == 0:
            blk = blk - sigma_L
        if i == l - 1:
            blk = blk - sigma_R
        return blk

    return M


def dense_matrix(H, w, E, sigma_L, sigma_R, eta_d=0.0) -> np.ndarray:
    l, b = H.shape[1], H.shape[2]
    Mb = block_accessor(H, w, E, sigma_L, sigma_R, eta_d)
    M = np.zeros((l * b, l * b), dtype=np.complex128)
    for i in range(l):
        for j in range(max(0, i - w), min(l, i + w + 1)):
            M[i * b:(i + 1) * b, j * b:(j + 1) * b] = Mb(i, j)
    return M


def _band_of_dense(G: np.ndarray, l: int, b: int, w: int) -> np.ndarray:
    out = np.zeros((2 * w + 1, l, b, b), dtype=np.complex128)
    for i in range(l):
        for k in range(-w, w + 1):
            j = i + k
            if 0 <= j < l:
                out[w + k, i] = G[i * b:(i + 1) * b, j * b:(j + 1) * b]
    return out


def dense_selected(H, w, E, sigma_L, sigma_R, eta_d=0.0, full: bool = False):
    """Definition (Sec. 2 intro): bndiag(M^{-1}) from a dense inverse.  Tiny systems only."""
    l, b = H.shape[1], H.shape[2]
    M = dense_matrix(H, w, E, sigma_L, sigma_R, eta_d)
    G = np.linalg.inv(M)
    band = _band_of_dense(G, l, b, w)
    if full:
        return band, G
    return band


# ----------------------------------------------------------------------------
# RGF for block tridiagonal systems (Sec. 2.2, Algorithm 1)
# ----------------------------------------------------------------------------

def rgf(H, E, sigma_L, sigma_R, eta_d=0.0, counter: Optional[OpCounter] = None,
        extras: bool = True, pivot_cond: bool = False,
        pivot_noise: Optional[int] = None, noise_scale: float = 2.0 ** -53) -> Dict[str, np.ndarray]:
    """Sequential RGF, w = 1.

    Upward pass (eliminate layer l-1 first, then l-2, ... 0): the Schur pivot of the
    last layer is its own diagonal block; for each earlier layer the right multiplier
    U_{i+1} = M_{i,i+1} S_{i+1}^{-1} and left multiplier L_{i+1} = S_{i+1}^{-1} M_{i+1,i}
    are obtained by solves with the LU of S_{i+1}, and S_i = M_ii - M_{i,i+1} L_{i+1}.
    Downward pass: G_00 = S_0^{-1}; for i >= 1, G_{i-1,i} = -G_{i-1,i-1} U_i,
    G_{i,i-1} = -L_i G_{i-1,i-1}, G_ii = S_i^{-1} - L_i G_{i-1,i}.

    ``pivot_cond`` also returns max_i kappa_1(S_i); ``pivot_noise`` perturbs every
    Schur pivot by a relative Gaussian of size ``noise_scale`` (default u) before
    factorisation (both as in :func:`nrgf`).

    With ``extras`` also the first block row/column and last block row/column of
    G = M^{-1}, propagated with the same multipliers (these are the far-corner
    entries of eq. 4x4_exact_RGF):  G_{0,i} = -G_{0,i-1} U_i,  G_{i,0} = -L_i G_{i-1,0},
    G_{i,l-1} = G_ii P_i with P_{l-1} = I, P_i = -U_{i+1} P_{i+1}, and
    G_{l-1,i} = Q_i G_ii with Q_{l-1} = I, Q_i = -Q_{i+1} L_{i+1}.
    """
    w = 1
    l, b = H.shape[1], H.shape[2]
    M = block_accessor(H, w, E, sigma_L, sigma_R, eta_d)
    ops = _Ops(counter)
    xops = _Ops(counter, extra=True)

    lu = [None] * l
    U = [None] * l       # U[i] = M_{i-1,i} S_i^{-1}
    L = [None] * l       # L[i] = S_i^{-1} M_{i,i-1}
    nrng = None if pivot_noise is None else np.random.default_rng(pivot_noise)

    def noisy(S):
        if nrng is None:
            return S
        xi = nrng.standard_normal((b, b)) + 1j * nrng.standard_normal((b, b))
        return S * (1.0 + noise_scale * xi)

    lu[l - 1] = ops.lu(noisy(M(l - 1, l - 1)))
    for i in range(l - 2, -1, -1):
        U[i + 1] = ops.solve_right(M(i, i + 1), lu[i + 1])
        L[i + 1] = ops.solve_left(lu[i + 1], M(i + 1, i))
        S = M(i, i) - ops.gemm(M(i, i + 1), L[i + 1])
        lu[i] = ops.lu(noisy(S))

    eye = np.eye(b, dtype=np.complex128)
    G = np.zeros((3, l, b, b), dtype=np.complex128)
    G[1, 0] = ops.solve_left(lu[0], eye)
    for i in range(1, l):
        G[2, i - 1] = -ops.gemm(G[1, i - 1], U[i])          # G_{i-1,i}
        G[0, i] = -ops.gemm(L[i], G[1, i - 1])              # G_{i,i-1}
        G[1, i] = ops.solve_left(lu[i], eye) - ops.gemm(L[i], G[2, i - 1])
    out = {"G": G}
    if pivot_cond:
        out["pivot_cond"] = max(_pivot_kappa(lu[i], b) for i in range(l))
    if not extras:
        return out

    row0 = np.zeros((l, b, b), dtype=np.complex128)
    col0 = np.zeros((l, b, b), dtype=np.complex128)
    row0[0] = G[1, 0]
    col0[0] = G[1, 0]
    for i in range(1, l):
        row0[i] = -xops.gemm(row0[i - 1], U[i])
        col0[i] = -xops.gemm(L[i], col0[i - 1])
    colL = np.zeros((l, b, b), dtype=np.complex128)
    rowL = np.zeros((l, b, b), dtype=np.complex128)
    P = eye.copy()
    Q = eye.copy()
    for i in range(l - 1, -1, -1):
        if i < l - 1:
            P = -xops.gemm(U[i + 1], P)
            Q = -xops.gemm(Q, L[i + 1])
        colL[i] = xops.gemm(G[1, i], P)
        rowL[i] = xops.gemm(Q, G[1, i])
    out.update(row0=row0, col0=col0, colL=colL, rowL=rowL)
    return out


def rgf_mixed_products(H, E, sigma_L, sigma_R, eta_d=0.0) -> Dict[str, np.ndarray]:
    """Algorithm 1 with every block product rounded to FP32 (operands rounded to
    complex64, product accumulated in single precision by NumPy/BLAS cgemm, result
    widened to complex128), while each Schur pivot is inverted in FP64 and refined
    once in FP64, g <- g + g (I - S g).  This is the definition of the mixed
    precision variant (the paper has none; its code is only type-generic, Sec. 4),
    written out so the GPU's mixed path can be compared with the same arithmetic.
    Returns the band and the first block row's last block (for T)."""
    l, b = H.shape[1], H.shape[2]
    M = block_accessor(H, 1, E, sigma_L, sigma_R, eta_d)
    eye = np.eye(b, dtype=np.complex128)

    def p32(A, B):
        return (A.astype(np.complex64) @ B.astype(np.complex64)).astype(np.complex128)

    g = [None] * l
    U = [None] * l
    L = [None] * l
    S = M(l - 1, l - 1)
    for i in range(l - 1, -1, -1):
        gi = np.linalg.inv(S)
        gi = gi + gi @ (eye - S @ gi)
        g[i] = gi
        if i == 0:
            break
        L[i] = p32(gi, M(i, i - 1))
        U[i] = p32(M(i - 1, i), gi)
        S = M(i - 1, i - 1) - p32(M(i - 1, i), L[i])
    G = np.zeros((3, l, b, b), dtype=np.complex128)
    G[1, 0] = g[0]
    R = g[0]
    for i in range(1, l):
        G[2, i - 1] = -p32(G[1, i - 1], U[i])
        G[0, i] = -p32(L[i], G[1, i - 1])
        R = -p32(R, U[i])
        G[1, i] = g[i] - p32(L[i], G[2, i - 1])
    return {"G": G, "G_0_last": R}


# ----------------------------------------------------------------------------
# RGF for block n-diagonal systems (Sec. 2.3)
# ----------------------------------------------------------------------------

def nrgf(Mb: Callable[[int, int], Optional[np.ndarray]], l: int, b: int, w: int,
         counter: Optional[OpCounter] = None, halo: int = 0,
         pivot_cond: bool = False, pivot_noise: Optional[int] = None,
         noise_scale: float = 2.0 ** -53) -> Dict[str, np.ndarray]:
    """Native n-diagonal RGF (n = 2w + 1) on the blocks returned by ``Mb``.

    Upward pass (Proposition 3): eliminate layers l-1, ..., 0.  When layer i is
    eliminated its Schur pivot S_ii is factorised, the multipliers
    U_{c,i} = S_{c,i} S_ii^{-1} and L_{i,c} = S_ii^{-1} S_{i,c} are formed for the
    in-band neighbours c in C_i = [max(0, i-w), i-1], and the trailing w x w window
    is updated S_{a,c} -= S_{a,i} L_{i,c} (a, c in C_i); the band is preserved.

    Downward pass (the paper's prose description for n > 3): with M = U~ D L~
    (U~ unit block upper, U~_{c,i} = U_{c,i}; D = diag(S_ii); L~ unit block lower,
    L~_{i,c} = L_{i,c}), G U~ is block lower and L~ G block upper triangular, so
    for a in C_i:  G_{a,i} = -sum_{c in C_i} G_{a,c} U_{c,i},
                   G_{i,a} = -sum_{c in C_i} L_{i,c} G_{c,a},
    and G_ii = S_ii^{-1} - sum_{c in C_i} L_{i,c} G_{c,i}.  Only blocks within the
    band are read.

    ``pivot_cond`` also returns max_i kappa_1(S_ii), the condition number of the
    worst Schur pivot: the block elimination does not pivot across blocks, so
    rounding errors are amplified by it (not by kappa(M)).

    ``pivot_noise`` (a seed) multiplies every entry of every Schur pivot by
    (1 + s xi), xi ~ N(0, 1), s = ``noise_scale`` (default u = 2^-53), before it
    is factorised: a second run of the same algorithm with independent
    rounding-sized perturbations, whose distance to the unperturbed run estimates
    the algorithm's rounding error at that precision (s = 2^-24 for FP32 products).

    ``halo`` > 0 additionally returns the first/last ``halo`` block rows and
    columns of M^{-1} (the "internal halos" that DDRGF needs from each interior):
      first rows   G_{a,i} = -sum_{c in C_i} G_{a,c} U_{c,i}         (a < i)
      first cols   G_{i,a} = -sum_{c in C_i} L_{i,c} G_{c,a}         (a < i)
      last cols    G_{i,t} = S_ii^{-1} y_i - sum_{c in C_i} L_{i,c} G_{c,t},
                   y = U~^{-1} e_t (back substitution from y_t = I)
      last rows    G_{t,i} = z_i S_ii^{-1} - sum_{c in C_i} G_{t,c} U_{c,i},
                   z = e_t^T L~^{-1}.
    """
    ops = _Ops(counter)
    xops = _Ops(counter, extra=True)
    S: Dict[tuple, np.ndarray] = {}
    for i in range(l):
        for j in range(max(0, i - w), min(l, i + w + 1)):
            blk = Mb(i, j)
            S[(i, j)] = np.array(blk, dtype=np.complex128, copy=True)

    lu = [None] * l
    U: Dict[tuple, np.ndarray] = {}
    L: Dict[tuple, np.ndarray] = {}
    nrng = None if pivot_noise is None else np.random.default_rng(pivot_noise)
    for i in range(l - 1, -1, -1):
        if nrng is not None:
            xi = nrng.standard_normal((b, b)) + 1j * nrng.standard_normal((b, b))
            S[(i, i)] = S[(i, i)] * (1.0 + noise_scale * xi)
        lu[i] = ops.lu(S[(i, i)])
        C = range(max(0, i - w), i)
        for c in C:
            U[(c, i)] = ops.solve_right(S[(c, i)], lu[i])
            L[(i, c)] = ops.solve_left(lu[i], S[(i, c)])
        for a in C:
            for c in C:
                S[(a, c)] = S[(a, c)] - ops.gemm(S[(a, i)], L[(i, c)])

    eye = np.eye(b, dtype=np.complex128)
    G: Dict[tuple, np.ndarray] = {}
    G[(0, 0)] = ops.solve_left(lu[0], eye)
    for i in range(1, l):
        C = list(range(max(0, i - w), i))
        for a in C:
            acc = np.zeros((b, b), dtype=np.complex128)
            for c in C:
                acc -= ops.gemm(G[(a, c)], U[(c, i)])
            G[(a, i)] = acc
        for a in C:
            acc = np.zeros((b, b), dtype=np.complex128)
            for c in C:
                acc -= ops.gemm(L[(i, c)], G[(c, a)])
            G[(i, a)] = acc
        acc = ops.solve_left(lu[i], eye)
        for c in C:
            acc = acc - ops.gemm(L[(i, c)], G[(c, i)])
        G[(i, i)] = acc

    band = np.zeros((2 * w + 1, l, b, b), dtype=np.complex128)
    for (i, j), blk in G.items():
        band[w + j - i, i] = blk
    out = {"G": band}
    if pivot_cond:
        kap = 0.0
        for i in range(l):
            kap = max(kap, _pivot_kappa(lu[i], b))
        out["pivot_cond"] = kap
    if halo <= 0:
        return out

    h = min(halo, l)
    # first rows / first columns
    for i in range(1, l):
        C = range(max(0, i - w), i)
        for a in range(0, min(h, i)):
            if (a, i) not in G:
                acc = np.zeros((b, b), dtype=np.complex128)
                for c in C:
                    acc -= xops.gemm(G[(a, c)], U[(c, i)])
                G[(a, i)] = acc
            if (i, a) not in G:
                acc = np.zeros((b, b), dtype=np.complex128)
                for c in C:
                    acc -= xops.gemm(L[(i, c)], G[(c, a)])
                G[(i, a)] = acc
    # last columns / last rows
    for t in range(l - h, l):
        y: Dict[int, np.ndarray] = {t: eye}
        z: Dict[int, np.ndarray] = {t: eye}
        for c in range(t - 1, -1, -1):
            accy = np.zeros((b, b), dtype=np.complex128)
            accz = np.zeros((b, b), dtype=np.complex128)
            for i in range(c + 1, min(c + w, t) + 1):
                accy -= xops.gemm(U[(c, i)], y[i])
                accz -= xops.gemm(z[i], L[(i, c)])
            y[c] = accy
            z[c] = accz
        for i in range(0, t + 1):
            C = range(max(0, i - w), i)
            if (i, t) not in G:
                acc = ops.solve_left(lu[i], y[i])
                for c in C:
                    acc = acc - xops.gemm(L[(i, c)], G[(c, t)])
                G[(i, t)] = acc
            if (t, i) not in G:
                acc = sla.lu_solve(lu[i], z[i].T, trans=1, check_finite=False).T
                for c in C:
                    acc = acc - xops.gemm(G[(t, c)], U[(c, i)])
                G[(t, i)] = acc
    first_rows = np.zeros((h, l, b, b), dtype=np.complex128)
    first_cols = np.zeros((h, l, b, b), dtype=np.complex128)
    last_rows = np.zeros((h, l, b, b), dtype=np.complex128)
    last_cols = np.zeros((h, l, b, b), dtype=np.complex128)
    for a in range(h):
        for i in range(l):
            first_rows[a, i] = G[(a, i)]
            first_cols[a, i] = G[(i, a)]
            last_rows[a, i] = G[(l - h + a, i)]
            last_cols[a, i] = G[(i, l - h + a)]
    out.update(first_rows=first_rows, first_cols=first_cols, last_rows=last_rows,
               last_cols=last_cols)
    return out


def _pivot_kappa(lu, b) -> float:
    """kappa_1 of the matrix whose LU is ``lu`` (rebuilt from the factors)."""
    LU, piv = lu
    Lf = np.tril(LU, -1) + np.eye(b)
    Uf = np.triu(LU)
    A = Lf @ Uf
    perm = np.arange(b)
    for k, pk in enumerate(piv):
        perm[k], perm[pk] = perm[pk], perm[k]
    Afull = np.empty_like(A)
    Afull[perm] = A
    return float(np.linalg.norm(Afull, 1) * np.linalg.norm(np.linalg.inv(Afull), 1))


# ----------------------------------------------------------------------------
# DDRGF, one level (Sec. 3, Algorithm 2)
# ----------------------------------------------------------------------------

def domain_layout(l: int, n_pairs: int, s1: int):
    """Alternating (interior D2^k, separator D1^k), k = 0..m-1, starting with an
    interior at the first layer and ending with a separator at the last layer
    (the figure of Sec. 3).  Separators have s1 layers; the l - m*s1 interior layers
    are split as evenly as possible (the first ones take one extra layer).
    Returns a list of (a_k, e_k, p_k) with interior [a_k, e_k] and separator
    [p_k, p_k + s1 - 1]."""
    m = n_pairs
    tot = l - m * s1
    if m < 1 or s1 < 1 or tot < m:
        raise ValueError(f"cannot split l={l} into {m} pairs with s1={s1}")
    base, rem = divmod(tot, m)
    out = []
    pos = 0
    for k in range(m):
        s2 = base + (1 if k < rem else 0)
        a, e = pos, pos + s2 - 1
        p = e + 1
        out.append((a, e, p))
        pos = p + s1
    assert pos == l
    return out


def ddrgf(H, w, E, sigma_L, sigma_R, eta_d=0.0, n_pairs=2, s1: Optional[int] = None,
          drop_orange: bool = False, return_parts: bool = False, pivot_cond: bool = False,
          inner_pairs: Sequence[int] = ()):
    """DDRGF (Algorithm 2) of M(E) = (E + i eta_d) I - H - Sigma; see ddrgf_blocks."""
    l, b = H.shape[1], H.shape[2]
    Mb = block_accessor(H, w, E, sigma_L, sigma_R, eta_d)
    return ddrgf_blocks(Mb, l, b, w, n_pairs, s1, drop_orange, return_parts, pivot_cond, inner_pairs)


def ddrgf_blocks(Mb: Callable[[int, int], Optional[np.ndarray]], l: int, b: int, w: int, n_pairs=2,
                 s1: Optional[int] = None, drop_orange: bool = False, return_parts: bool = False,
                 pivot_cond: bool = False, inner_pairs: Sequence[int] = ()):
    """DDRGF (Algorithm 2), block n-diagonal, separators of s1 = w layers, on the
    blocks returned by Mb.

    Step 1: for every interior D2^k, X^(k) = (M_{D2^k})^{-1} restricted to the band
            plus its first/last w block rows and columns (extended RGF).
    Step 2: Schur complement on the separators,
            T_S = T_11 - T_12 T_22^{-1} T_21; with the separators of pair k grouped
            into one block of size w*b it is block tridiagonal (Proposition 4),
            including the couplings between neighbouring separators through one
            interior (the "orange" blocks, which cannot be dropped).
    Step 3: band of T_S^{-1} by RGF on the reduced system (plus its first row, used
            for the first-layer-to-last-layer block needed by the transmission).
    Step 4: recover the wanted blocks:  G_{D2,D1} = -X T_21 G_S,
            G_{D1,D2} = -G_S T_12 X,  G_{D2,D2} = X + X T_21 G_S T_12 X,
            each only inside the band.
    Step 5: everything is written straight into natural layer order.

    Multi-level (the recursion of Algorithm 2's step 3): with ``inner_pairs`` =
    (m2, m3, ...) the reduced system is itself solved by DDRGF with m2 pairs (its
    own reduced system with m3 pairs, and so on), and by RGF at the last level.
    The outer level needs from the reduced inverse only its band and the block
    (first separator, last separator), which DDRGF returns as G_0_last.
    """
    if s1 is None:
        s1 = w
    if s1 != w:
        raise ValueError("this oracle uses separators of exactly w layers")
    lay = domain_layout(l, n_pairs, s1)
    m = len(lay)
    for (a, e, p) in lay:
        if e - a + 1 < w:
            raise ValueError("interiors must hold at least w layers")
    wb = w * b

    def dense(rows: List[int], cols: List[int]) -> np.ndarray:
        out = np.zeros((len(rows) * b, len(cols) * b), dtype=np.complex128)
        for r, i in enumerate(rows):
            for c, j in enumerate(cols):
                blk = Mb(i, j)
                if blk is not None:
                    out[r * b:(r + 1) * b, c * b:(c + 1) * b] = blk
        return out

    # ---- Step 1 -------------------------------------------------------------
    X = []
    for (a, e, p) in lay:
        n = e - a + 1
        sub = (lambda a0: (lambda i, j: Mb(a0 + i, a0 + j)))(a)
        X.append(nrgf(sub, n, b, w, halo=w, pivot_cond=pivot_cond))

    def Xcorner(k: int, first_rows: bool, first_cols: bool) -> np.ndarray:
        """w*b x w*b corner of X^(k): rows first/last w, cols first/last w."""
        a, e, p = lay[k]
        n = e - a + 1
        rows = list(range(w)) if first_rows else list(range(n - w, n))
        cols = list(range(w)) if first_cols else list(range(n - w, n))
        out = np.zeros((wb, wb), dtype=np.complex128)
        fr, fc, lr, lc = (X[k]["first_rows"], X[k]["first_cols"], X[k]["last_rows"],
                          X[k]["last_cols"])
        for r, i in enumerate(rows):
            for c, j in enumerate(cols):
                if first_rows:
                    blk = fr[i, j]
                elif first_cols:
                    blk = fc[j, i]
                else:
                    blk = lr[i - (n - w), j]
                out[r * b:(r + 1) * b, c * b:(c + 1) * b] = blk
        return out

    sep = [list(range(p, p + s1)) for (a, e, p) in lay]
    first_w = [list(range(a, a + w)) for (a, e, p) in lay]
    last_w = [list(range(e - w + 1, e + 1)) for (a, e, p) in lay]

    # couplings interior <-> neighbouring separators
    Lin = [None] * m     # M[first w of D2^k, D1^{k-1}]
    Lout = [None] * m    # M[D1^{k-1}, first w of D2^k]
    Rin = [None] * m     # M[last w of D2^k, D1^k]
    Rout = [None] * m    # M[D1^k, last w of D2^k]
    for k in range(m):
        if k >= 1:
            Lin[k] = dense(first_w[k], sep[k - 1])
            Lout[k] = dense(sep[k - 1], first_w[k])
        Rin[k] = dense(last_w[k], sep[k])
        Rout[k] = dense(sep[k], last_w[k])

    # ---- Step 2 -------------------------------------------------------------
    S_diag = []
    S_up = []     # S_{k,k+1}
    S_lo = []     # S_{k+1,k}
    for k in range(m):
        Skk = dense(sep[k], sep[k])
        Skk = Skk - Rout[k] @ Xcorner(k, False, False) @ Rin[k]
        if k + 1 < m:
            Skk = Skk - Lout[k + 1] @ Xcorner(k + 1, True, True) @ Lin[k + 1]
        S_diag.append(Skk)
        if k + 1 < m:
            up = -(Lout[k + 1] @ Xcorner(k + 1, True, False) @ Rin[k + 1])
            lo = -(Rout[k + 1] @ Xcorner(k + 1, False, True) @ Lin[k + 1])
            if drop_orange:
                up = np.zeros_like(up)
                lo = np.zeros_like(lo)
            S_up.append(up)
            S_lo.append(lo)

    # ---- Step 3 -------------------------------------------------------------
    def Sb(i, j):
        if i == j:
            return S_diag[i]
        if j == i + 1:
            return S_up[i]
        if i == j + 1:
            return S_lo[j]
        return None

    if inner_pairs:
        # multi-level: the reduced (block tridiagonal, w b blocks) system by DDRGF
        red = ddrgf_blocks(Sb, m, wb, 1, inner_pairs[0], None, False, return_parts, pivot_cond,
                           tuple(inner_pairs[1:]))
        GS = red["G"]
        GS_0_last = red["G_0_last"]
    else:
        red = nrgf(Sb, m, wb, 1, halo=1, pivot_cond=pivot_cond)
        GS = red["G"]                                # [3, m, wb, wb]
        GS_0_last = red["first_rows"][0][m - 1]      # G_S(0, m-1)

    def gs(i, j):
        if i == j:
            return GS[1, i]
        if j == i + 1:
            return GS[2, i]
        if i == j + 1:
            return GS[0, i]
        if i == 0 and j == m - 1:
            return GS_0_last
        raise KeyError((i, j))

    # ---- Steps 4 and 5 ------------------------------------------------------
    band = np.zeros((2 * w + 1, l, b, b), dtype=np.complex128)

    def put(i, j, blk):
        if abs(j - i) <= w and 0 <= i < l and 0 <= j < l:
            band[w + j - i, i] = blk

    # separator <-> separator blocks from G_S
    for k in range(m):
        for kk in (k - 1, k, k + 1):
            if 0 <= kk < m:
                Z = gs(k, kk)
                for r, i in enumerate(sep[k]):
                    for c, j in enumerate(sep[kk]):
                        put(i, j, Z[r * b:(r + 1) * b, c * b:(c + 1) * b])

    for k in range(m):
        a, e, p = lay[k]
        n = e - a + 1
        Xb = X[k]["G"]
        fr, fc, lr, lc = (X[k]["first_rows"], X[k]["first_cols"], X[k]["last_rows"],
                          X[k]["last_cols"])
        groups = ([k - 1] if k >= 1 else []) + [k]
        Z = np.block([[gs(g1, g2) for g2 in groups] for g1 in groups])
        for il in range(n):
            parts = []
            if k >= 1:
                parts.append(np.hstack([fc[t, il] for t in range(w)]) @ Lin[k])
            parts.append(np.hstack([lc[t, il] for t in range(w)]) @ Rin[k])
            A_i = np.hstack(parts)                      # (X T_21)_{i, B_k}
            AZ = A_i @ Z
            for jl in range(max(0, il - w), min(n, il + w + 1)):
                parts = []
                if k >= 1:
                    parts.append(Lout[k] @ np.vstack([fr[t, jl] for t in range(w)]))
                parts.append(Rout[k] @ np.vstack([lr[t, jl] for t in range(w)]))
                B_j = np.vstack(parts)                  # (T_12 X)_{B_k, j}
                put(a + il, a + jl, Xb[w + jl - il, il] + AZ @ B_j)
            # interior -> separator and separator -> interior (edges only)
            col = 0
            for g in groups:
                for r, q in enumerate(sep[g]):
                    if abs(q - (a + il)) <= w:
                        put(a + il, q, -AZ[:, (col + r) * b:(col + r + 1) * b])
                col += len(sep[g])
        # G_{q, j} for separators q next to this interior
        for jl in range(n):
            parts = []
            if k >= 1:
                parts.append(Lout[k] @ np.vstack([fr[t, jl] for t in range(w)]))
            parts.append(Rout[k] @ np.vstack([lr[t, jl] for t in range(w)]))
            B_j = np.vstack(parts)
            ZB = Z @ B_j
            row = 0
            for g in groups:
                for r, q in enumerate(sep[g]):
                    if abs(q - (a + jl)) <= w:
                        put(q, a + jl, -ZB[(row + r) * b:(row + r + 1) * b, :])
                row += len(sep[g])

    # first layer -> last layer block (for the transmission):
    # G_{0, D1^{m-1}} = -(X^(0) T_21)_{0, D1^0} G_S(0, m-1)
    a0, e0, p0 = lay[0]
    lc0 = X[0]["last_cols"]
    A0 = np.hstack([lc0[t, 0] for t in range(w)]) @ Rin[0]
    G_first_last = -(A0 @ gs(0, m - 1))[:, (w - 1) * b: w * b]
    out = {"G": band, "G_0_last": G_first_last}
    if pivot_cond:
        out["pivot_cond"] = max([x["pivot_cond"] for x in X] + [red["pivot_cond"]])
    if return_parts:
        out.update(X=X, S_diag=S_diag, S_up=S_up, S_lo=S_lo, GS=GS, layout=lay)
        if inner_pairs:
            out["inner"] = red
    return out


# ----------------------------------------------------------------------------
# Transmission (Caroli trace) and the on-site gradient
# ----------------------------------------------------------------------------

def gamma_of(sigma: np.ndarray) -> np.ndarray:
    """Broadening Gamma = i (Sigma - Sigma^H)."""
    return 1j * (sigma - sigma.conj().T)


def transmission(G_first_last, sigma_L, sigma_R) -> float:
    """T(E) = Re Tr[Gamma_L G_{0,l-1} Gamma_R G_{0,l-1}^H] (leads on first/last layer)."""
    gl, gr = gamma_of(sigma_L), gamma_of(sigma_R)
    return float(np.real(np.trace(gl @ G_first_last @ gr @ G_first_last.conj().T)))


def transmission_g11(G00, sigma_L) -> float:
    """Same T from the first diagonal block only (needs Hermitian H and eta_d = 0):
    T = Re Tr[Gamma_L (i (G_00 - G_00^H) - G_00 Gamma_L G_00^H)]."""
    gl = gamma_of(sigma_L)
    A = 1j * (G00 - G00.conj().T) - G00 @ gl @ G00.conj().T
    return float(np.real(np.trace(gl @ A)))


def grad_onsite(H, E, sigma_L, sigma_R, eta_d=0.0):
    """dT/d eps_s for on-site shifts H_ii,ss += eps_s (all layers i, orbitals s), w = 1.

    From dG = G dH G (M = E - H - Sigma):  dT/d eps_s = 2 Re[(G_{i,l-1} X G_{0,i})_{ss}]
    with X = Gamma_R G_{0,l-1}^H Gamma_L.  Returns (T, grad[l, b])."""
    res = rgf(H, E, sigma_L, sigma_R, eta_d, extras=True)
    l, b = H.shape[1], H.shape[2]
    G0L = res["row0"][l - 1]
    gl, gr = gamma_of(sigma_L), gamma_of(sigma_R)
    Xm = gr @ G0L.conj().T @ gl
    grad = np.zeros((l, b), dtype=np.float64)
    for i in range(l):
        Y = res["colL"][i] @ Xm @ res["row0"][i]
        grad[i] = 2.0 * np.real(np.diag(Y))
    T = float(np.real(np.trace(gl @ G0L @ gr @ G0L.conj().T)))
    return T, grad


def grad_band(H, E, sigma_L, sigma_R, eta_d=0.0):
    """dT/dH for every entry of every band block of a block tridiagonal H (w = 1),
    each entry an independent complex parameter h = x + i y, in PyTorch's complex
    convention dT/dx + i dT/dy.

    M = (E + i eta_d) I - H - Sigma, so dG = G dH G and, with Gamma Hermitian,
    dT = 2 Re Tr[Gamma_L dG_{0,l-1} Gamma_R G_{0,l-1}^H]
       = 2 Re sum_{i,j} Tr[dH_ij Y_ij],   Y_ij = G_{j,l-1} X G_{0,i},
    X = Gamma_R G_{0,l-1}^H Gamma_L.  For one entry (a, c) of block (i, j) this gives
    dT/dx = 2 Re (Y_ij)_{c,a} and dT/dy = -2 Im (Y_ij)_{c,a}, i.e. the gradient block
    dT/dH_ij = 2 Y_ij^H.  The first block row G_{0,i} and the last block column
    G_{j,l-1} come from Algorithm 1's extras (:func:`rgf`).
    Returns (T, band [3, l, b, b]) with blocks outside the matrix zero."""
    res = rgf(H, E, sigma_L, sigma_R, eta_d, extras=True)
    l, b = H.shape[1], H.shape[2]
    G0L = res["row0"][l - 1]
    gl, gr = gamma_of(sigma_L), gamma_of(sigma_R)
    Xm = gr @ G0L.conj().T @ gl
    out = np.zeros((3, l, b, b), dtype=np.complex128)
    for i in range(l):
        for k in (-1, 0, 1):
            j = i + k
            if 0 <= j < l:
                Y = res["colL"][j] @ Xm @ res["row0"][i]
                out[1 + k, i] = 2.0 * Y.conj().T
    T = float(np.real(np.trace(gl @ G0L @ gr @ G0L.conj().T)))
    return T, out


# ----------------------------------------------------------------------------
# Convenience: one energy of a workload through a chosen method
# ----------------------------------------------------------------------------

def solve_energy(H, w, E, sigma_L, sigma_R, eta_d=0.0, method="rgf", n_pairs=2):
    """Return (G band, T) for one energy with method in {'dense','rgf','nrgf','ddrgf'}."""
    l, b = H.shape[1], H.shape[2]
    if method == "dense":
        band, G = dense_selected(H, w, E, sigma_L, sigma_R, eta_d, full=True)
        return band, transmission(G[:b, (l - 1) * b:], sigma_L, sigma_R)
    if method == "rgf":
        if w != 1:
            raise ValueError("rgf is the block-tridiagonal method")
        r = rgf(H, E, sigma_L, sigma_R, eta_d, extras=True)
        return r["G"], transmission(r["row0"][l - 1], sigma_L, sigma_R)
    if method == "nrgf":
        Mb = block_accessor(H, w, E, sigma_L, sigma_R, eta_d)
        r = nrgf(Mb, l, b, w, halo=1)
        return r["G"], transmission(r["first_rows"][0, l - 1], sigma_L, sigma_R)
    if method == "ddrgf":
        r = ddrgf(H, w, E, sigma_L, sigma_R, eta_d, n_pairs=n_pairs)
        return r["G"], transmission(r["G_0_last"], sigma_L, sigma_R)
    raise ValueError(method)
