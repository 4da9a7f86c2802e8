"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each check is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, a transposed operand, a wrong index in a recurrence) fails at least
one of them:
  * dense inversion (the definition of bndiag(M^{-1}), Sec. 2 intro) on tiny systems;
  * the printed symbolic inverses for 2 and 4 layers (eqs. 2x2_exact_RGF,
    4x4_exact_RGF, Sec. 2.2);
  * the closed-form Green's function of a uniform chain and its integer transmission;
  * the identity G^R - G^A = G^R (Sigma^R - Sigma^A) G^A;
  * the op counts of eqs. cost_model_RGF and cost_model_general_RGF;
  * native n-diagonal RGF == block-fused tridiagonal RGF (Sec. 2.3);
  * DDRGF == RGF, and dropping the inter-separator couplings breaks it (Sec. 3);
  * the on-site gradient against central finite differences.
"""
import numpy as np
import pytest

import oracle as O
from workloads import (lead_sigma, make_config, make_random, make_uniform_chain,
                       midpoint_grid, random_hermitian_band, surface_sigma)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dense_block(G, b, i, j):
    return G[i * b:(i + 1) * b, j * b:(j + 1) * b]


# ----------------------------------------------------------------------------
# generators
# ----------------------------------------------------------------------------

def test_generator_hermitian_and_band():
    H = random_hermitian_band(7, 5, 2, seed=1)
    w = 2
    for i in range(7):
        np.testing.assert_allclose(H[w, i], H[w, i].conj().T, atol=0)
        for k in (1, 2):
            if i + k < 7:
                np.testing.assert_allclose(H[w - k, i + k], H[w + k, i].conj().T, atol=0)
    # out-of-range blocks are zero
    assert np.all(H[w + 1, 6] == 0) and np.all(H[w - 2, :2] == 0)
    # far band is scaled down
    assert np.std(H[w + 2, :5]) < 0.5 * np.std(H[w + 1, :6])


def test_surface_sigma_branch():
    E = np.linspace(-3.5, 3.5, 141)
    s = surface_sigma(E + 1e-9j)
    inband = np.abs(E) < 2
    assert np.all(s.imag[inband] < 0)
    assert np.all(np.abs(s[~inband]) <= 1 + 1e-6)
    # sigma solves sigma^2 - z sigma + 1 = 0 (Dyson equation of the semi-infinite chain)
    z = E + 1e-9j
    np.testing.assert_allclose(s * s - z * s + 1, 0, atol=1e-12)


def test_midpoint_grid_config1():
    np.testing.assert_allclose(midpoint_grid(-1, 1, 4), [-0.75, -0.25, 0.25, 0.75])


# ----------------------------------------------------------------------------
# P1: dense inversion on tiny systems (all methods)
# ----------------------------------------------------------------------------

CASES = [(1, 3, 1), (2, 4, 1), (5, 1, 1), (7, 5, 1), (12, 8, 1), (9, 3, 2), (11, 2, 2),
         (10, 4, 3), (6, 16, 1), (8, 5, 2)]


@pytest.mark.parametrize("l,b,w", CASES)
def test_nrgf_matches_dense(l, b, w):
    wl = make_random(l, b, w, 3, seed=1000 + 10 * l + b, eta=1e-3)
    for e in range(wl.ne):
        args = (wl.H, w, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        band, G = O.dense_selected(*args, full=True)
        Mb = O.block_accessor(*args)
        r = O.nrgf(Mb, l, b, w, halo=min(w, l))
        assert rel(r["G"], band) < 1e-11
        h = min(w, l)
        for a in range(h):
            t = l - h + a
            assert rel(r["first_rows"][a], np.stack([dense_block(G, b, a, j) for j in range(l)])) < 1e-11
            assert rel(r["first_cols"][a], np.stack([dense_block(G, b, j, a) for j in range(l)])) < 1e-11
            assert rel(r["last_rows"][a], np.stack([dense_block(G, b, t, j) for j in range(l)])) < 1e-11
            assert rel(r["last_cols"][a], np.stack([dense_block(G, b, j, t) for j in range(l)])) < 1e-11


@pytest.mark.parametrize("l,b", [(1, 4), (2, 3), (6, 5), (16, 16), (23, 7)])
def test_rgf_matches_dense(l, b):
    wl = make_random(l, b, 1, 2, seed=77 + l, eta=1e-3)
    for e in range(wl.ne):
        args = (wl.H, 1, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        band, G = O.dense_selected(*args, full=True)
        r = O.rgf(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        assert rel(r["G"], band) < 1e-11
        for key, f in [("row0", lambda j: dense_block(G, b, 0, j)),
                       ("col0", lambda j: dense_block(G, b, j, 0)),
                       ("colL", lambda j: dense_block(G, b, j, l - 1)),
                       ("rowL", lambda j: dense_block(G, b, l - 1, j))]:
            assert rel(r[key], np.stack([f(j) for j in range(l)])) < 1e-11


def test_config1_dense_all_methods():
    wl = make_config(1)
    for e in range(wl.ne):
        args = (wl.H, 1, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        band, T = O.solve_energy(*args, method="dense")
        for method in ("rgf", "nrgf", "ddrgf"):
            b2, T2 = O.solve_energy(*args, method=method, n_pairs=wl.domains)
            assert rel(b2, band) < 1e-11, method
            assert abs(T2 - T) <= 1e-11 * max(1.0, abs(T)), method


# ----------------------------------------------------------------------------
# P2: printed closed forms for one, two and four layers
# ----------------------------------------------------------------------------

def test_single_layer():
    wl = make_random(1, 6, 1, 2, seed=5, eta=1e-3)
    for e in range(2):
        E = wl.energies[e]
        M = E * np.eye(6) - wl.H[1, 0] - wl.sigma_L[e] - wl.sigma_R[e]
        r = O.rgf(wl.H, E, wl.sigma_L[e], wl.sigma_R[e])
        np.testing.assert_allclose(r["G"][1, 0], np.linalg.inv(M), rtol=0, atol=1e-12)


def _right_connected(T, l):
    """t_ll = T_ll^{-1}; t_ii = (T_ii - T_{i,i+1} t_{i+1,i+1} T_{i+1,i})^{-1}  (Sec. 2.2)."""
    t = [None] * l
    t[l - 1] = np.linalg.inv(T[(l - 1, l - 1)])
    for i in range(l - 2, -1, -1):
        t[i] = np.linalg.inv(T[(i, i)] - T[(i, i + 1)] @ t[i + 1] @ T[(i + 1, i)])
    return t


def _blocks(wl, e):
    Mb = O.block_accessor(wl.H, 1, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
    return {(i, j): Mb(i, j) for i in range(wl.l) for j in range(wl.l) if abs(i - j) <= 1}


def test_two_layer_closed_form():
    """eq. 2x2_exact_RGF."""
    wl = make_random(2, 5, 1, 2, seed=11, eta=1e-3)
    for e in range(2):
        T = _blocks(wl, e)
        t = _right_connected(T, 2)
        t11, t22 = t
        exact = {
            (0, 0): t11,
            (0, 1): -t11 @ T[(0, 1)] @ t22,
            (1, 0): -t22 @ T[(1, 0)] @ t11,
            (1, 1): t22 + t22 @ T[(1, 0)] @ t11 @ T[(0, 1)] @ t22,
        }
        r = O.rgf(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        G = r["G"]
        np.testing.assert_allclose(G[1, 0], exact[(0, 0)], atol=1e-12)
        np.testing.assert_allclose(G[2, 0], exact[(0, 1)], atol=1e-12)
        np.testing.assert_allclose(G[0, 1], exact[(1, 0)], atol=1e-12)
        np.testing.assert_allclose(G[1, 1], exact[(1, 1)], atol=1e-12)


def test_four_layer_closed_form_all_16_blocks():
    """All 16 blocks of eq. 4x4_exact_RGF, in terms of the right-connected t_ii,
    tilde t_ii = t_ii + t_ii T_{i,i-1} tilde t_{i-1,i-1} T_{i-1,i} t_ii and T_ij."""
    wl = make_random(4, 4, 1, 2, seed=13, eta=1e-3)
    for e in range(2):
        T = _blocks(wl, e)
        t = _right_connected(T, 4)
        tt = [t[0]]
        for i in range(1, 4):
            tt.append(t[i] + t[i] @ T[(i, i - 1)] @ tt[i - 1] @ T[(i - 1, i)] @ t[i])
        T12, T23, T34 = T[(0, 1)], T[(1, 2)], T[(2, 3)]
        T21, T32, T43 = T[(1, 0)], T[(2, 1)], T[(3, 2)]
        t11, t22, t33, t44 = t
        X = [[None] * 4 for _ in range(4)]
        X[0][0] = tt[0]
        X[0][1] = -t11 @ T12 @ t22
        X[0][2] = t11 @ T12 @ t22 @ T23 @ t33
        X[0][3] = -t11 @ T12 @ t22 @ T23 @ t33 @ T34 @ t44
        X[1][0] = -t22 @ T21 @ t11
        X[1][1] = tt[1]
        X[1][2] = -tt[1] @ T23 @ t33
        X[1][3] = tt[1] @ T23 @ t33 @ T34 @ t44
        X[2][0] = t33 @ T32 @ t22 @ T21 @ t11
        X[2][1] = -t33 @ T32 @ tt[1]
        X[2][2] = tt[2]
        X[2][3] = -tt[2] @ T34 @ t44
        X[3][0] = -t44 @ T43 @ t33 @ T32 @ t22 @ T21 @ t11
        X[3][1] = t44 @ T43 @ t33 @ T32 @ tt[1]
        X[3][2] = -t44 @ T43 @ tt[2]
        X[3][3] = tt[3]
        r = O.rgf(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        # oracle band
        for i in range(4):
            for k in (-1, 0, 1):
                j = i + k
                if 0 <= j < 4:
                    np.testing.assert_allclose(r["G"][1 + k, i], X[i][j], atol=1e-12)
        # oracle far corners (first/last rows and columns)
        for j in range(4):
            np.testing.assert_allclose(r["row0"][j], X[0][j], atol=1e-12)
            np.testing.assert_allclose(r["col0"][j], X[j][0], atol=1e-12)
            np.testing.assert_allclose(r["colL"][j], X[j][3], atol=1e-12)
            np.testing.assert_allclose(r["rowL"][j], X[3][j], atol=1e-12)
        # and the printed forms are the inverse
        Gd = np.linalg.inv(O.dense_matrix(wl.H, 1, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e]))
        for i in range(4):
            for j in range(4):
                np.testing.assert_allclose(dense_block(Gd, 4, i, j), X[i][j], atol=1e-12)


# ----------------------------------------------------------------------------
# P3 / P4: uniform chain, closed form at every block; integer transmission
# ----------------------------------------------------------------------------

def _chain_exact(wl, e, i, j):
    V, eps = wl.meta["V"], wl.meta["eps"]
    z = wl.energies[e] + 1j * wl.eta - eps
    s = np.sqrt(z - 2.0) * np.sqrt(z + 2.0)
    sig = surface_sigma(z)
    return (V * (sig ** abs(i - j) / s)[None, :]) @ V.conj().T


@pytest.mark.parametrize("l,b,ne", [(64, 16, 5), (40, 12, 3)])
def test_uniform_chain_closed_form(l, b, ne):
    wl = make_uniform_chain(l, b, ne, eta=1e-3)
    for e in range(ne):
        args = (wl.H, 1, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        r = O.rgf(wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], eta_d=wl.eta)
        worst = 0.0
        for i in range(l):
            for k in (-1, 0, 1):
                j = i + k
                if 0 <= j < l:
                    ex = _chain_exact(wl, e, i, j)
                    worst = max(worst, np.abs(r["G"][1 + k, i] - ex).max() / np.abs(ex).max())
        assert worst < 1e-10
        ex = _chain_exact(wl, e, 0, l - 1)
        assert np.abs(r["row0"][l - 1] - ex).max() <= 1e-10 * np.abs(ex).max()
        d = O.ddrgf(wl.H, 1, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], eta_d=wl.eta, n_pairs=4)
        assert rel(d["G"], r["G"]) < 1e-11


def test_uniform_chain_integer_transmission():
    b, l = 16, 48
    wl = make_uniform_chain(l, b, 32, eta=1e-6)
    eps = wl.meta["eps"]
    for e in range(wl.ne):
        E = wl.energies[e]
        _, T = O.solve_energy(wl.H, 1, E, wl.sigma_L[e], wl.sigma_R[e], method="rgf")
        n_open = int(np.sum(np.abs(E - eps) < 2))
        assert abs(T - n_open) < 1e-6, (E, T, n_open)


# ----------------------------------------------------------------------------
# P5 / P6: G^R - G^A identity and invariants
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("l,b", [(20, 8), (9, 16)])
def test_retarded_minus_advanced_identity(l, b):
    wl = make_random(l, b, 1, 4, seed=31, eta=1e-3)
    for e in range(wl.ne):
        sL, sR = wl.sigma_L[e], wl.sigma_R[e]
        gl, gr = O.gamma_of(sL), O.gamma_of(sR)
        r = O.rgf(wl.H, wl.energies[e], sL, sR)
        G = r["G"]
        c0, cL = r["col0"], r["colL"]
        for i in range(l):
            for k in (-1, 0, 1):
                j = i + k
                if not (0 <= j < l):
                    continue
                lhs = G[1 + k, i] - G[1 - k, j].conj().T
                rhs = -1j * (c0[i] @ gl @ c0[j].conj().T + cL[i] @ gr @ cL[j].conj().T)
                assert np.abs(lhs - rhs).max() <= 1e-11 * max(1.0, np.abs(G[1 + k, i]).max())


def test_invariants_config1():
    wl = make_config(1)
    for e in range(wl.ne):
        sL, sR = wl.sigma_L[e], wl.sigma_R[e]
        r = O.rgf(wl.H, wl.energies[e], sL, sR)
        G = r["G"]
        for i in range(wl.l):
            assert np.all(np.diag(G[1, i]).imag <= 1e-14)
        T = O.transmission(r["row0"][wl.l - 1], sL, sR)
        T11 = O.transmission_g11(G[1, 0], sL)
        TRL = float(np.real(np.trace(O.gamma_of(sR) @ r["rowL"][0] @ O.gamma_of(sL) @ r["rowL"][0].conj().T)))
        assert 0 <= T <= wl.b
        assert abs(T - T11) < 1e-10 * max(1, T)
        assert abs(T - TRL) < 1e-10 * max(1, T)


# ----------------------------------------------------------------------------
# P7: op counts (eqs. cost_model_RGF, cost_model_general_RGF)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("l", [1, 2, 3, 9])
def test_rgf_op_counts(l):
    wl = make_random(l, 3, 1, 1, seed=2)
    c = O.OpCounter()
    O.rgf(wl.H, wl.energies[0], wl.sigma_L[0], wl.sigma_R[0], counter=c, extras=False)
    assert c.as_tuple() == (l, 3 * l - 2, 4 * (l - 1))


@pytest.mark.parametrize("l,w", [(8, 1), (9, 2), (13, 3), (5, 2), (4, 3)])
def test_nrgf_op_counts(l, w):
    wl = make_random(l, 2, w, 1, seed=3)
    Mb = O.block_accessor(wl.H, w, wl.energies[0], wl.sigma_L[0], wl.sigma_R[0])
    c = O.OpCounter()
    O.nrgf(Mb, l, 2, w, counter=c)
    assert c.lu == l
    assert c.getrs == l * (2 * w + 1) - w * w - w
    assert c.gemm == (3 * w * w + w) * l - 2 * w ** 3 - 2 * w * w


def test_config_op_counts():
    """The counts quoted for the benchmark sizes: l=256 tridiagonal, l=512 pentadiagonal."""
    assert (256, 3 * 256 - 2, 4 * 255) == (256, 766, 1020)
    l, w = 512, 2
    assert (l * (2 * w + 1) - w * w - w, (3 * w * w + w) * l - 2 * w ** 3 - 2 * w * w) == (2554, 7144)


# ----------------------------------------------------------------------------
# P8: native n-diagonal == block-fused tridiagonal (Sec. 2.3)
# ----------------------------------------------------------------------------

def test_native_pentadiagonal_equals_fused():
    l, b, w = 10, 3, 2
    wl = make_random(l, b, w, 2, seed=17, eta=1e-3)
    lf, bf = l // w, w * b
    for e in range(wl.ne):
        Mb = O.block_accessor(wl.H, w, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        native = O.nrgf(Mb, l, b, w)["G"]

        def Mf(I, J):
            if abs(I - J) > 1:
                return None
            out = np.zeros((bf, bf), dtype=np.complex128)
            for r in range(w):
                for c in range(w):
                    blk = Mb(I * w + r, J * w + c)
                    if blk is not None:
                        out[r * b:(r + 1) * b, c * b:(c + 1) * b] = blk
            return out

        fused = O.nrgf(Mf, lf, bf, 1)["G"]
        for i in range(l):
            for k in range(-w, w + 1):
                j = i + k
                if not (0 <= j < l):
                    continue
                I, J = i // w, j // w
                fb = fused[1 + J - I, I][(i % w) * b:(i % w + 1) * b, (j % w) * b:(j % w + 1) * b]
                np.testing.assert_allclose(native[w + k, i], fb, atol=1e-11)


# ----------------------------------------------------------------------------
# P9: DDRGF == RGF; dropping the orange couplings fails (Sec. 3)
# ----------------------------------------------------------------------------

DD_CASES = [(16, 16, 1, 2), (33, 6, 1, 4), (40, 5, 2, 4), (24, 4, 2, 3), (31, 3, 3, 3),
            (10, 4, 1, 5)]


@pytest.mark.parametrize("l,b,w,m", DD_CASES)
def test_ddrgf_equals_rgf(l, b, w, m):
    """With a device broadening eta_d every Schur pivot of every closed interior is
    bounded (||S_ii^{-1}|| <= 1/eta_d), so DDRGF and RGF agree to rounding."""
    wl = make_random(l, b, w, 2, seed=300 + l, eta=1e-3)
    for e in range(wl.ne):
        args = (wl.H, w, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], 0.05)
        Mb = O.block_accessor(*args)
        ref = O.nrgf(Mb, l, b, w, halo=1)
        d = O.ddrgf(*args, n_pairs=m)
        dense = O.dense_selected(*args)
        assert rel(d["G"], dense) < 1e-12
        assert rel(d["G"], ref["G"]) < 1e-12
        assert rel(d["G_0_last"], ref["first_rows"][0, l - 1]) < 1e-12
        bad = O.ddrgf(*args, n_pairs=m, drop_orange=True)
        assert rel(bad["G"], ref["G"]) > 1e-3


ML_CASES = [(40, 4, 1, 8, (2,)), (64, 3, 1, 16, (4, 2)), (48, 5, 2, 6, (2,)), (33, 6, 1, 8, (3,)),
            (80, 2, 1, 20, (5, 2))]


@pytest.mark.parametrize("l,b,w,m,inner", ML_CASES)
def test_multilevel_ddrgf_equals_rgf(l, b, w, m, inner):
    """Multi-level DDRGF (the reduced system solved by DDRGF again, down to RGF at the
    last level): the same band and first-to-last block as RGF and the dense inverse."""
    wl = make_random(l, b, w, 2, seed=500 + l, eta=1e-3)
    for e in range(wl.ne):
        args = (wl.H, w, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], 0.05)
        ref = O.nrgf(O.block_accessor(*args), l, b, w, halo=1)
        d = O.ddrgf(*args, n_pairs=m, inner_pairs=inner)
        one = O.ddrgf(*args, n_pairs=m)
        assert rel(d["G"], O.dense_selected(*args)) < 1e-12
        assert rel(d["G"], ref["G"]) < 1e-12
        assert rel(d["G_0_last"], ref["first_rows"][0, l - 1]) < 1e-12
        # and the single-level result
        assert rel(d["G"], one["G"]) < 1e-12


@pytest.mark.parametrize("l,b,w,m", DD_CASES)
def test_ddrgf_without_broadening_within_pivot_bound(l, b, w, m):
    """With eta_d = 0 a closed interior can have a nearly singular Schur pivot even when
    M is well conditioned (no pivoting across blocks); the error then scales with the
    worst pivot condition number, which the oracle reports."""
    wl = make_random(l, b, w, 2, seed=300 + l, eta=1e-3)
    for e in range(wl.ne):
        args = (wl.H, w, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        dense = O.dense_selected(*args)
        d = O.ddrgf(*args, n_pairs=m, pivot_cond=True)
        kap = d["pivot_cond"]
        assert rel(d["G"], dense) < max(1e-12, 1e-14 * kap * 10), kap


def test_ddrgf_layout():
    lay = O.domain_layout(256, 8, 1)
    assert lay[0] == (0, 30, 31) and lay[-1] == (224, 254, 255)
    lay = O.domain_layout(512, 16, 2)
    assert lay[0] == (0, 29, 30) and lay[-1][2] == 510
    with pytest.raises(ValueError):
        O.domain_layout(5, 3, 1)


# ----------------------------------------------------------------------------
# P10: on-site gradient
# ----------------------------------------------------------------------------

def test_gradient_finite_difference_and_dense():
    wl = make_random(12, 6, 1, 2, seed=41, eta=1e-3)
    rng = np.random.default_rng(0)
    for e in range(wl.ne):
        E, sL, sR = wl.energies[e], wl.sigma_L[e], wl.sigma_R[e]
        T, g = O.grad_onsite(wl.H, E, sL, sR)
        # dense gradient: dT/deps_s = 2 Re Tr[Gamma_L dG Gamma_R G^H], dG = G e_s e_s^T G
        _, Gd = O.dense_selected(wl.H, 1, E, sL, sR, full=True)
        n, b = Gd.shape[0], 6
        G0L = Gd[:b, n - b:]
        gl, gr = O.gamma_of(sL), O.gamma_of(sR)
        for idx in rng.choice(n, 8, replace=False):
            dG0L = np.outer(Gd[:b, idx], Gd[idx, n - b:])
            dense_g = 2 * np.real(np.trace(gl @ dG0L @ gr @ G0L.conj().T))
            i, s = divmod(int(idx), b)
            assert abs(g[i, s] - dense_g) < 1e-10 * max(1, abs(dense_g))
            h = 1e-6
            Hp, Hm = wl.H.copy(), wl.H.copy()
            Hp[1, i, s, s] += h
            Hm[1, i, s, s] -= h
            Tp = O.solve_energy(Hp, 1, E, sL, sR)[1]
            Tm = O.solve_energy(Hm, 1, E, sL, sR)[1]
            assert abs((Tp - Tm) / (2 * h) - g[i, s]) < 1e-7


def test_pivot_noise_estimator_is_rounding_sized():
    """The u-perturbed second run used as a rounding-spread yardstick differs from the
    clean run by a rounding-sized amount on a well-conditioned system, and is a
    different computation (not bitwise equal)."""
    wl = make_random(12, 8, 1, 1, seed=21, eta=1e-3)
    args = (wl.H, wl.energies[0], wl.sigma_L[0], wl.sigma_R[0], 0.1)
    r = O.rgf(*args, extras=False)
    rn = O.rgf(*args, extras=False, pivot_noise=3)
    d = rel(rn["G"], r["G"])
    assert 0 < d < 1e-13
    Mb = O.block_accessor(wl.H, 1, *args[1:])
    r2 = O.nrgf(Mb, 12, 8, 1)
    rn2 = O.nrgf(Mb, 12, 8, 1, pivot_noise=3)
    assert 0 < rel(rn2["G"], r2["G"]) < 1e-13
