"""Pins of the oracle's extended-precision reference, its mixed-precision variant and
its band gradient against facts that do not come from the oracle itself:

  * exact integer inverses: the symmetric Pascal matrix (inverse known in closed
    form) for the long-double LU and solves, and block tridiagonal integer systems
    M = U~ D L~ (unit block bidiagonal U~, L~, unimodular integer pivots D_i), whose
    inverse is an integer matrix computed here with exact rational arithmetic.  The
    RGF of Algorithm 1 eliminates from the last layer, so its Schur pivots are
    exactly the D_i and their conditioning is set by construction;
  * dense FP64 inversion of small complex systems (the definition of bndiag(M^{-1}),
    Sec. 2 introduction), for w = 1, 2, 3;
  * central finite differences of T for the band gradient dT/dH.
"""
from fractions import Fraction
from math import comb

import numpy as np
import pytest

import oracle as O
from workloads import make_random


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, dtype=np.complex128) - b) / np.linalg.norm(b))


# ----------------------------------------------------------------------------
# exact integer test systems
# ----------------------------------------------------------------------------

def _unit_triangular(rng, b, k, lower):
    A = np.eye(b, dtype=np.int64)
    for i in range(b):
        for j in range(b):
            if (i > j) if lower else (i < j):
                A[i, j] = rng.integers(-k, k + 1)
    return A


def integer_udl(l, b, kd, ko, seed):
    """Integer block tridiagonal M = U~ D L~ as a band (M itself, not H) plus the
    dense integer matrix.  D_i = (unit lower)(unit upper) with entries in [-kd, kd]
    (determinant 1), U~_{i,i+1}, L~_{i+1,i} with entries in [-ko, ko]."""
    rng = np.random.default_rng(seed)
    D = [_unit_triangular(rng, b, kd, True) @ _unit_triangular(rng, b, kd, False) for _ in range(l)]
    X = [rng.integers(-ko, ko + 1, (b, b)) for _ in range(l - 1)]
    Y = [rng.integers(-ko, ko + 1, (b, b)) for _ in range(l - 1)]
    n = l * b
    Ut = np.eye(n, dtype=object)
    Lt = np.eye(n, dtype=object)
    Dd = np.zeros((n, n), dtype=object)
    for i in range(l):
        Dd[i * b:(i + 1) * b, i * b:(i + 1) * b] = D[i]
        if i + 1 < l:
            Ut[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = X[i]
            Lt[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = Y[i]
    return Ut.dot(Dd).dot(Lt)


def exact_inverse(M):
    """Inverse of an integer matrix by Gauss-Jordan elimination over the rationals."""
    n = M.shape[0]
    A = [[Fraction(int(M[i, j])) for j in range(n)] + [Fraction(int(i == j)) for j in range(n)]
         for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[p] = A[p], A[c]
        pv = A[c][c]
        A[c] = [x / pv for x in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return np.array([[A[i][n + j] for j in range(n)] for i in range(n)], dtype=object)


def as_oracle_input(M, l, b):
    """(H, sigma) such that M(E = 0) = -H with zero self-energies: H = -M."""
    Mf = np.array(M, dtype=np.float64)
    H = np.zeros((3, l, b, b), dtype=np.complex128)
    for i in range(l):
        for k in (-1, 0, 1):
            j = i + k
            if 0 <= j < l:
                H[1 + k, i] = -Mf[i * b:(i + 1) * b, j * b:(j + 1) * b]
    return H, np.zeros((b, b), dtype=np.complex128)


def band_of(Gdense, l, b):
    out = np.zeros((3, l, b, b), dtype=np.complex128)
    for i in range(l):
        for k in (-1, 0, 1):
            j = i + k
            if 0 <= j < l:
                out[1 + k, i] = np.array(Gdense[i * b:(i + 1) * b, j * b:(j + 1) * b], dtype=np.float64)
    return out


# ----------------------------------------------------------------------------
# extended-precision LU and solves
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n", [8, 10, 12])
def test_ext_lu_inverts_pascal_matrix(n):
    """P_n[i][j] = C(i+j, i) = L L^T with L[i][j] = C(i, j), so P_n^{-1} = L^{-T} L^{-1}
    with L^{-1}[i][j] = (-1)^(i-j) C(i, j): an exact integer inverse with kappa up to
    ~1e12.  The long-double LU must beat LAPACK's FP64 inverse by the ratio of the
    two unit roundoffs (2^-53 / 2^-64 = 2048, asserted with margin: 200) and stay
    within n * 2^-64 * kappa."""
    P = np.array([[comb(i + j, i) for j in range(n)] for i in range(n)], dtype=np.float64)
    Linv = np.array([[(-1) ** (i - j) * comb(i, j) for j in range(n)] for i in range(n)], dtype=object)
    Pinv = Linv.T.dot(Linv).astype(np.float64)
    kappa = np.linalg.norm(P, 1) * np.linalg.norm(Pinv, 1)
    e64 = rel(np.linalg.inv(P), Pinv)
    lu = O.lu_factor_ext(P.astype(np.complex128))
    X = O.lu_solve_ext(lu, np.eye(n, dtype=np.complex128))
    Y = O.lu_solve_right_ext(np.eye(n, dtype=np.complex128), lu)
    for Z in (X, Y):
        ez = rel(Z, Pinv)
        assert ez <= e64 / 200.0, (ez, e64)
        assert ez <= n * 2.0 ** -64 * kappa, (ez, kappa)


def test_ext_solves_complex_random():
    """Left and right solves on a random complex matrix with row pivoting actually
    needed (small leading entry): residuals at the long-double level."""
    rng = np.random.default_rng(5)
    n = 9
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A[0, 0] = 1e-9
    B = rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4))
    lu = O.lu_factor_ext(A)
    assert lu[1][0] != 0                     # the first pivot row was swapped
    X = O.lu_solve_ext(lu, B)
    Al = A.astype(np.clongdouble)
    assert np.abs(Al @ X - B).max() < 1e-16 * np.abs(B).max() * n
    Y = O.lu_solve_right_ext(B.T.copy(), lu)
    assert np.abs(Y @ Al - B.T).max() < 1e-16 * np.abs(B).max() * n


# ----------------------------------------------------------------------------
# extended-precision selected inverse
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("l,b,w", [(1, 4, 1), (2, 3, 1), (9, 5, 1), (12, 8, 1), (7, 4, 2), (10, 3, 3)])
def test_ext_matches_dense(l, b, w):
    wl = make_random(l, b, w, 2, seed=3100 + 10 * l + b, eta=1e-3)
    for e in range(wl.ne):
        args = (wl.H, w, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e])
        ref, G = O.dense_selected(*args, full=True)
        Gx, Tx = O.solve_energy_ext(*args)
        assert rel(Gx, ref) < 1e-13
        Tref = O.transmission(G[:b, (l - 1) * b:], wl.sigma_L[e], wl.sigma_R[e])
        assert abs(Tx - Tref) < 1e-12 * max(1.0, abs(Tref))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_ext_matches_exact_integer_inverse(seed):
    """Ill-conditioned integer systems (pivot kappa 3e2..3e3, |G| up to ~1e6): the
    extended-precision RGF reproduces the exact rational inverse's band."""
    l, b = 6, 4
    M = integer_udl(l, b, 2, 2, seed)
    exact = band_of(exact_inverse(M), l, b)
    H, z = as_oracle_input(M, l, b)
    Gx, _ = O.solve_energy_ext(H, 1, 0.0, z, z)
    assert rel(Gx, exact) < 1e-12


# ----------------------------------------------------------------------------
# mixed-precision variant
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed,kd", [(0, 2), (1, 2), (2, 4), (3, 4), (4, 4)])
def test_mixed_products_exact_where_fp32_products_are_exact(seed, kd):
    """On integer systems whose multipliers, Schur updates and band blocks are
    integers below 2^24, every FP32 product is exact (operands round to the same
    integers), so the written-out mixed variant must reproduce the exact inverse:
    any dropped term, wrong sign or transposed operand in it shows up as an O(1)
    difference."""
    l, b = 6, 4
    M = integer_udl(l, b, kd, 2, seed)
    Gex = exact_inverse(M)
    assert max(abs(int(x)) for x in Gex.flat) < 2 ** 24
    exact = band_of(Gex, l, b)
    H, z = as_oracle_input(M, l, b)
    m = O.rgf_mixed_products(H, 0.0, z, z)
    assert rel(m["G"], exact) < 1e-14
    # the first block row's last block (behind T) as well
    np.testing.assert_allclose(m["G_0_last"], np.array(Gex[:b, (l - 1) * b:], dtype=np.float64), rtol=0,
                               atol=1e-14 * np.abs(exact).max())


def test_mixed_products_error_is_fp32_rounding_times_pivot_conditioning():
    """On a well-conditioned random system the mixed variant differs from the FP64
    RGF by FP32 rounding (2^-24 ~ 6e-8) amplified at most by the worst Schur pivot's
    condition number: more than 1e-9 (the products really are rounded) and less than
    10 * kappa * 2^-24."""
    wl = make_random(16, 16, 1, 3, seed=77, eta=1e-3)
    for e in range(wl.ne):
        args = (wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], 0.5)
        r = O.rgf(*args, extras=False, pivot_cond=True)
        m = O.rgf_mixed_products(*args)
        err = rel(m["G"], r["G"])
        assert 1e-9 < err < 10.0 * r["pivot_cond"] * 2.0 ** -24, (err, r["pivot_cond"])


# ----------------------------------------------------------------------------
# band gradient dT/dH
# ----------------------------------------------------------------------------

def test_grad_band_finite_differences():
    """dT/dH for entries of every kind of band block (lower, diagonal, upper), real
    and imaginary parts separately, against central differences of T."""
    wl = make_random(5, 3, 1, 2, seed=61, eta=1e-3)
    rng = np.random.default_rng(1)
    h = 1e-6
    for e in range(wl.ne):
        E, sL, sR = wl.energies[e], wl.sigma_L[e], wl.sigma_R[e]
        T, gH = O.grad_band(wl.H, E, sL, sR)
        assert abs(T - O.solve_energy(wl.H, 1, E, sL, sR)[1]) < 1e-13
        for _ in range(12):
            k = int(rng.integers(-1, 2))
            i = int(rng.integers(max(0, -k), 5 - max(0, k)))
            a, c = (int(x) for x in rng.integers(0, 3, 2))
            for part, unit in (("re", 1.0), ("im", 1j)):
                Hp, Hm = wl.H.copy(), wl.H.copy()
                Hp[1 + k, i, a, c] += h * unit
                Hm[1 + k, i, a, c] -= h * unit
                fd = (O.solve_energy(Hp, 1, E, sL, sR)[1] - O.solve_energy(Hm, 1, E, sL, sR)[1]) / (2 * h)
                g = gH[1 + k, i, a, c]
                an = g.real if part == "re" else g.imag
                assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (k, i, a, c, part, fd, an)
        # blocks outside the matrix are zero; the diagonal's real part is the on-site gradient
        assert np.all(gH[0, 0] == 0) and np.all(gH[2, 4] == 0)
        _, g_on = O.grad_onsite(wl.H, E, sL, sR)
        np.testing.assert_allclose(np.real(np.diagonal(gH[1], axis1=1, axis2=2)), g_on, rtol=0, atol=1e-12)
