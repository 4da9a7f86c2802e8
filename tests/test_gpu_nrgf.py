"""GPU parity of the block n-diagonal paths (n = 2w + 1) against the FP64 oracle.

* sequential: the native n-diagonal sweep (Sec. 2.3) vs the oracle's n-RGF; bound
  1e-10 per energy, at the full size max(1e-10, 2 e_noise) with e_noise the
  oracle's own rounding spread (the largest of three runs with u-perturbed Schur pivots);
* DDRGF with separators of w layers: distance to the exact band no larger than
  4x the oracle DDRGF's own (see test_gpu_ddrgf).
"""
import numpy as np
import pytest

import oracle
from workloads import make_config, make_random

from test_gpu_rgf import mask_band, rel, run_gpu

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


def check_seq(wl, G, T, info, energies, eta_d=0.0, noise=False):
    assert np.all(info == 0), info
    for e in energies:
        Mb = oracle.block_accessor(wl.H, wl.w, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], eta_d)
        r = oracle.nrgf(Mb, wl.l, wl.b, wl.w, halo=1)
        Tref = oracle.transmission(r["first_rows"][0, wl.l - 1], wl.sigma_L[e], wl.sigma_R[e])
        tol = 1e-10
        if noise:
            # the largest of three perturbed oracle runs (see test_gpu_rgf.check_energies)
            # (drawn until the bound holds: the maximum of three is never below them)
            err0 = rel(mask_band(G[e], wl.w), r["G"])
            terr0 = abs(T[e] - Tref) / max(1.0, abs(Tref))
            for s in range(3):
                rn = oracle.nrgf(Mb, wl.l, wl.b, wl.w, halo=1, pivot_noise=1000 + e + 100000 * s)
                Tn = oracle.transmission(rn["first_rows"][0, wl.l - 1], wl.sigma_L[e], wl.sigma_R[e])
                tol = max(tol, 2.0 * max(rel(rn["G"], r["G"]), abs(Tn - Tref) / max(1.0, abs(Tref))))
                print(f"energy {e}: |dG|/|G| {err0:.2e}, bound {tol:.2e} after {s + 1} samples", flush=True)
                if err0 <= tol and terr0 <= tol:
                    break
        err = rel(mask_band(G[e], wl.w), r["G"])
        assert err <= tol, (e, err, tol)
        assert abs(T[e] - Tref) <= tol * max(1.0, abs(Tref)), (e, T[e], Tref)


def check_dd(wl, G, T, info, energies, m, eta_d=0.0):
    assert np.all(info == 0), info
    for e in energies:
        args = (wl.H, wl.w, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], eta_d)
        if wl.l * wl.b <= 2500:
            ref, Gf = oracle.dense_selected(*args, full=True)
            n, b = wl.l * wl.b, wl.b
            Tref = oracle.transmission(Gf[:b, n - b:], wl.sigma_L[e], wl.sigma_R[e])
        else:
            Mb = oracle.block_accessor(*args)
            r = oracle.nrgf(Mb, wl.l, wl.b, wl.w, halo=1)
            ref = r["G"]
            Tref = oracle.transmission(r["first_rows"][0, wl.l - 1], wl.sigma_L[e], wl.sigma_R[e])
        d = oracle.ddrgf(*args, n_pairs=m)
        tol = max(1e-10, 4.0 * rel(d["G"], ref))
        err = rel(mask_band(G[e], wl.w), ref)
        assert err <= tol, (e, err, tol)
        assert abs(T[e] - Tref) <= tol * max(1.0, abs(Tref)), (e, T[e], Tref)


@pytest.mark.parametrize("l,b,w", [(3, 8, 2), (9, 16, 2), (14, 20, 2), (11, 37, 3), (8, 64, 2),
                                   (6, 100, 2), (10, 5, 4), (7, 128, 2)])
def test_native_ndiagonal(lib, l, b, w):
    wl = make_random(l, b, w, 2, seed=1300 + l * 3 + b + w, eta=1e-3)
    G, T, info = run_gpu(lib, wl)
    check_seq(wl, G, T, info, range(2))


@pytest.mark.parametrize("l,b,w,m", [(8, 8, 2, 2), (20, 16, 2, 4), (24, 20, 2, 5), (18, 12, 3, 2),
                                     (40, 64, 2, 8), (12, 32, 2, 3)])
def test_ddrgf_ndiagonal(lib, l, b, w, m):
    wl = make_random(l, b, w, 2, seed=1700 + l + b + w + m, eta=1e-3)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=m)
    check_dd(wl, G, T, info, range(2), m)


def test_config3_full_size_sequential(lib):
    """Block pentadiagonal, 512 layers x 64, 128 energies, native n-diagonal sweep."""
    wl = make_config(3)
    G, T, info = run_gpu(lib, wl)
    check_seq(wl, G, T, info, [127], noise=True)


def test_config3_full_size_ddrgf(lib):
    """Same system, DDRGF with 16 domains (separators of 2 layers; the reduced system
    is block tridiagonal in 2-layer groups)."""
    wl = make_config(3)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=16)
    check_dd(wl, G, T, info, [64], 16)
