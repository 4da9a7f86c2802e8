"""GPU parity of DDRGF (Algorithm 2) against the FP64 oracle, through the C ABI.

DDRGF inverts closed interiors (no lead, no broadening).  For the random,
non-diagonally-dominant generator used here their Schur pivots are at some
energies far worse conditioned than M itself, and the method's own rounding
error - measured with the oracle's DDRGF against the exact band - reaches
1e-10..1e-7 where sequential RGF stays near 1e-13.  Bound per energy, with
ref = the exact band (dense inverse when small, else the oracle's RGF, accurate
to ~1e-12 here) and e_dd = |oracle DDRGF - ref| / |ref|:
    |G_gpu - ref| / |ref| <= max(1e-10, 4 e_dd),   same relative bound for T.
"""
import numpy as np
import pytest

import oracle
from workloads import make_config, make_random

from test_gpu_rgf import mask_band, rel, run_gpu

pytestmark = pytest.mark.gpu


def check(wl, G, T, info, energies, m, eta_d=0.0):
    assert np.all(info == 0), info
    for e in energies:
        args = (wl.H, wl.w, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], eta_d)
        if wl.l * wl.b <= 2500:
            ref, G_full = oracle.dense_selected(*args, full=True)
            b, n = wl.b, wl.l * wl.b
            Tref = oracle.transmission(G_full[:b, n - b:], wl.sigma_L[e], wl.sigma_R[e])
        else:
            ref, Tref = oracle.solve_energy(*args, method="rgf")
        d = oracle.ddrgf(*args, n_pairs=m)
        e_dd = rel(d["G"], ref)
        tol = max(1e-10, 4.0 * e_dd)
        err = rel(mask_band(G[e], wl.w), ref)
        assert err <= tol, (e, err, e_dd)
        assert abs(T[e] - Tref) <= tol * max(1.0, abs(Tref)), (e, T[e], Tref, e_dd)


def test_config1_two_domains(lib):
    wl = make_config(1)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=wl.domains)
    check(wl, G, T, info, range(wl.ne), wl.domains)


@pytest.mark.parametrize("l,b,m", [(5, 8, 1), (2, 4, 1), (10, 20, 3), (9, 64, 4), (33, 37, 4),
                                   (40, 48, 8), (7, 128, 3), (20, 100, 5), (12, 1, 2)])
def test_ragged_layouts(lib, l, b, m):
    wl = make_random(l, b, 1, 2, seed=900 + l + b, eta=1e-3)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=m)
    check(wl, G, T, info, range(2), m)


def test_with_device_broadening(lib):
    wl = make_random(30, 32, 1, 3, seed=77, eta=1e-3)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=4, eta_d=0.02)
    check(wl, G, T, info, range(3), 4, eta_d=0.02)


def test_config2_full_size_sampled(lib):
    """The 256 x 128 system with 8 domains over all 64 energies (the benchmark launch);
    three energies compared with the oracle block by block."""
    wl = make_config(2)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=8)
    check(wl, G, T, info, [0, 33, 63], 8)


def test_singular_interior_pivot_reported(lib):
    """A closed interior whose last layer is exactly E I - H = 0: the first pivot of
    that interior is singular and its global layer is reported."""
    wl = make_random(10, 8, 1, 2, seed=5, eta=1e-3)
    # 2 pairs: interiors [0..3], [5..8]; separators 4, 9.  Zero the pivot of layer 3.
    wl.H[1, 3] = wl.energies[0] * np.eye(8)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=2)
    assert info[0] == 4 and info[1] == 0
    assert np.all(np.isnan(G[0])) and np.isnan(T[0])


def test_kernel_timing_marks(lib):
    """With timing enabled, every DDRGF kernel is reported once per solve with a
    positive duration, and the results are bitwise those of an untimed solve."""
    import torch
    from paper_2605_19910_amd import binding
    wl = make_random(12, 24, 1, 3, seed=31, eta=1e-3)
    G0, T0, info0 = run_gpu(lib, wl, method="ddrgf", domains=3)
    dev = torch.device("cuda:0")
    H, sL, sR, E = (torch.from_numpy(x).to(dev) for x in (wl.H, wl.sigma_L, wl.sigma_R, wl.energies))
    plan = binding.Plan(wl.l, wl.b, wl.w, wl.ne, method="ddrgf", domains=3)
    plan.set_timing(True, 64)
    for _ in range(2):
        G, T, info = binding.solve(H, sL, sR, E, eta_d=wl.eta_d, plan=plan)
    times = plan.kernel_times()
    torch.cuda.synchronize()
    for k in ("ddrgf_interior_kernel", "ddrgf_schur_kernel", "rgf_sweep_kernel", "ddrgf_recover_kernel",
              "ddrgf_finalize_kernel"):
        assert k in times, times
        assert times[k][1] == 2 and times[k][0] > 0.0, (k, times[k])
    assert np.all(info.cpu().numpy() == 0)
    # blocks outside the matrix are never written: compare inside the band only
    assert np.array_equal(mask_band(G.cpu().numpy(), wl.w), mask_band(G0, wl.w))
    assert np.array_equal(T.cpu().numpy(), T0)
    plan.set_timing(False)
    plan.close()
