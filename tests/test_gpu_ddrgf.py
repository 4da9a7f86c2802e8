"""GPU parity of DDRGF (Algorithm 2) against the FP64 oracle, through the C ABI.

The GPU runs the same algorithm as oracle.ddrgf (closed interiors, reduced
separator system with the inter-separator couplings, recovery), so it is compared
with it element by element, under the DDRGF rule of tests/parity.py: within
max(2 b u kappa_max, 8 e_method), e_method being the oracle DDRGF's own distance to
the exact band.  DDRGF's closed interiors have no lead and no broadening; near
their eigenvalues the recovery cancels a large interior inverse and the method is
much less accurate than sequential RGF.  The GPU's distance to the exact band is
printed beside the comparison.
"""
import numpy as np
import pytest

from parity import check_dd, oracle_results
from test_gpu_rgf import free_gpu, run_gpu, run_gpu_dev
from workloads import make_config, make_dominant, make_random

pytestmark = pytest.mark.gpu


def check_small(label, wl, G, T, info, m, eta_d=None):
    assert np.all(info == 0), info
    es = range(wl.ne)
    refs = oracle_results("ddrgf", wl, es, eta_d=eta_d, m=m)
    exact = oracle_results("dense", wl, es, eta_d=eta_d)
    check_dd(label, G, T, es, refs, exact, wl.w)


def test_config1_two_domains(lib):
    wl = make_config(1)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=wl.domains)
    check_small("config1 ddrgf", wl, G, T, info, wl.domains)


@pytest.mark.parametrize("l,b,m", [(5, 8, 1), (2, 4, 1), (10, 20, 3), (9, 64, 4), (33, 37, 4),
                                   (40, 48, 8), (7, 128, 3), (20, 100, 5), (12, 1, 2)])
def test_ragged_layouts(lib, l, b, m):
    wl = make_random(l, b, 1, 2, seed=900 + l + b, eta=1e-3)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=m)
    check_small(f"ddrgf l={l} b={b} m={m}", wl, G, T, info, m)


def test_with_device_broadening(lib):
    wl = make_random(30, 32, 1, 3, seed=77, eta=1e-3)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=4, eta_d=0.02)
    check_small("ddrgf eta_d", wl, G, T, info, 4, eta_d=0.02)


def test_non_hermitian_h(lib):
    """H not Hermitian (the library does not assume it): the interiors take the
    general path instead of the Hermitian one, against the oracle's DDRGF."""
    wl = make_random(20, 24, 1, 2, seed=33, eta=1e-3)
    rng = np.random.default_rng(4)
    wl.H[2, :19] += 0.05 * (rng.standard_normal((19, 24, 24)) + 1j * rng.standard_normal((19, 24, 24)))
    wl.H[1, 7, 3, 5] += 0.1
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=4)
    check_small("ddrgf non-Hermitian H", wl, G, T, info, 4)


def test_config2_all_energies(lib):
    """The 256 x 128 system with 8 domains over all 64 energies (the benchmark
    launch), every band block and T against the oracle's DDRGF."""
    wl = make_config(2)
    G, T, info = run_gpu_dev(lib, wl, method="ddrgf", domains=8)
    assert bool((info == 0).all())
    refs = oracle_results("ddrgf", ("config", 2), range(wl.ne), m=8)
    exact = oracle_results("rgf", ("config", 2), range(wl.ne))
    check_dd("config2 ddrgf", G, T.cpu().numpy(), range(wl.ne), refs, exact, 1)
    del G
    free_gpu()


def test_dominant_full_size(lib):
    """256 x 128, 64 energies, 8 domains on a block diagonally dominant system (the
    paper's class of test matrices): every energy within the DDRGF rule, which here
    comes down to the FP64 target, against the oracle's DDRGF and the exact band."""
    src = ("dominant", 256, 128, 1, 64, 202)
    wl = make_dominant(*src[1:])
    G, T, info = run_gpu_dev(lib, wl, method="ddrgf", domains=8)
    assert bool((info == 0).all())
    refs = oracle_results("ddrgf", src, range(wl.ne), m=8)
    exact = oracle_results("rgf", src, range(wl.ne))
    rows = check_dd("dominant 256x128 ddrgf", G, T.cpu().numpy(), range(wl.ne), refs, exact, 1)
    assert max(r[3] for r in rows) <= 1e-9, "the rule should be tight on a well-conditioned system"
    del G
    free_gpu()


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
    from parity import mask_band
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
